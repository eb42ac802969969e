"""GPU time steps with Dirichlet walls through the C-ABI against the FP64 oracle.

The walls hold the homogeneous condition of the shifted variable (v = u + 1,
eq. CahnHilliard_v; the vector model's v = u - z3), so the inputs carry
u = -1 (u = z3) on every wall node.  Bars: FP64 <= 1e-12 relative at equal
iteration counts, FP32 <= 1e-5 max-abs on u; the walls keep their value.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1611_04214_amd import molt, synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
Z3 = (-0.5, -np.sqrt(3.0) / 2.0)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    molt.load()
    oracle.build(force=False)


def _og(g):
    return oracle.Grid(nx=g.nx, ny=g.ny, x0=g.x0, x1=g.x1, y0=g.y0, y1=g.y1, bc=g.bc, M=g.order_M)


def _walls(a):
    a = np.asarray(a)
    if a.ndim == 1:
        return a[[0, -1]]
    return np.concatenate([a[0, :], a[-1, :], a[:, 0], a[:, -1]])


CASES = [
    # (name, nx, ny, y1, eps, dt, M): both branches, 1D and 2D, ragged shapes
    ("1d_cs", 129, 1, 1.0, 0.05, 1e-3, 4),
    ("1d_fact", 129, 1, 1.0, 0.05, 5e-3, 6),
    ("2d_cs", 45, 33, 0.7, 0.03, 2e-4, 4),
    ("2d_fact", 45, 33, 0.7, 0.03, 2e-3, 2),
]
# several x tiles and y segments and a ragged tail: one stepper, one initial iterate
TILES = ("2d_tiles", 530, 300, 0.56, 0.01, 1e-4, 4)
STEPPERS = {"BE": (molt.MOLT_BE, oracle.BE), "BDF2": (molt.MOLT_BDF2, oracle.BDF2),
            "BDF3": (molt.MOLT_BDF3, oracle.BDF3)}


def _fields(nx, ny, seed):
    rng = np.random.default_rng(seed)
    sh = (nx,) if ny == 1 else (ny, nx)
    u = synth.with_walls(0.4 * rng.uniform(-1, 1, sh), -1.0)
    up = synth.with_walls(u + 0.01 * rng.uniform(-1, 1, sh), -1.0)
    up2 = synth.with_walls(up + 0.01 * rng.uniform(-1, 1, sh), -1.0)
    return u, up, up2


STEP_PARAMS = [(c, s, i) for c in CASES for s in STEPPERS for i in (molt.MOLT_INIT_PREV, molt.MOLT_INIT_LINEAR)]
STEP_PARAMS.append((TILES, "BDF2", molt.MOLT_INIT_LINEAR))


@pytest.mark.parametrize("c,stepper,init", STEP_PARAMS, ids=[f"{c[0]}-{s}-{i}" for c, s, i in STEP_PARAMS])
def test_dirichlet_step_fixed_iterations_fp64(c, stepper, init):
    name, nx, ny, y1, eps, dt, M = c
    g = molt.make_grid(nx, ny, 0.0, 1.0, 0.0, y1, molt.MOLT_BC_DIRICHLET, M)
    u, up, up2 = _fields(nx, ny, 51)
    ms, os_ = STEPPERS[stepper]
    nh = {"BE": 0, "BDF2": 1, "BDF3": 2}[stepper]
    print(f"dirichlet step {name} {stepper} init={init}", flush=True)
    for fi in (1, 4):
        po = oracle.Params(eps=eps, dt=dt, stepper=os_, init=init, fixed_iters=fi)
        if stepper == "BDF3":
            ref, rinfo = oracle.bdf3_step(_og(g), po, u, up, up2)
            hist = torch.tensor(np.stack([up, up2]), dtype=torch.float64, device=DEV)
        else:
            ref, rinfo = oracle.step(_og(g), po, u, up if nh else None)
            hist = torch.tensor(up, dtype=torch.float64, device=DEV)
        p = molt.make_params(eps, dt, stepper=ms, init=init, precision=molt.MOLT_F64, fixed_iters=fi,
                             have_prev=nh)
        x = torch.tensor(u, dtype=torch.float64, device=DEV)
        info = molt.step(x, g, p, hist)
        got = x.cpu().numpy()
        assert info.iters == fi
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), (fi, np.abs(got - ref).max())
        assert np.abs(_walls(got) + 1.0).max() <= 1e-13
        # history rotated (through the in-place shift: to one rounding)
        h = hist.cpu().numpy()
        h0 = h[0] if stepper == "BDF3" else h
        assert np.abs(h0 - u).max() <= 4e-16
        if stepper == "BDF3":
            assert np.abs(h[1] - up).max() <= 4e-16
        assert abs(info.s1 - rinfo.s1) <= 1e-14 * rinfo.s1 and abs(info.sigma - rinfo.sigma) <= 1e-14 * rinfo.sigma
        assert abs(info.mass - rinfo.mass) <= 1e-12 * max(1.0, abs(rinfo.mass))
        assert abs(info.energy - rinfo.energy) <= 1e-12 * abs(rinfo.energy)


@pytest.mark.parametrize("stepper", ["BDF2", "BDF3"])
def test_dirichlet_solve_to_tolerance_fp64(stepper):
    g = molt.make_grid(40, 36, 0.0, 1.0, 0.0, 0.9, molt.MOLT_BC_DIRICHLET, 4)
    u0 = synth.with_walls(synth.u0_uniform_noise(synth.BASE_SEED + 52, 36, 40, 0.3), -1.0)
    ms, os_ = STEPPERS[stepper]
    po = oracle.Params(eps=0.04, dt=3e-4, tol=1e-11, stepper=os_, max_iter=4000)
    ref, rinf = oracle.solve(_og(g), po, u0, 6)
    x = torch.tensor(u0, dtype=torch.float64, device=DEV)
    p = molt.make_params(0.04, 3e-4, tol=1e-11, stepper=ms, max_iter=4000, precision=molt.MOLT_F64)
    st, infos = molt.solve(x, g, p, 6)
    print(f"dirichlet solve {stepper} iters gpu", [i.iters for i in infos], "oracle", [i.iters for i in rinf],
          flush=True)
    assert st == molt.MOLT_OK
    assert [i.iters for i in infos] == [i.iters for i in rinf]
    got = x.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(_walls(got) + 1.0).max() <= 1e-13
    for a, b in zip(infos, rinf):
        assert abs(a.energy - b.energy) <= 1e-12 * abs(b.energy)


def test_dirichlet_solve_fp32_against_fp64_oracle():
    """FP32 sweeps, 20 BDF2 steps of a 96^2 quench between walls at -1 (tol
    1e-8 vs the oracle's 1e-11): max-abs error on u <= 1e-5."""
    n = 96
    g = molt.make_grid(n, n, 0.0, 1.0, 0.0, 1.0, molt.MOLT_BC_DIRICHLET, 4)
    u0 = synth.with_walls(synth.u0_uniform_noise(synth.BASE_SEED + 53, n, n, 0.05), -1.0)
    po = oracle.Params(eps=0.02, dt=5e-5, tol=1e-11, stepper=oracle.BDF2, max_iter=5000, init=oracle.INIT_LINEAR)
    ref, rinf = oracle.solve(_og(g), po, u0, 20)
    x = torch.tensor(u0, dtype=torch.float32, device=DEV)
    p = molt.make_params(0.02, 5e-5, tol=1e-8, stepper=molt.MOLT_BDF2, max_iter=5000, init=molt.MOLT_INIT_LINEAR,
                         precision=molt.MOLT_F32)
    st, infos = molt.solve(x, g, p, 20)
    err = np.abs(x.cpu().double().numpy() - ref)
    print(f"dirichlet fp32: max-abs {err.max():.3e} iters gpu {[i.iters for i in infos][:5]} "
          f"oracle {[i.iters for i in rinf][:5]}", flush=True)
    assert st == molt.MOLT_OK
    assert err.max() <= 1e-5


VCH_CASES = [  # (name, nx, ny, eps, dt): dt >= eps^2/81 is the factorization branch
    ("vch_cs", 40, 36, 0.03, 5e-6),
    ("vch_fact", 40, 36, 0.03, 5e-5),
    ("vch_1d", 96, 1, 0.03, 2e-5),
]


@pytest.mark.parametrize("name,nx,ny,eps,dt", VCH_CASES, ids=[c[0] for c in VCH_CASES])
@pytest.mark.parametrize("stepper", ["BE", "BDF2"])
def test_vch_dirichlet_step_fixed_iterations_fp64(name, nx, ny, eps, dt, stepper):
    g = molt.make_grid(nx, ny, 0.0, 1.0, 0.0, max(ny, 2) / nx, molt.MOLT_BC_DIRICHLET, 4)
    u = synth.with_walls(synth.u0_vch(synth.BASE_SEED + 54, ny, nx), Z3)
    up = synth.with_walls(synth.u0_vch(synth.BASE_SEED + 55, ny, nx), Z3)
    bdf2 = stepper == "BDF2"
    for fi in (1, 4):
        po = oracle.Params(eps=eps, dt=dt, stepper=oracle.BDF2 if bdf2 else oracle.BE, fixed_iters=fi,
                           sigma0=oracle.VCH_SIGMA0)
        ref, rinfo = oracle.vch_step(_og(g), po, u, up if bdf2 else None)
        p = molt.make_params(eps, dt, stepper=molt.MOLT_BDF2 if bdf2 else molt.MOLT_BE, precision=molt.MOLT_F64,
                             fixed_iters=fi, have_prev=1 if bdf2 else 0, model=molt.MOLT_MODEL_VCH)
        x = torch.tensor(u, dtype=torch.float64, device=DEV)
        xp = torch.tensor(up, dtype=torch.float64, device=DEV)
        info = molt.step(x, g, p, xp)
        got = x.cpu().numpy()
        assert info.iters == fi
        err = np.abs(got - ref).max()
        assert err <= 1e-12 * np.abs(ref).max(), (fi, err)
        for k in range(2):
            assert np.abs(_walls(got[k].squeeze()) - Z3[k]).max() <= 1e-13
        assert abs(info.mass - rinfo.mass) <= 1e-12 * max(1.0, abs(rinfo.mass))
        assert abs(info.mass2 - rinfo.mass2) <= 1e-12 * max(1.0, abs(rinfo.mass2))
        assert abs(info.energy - rinfo.energy) <= 1e-12 * abs(rinfo.energy)


def test_dirichlet_adaptive_matches_oracle_fp64():
    """Algorithm 1 between Dirichlet walls: the oracle driver's trial steps,
    decisions and iteration counts, and its final field."""
    g = molt.make_grid(45, 33, 0.0, 1.0, 0.0, 33 / 45, molt.MOLT_BC_DIRICHLET, 4)
    u0 = synth.with_walls(synth.u0_uniform_noise(synth.BASE_SEED + 56, 33, 45, 0.05), -1.0)
    eps, t_end, dt0, tol, nmaxit = 0.04, 3e-3, 2e-5, 5e-4, 400
    po = oracle.Params(eps=eps, dt=dt0, tol=1e-11)
    ref, rrec = oracle.adaptive_solve(_og(g), po, u0, oracle.AdaptParams(t_end=t_end, dt0=dt0, lte_tol=tol,
                                                                         nmaxit=nmaxit))
    x = torch.tensor(u0, dtype=torch.float64, device=DEV)
    p = molt.make_params(eps, dt0, tol=1e-11, precision=molt.MOLT_F64)
    st, rec, tf = molt.solve_adaptive(x, g, p, molt.make_adapt(t_end, dt0, tol, nmaxit=nmaxit))
    print(f"dirichlet adaptive: {len(rec)} attempts", flush=True)
    assert st == molt.MOLT_OK and abs(tf - t_end) <= 1e-12 * t_end
    assert len(rec) == len(rrec)
    for r, (t, dt, eta, nit, ok) in zip(rec, rrec):
        assert bool(r.accepted) == ok and r.iters == nit
        assert abs(r.dt - dt) <= 1e-10 * dt
    assert np.abs(x.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()
