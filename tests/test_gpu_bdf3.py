"""GPU tests of the third-order stepper through the C-ABI: BDF3 (Sec. 4.1)
with two SDIRK2 start-up steps (Sec. 4.2, 4.4), against the FP64 oracle.

  - one BDF3 step and one SDIRK2 step at fixed iteration counts:
    <= 1e-12 relative, histories rotated in place;
  - ch_solve to tolerance: identical iteration counts, <= 1e-12 relative;
  - FP32 sweeps against the FP64 oracle: max-abs error on u <= 1e-5.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1611_04214_amd import molt, synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    molt.load()
    oracle.build(force=False)


def _og(g):
    return oracle.Grid(nx=g.nx, ny=g.ny, x0=g.x0, x1=g.x1, y0=g.y0, y1=g.y1, bc=g.bc, M=g.order_M)


CASES = [
    # (name, nx, ny, x1, y1, bc, eps, dt): both branches of the stepper
    # (beta*dt below and above eps^2), both boundary kinds, 1D and 2D
    ("1d_periodic", 256, 1, 2 * np.pi, 1.0, 0, 0.05, 1e-3),
    ("2d_periodic_cs", 48, 40, 1.0, 0.8, 0, 0.02, 1e-4),
    ("2d_periodic_fact", 48, 40, 1.0, 0.8, 0, 0.02, 1e-3),
    ("2d_neumann_fact", 45, 33, 1.0, 0.7, 1, 0.03, 2e-3),
]


def _fields(c, seed=31):
    _, nx, ny = c[:3]
    rng = np.random.default_rng(seed)
    u = 0.4 * rng.uniform(-1, 1, (ny, nx)).squeeze()
    up = u + 0.01 * rng.uniform(-1, 1, u.shape)
    up2 = up + 0.01 * rng.uniform(-1, 1, u.shape)
    return u, up, up2


def _grid(c, M=4):
    _, nx, ny, x1, y1, bc = c[:6]
    return molt.make_grid(nx, ny, 0.0, x1, 0.0, y1, bc, M)


@pytest.mark.parametrize("c", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("init", [molt.MOLT_INIT_PREV, molt.MOLT_INIT_LINEAR])
def test_bdf3_step_fixed_iterations_fp64(c, init):
    g = _grid(c)
    eps, dt = c[6], c[7]
    u, up, up2 = _fields(c)
    print(f"bdf3 step {c[0]} init={init}", flush=True)
    for fi in (1, 3):
        po = oracle.Params(eps=eps, dt=dt, stepper=oracle.BDF3, init=init, fixed_iters=fi)
        ref, rinfo = oracle.bdf3_step(_og(g), po, u, up, up2)
        p = molt.make_params(eps, dt, stepper=molt.MOLT_BDF3, init=init, precision=molt.MOLT_F64,
                             fixed_iters=fi, have_prev=2)
        x = torch.tensor(u, dtype=torch.float64, device=DEV)
        hist = torch.tensor(np.stack([up, up2]), dtype=torch.float64, device=DEV)
        info = molt.step(x, g, p, hist)
        got = x.cpu().numpy()
        assert info.iters == fi
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), (fi, np.abs(got - ref).max())
        h = hist.cpu().numpy()
        assert np.array_equal(h[0], u) and np.array_equal(h[1], up)  # [u^n | u^{n-1}]
        assert abs(info.s1 - rinfo.s1) <= 1e-14 * rinfo.s1 and abs(info.sigma - rinfo.sigma) <= 1e-14 * rinfo.sigma
        assert abs(info.mass - rinfo.mass) <= 1e-12 * max(1.0, abs(rinfo.mass))
        assert abs(info.energy - rinfo.energy) <= 1e-12 * abs(rinfo.energy)


@pytest.mark.parametrize("c", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("have_prev", [0, 1])
def test_sdirk2_step_fixed_iterations_fp64(c, have_prev):
    """Fewer than two histories: an SDIRK2 step (two BE stages of eta*dt)."""
    g = _grid(c)
    eps, dt = c[6], c[7]
    u, up, _ = _fields(c, seed=32)
    fi = 3
    po = oracle.Params(eps=eps, dt=dt, stepper=oracle.BDF3, fixed_iters=fi)
    ref, rinfo = oracle.sdirk2_step(_og(g), po, u)
    p = molt.make_params(eps, dt, stepper=molt.MOLT_BDF3, precision=molt.MOLT_F64, fixed_iters=fi,
                         have_prev=have_prev)
    x = torch.tensor(u, dtype=torch.float64, device=DEV)
    hist = torch.tensor(np.stack([up, np.zeros_like(up)]), dtype=torch.float64, device=DEV)
    info = molt.step(x, g, p, hist)
    got = x.cpu().numpy()
    assert info.iters == 2 * fi == rinfo.iters
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), np.abs(got - ref).max()
    h = hist.cpu().numpy()
    assert np.array_equal(h[0], u) and np.array_equal(h[1], up)
    assert abs(info.energy - rinfo.energy) <= 1e-12 * abs(rinfo.energy)
    # without a history buffer the step is the same
    x2 = torch.tensor(u, dtype=torch.float64, device=DEV)
    molt.step(x2, g, p, None)
    assert torch.equal(x2, x)


@pytest.mark.parametrize("bc,M", [(molt.MOLT_BC_NEUMANN, 4), (molt.MOLT_BC_PERIODIC, 6)])
def test_bdf3_solve_to_tolerance_fp64(bc, M):
    """Two SDIRK2 steps then BDF3, tol 1e-11: the oracle's iteration counts,
    <= 1e-12 relative, mass and energy."""
    g = molt.make_grid(40, 36, 0.0, 1.0, 0.0, 0.9, bc, M)
    u0 = synth.u0_uniform_noise(synth.BASE_SEED + 41, 36, 40, 0.3)
    po = oracle.Params(eps=0.04, dt=3e-4, tol=1e-11, stepper=oracle.BDF3, max_iter=4000)
    ref, rinf = oracle.solve(_og(g), po, u0, 7)
    x = torch.tensor(u0, dtype=torch.float64, device=DEV)
    p = molt.make_params(0.04, 3e-4, tol=1e-11, stepper=molt.MOLT_BDF3, max_iter=4000, precision=molt.MOLT_F64)
    st, infos = molt.solve(x, g, p, 7)
    print("bdf3 solve iters gpu", [i.iters for i in infos], "oracle", [i.iters for i in rinf], flush=True)
    assert st == molt.MOLT_OK
    assert [i.iters for i in infos] == [i.iters for i in rinf]
    assert np.abs(x.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    for a, b in zip(infos, rinf):
        assert abs(a.mass - b.mass) <= 1e-12 * max(1.0, abs(b.mass))
        assert abs(a.energy - b.energy) <= 1e-12 * abs(b.energy)


@pytest.mark.parametrize("bc", [molt.MOLT_BC_PERIODIC, molt.MOLT_BC_NEUMANN])
def test_bdf3_solve_fp32_against_fp64_oracle(bc):
    """FP32 sweeps, 12 BDF3 steps of a 96^2 quench (tol 1e-8 vs the oracle's
    1e-11): max-abs error on u <= 1e-5."""
    n = 96
    g = molt.make_grid(n, n, 0.0, 1.0, 0.0, 1.0, bc, 4)
    u0 = synth.u0_uniform_noise(synth.BASE_SEED + 42, n, n, 0.05)
    po = oracle.Params(eps=0.02, dt=5e-5, tol=1e-11, stepper=oracle.BDF3, max_iter=5000, init=oracle.INIT_LINEAR)
    ref, rinf = oracle.solve(_og(g), po, u0, 12)
    x = torch.tensor(u0, dtype=torch.float32, device=DEV)
    p = molt.make_params(0.02, 5e-5, tol=1e-8, stepper=molt.MOLT_BDF3, max_iter=5000, init=molt.MOLT_INIT_LINEAR,
                         precision=molt.MOLT_F32)
    st, infos = molt.solve(x, g, p, 12)
    err = np.abs(x.cpu().double().numpy() - ref)
    print(f"bdf3 fp32 bc={bc}: max-abs {err.max():.3e} iters gpu {[i.iters for i in infos][:5]} "
          f"oracle {[i.iters for i in rinf][:5]}", flush=True)
    assert st == molt.MOLT_OK
    assert err.max() <= 1e-5
