"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Tolerances (stated here, derived in the design notes):
  FP64 mode: max|gpu - oracle| <= 1e-12 * max|oracle| (relative), at equal
             iteration counts (fixed_iters, or identical counts under tol).
  FP32 sweeps: max abs error <= 6e-8 * (M + 4 + 2/(1 - d)) * max|in|: a few
             ulps per stencil term plus the scan's accumulation over the
             decay length 1/(1-d) of the recursion.
  FP32 steps: max abs error on u <= 1e-5 (the target), stated per case.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1611_04214_amd import molt, synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
BCS = [molt.MOLT_BC_PERIODIC, molt.MOLT_BC_NEUMANN, molt.MOLT_BC_DIRICHLET]


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    molt.load()
    oracle.build(force=False)


def _og(g: molt.molt_grid) -> oracle.Grid:
    return oracle.Grid(nx=g.nx, ny=g.ny, x0=g.x0, x1=g.x1, y0=g.y0, y1=g.y1, bc=g.bc, M=g.order_M)


def _f32_sweep_tol(M, nu, scale):
    d = np.exp(-nu)
    return 6e-8 * (M + 4 + 2.0 / (1.0 - d)) * scale


def _h(g, axis):
    n = g.nx if axis == 0 else g.ny
    a, b = (g.x0, g.x1) if axis == 0 else (g.y0, g.y1)
    return (b - a) / (n if g.bc == molt.MOLT_BC_PERIODIC else n - 1)


# ------------------------------------------------------------------ sweeps --
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("M", [2, 4, 6])
@pytest.mark.parametrize("shape", [(37, 300), (530, 1030), (7, 9)])
def test_sweep_matches_oracle(bc, M, shape):
    """Both axes, both precisions, ragged sizes spanning several threads,
    waves and y-segments; nu from 0.07 to 2.5."""
    ny, nx = shape
    if min(nx, ny) < M + 1:
        pytest.skip("line shorter than M+1")
    g = molt.make_grid(nx, ny, 0.0, 1.3, -0.2, 0.9, bc, M)
    u = synth.u0_uniform_noise(synth.BASE_SEED + 17, ny, nx, 1.0)
    print(f"sweep case bc={bc} M={M} shape={shape}", flush=True)
    for axis in (0, 1):
        h = _h(g, axis)
        for nu in (0.07, 2.5):
            alpha = nu / h
            ref = oracle.sweep(_og(g), axis, alpha, u)
            scale = np.abs(ref).max()
            for dt, prec in ((torch.float64, molt.MOLT_F64), (torch.float32, molt.MOLT_F32)):
                x = torch.tensor(u, dtype=dt, device=DEV)
                y = molt.sweep(x, g, axis, alpha)
                torch.cuda.synchronize()
                err = np.abs(y.cpu().double().numpy() - ref).max()
                tol = 1e-12 * scale if prec == molt.MOLT_F64 else _f32_sweep_tol(M, nu, 1.0)
                assert err <= tol, (axis, nu, prec, err, tol)


def test_sweep_batch_and_in_place():
    g = molt.make_grid(96, 70, 0.0, 1.0, 0.0, 2.0, molt.MOLT_BC_NEUMANN, 4)
    u = synth.u0_uniform_noise(synth.BASE_SEED + 5, 3 * 70, 96, 1.0).reshape(3, 70, 96)
    for axis in (0, 1):
        ref = np.stack([oracle.sweep(_og(g), axis, 40.0, u[b]) for b in range(3)])
        x = torch.tensor(u, dtype=torch.float64, device=DEV)
        molt.sweep(x, g, axis, 40.0, out=x)  # in place
        torch.cuda.synchronize()
        assert np.abs(x.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


def test_sweep_full_size_sampled_lines():
    """The 4096^2 periodic FP32 field of the roofline workload, in the launch
    configuration the benchmark times: sampled rows and columns against the
    oracle applied to those lines alone."""
    n = 4096
    g = molt.make_grid(n, n, 0.0, 1.0, 0.0, 1.0, molt.MOLT_BC_PERIODIC, 4)
    u = synth.workload_u0("ch2d_periodic_bdf2_4096")
    x = torch.tensor(u, dtype=torch.float32, device=DEV)
    alpha = 278.3
    yx = molt.sweep(x, g, 0, alpha).cpu().double().numpy()
    yy = molt.sweep(x, g, 1, alpha).cpu().double().numpy()
    rng = np.random.default_rng(3)
    lg = oracle.Grid(nx=n, x0=0.0, x1=1.0, bc=0, M=4)
    nu = alpha / n
    tol = _f32_sweep_tol(4, nu, np.abs(u).max())
    for r in rng.choice(n, 6, replace=False):
        ref = oracle.sweep(lg, 0, alpha, u[r])
        assert np.abs(yx[r] - ref).max() <= tol
        ref = oracle.sweep(lg, 0, alpha, u[:, r])
        assert np.abs(yy[:, r] - ref).max() <= tol
    # mass of a periodic sweep equals the mass of its input (mean preserved)
    assert abs(yx.mean() - u.mean()) < 1e-6 and abs(yy.mean() - u.mean()) < 1e-6


# ------------------------------------------------------------------- steps --
STEP_CASES = [
    # (name, grid kwargs, eps, dt)
    ("1d_periodic_cs", dict(nx=256, ny=1, x1=2 * np.pi, bc=0), 0.05, 1e-3),
    ("1d_neumann_fact", dict(nx=129, ny=1, x1=1.0, bc=1), 0.05, 5e-3),
    ("2d_periodic_cs", dict(nx=48, ny=40, x1=1.0, y1=0.8, bc=0), 0.02, 1e-4),
    ("2d_periodic_fact", dict(nx=48, ny=40, x1=1.0, y1=0.8, bc=0), 0.02, 1e-3),
    ("2d_neumann_cs", dict(nx=45, ny=33, x1=1.0, y1=0.7, bc=1), 0.03, 2e-4),
    ("2d_neumann_fact", dict(nx=45, ny=33, x1=1.0, y1=0.7, bc=1), 0.03, 2e-3),
]


def _mk(kw, M=4):
    return molt.make_grid(kw["nx"], kw["ny"], 0.0, kw["x1"], 0.0, kw.get("y1", 1.0), kw["bc"], M)


@pytest.mark.parametrize("name,kw,eps,dt", STEP_CASES, ids=[c[0] for c in STEP_CASES])
@pytest.mark.parametrize("stepper", ["BE", "BDF2"])
@pytest.mark.parametrize("init", [molt.MOLT_INIT_PREV, molt.MOLT_INIT_LINEAR])
def test_step_fixed_iterations_fp64(name, kw, eps, dt, stepper, init):
    """One step at fixed iteration counts (1, 2, 6): <= 1e-12 relative."""
    g = _mk(kw)
    rng = np.random.default_rng(21)
    u = 0.4 * rng.uniform(-1, 1, (g.ny, g.nx)).squeeze()
    up = u + 0.01 * rng.uniform(-1, 1, u.shape)
    bdf2 = stepper == "BDF2"
    print(f"step case {name} {stepper} init={init}", flush=True)
    for fi in (1, 2, 6):
        po = oracle.Params(eps=eps, dt=dt, stepper=oracle.BDF2 if bdf2 else oracle.BE, init=init, fixed_iters=fi)
        ref, rinfo = oracle.step(_og(g), po, u, up if bdf2 else None)
        p = molt.make_params(eps, dt, stepper=molt.MOLT_BDF2 if bdf2 else molt.MOLT_BE, init=init,
                             precision=molt.MOLT_F64, fixed_iters=fi, have_prev=1 if bdf2 else 0)
        x = torch.tensor(u, dtype=torch.float64, device=DEV)
        xp = torch.tensor(up, dtype=torch.float64, device=DEV)
        info = molt.step(x, g, p, xp)
        got = x.cpu().numpy()
        assert info.iters == fi
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), (fi, np.abs(got - ref).max())
        assert np.abs(xp.cpu().numpy() - u).max() == 0.0  # history rotated: u_prev <- u^n
        assert abs(info.s1 - rinfo.s1) <= 1e-14 * rinfo.s1 and abs(info.s2 - rinfo.s2) <= 1e-14 * rinfo.s1
        assert abs(info.mass - rinfo.mass) <= 1e-12 * max(1.0, abs(rinfo.mass))
        assert abs(info.energy - rinfo.energy) <= 1e-12 * abs(rinfo.energy)


@pytest.mark.parametrize("M", [2, 6])
def test_step_to_tolerance_fp64(M):
    """Converged steps (tol 1e-11): same iteration count and <= 1e-12 relative."""
    g = molt.make_grid(40, 36, 0.0, 1.0, 0.0, 0.9, molt.MOLT_BC_NEUMANN, M)
    u = synth.u0_uniform_noise(synth.BASE_SEED + 9, 36, 40, 0.3)
    po = oracle.Params(eps=0.04, dt=3e-4, tol=1e-11, stepper=oracle.BE, max_iter=2000)
    ref, rinfo = oracle.step(_og(g), po, u)
    x = torch.tensor(u, dtype=torch.float64, device=DEV)
    info = molt.step(x, g, molt.make_params(0.04, 3e-4, tol=1e-11, max_iter=2000, precision=molt.MOLT_F64))
    assert info.converged == 1
    # the oracle's last increment is under the tolerance by far more than
    # FP64 rounding of an increment (~1e-16 absolute), so rounding cannot move
    # the stopping iteration: the counts must be equal
    assert po.tol - rinfo.residual > 1e-3 * po.tol
    assert info.iters == rinfo.iters
    assert abs(info.residual - rinfo.residual) <= 1e-3 * po.tol
    assert np.abs(x.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


def test_not_converged_status():
    """max_iter reached: the state is advanced and ch_step returns +1."""
    g = molt.make_grid(32, 32, 0.0, 1.0, 0.0, 1.0, molt.MOLT_BC_PERIODIC, 4)
    u = synth.u0_uniform_noise(synth.BASE_SEED + 1, 32, 32, 0.3)
    x = torch.tensor(u, dtype=torch.float64, device=DEV)
    p = molt.make_params(0.02, 1e-4, tol=0.0, max_iter=3, precision=molt.MOLT_F64)
    work = molt.workspace(molt.ch_workspace_bytes(g, p))
    info = molt.molt_step_info()
    rc = molt.ch_step(g, p, x.data_ptr(), 0, work.data_ptr(), work.numel(), info,
                      torch.cuda.current_stream().cuda_stream)
    assert rc == molt.MOLT_NOT_CONVERGED and info.iters == 3 and info.converged == 0
    po = oracle.Params(eps=0.02, dt=1e-4, fixed_iters=3)
    ref, _ = oracle.step(_og(g), po, u)
    assert np.abs(x.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


def test_solve_1d_workload_fp64():
    """The 1D workload (N=256 periodic, eps 0.05, dt 1e-3, BE, tol 1e-10, 200
    steps, M=4, FP64) end to end: same iteration counts, <= 1e-12 relative."""
    w = synth.WORKLOADS["ch1d_be_n256"]
    g = molt.make_grid(256, 1, 0.0, 2 * np.pi, 0.0, 1.0, molt.MOLT_BC_PERIODIC, 4)
    u0 = synth.workload_u0("ch1d_be_n256")
    po = oracle.Params(eps=w["eps"], dt=w["dt"], tol=w["tol"], stepper=oracle.BE, max_iter=1000)
    ref, rinf = oracle.solve(_og(g), po, u0, w["steps"])
    x = torch.tensor(u0, dtype=torch.float64, device=DEV)
    p = molt.make_params(w["eps"], w["dt"], tol=w["tol"], max_iter=1000, precision=molt.MOLT_F64)
    st, infos = molt.solve(x, g, p, w["steps"])
    it_g = [i.iters for i in infos]
    it_o = [i.iters for i in rinf]
    assert st == molt.MOLT_OK
    assert it_g == it_o
    assert np.abs(x.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    e = [i.energy for i in infos]
    assert all(e[k + 1] <= e[k] + 1e-12 * abs(e[k]) for k in range(len(e) - 1))


@pytest.mark.parametrize("bc", [molt.MOLT_BC_PERIODIC, molt.MOLT_BC_NEUMANN])
def test_solve_fp32_against_fp64_oracle(bc):
    """FP32 sweeps (increment form) vs the FP64 oracle over 20 BDF2 steps of a
    96^2 noisy quench (tol 1e-8 vs 1e-11): max-abs error on u <= 1e-5."""
    n = 96
    g = molt.make_grid(n, n, 0.0, 1.0, 0.0, 1.0, bc, 4)
    u0 = synth.u0_uniform_noise(synth.BASE_SEED + 2, n, n, 0.05)
    po = oracle.Params(eps=0.02, dt=5e-5, tol=1e-11, stepper=oracle.BDF2, max_iter=5000, init=oracle.INIT_LINEAR)
    ref, rinf = oracle.solve(_og(g), po, u0, 20)
    x = torch.tensor(u0, dtype=torch.float32, device=DEV)
    p = molt.make_params(0.02, 5e-5, tol=1e-8, stepper=molt.MOLT_BDF2, max_iter=5000, init=molt.MOLT_INIT_LINEAR,
                         precision=molt.MOLT_F32)
    st, infos = molt.solve(x, g, p, 20)
    err = np.abs(x.cpu().double().numpy() - ref)
    print(f"fp32 bc={bc}: max-abs {err.max():.3e}  L2 {np.sqrt((err ** 2).mean()):.3e}  "
          f"iters gpu {[i.iters for i in infos][:6]} oracle {[i.iters for i in rinf][:6]}", flush=True)
    assert st == molt.MOLT_OK
    assert err.max() <= 1e-5


@pytest.mark.parametrize("bc", [molt.MOLT_BC_PERIODIC, molt.MOLT_BC_NEUMANN])
@pytest.mark.parametrize("shape", [(256, 300), (200, 320), (520, 192)])
def test_deferred_ypass_ragged_shapes(shape, bc):
    """The single-read y-pass leaves segment-local scans and seeds that the next
    x-pass adds: ragged column strips, a ragged last segment and rows of a
    segment spread over several x-pass blocks, against the oracle at fixed
    iteration counts (one BE step of 4 iterations, then 3 BDF2 steps of 40):
    FP64 <= 1e-12 relative, FP32 <= 1e-5."""
    ny, nx = shape
    g = molt.make_grid(nx, ny, 0.0, 1.0, 0.0, ny / nx, bc, 4)
    u0 = synth.u0_uniform_noise(synth.BASE_SEED + 31, ny, nx, 0.3, mean=0.1)
    ref, _ = oracle.step(_og(g), oracle.Params(eps=0.02, dt=2e-4, fixed_iters=4), u0)
    ref3, _ = oracle.solve(_og(g), oracle.Params(eps=0.02, dt=2e-4, stepper=oracle.BDF2, fixed_iters=40), u0, 3)
    for prec, dt in ((molt.MOLT_F64, torch.float64), (molt.MOLT_F32, torch.float32)):
        x = torch.tensor(u0, dtype=dt, device=DEV)
        info = molt.step(x, g, molt.make_params(0.02, 2e-4, precision=prec, fixed_iters=4))
        assert info.iters == 4
        x2 = torch.tensor(u0, dtype=dt, device=DEV)
        p = molt.make_params(0.02, 2e-4, stepper=molt.MOLT_BDF2, precision=prec, fixed_iters=40)
        st, infos = molt.solve(x2, g, p, 3)
        assert st == molt.MOLT_OK and [i.iters for i in infos] == [40, 40, 40]
        e1 = np.abs(x.cpu().double().numpy() - ref).max()
        e3 = np.abs(x2.cpu().double().numpy() - ref3).max()
        print(f"deferred y-pass shape={shape} bc={bc} prec={prec}: step {e1:.2e} solve {e3:.2e}", flush=True)
        if prec == molt.MOLT_F64:
            assert e1 <= 1e-12 * np.abs(ref).max() and e3 <= 1e-12 * np.abs(ref3).max()
        else:
            assert e1 <= 1e-5 and e3 <= 1e-5
