"""GPU parity of the vector (three-phase) Cahn-Hilliard model (Sec. 5.2)
through the C-ABI against the FP64 oracle: <= 1e-12 relative in FP64 at equal
iteration counts, <= 1e-5 max-abs on u in FP32; the batched path bitwise
equal to ch_solve for vector-model instances mixed with scalar ones."""
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


CASES = [  # (name, nx, ny, bc, eps, dt): dt >= eps^2/81 is the factorization branch
    ("per_cs", 40, 36, 0, 0.03, 5e-6),
    ("per_fact", 40, 36, 0, 0.03, 5e-5),
    ("neu_cs", 45, 33, 1, 0.04, 1e-5),
    ("neu_fact", 45, 33, 1, 0.02, 2e-5),
    ("1d_per", 96, 1, 0, 0.03, 2e-5),
]


@pytest.mark.parametrize("name,nx,ny,bc,eps,dt", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("stepper", ["BE", "BDF2"])
@pytest.mark.parametrize("init", [molt.MOLT_INIT_PREV, molt.MOLT_INIT_LINEAR])
def test_vch_step_fixed_iterations_fp64(name, nx, ny, bc, eps, dt, stepper, init):
    g = molt.make_grid(nx, ny, 0.0, 1.0, 0.0, max(ny, 2) / nx, bc, 4)
    u = synth.u0_vch(synth.BASE_SEED + 70, ny, nx)
    up = synth.u0_vch(synth.BASE_SEED + 71, ny, nx)
    bdf2 = stepper == "BDF2"
    print(f"vch step {name} {stepper} init={init}", flush=True)
    for fi in (1, 2, 5):
        po = oracle.Params(eps=eps, dt=dt, stepper=oracle.BDF2 if bdf2 else oracle.BE, init=init, fixed_iters=fi,
                           sigma0=oracle.VCH_SIGMA0)
        ref, rinfo = oracle.vch_step(_og(g), po, u, up if bdf2 else None)
        p = molt.make_params(eps, dt, stepper=molt.MOLT_BDF2 if bdf2 else molt.MOLT_BE, init=init,
                             precision=molt.MOLT_F64, fixed_iters=fi, have_prev=1 if bdf2 else 0,
                             model=molt.MOLT_MODEL_VCH)
        x = torch.tensor(u, dtype=torch.float64, device=DEV)
        xp = torch.tensor(up, dtype=torch.float64, device=DEV)
        info = molt.step(x, g, p, xp)
        got = x.cpu().numpy()
        assert info.iters == fi
        err = np.abs(got - ref).max()
        assert err <= 1e-12 * np.abs(ref).max(), (fi, err)
        assert np.array_equal(xp.cpu().numpy(), u)  # history rotated
        assert abs(info.sigma - rinfo.sigma) <= 1e-14 * rinfo.sigma
        assert abs(info.mass - rinfo.mass) <= 1e-12 * max(1.0, abs(rinfo.mass))
        assert abs(info.mass2 - rinfo.mass2) <= 1e-12 * max(1.0, abs(rinfo.mass2))
        assert abs(info.energy - rinfo.energy) <= 1e-12 * abs(rinfo.energy)


@pytest.mark.parametrize("bc", [molt.MOLT_BC_PERIODIC, molt.MOLT_BC_NEUMANN])
def test_vch_solve_to_tolerance_fp64(bc):
    g = molt.make_grid(48, 40, 0.0, 1.0, 0.0, 40 / 48, bc, 4)
    u0 = synth.u0_vch(synth.BASE_SEED + 72, 40, 48)
    po = oracle.Params(eps=0.03, dt=2e-5, tol=1e-11, stepper=oracle.BDF2, max_iter=5000, init=oracle.INIT_LINEAR,
                       sigma0=oracle.VCH_SIGMA0)
    ref, rinf = oracle.vch_solve(_og(g), po, u0, 4)
    x = torch.tensor(u0, dtype=torch.float64, device=DEV)
    p = molt.make_params(0.03, 2e-5, tol=1e-11, stepper=molt.MOLT_BDF2, max_iter=5000, init=molt.MOLT_INIT_LINEAR,
                         precision=molt.MOLT_F64, model=molt.MOLT_MODEL_VCH)
    st, infos = molt.solve(x, g, p, 4)
    assert st == molt.MOLT_OK
    assert [i.iters for i in infos] == [i.iters for i in rinf]
    assert np.abs(x.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    e = [i.energy for i in infos]
    assert all(e[k + 1] <= e[k] for k in range(len(e) - 1))


@pytest.mark.parametrize("bc", [molt.MOLT_BC_PERIODIC, molt.MOLT_BC_NEUMANN])
def test_vch_fp32_against_fp64_oracle(bc):
    n = 80
    g = molt.make_grid(n, n, 0.0, 1.0, 0.0, 1.0, bc, 4)
    u0 = synth.u0_vch(synth.BASE_SEED + 73, n, n)
    po = oracle.Params(eps=0.02, dt=1e-5, tol=1e-11, stepper=oracle.BDF2, max_iter=8000, init=oracle.INIT_LINEAR,
                       sigma0=oracle.VCH_SIGMA0)
    ref, rinf = oracle.vch_solve(_og(g), po, u0, 8)
    x = torch.tensor(u0, dtype=torch.float32, device=DEV)
    p = molt.make_params(0.02, 1e-5, tol=1e-8, stepper=molt.MOLT_BDF2, max_iter=8000, init=molt.MOLT_INIT_LINEAR,
                         precision=molt.MOLT_F32, model=molt.MOLT_MODEL_VCH)
    st, infos = molt.solve(x, g, p, 8)
    err = np.abs(x.cpu().double().numpy() - ref)
    print(f"vch fp32 bc={bc}: max-abs {err.max():.3e} L2 {np.sqrt((err ** 2).mean()):.3e} "
          f"iters {[i.iters for i in infos]} oracle {[i.iters for i in rinf]}", flush=True)
    assert st == molt.MOLT_OK
    assert err.max() <= 1e-5


@pytest.mark.parametrize("prec", [molt.MOLT_F32, molt.MOLT_F64], ids=["f32", "f64"])
def test_vch_batch_equals_single_problem_path(prec):
    dt_ = torch.float64 if prec == molt.MOLT_F64 else torch.float32
    tol = 1e-11 if prec == molt.MOLT_F64 else 1e-8
    cases = [(64, 48, 0, molt.MOLT_MODEL_VCH, 3), (90, 70, 1, molt.MOLT_MODEL_VCH, 2),
             (70, 64, 0, molt.MOLT_MODEL_CH, 3), (40, 120, 1, molt.MOLT_MODEL_VCH, 4)]
    specs, plain = [], []
    for i, (nx, ny, bc, model, ns) in enumerate(cases):
        g = molt.make_grid(nx, ny, 0.0, 1.0, 0.0, ny / nx, bc, 4)
        p = molt.make_params(0.03, 2e-5, tol=tol, stepper=molt.MOLT_BDF2, max_iter=6000, init=molt.MOLT_INIT_LINEAR,
                             precision=prec, model=model)
        u0 = (synth.u0_vch(synth.BASE_SEED + 80 + i, ny, nx) if model == molt.MOLT_MODEL_VCH
              else synth.u0_uniform_noise(synth.BASE_SEED + 80 + i, ny, nx, 0.05))
        x = torch.tensor(u0, dtype=dt_, device=DEV)
        _, infos = molt.solve(x, g, p, ns)
        plain.append((x.cpu(), [r.iters for r in infos], [r.mass2 for r in infos]))
        specs.append((g, p, torch.tensor(u0, dtype=dt_, device=DEV), ns))
    st, recs = molt.solve_batch(specs)
    assert st == molt.MOLT_OK
    for k, (_, _, x, _) in enumerate(specs):
        assert [r.iters for r in recs[k]] == plain[k][1], k
        assert [r.mass2 for r in recs[k]] == plain[k][2], k
        assert torch.equal(x.cpu(), plain[k][0]), k
