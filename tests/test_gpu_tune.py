"""GPU tests of the line-block shape table: every shape against the FP64
oracle, the single-problem and batched paths bitwise equal under a non-default
table, and the autotuner producing a valid table."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1611_04214_amd import molt, synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(autouse=True)
def _restore_table():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    molt.load()
    oracle.build(force=False)
    saved = {p: molt.tune_table(p) for p in (molt.MOLT_F32, molt.MOLT_F64)}
    yield
    for p, tab in saved.items():
        for c, (kx, ky) in enumerate(tab):
            assert molt.molt_tune_set(p, c, kx, ky) == 0


def _og(g):
    return oracle.Grid(nx=g.nx, ny=g.ny, x0=g.x0, x1=g.x1, y0=g.y0, y1=g.y1, bc=g.bc, M=g.order_M)


SHAPES = {molt.MOLT_F32: [(4, 4), (8, 8), (16, 16), (32, 4)], molt.MOLT_F64: [(4, 4), (8, 8), (16, 4)]}


@pytest.mark.parametrize("prec", [molt.MOLT_F32, molt.MOLT_F64], ids=["f32", "f64"])
@pytest.mark.parametrize("bc", [molt.MOLT_BC_PERIODIC, molt.MOLT_BC_NEUMANN])
def test_every_shape_matches_oracle(prec, bc):
    """Sweeps along both axes and one fixed-iteration step, for every (kx, ky)
    on a 150 x 130 grid (class 1: ragged threads, segments and strips)."""
    g = molt.make_grid(150, 130, 0.0, 1.0, 0.0, 0.9, bc, 4)
    u = synth.u0_uniform_noise(synth.BASE_SEED + 41, 130, 150, 0.3, mean=0.1)
    dt = torch.float64 if prec == molt.MOLT_F64 else torch.float32
    po = oracle.Params(eps=0.02, dt=2e-4, stepper=oracle.BE, fixed_iters=3)
    ref_step, _ = oracle.step(_og(g), po, u)
    refs = [oracle.sweep(_og(g), ax, 90.0, u) for ax in (0, 1)]
    for kx, ky in SHAPES[prec]:
        assert molt.molt_tune_set(prec, 1, kx, ky) == 0
        print(f"shape kx={kx} ky={ky} prec={prec} bc={bc}", flush=True)
        for ax in (0, 1):
            y = molt.sweep(torch.tensor(u, dtype=dt, device=DEV), g, ax, 90.0)
            err = np.abs(y.cpu().double().numpy() - refs[ax]).max()
            tol = 1e-12 * np.abs(refs[ax]).max() if prec == molt.MOLT_F64 else 2e-6
            assert err <= tol, (kx, ky, ax, err)
        x = torch.tensor(u, dtype=dt, device=DEV)
        molt.step(x, g, molt.make_params(0.02, 2e-4, precision=prec, fixed_iters=3))
        err = np.abs(x.cpu().double().numpy() - ref_step).max()
        tol = 1e-12 * np.abs(ref_step).max() if prec == molt.MOLT_F64 else 1e-5
        assert err <= tol, (kx, ky, err)


def test_batch_equals_single_under_a_tuned_table():
    for c in range(4):
        assert molt.molt_tune_set(molt.MOLT_F32, c, 8, 4) == 0
    specs, plain = [], []
    for i, (nx, ny, bc) in enumerate([(100, 90, 0), (300, 257, 1), (64, 700, 0)]):
        g = molt.make_grid(nx, ny, 0.0, 1.0, 0.0, ny / nx, bc, 4)
        p = molt.make_params(0.02, 5e-5, tol=1e-8, stepper=molt.MOLT_BDF2, max_iter=5000,
                             init=molt.MOLT_INIT_LINEAR, precision=molt.MOLT_F32)
        u0 = synth.u0_uniform_noise(synth.BASE_SEED + 60 + i, ny, nx, 0.05)
        x = torch.tensor(u0, dtype=torch.float32, device=DEV)
        _, infos = molt.solve(x, g, p, 3)
        plain.append((x.cpu(), [r.iters for r in infos]))
        specs.append((g, p, torch.tensor(u0, dtype=torch.float32, device=DEV), 3))
    st, recs = molt.solve_batch(specs)
    assert st == molt.MOLT_OK
    for k, (_, _, x, _) in enumerate(specs):
        assert [r.iters for r in recs[k]] == plain[k][1]
        assert torch.equal(x.cpu(), plain[k][0]), k


def test_autotune_gives_a_valid_table():
    tab = molt.autotune(molt.MOLT_F32, 1024)
    print("tuned FP32 table", tab, flush=True)
    for c, (kx, ky) in enumerate(tab[:4]):
        assert kx in (4, 8, 16, 32) and ky in (4, 8, 16) and 128 << c <= 256 * kx
    # a step under the tuned table still matches the oracle
    g = molt.make_grid(96, 96, 0.0, 1.0, 0.0, 1.0, molt.MOLT_BC_NEUMANN, 4)
    u = synth.u0_uniform_noise(synth.BASE_SEED + 43, 96, 96, 0.3)
    ref, _ = oracle.step(_og(g), oracle.Params(eps=0.02, dt=2e-4, fixed_iters=4), u)
    x = torch.tensor(u, dtype=torch.float32, device=DEV)
    molt.step(x, g, molt.make_params(0.02, 2e-4, precision=molt.MOLT_F32, fixed_iters=4))
    assert np.abs(x.cpu().double().numpy() - ref).max() <= 1e-5
