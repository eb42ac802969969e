"""GPU tests of ch_solve_batch (batched independent instances) through the C-ABI.

  - FP64 instances against the FP64 oracle at fixed iteration counts and to
    tolerance: <= 1e-12 relative, identical iteration counts.
  - FP32 instances against the FP64 oracle: max-abs error on u <= 1e-5.
  - An instance's result is bitwise the same alone and in a mixed batch, with
    the ticks launched one by one or replayed as a HIP graph, and bitwise the
    same as the single-problem ch_solve path.
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
    yield
    molt.molt_set_option(molt.MOLT_OPT_BATCH_TICKS, 8)
    molt.molt_set_option(molt.MOLT_OPT_BATCH_GRAPH, 1)
    molt.molt_set_option(molt.MOLT_OPT_BATCH_LEAN, LEAN_DEFAULT)


def _og(g):
    return oracle.Grid(nx=g.nx, ny=g.ny, x0=g.x0, x1=g.x1, y0=g.y0, y1=g.y1, bc=g.bc, M=g.order_M)


# (nx, ny, bc, M, eps, dt, stepper, init, nsteps): uneven shapes, both
# boundary kinds, all orders, both steppers and initial iterates, both
# branches of the stepper (factorization when beta*dt >= eps^2)
MIX = [
    (64, 48, 0, 4, 0.03, 1e-4, "BDF2", 1, 4),
    (97, 130, 1, 4, 0.02, 5e-5, "BE", 1, 3),
    (45, 33, 1, 2, 0.03, 2e-3, "BDF2", 0, 3),
    (200, 70, 0, 6, 0.01, 2e-5, "BE", 0, 2),
    (33, 260, 0, 4, 0.02, 1e-3, "BDF2", 1, 5),
    (130, 129, 1, 6, 0.02, 3e-5, "BDF2", 1, 1),
]


def _case(c, prec, tol, fixed=0, max_iter=4000):
    nx, ny, bc, M, eps, dt, stp, init, ns = c
    g = molt.make_grid(nx, ny, 0.0, 1.0, 0.0, ny / nx, bc, M)
    p = molt.make_params(eps, dt, tol=tol, stepper=molt.MOLT_BDF2 if stp == "BDF2" else molt.MOLT_BE,
                         max_iter=max_iter, init=init, precision=prec, fixed_iters=fixed)
    return g, p, ns


def _u0(i, c):
    nx, ny = c[0], c[1]
    return synth.u0_uniform_noise(synth.BASE_SEED + 100 + i, ny, nx, 0.3, mean=0.05)


def _oracle(c, g, u0, tol, fixed=0, max_iter=4000):
    stp = oracle.BDF2 if c[6] == "BDF2" else oracle.BE
    po = oracle.Params(eps=c[4], dt=c[5], tol=tol, stepper=stp, max_iter=max_iter, init=c[7], fixed_iters=fixed)
    return oracle.solve(_og(g), po, u0, c[8])


@pytest.mark.parametrize("fixed", [3, 0], ids=["fixed3", "to_tol"])
def test_batch_fp64_matches_oracle(fixed):
    tol = 1e-11
    specs, refs = [], []
    for i, c in enumerate(MIX):
        g, p, ns = _case(c, molt.MOLT_F64, tol, fixed)
        u0 = _u0(i, c)
        refs.append(_oracle(c, g, u0, tol, fixed))
        specs.append((g, p, torch.tensor(u0, dtype=torch.float64, device=DEV), ns))
    print(f"batch fp64 vs oracle fixed={fixed}", flush=True)
    st, recs = molt.solve_batch(specs)
    assert st == molt.MOLT_OK
    for i, ((g, p, x, ns), (ref, rinf)) in enumerate(zip(specs, refs)):
        assert [r.iters for r in recs[i]] == [r.iters for r in rinf], i
        err = np.abs(x.cpu().numpy() - ref).max()
        assert err <= 1e-12 * np.abs(ref).max(), (i, err)
        for a, b in zip(recs[i], rinf):
            assert a.converged == 1
            assert abs(a.mass - b.mass) <= 1e-12 * max(1.0, abs(b.mass))
            assert abs(a.energy - b.energy) <= 1e-12 * abs(b.energy)
            assert abs(a.s1 - b.s1) <= 1e-14 * b.s1 and abs(a.sigma - b.sigma) <= 1e-14 * b.sigma


def test_batch_fp32_against_fp64_oracle():
    """FP32 sweeps, tolerance 1e-8 (oracle 1e-11): max-abs error on u <= 1e-5."""
    specs, refs = [], []
    for i, c in enumerate(MIX[:4]):
        g, p, ns = _case(c, molt.MOLT_F32, 1e-8)
        u0 = _u0(i, c)
        refs.append(_oracle(c, g, u0, 1e-11))
        specs.append((g, p, torch.tensor(u0, dtype=torch.float32, device=DEV), ns))
    st, recs = molt.solve_batch(specs)
    assert st == molt.MOLT_OK
    for i, ((g, p, x, ns), (ref, rinf)) in enumerate(zip(specs, refs)):
        err = np.abs(x.cpu().double().numpy() - ref)
        print(f"fp32 batch instance {i}: max-abs {err.max():.3e} L2 {np.sqrt((err ** 2).mean()):.3e} "
              f"iters {[r.iters for r in recs[i]]} oracle {[r.iters for r in rinf]}", flush=True)
        assert err.max() <= 1e-5, (i, err.max())


LEAN_DEFAULT = 16  # the library's default for MOLT_OPT_BATCH_LEAN


def _run_batch(idx, prec, ticks=8, graph=1, lean=LEAN_DEFAULT):
    assert molt.molt_set_option(molt.MOLT_OPT_BATCH_TICKS, ticks) == 0
    assert molt.molt_set_option(molt.MOLT_OPT_BATCH_GRAPH, graph) == 0
    assert molt.molt_set_option(molt.MOLT_OPT_BATCH_LEAN, lean) == 0
    dt = torch.float64 if prec == molt.MOLT_F64 else torch.float32
    specs = []
    for i in idx:
        g, p, ns = _case(MIX[i], prec, 1e-8 if prec == molt.MOLT_F32 else 1e-11)
        specs.append((g, p, torch.tensor(_u0(i, MIX[i]), dtype=dt, device=DEV), ns))
    s = torch.cuda.Stream()  # a non-default stream, so the graph path is taken
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        st, recs = molt.solve_batch(specs)
    torch.cuda.synchronize()
    return st, [x.cpu() for (_, _, x, _) in specs], recs


@pytest.mark.parametrize("prec", [molt.MOLT_F32, molt.MOLT_F64], ids=["f32", "f64"])
def test_batch_alone_equals_in_batch_bitwise(prec):
    full = list(range(len(MIX)))
    st, xs, recs = _run_batch(full, prec)
    assert st == molt.MOLT_OK
    for i in (0, 3, 5):
        st1, x1, r1 = _run_batch([i], prec)
        assert st1 == molt.MOLT_OK
        assert torch.equal(x1[0], xs[i]), i
        assert [(r.iters, r.residual, r.mass, r.energy) for r in r1[0]] == \
               [(r.iters, r.residual, r.mass, r.energy) for r in recs[i]]
    # reversed order, one tick per check, kernels launched one by one
    st2, xr, _ = _run_batch(full[::-1], prec, ticks=1, graph=0)
    for k, i in enumerate(full[::-1]):
        assert torch.equal(xr[k], xs[i]), i
    # lean ticks from the start (graph replay, and launched one by one), and never
    for lean, graph in ((1024, 1), (1024, 0), (0, 1)):
        st3, xl, rl = _run_batch(full, prec, graph=graph, lean=lean)
        assert st3 == molt.MOLT_OK
        for i in full:
            assert torch.equal(xl[i], xs[i]), (lean, graph, i)
            assert [(r.iters, r.residual, r.mass, r.energy) for r in rl[i]] == \
                   [(r.iters, r.residual, r.mass, r.energy) for r in recs[i]], (lean, graph, i)


@pytest.mark.parametrize("prec", [molt.MOLT_F32, molt.MOLT_F64], ids=["f32", "f64"])
def test_batch_equals_single_problem_path(prec):
    """The batched kernels run the single-problem kernels' device code: same
    fields bit for bit and the same iteration counts as ch_solve."""
    idx = list(range(len(MIX)))
    st, xs, recs = _run_batch(idx, prec)
    dt = torch.float64 if prec == molt.MOLT_F64 else torch.float32
    for i in idx:
        g, p, ns = _case(MIX[i], prec, 1e-8 if prec == molt.MOLT_F32 else 1e-11)
        x = torch.tensor(_u0(i, MIX[i]), dtype=dt, device=DEV)
        st1, infos = molt.solve(x, g, p, ns)
        assert [r.iters for r in infos] == [r.iters for r in recs[i]], i
        diff = (x.cpu() - xs[i]).abs().max().item()
        assert torch.equal(x.cpu(), xs[i]), (i, diff)


def test_batch_zero_steps_and_not_converged():
    g = molt.make_grid(64, 64, 0.0, 1.0, 0.0, 1.0, molt.MOLT_BC_PERIODIC, 4)
    u0 = synth.u0_uniform_noise(synth.BASE_SEED + 7, 64, 64, 0.3)
    p_ok = molt.make_params(0.02, 1e-4, tol=1e-11, max_iter=4000, precision=molt.MOLT_F64)
    p_cap = molt.make_params(0.02, 1e-4, tol=0.0, max_iter=3, precision=molt.MOLT_F64)
    xs = [torch.tensor(u0, dtype=torch.float64, device=DEV) for _ in range(3)]
    st, recs = molt.solve_batch([(g, p_ok, xs[0], 0), (g, p_cap, xs[1], 2), (g, p_ok, xs[2], 1)])
    assert st == molt.MOLT_NOT_CONVERGED
    assert np.array_equal(xs[0].cpu().numpy(), u0)  # no steps: unchanged
    assert [r.iters for r in recs[1]] == [3, 3] and all(r.converged == 0 for r in recs[1])
    ref, _ = oracle.solve(_og(g), oracle.Params(eps=0.02, dt=1e-4, fixed_iters=3), u0, 2)
    assert np.abs(xs[1].cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    assert recs[2][0].converged == 1


def test_batch_workload_sample_fp32():
    """Eight instances of the seeded 256-instance workload (sides 65..982),
    3 steps each, against plain ch_solve: identical fields and iterations."""
    inst = synth.batch_instances()
    pick = [0, 13, 37, 64, 101, 150, 199, 255]
    specs, plain = [], []
    for i in pick:
        d = inst[i]
        bc = molt.MOLT_BC_PERIODIC if d["bc"] == "periodic" else molt.MOLT_BC_NEUMANN
        g = molt.make_grid(d["n"], d["n"], 0.0, 1.0, 0.0, 1.0, bc, 4)
        p = molt.make_params(d["eps"], d["dt"], tol=d["tol"], max_iter=20000, init=molt.MOLT_INIT_LINEAR,
                             stepper=molt.MOLT_BDF2 if d["stepper"] == "BDF2" else molt.MOLT_BE,
                             precision=molt.MOLT_F32)
        u0 = synth.instance_u0(d)
        specs.append((g, p, torch.tensor(u0, dtype=torch.float32, device=DEV), 3))
        x = torch.tensor(u0, dtype=torch.float32, device=DEV)
        _, infos = molt.solve(x, g, p, 3)
        plain.append((x.cpu(), [r.iters for r in infos]))
    print("workload sample sides", [inst[i]["n"] for i in pick], flush=True)
    st, recs = molt.solve_batch(specs)
    assert st == molt.MOLT_OK
    for k, (g, p, x, ns) in enumerate(specs):
        assert [r.iters for r in recs[k]] == plain[k][1], k
        assert torch.equal(x.cpu(), plain[k][0]), k
