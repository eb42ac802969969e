"""Runs of increment iterations launched as captured graphs (ch_step /
ch_solve) give bit-for-bit the results of launching every kernel on the
caller's stream: per step (graph replays between eager kernels and host
reads of the device state), on the default and on a side stream, after the
workspace or the line-block shape changes (new cache keys), and for more
distinct problems than the cache holds (evictions)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1611_04214_amd import molt, synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    molt.load()
    yield
    assert molt.molt_set_option(molt.MOLT_OPT_STEP_GRAPH, 1) == molt.MOLT_OK


def _graphs(on):
    assert molt.molt_set_option(molt.MOLT_OPT_STEP_GRAPH, 1 if on else 0) == molt.MOLT_OK


def _steps(u0, g, p, nsteps, work=None, stream=None):
    """nsteps single ch_step calls (BE start, then BDF2 with the history);
    the field after every step and the iteration counts."""
    dt = torch.float64 if p.precision == molt.MOLT_F64 else torch.float32
    x = torch.tensor(u0, dtype=dt, device=DEV)
    prev = torch.zeros_like(x)
    fields, iters = [], []
    ctx = torch.cuda.stream(stream) if stream is not None else torch.cuda.stream(torch.cuda.current_stream())
    with ctx:
        for k in range(nsteps):
            p.have_prev = 1 if k > 0 else 0
            info = molt.step(x, g, p, prev if p.stepper == molt.MOLT_BDF2 else None, work=work)
            assert info.converged == 1
            iters.append(info.iters)
            fields.append(x.cpu().numpy().copy())
    torch.cuda.synchronize()
    return fields, iters


@pytest.mark.parametrize("prec", [molt.MOLT_F64, molt.MOLT_F32])
@pytest.mark.parametrize("bc", [molt.MOLT_BC_PERIODIC, molt.MOLT_BC_NEUMANN])
def test_step_graph_equals_eager_launches(prec, bc):
    g = molt.make_grid(96, 80, 0.0, 1.0, 0.0, 0.8, bc, 4)
    u0 = synth.u0_uniform_noise(synth.BASE_SEED + 31, 80, 96, 0.3)
    # (the oracle takes 167, 111, 102, 83, 67 iterations periodic and
    # 592, 317, 290, 183, 137 with Neumann walls at tol 1e-10)
    p = molt.make_params(0.03, 1e-5, tol=1e-10 if prec == molt.MOLT_F64 else 1e-7, stepper=molt.MOLT_BDF2,
                         precision=prec, max_iter=5000)
    print(f"step graph case prec={prec} bc={bc}", flush=True)
    _graphs(False)
    ref, it_ref = _steps(u0, g, p, 5)
    _graphs(True)
    side = torch.cuda.Stream()
    for stream in (None, side):
        got, it_got = _steps(u0, g, p, 5, stream=stream)
        assert it_got == it_ref
        assert max(it_ref) >= 8  # runs of increment iterations were replayed
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)


def test_step_graph_new_workspace_and_shape():
    g = molt.make_grid(128, 128, 0.0, 1.0, 0.0, 1.0, molt.MOLT_BC_PERIODIC, 4)
    u0 = synth.u0_uniform_noise(synth.BASE_SEED + 32, 128, 128, 0.3)
    p = molt.make_params(0.02, 2e-5, tol=1e-8, stepper=molt.MOLT_BDF2, precision=molt.MOLT_F32, max_iter=5000)
    need = molt.ch_workspace_bytes(g, p)
    wa = molt.workspace(need, torch.device(DEV))
    wb = molt.workspace(need, torch.device(DEV))
    cls = 0
    while (128 << cls) < 128:
        cls += 1
    kx0, ky0 = molt.molt_tune_get(molt.MOLT_F32, cls)
    print("step graph case: workspaces and shapes", flush=True)
    try:
        for shape in ((kx0, ky0), (8, 4)):
            assert molt.molt_tune_set(molt.MOLT_F32, cls, *shape) == molt.MOLT_OK
            _graphs(False)
            ref, it_ref = _steps(u0, g, p, 3, work=wa)
            _graphs(True)
            for work in (wa, wb, wa):
                got, it_got = _steps(u0, g, p, 3, work=work)
                assert it_got == it_ref
                for a, b in zip(got, ref):
                    assert np.array_equal(a, b)
    finally:
        assert molt.molt_tune_set(molt.MOLT_F32, cls, kx0, ky0) == molt.MOLT_OK


def test_step_graph_evictions():
    """Ten distinct problems (more than the cache holds), each solved twice
    with graphs and once without: all three equal."""
    print("step graph case: evictions", flush=True)
    for i in range(10):
        n = 48 + 8 * i
        g = molt.make_grid(n, n, 0.0, 1.0, 0.0, 1.0, molt.MOLT_BC_PERIODIC, 4)
        u0 = synth.u0_uniform_noise(synth.BASE_SEED + 40 + i, n, n, 0.3)
        p = molt.make_params(0.03, 1e-5, tol=1e-10, stepper=molt.MOLT_BE, precision=molt.MOLT_F64, max_iter=5000)
        outs = []
        for on in (True, False, True):
            _graphs(on)
            x = torch.tensor(u0, dtype=torch.float64, device=DEV)
            st, infos = molt.solve(x, g, p, 2)
            assert st == molt.MOLT_OK
            outs.append((x.cpu().numpy(), [k.iters for k in infos]))
        assert outs[0][1] == outs[1][1] == outs[2][1]
        assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[2][0], outs[1][0])
    _graphs(True)
