"""GPU tests of the continuous-batching server (molt_server_*): requests that
arrive while others run are admitted as slots and memory free up, and every
result is bitwise the same alone and in the mix (and the same as ch_solve)."""
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


def _req(i, n, steps, bc, stepper, prec=molt.MOLT_F32, model=molt.MOLT_MODEL_VCH, eps=0.03, dt=2e-5):
    g = molt.make_grid(n, n, 0.0, 1.0, 0.0, 1.0, bc, 4)
    tol = 1e-8 if prec == molt.MOLT_F32 else 1e-11
    p = molt.make_params(eps, dt, tol=tol, max_iter=6000, init=molt.MOLT_INIT_LINEAR, precision=prec, model=model,
                         stepper=molt.MOLT_BDF2 if stepper == "BDF2" else molt.MOLT_BE)
    u0 = (synth.u0_vch(synth.BASE_SEED + 200 + i, n, n) if model == molt.MOLT_MODEL_VCH
          else synth.u0_uniform_noise(synth.BASE_SEED + 200 + i, n, n, 0.05))
    return g, p, u0, steps


def _serve(reqs, max_slots, pool_bytes, arrivals=None, prec=molt.MOLT_F32):
    """Submit request k before round arrivals[k] (default: all at once); run to
    completion; returns ({id: result}, {id: field}, max admitted at once)."""
    dt_ = torch.float32 if prec == molt.MOLT_F32 else torch.float64
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    out, fields, most = {}, {}, 0
    with torch.cuda.stream(s):
        srv = molt.Server(prec, max_slots, pool_bytes)
        order = sorted(range(len(reqs)), key=lambda k: arrivals[k] if arrivals else 0)
        rnd, k = 0, 0
        while len(out) < len(reqs):
            while k < len(order) and (arrivals is None or arrivals[order[k]] <= rnd):
                i = order[k]
                g, p, u0, ns = reqs[i]
                fields[i] = torch.tensor(u0, dtype=dt_, device=DEV)
                srv.submit(g, p, fields[i], ns, i)
                k += 1
            active, queued = srv.run(1)
            most = max(most, active)
            for r in srv.poll():
                out[r.id] = r
            rnd += 1
            assert rnd < 200000
        srv.close()
    torch.cuda.synchronize()
    return out, {i: f.cpu() for i, f in fields.items()}, most


MIX = [(0, 64, 5, 0, "BDF2"), (1, 96, 3, 1, "BE"), (2, 130, 6, 0, "BDF2"), (3, 72, 4, 1, "BDF2"),
       (4, 150, 2, 0, "BE"), (5, 80, 5, 1, "BDF2")]


@pytest.mark.parametrize("ticks", [8, 1])
def test_served_results_equal_alone_and_plain(ticks):
    assert molt.molt_set_option(molt.MOLT_OPT_BATCH_TICKS, ticks) == 0
    reqs = [_req(i, n, st, bc, stp) for (i, n, st, bc, stp) in MIX]
    arrivals = [0, 0, 3, 10, 25, 40]  # rounds: later requests arrive while earlier ones run
    res, fields, most = _serve(reqs, max_slots=8, pool_bytes=256 << 20, arrivals=arrivals)
    assert most >= 2
    for i, r in res.items():
        assert r.status == molt.MOLT_OK and r.steps == reqs[i][3]
    for i in (0, 2, 4):
        alone, af, _ = _serve([reqs[i]], max_slots=2, pool_bytes=128 << 20)
        assert torch.equal(af[0], fields[i]), i
        assert alone[0].iters == res[i].iters and alone[0].last.energy == res[i].last.energy
        g, p, u0, ns = reqs[i]
        x = torch.tensor(u0, dtype=torch.float32, device=DEV)
        _, infos = molt.solve(x, g, p, ns)
        assert torch.equal(x.cpu(), fields[i]), i
        assert sum(x.iters for x in infos) == res[i].iters


def test_admission_is_bounded_by_the_pool():
    reqs = [_req(i, 128, 3, i % 2, "BDF2") for i in range(5)]
    fp = molt.molt_server_footprint(molt.molt_instance(reqs[0][0], reqs[0][1], 4096, 3))
    res, fields, most = _serve(reqs, max_slots=16, pool_bytes=2 * fp + fp // 2)
    assert most == 2  # two requests fit the pool at once
    assert sorted(res) == list(range(5)) and all(r.status == molt.MOLT_OK for r in res.values())
    for i in (1, 4):
        g, p, u0, ns = reqs[i]
        x = torch.tensor(u0, dtype=torch.float32, device=DEV)
        molt.solve(x, g, p, ns)
        assert torch.equal(x.cpu(), fields[i])


def test_served_vch_fp64_matches_oracle():
    reqs = [_req(i, 48, 3, i % 2, "BDF2", prec=molt.MOLT_F64) for i in range(3)]
    res, fields, _ = _serve(reqs, max_slots=4, pool_bytes=64 << 20, arrivals=[0, 2, 5], prec=molt.MOLT_F64)
    for i, (g, p, u0, ns) in enumerate(reqs):
        og = oracle.Grid(nx=g.nx, ny=g.ny, x0=g.x0, x1=g.x1, y0=g.y0, y1=g.y1, bc=g.bc, M=4)
        po = oracle.Params(eps=p.eps, dt=p.dt, tol=p.tol, stepper=oracle.BDF2, max_iter=6000,
                           init=oracle.INIT_LINEAR, sigma0=oracle.VCH_SIGMA0)
        ref, rinf = oracle.vch_solve(og, po, u0, ns)
        assert res[i].iters == sum(x.iters for x in rinf)
        assert np.abs(fields[i].numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


def test_unfit_request_is_rejected():
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        srv = molt.Server(molt.MOLT_F32, 2, 1 << 20)
        g, p, u0, ns = _req(0, 256, 3, 0, "BE")
        x = torch.tensor(u0, dtype=torch.float32, device=DEV)
        with pytest.raises(molt.MoltError):
            srv.submit(g, p, x, ns, 0)
        assert srv.run(1) == (0, 0)
        srv.close()
