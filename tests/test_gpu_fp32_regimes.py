"""FP32 steps solved to tolerance in the regimes of the 4096^2 and 512^2
workloads, against the FP64 oracle at the same tolerance.

The 4096^2 workload (eps 0.005, BDF2 dt 1e-5, h = 1/4096, alpha*h ~ 0.068) is
run on a periodic 512^2 patch with the same grid spacing, eps, dt and initial
statistics, so every mode that is slow for the splitting's fixed point at full
size is present (the contraction of a mode depends on alpha*h and the
wavenumber times h only).  The 512^2 Neumann workload (eps 0.01, dt 5e-5) runs
at its full size.  Each test prints max-abs and L2 of u - u_oracle, both
iteration logs and the mass drift, and requires max-abs <= 1e-5 with the
oracle's iteration counts to within 2 %.
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


def _compare(name, g, u0, eps, dt, nsteps, tol=1e-8):
    po = oracle.Params(eps=eps, dt=dt, tol=tol, stepper=oracle.BDF2, max_iter=20000, init=oracle.INIT_LINEAR)
    ref, rinf = oracle.solve(_og(g), po, u0, nsteps)
    x = torch.tensor(u0, dtype=torch.float32, device=DEV)
    p = molt.make_params(eps, dt, tol=tol, stepper=molt.MOLT_BDF2, max_iter=20000, init=molt.MOLT_INIT_LINEAR,
                         precision=molt.MOLT_F32)
    st, infos = molt.solve(x, g, p, nsteps)
    got = x.cpu().double().numpy()
    err = np.abs(got - ref)
    gi, oi = [i.iters for i in infos], [i.iters for i in rinf]
    m0 = oracle.mass(_og(g), u0)
    print(f"{name}: max-abs {err.max():.3e}  L2 {np.sqrt((err ** 2).mean()):.3e}  iters gpu {gi} oracle {oi}  "
          f"mass drift gpu {infos[-1].mass - m0:.2e} oracle {rinf[-1].mass - m0:.2e}", flush=True)
    assert st == molt.MOLT_OK
    for a, b in zip(gi, oi):
        assert abs(a - b) <= max(2, 0.02 * b), (gi, oi)
    assert err.max() <= 1e-5


def test_fp32_at_the_4096_regime_on_a_512_patch():
    n = 512
    L = n / 4096
    g = molt.make_grid(n, n, 0.0, L, 0.0, L, molt.MOLT_BC_PERIODIC, 4)
    u0 = synth.u0_normal_noise(synth.BASE_SEED + 7, n, n, 0.3, 0.05)
    _compare("4096-regime patch 512^2", g, u0, 0.005, 1e-5, 3)


def test_fp32_neumann_512_workload():
    w = synth.WORKLOADS["ch2d_neumann_bdf2_512"]
    n = w["n"]
    g = molt.make_grid(n, n, 0.0, 1.0, 0.0, 1.0, molt.MOLT_BC_NEUMANN, w["M"])
    _compare("neumann 512^2 workload", g, synth.workload_u0("ch2d_neumann_bdf2_512"), w["eps"], w["dt"], 3)
