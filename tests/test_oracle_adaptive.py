"""Pins of the oracle's adaptive time stepping (Sec. 6, Algorithm 1) and its
variable-step BDF2 (reading: the paper writes BDF2 for constant steps)."""
import os

import numpy as np
import pytest

import oracle
from paper_1611_04214_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build(force=False)


@pytest.mark.parametrize("eta,nit,accept,fac", [
    (1e-4, 100, True, min(0.8 * np.sqrt(10.0), 1.3)),     # well inside: grow by at most gamma
    (9e-4, 100, True, 0.8 * np.sqrt(1e-3 / 9e-4)),         # close to tol: theta sqrt(tol/eta) < gamma
    (1e-5, 450, True, 1.0),                                # 0.7 <= N_it/N_maxit < 1: no growth
    (9.5e-4, 500, True, 0.8 * np.sqrt(1e-3 / 9.5e-4)),     # ... but shrink if theta sqrt(tol/eta) < 1
    (1e-5, 600, False, 1 / 1.3),                           # fixed point hit N_maxit: fail, 1/gamma
    (3e-3, 10, False, 1 / 1.3),                            # eta/tol > 2: fail, 1/gamma
    (1.5e-3, 10, False, 0.8 * np.sqrt(1e-3 / 1.5e-3)),     # eta/tol <= 2: fail, theta sqrt(tol/eta)
])
def test_step_size_control_follows_algorithm_1(eta, nit, accept, fac):
    ok, f = oracle.adapt_decision(eta, 1e-3, nit, 600, 0.8, 1.3)
    assert ok == accept and abs(f - fac) <= 1e-15 * fac


def _bdf2_run(nbase, ratio, T=0.4):
    """BDF2 over steps alternating a, ratio*a (2 steps = 2T/nbase), started with
    32 BE sub-steps; the Table 1 problem (1D, eps 0.18, N = 128, M = 6)."""
    g = oracle.Grid(nx=128, ny=1, x0=0.0, x1=2 * np.pi, bc=oracle.BC_PERIODIC, M=6)
    u = synth.u0_table1(np.arange(128) * 2 * np.pi / 128)
    h = T / nbase
    a = 2 * h / (1 + ratio)
    dts = [a, ratio * a] * (nbase // 2)
    up, dprev = None, None
    for d in dts:
        if up is None:
            v = u.copy()
            for _ in range(32):
                v, _ = oracle.step(g, oracle.Params(eps=0.18, dt=d / 32, tol=1e-13, max_iter=5000), v)
        else:
            v, _ = oracle.step(g, oracle.Params(eps=0.18, dt=d, tol=1e-13, max_iter=5000, stepper=oracle.BDF2,
                                                omega=d / dprev), u, up)
        up, u, dprev = u, v, d
    return u


def test_variable_step_bdf2_is_second_order():
    """Steps alternating by a factor 2: successive differences fall at least
    like dt^2 (the constant-step coefficients on the same steps give order 1)."""
    us = [_bdf2_run(n, 2.0) for n in (16, 32, 64, 128)]
    e = [np.abs(us[i] - us[i + 1]).max() for i in range(3)]
    orders = [np.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(orders) >= 1.9, (e, orders)


def test_variable_step_reduces_to_constant_step():
    g = oracle.Grid(nx=64, ny=48, x0=0.0, x1=1.0, y0=0.0, y1=0.75, bc=oracle.BC_NEUMANN, M=4)
    u = synth.u0_uniform_noise(synth.BASE_SEED + 90, 48, 64, 0.3)
    up = synth.u0_uniform_noise(synth.BASE_SEED + 91, 48, 64, 0.3)
    a, _ = oracle.step(g, oracle.Params(eps=0.03, dt=1e-4, stepper=oracle.BDF2, fixed_iters=3, omega=1.0), u, up)
    b, _ = oracle.step(g, oracle.Params(eps=0.03, dt=1e-4, stepper=oracle.BDF2, fixed_iters=3,
                                        omega=1.0 + 1e-12), u, up)
    assert np.abs(a - b).max() <= 1e-10


def test_adaptive_run_keeps_energy_decay_and_the_lte_bound():
    g = oracle.Grid(nx=48, ny=40, x0=0.0, x1=1.0, y0=0.0, y1=40 / 48, bc=oracle.BC_PERIODIC, M=4)
    u0 = synth.u0_uniform_noise(synth.BASE_SEED + 92, 40, 48, 0.05)
    ap = oracle.AdaptParams(t_end=2e-3, dt0=1e-5, lte_tol=1e-3, nmaxit=400)
    energies = []
    u, recs = oracle.adaptive_solve(g, oracle.Params(eps=0.03, dt=1e-5, tol=1e-11), u0, ap,
                                    stop=lambda t, u: energies.append(oracle.energy(g, 0.03, u)) and False)
    acc = [r for r in recs if r[4]]
    assert abs(sum(r[1] for r in acc) - 2e-3) <= 1e-15
    assert all(r[2] <= 1e-3 for r in acc)
    assert all(energies[k + 1] <= energies[k] + 1e-13 for k in range(len(energies) - 1))
    assert max(r[1] for r in acc) > 5 * 1e-5  # the step grows during coarsening


@pytest.mark.slow
def test_ripening_time_of_the_1d_problem():
    """Sec. 7.1 / Table 7: adaptive BE-BDF2 (delta_tol 1e-3, N_maxit 600, tol
    1e-11) ripens within 0.05% of the reference time and of the printed value."""
    golden = dict(line.split() for line in open(os.path.join(HERE, "golden", "ripening_1d.txt"))
                  if line.strip() and not line.startswith("#"))
    ref, printed = float(golden["reference_Tr"]), float(golden["table7_be_bdf2_Tr"])
    g = oracle.Grid(nx=128, ny=1, x0=0.0, x1=2 * np.pi, bc=oracle.BC_PERIODIC, M=4)
    u0 = synth.u0_table1(np.arange(128) * 2 * np.pi / 128)
    st = {"tr": None, "prev": (0.0, u0[64])}

    def stop(t, u):  # x = pi is node 64
        tp, upv = st["prev"]
        if upv > 0 >= u[64] and st["tr"] is None:
            st["tr"] = tp + (t - tp) * upv / (upv - u[64])
        st["prev"] = (t, u[64])
        return st["tr"] is not None

    ap = oracle.AdaptParams(t_end=9000.0, dt0=0.01, lte_tol=1e-3, nmaxit=600)
    oracle.adaptive_solve(g, oracle.Params(eps=0.18, dt=0.01, tol=1e-11), u0, ap, stop=stop)
    assert st["tr"] is not None
    assert abs(st["tr"] - ref) <= 5e-4 * ref and abs(st["tr"] - printed) <= 5e-4 * printed, st["tr"]
