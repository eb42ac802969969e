"""Pins of the oracle's vector Cahn-Hilliard model (Sec. 2 eq. CH_vector_reaction,
Sec. 5.2) against what the paper and the mathematics fix."""
import numpy as np
import pytest

import oracle
from paper_1611_04214_amd import synth

Z = synth.VCH_Z


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build(force=False)


def test_potential_is_the_cube_root_product():
    """prod |u - z_i|^2 over the cube roots of unity equals |w^3 - 1|^2, w = u1 + i u2."""
    rng = np.random.default_rng(3)
    for u1, u2 in rng.uniform(-1.5, 1.5, (50, 2)):
        w = complex(u1, u2)
        assert abs(oracle.vch_W(u1, u2) - abs(w ** 3 - 1) ** 2) <= 1e-13 * (1 + abs(w) ** 6)


def test_gradient_is_the_derivative_of_the_potential():
    rng = np.random.default_rng(4)
    h = 1e-6
    for u1, u2 in rng.uniform(-1.2, 1.2, (30, 2)):
        g = oracle.vch_gradW(u1, u2)
        fd = [(oracle.vch_W(u1 + h, u2) - oracle.vch_W(u1 - h, u2)) / (2 * h),
              (oracle.vch_W(u1, u2 + h) - oracle.vch_W(u1, u2 - h)) / (2 * h)]
        assert np.allclose(g, fd, rtol=1e-7, atol=1e-7)


@pytest.mark.parametrize("i", [0, 1, 2])
def test_minima_and_the_printed_jacobian(i):
    """W = 0, grad W = 0 and the Hessian of W is 18 I at every z_i (eq. Jacobian)."""
    z1, z2 = Z[i]
    assert oracle.vch_W(z1, z2) <= 1e-28
    assert np.abs(oracle.vch_gradW(z1, z2)).max() <= 1e-14
    h = 1e-5
    H = np.zeros((2, 2))
    for c in range(2):
        e = np.zeros(2)
        e[c] = h
        H[:, c] = (oracle.vch_gradW(z1 + e[0], z2 + e[1]) - oracle.vch_gradW(z1 - e[0], z2 - e[1])) / (2 * h)
    assert np.allclose(H, 18.0 * np.eye(2), atol=1e-7)


def _grid(nx=32, ny=24, bc=oracle.BC_PERIODIC):
    return oracle.Grid(nx=nx, ny=ny, x0=0.0, x1=1.0, y0=0.0, y1=ny / nx, bc=bc, M=4)


def test_real_axis_reduces_to_the_scalar_model():
    """u2 = 0 is invariant and u1 then follows the scalar equation with
    f(u) = dW/du1(u, 0) = 6(u^5 - u^2); the vector scheme (shift by z3, sigma0
    18) and the scalar scheme (shift by -1, reaction hook 2) reach the same BE
    solution at tight tolerance."""
    g = _grid()
    rng = np.random.default_rng(5)
    u1 = -0.5 + 0.1 * rng.uniform(-1, 1, (g.ny, g.nx))
    u = np.stack([u1, np.zeros_like(u1)])
    pv = oracle.Params(eps=0.03, dt=2e-5, tol=1e-13, max_iter=5000, sigma0=oracle.VCH_SIGMA0)
    uv, iv = oracle.vch_step(g, pv, u)
    ps = oracle.Params(eps=0.03, dt=2e-5, tol=1e-13, max_iter=5000, sigma0=oracle.VCH_SIGMA0, reaction=2)
    us, _ = oracle.step(g, ps, u1)
    assert np.abs(uv[1]).max() <= 1e-13
    assert np.abs(uv[0] - us).max() <= 1e-10


def test_rotation_by_a_third_turn_commutes_with_the_step():
    """W is invariant under w -> e^{2 pi i/3} w; at convergence the BE step is
    too, although the iteration's shift by z3 is not."""
    g = _grid()
    u = synth.u0_vch(synth.BASE_SEED + 9, g.ny, g.nx)
    c, s = np.cos(2 * np.pi / 3), np.sin(2 * np.pi / 3)
    rot = lambda v: np.stack([c * v[0] - s * v[1], s * v[0] + c * v[1]])
    p = oracle.Params(eps=0.03, dt=2e-5, tol=1e-13, max_iter=8000, sigma0=oracle.VCH_SIGMA0)
    a, _ = oracle.vch_step(g, p, u)
    b, _ = oracle.vch_step(g, p, rot(u))
    assert np.abs(b - rot(a)).max() <= 1e-10


@pytest.mark.parametrize("bc", [oracle.BC_PERIODIC, oracle.BC_NEUMANN])
def test_mass_of_each_component_and_energy_decrease(bc):
    g = _grid(bc=bc)
    u = synth.u0_vch(synth.BASE_SEED + 10, g.ny, g.nx)
    p = oracle.Params(eps=0.03, dt=5e-5, tol=1e-12, max_iter=8000, stepper=oracle.BDF2,
                      sigma0=oracle.VCH_SIGMA0, init=oracle.INIT_LINEAR)
    m0 = (oracle.mass(g, u[0]), oracle.mass(g, u[1]))
    e0 = oracle.vch_energy(g, 0.03, u)
    out, infos = oracle.vch_solve(g, p, u, 6)
    if bc == oracle.BC_PERIODIC:  # periodic: plain h-weighted sums are conserved
        for inf in infos:
            assert abs(inf.mass - m0[0]) <= 1e-12 and abs(inf.mass2 - m0[1]) <= 1e-12
    e = [e0] + [inf.energy for inf in infos]
    assert all(e[k + 1] <= e[k] + 1e-13 for k in range(len(e) - 1)), e
    assert e[-1] < e0
    assert abs(infos[0].sigma - 18.0) < 1e-15 or infos[0].sigma > 18.0


def test_vch_iteration_switch_point():
    """eqs. CH_vector_fixed1/2: factorization for dt >= eps^2/81 (BE)."""
    eps = 0.05
    s1, s2, sg = oracle.stepper_params(eps, 1.01 * eps ** 2 / 81, oracle.BE, True, 18.0)
    assert sg == 18.0 and s1 > s2
    dt = 1.01 * eps ** 2 / 81
    assert abs(s1 - (9 * dt + np.sqrt(81 * dt * dt - eps * eps * dt))) <= 1e-15 * s1
    s1, s2, sg = oracle.stepper_params(eps, 0.99 * eps ** 2 / 81, oracle.BE, True, 18.0)
    assert s1 == s2 and sg > 18.0
