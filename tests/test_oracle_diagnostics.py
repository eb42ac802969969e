"""Pins of the oracle's discrete mass and energy (the diagnostics of a step).

The paper defines the continuum energies (Sec. 2, eqs. EnergyFunctional and
EnergyFunctional_vector: the integral of eps^2/2 |grad u|^2 plus the potential)
and says that periodic and no-flux problems keep the volume (Sec. 7); it gives
no discrete formula.  The oracle's reading is forward differences for the
gradient and, off the periodic case, trapezoid end weights for both terms.
These tests fix that reading by results it must reproduce, not by restating
its sums:

* exact sums of the rule for data whose sums have closed forms (a constant,
  an exponential, single Fourier modes: the forward-difference symbol
  4 sin^2(theta/2)/h^2 and the midpoint sums of sin^2),
* the continuum integrals of eq. EnergyFunctional(_vector), evaluated by
  adaptive quadrature in 30 digits, reached at second order in h (smooth data)
  or exactly (trigonometric potentials below the grid's aliasing limit),
* the Euler-Maclaurin end correction of the trapezoid rule (weights 1/2 at the
  ends, nothing else).

A factor eps^2 in place of eps^2/2, a dropped h_x h_y, a wrong end weight, a
weight applied to the gradient term along its own axis, or a wrong potential
fails one of them.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from paper_1611_04214_amd import synth  # noqa: F401  (seeded inputs live there)


def _grid(oracle_mod, nx, ny, bc, Lx=1.0, Ly=1.0):
    return oracle_mod.Grid(nx=nx, ny=ny, bc=bc, M=4, x0=0.0, x1=Lx, y0=0.0, y1=Ly)


def _field(g, fx, fy=None):
    x = g.nodes_x()
    if g.ny == 1:
        return fx(x)[None, :]
    y = g.nodes_y()
    return fy(y)[:, None] * fx(x)[None, :] if fy is not None else np.broadcast_to(fx(x), (g.ny, g.nx)).copy()


def _mean_quartic(c, A):
    """(1/2pi) int_0^{2pi} 1/4 ((c + A cos t)^2 - 1)^2 dt in 30 digits."""
    mp.mp.dps = 30
    return float(mp.quad(lambda t: 0.25 * ((c + A * mp.cos(t)) ** 2 - 1) ** 2, [0, 2 * mp.pi]) / (2 * mp.pi))


# ------------------------------------------------------------------ mass ----
@pytest.mark.parametrize("bc", [0, 1, 2])
@pytest.mark.parametrize("shape", [(17, 1), (12, 9), (40, 33)])
def test_mass_of_a_constant_is_value_times_area(oracle_mod, bc, shape):
    nx, ny = shape
    Lx, Ly = 0.7, 1.3
    g = _grid(oracle_mod, nx, ny, bc, Lx, Ly)
    c = -0.37
    u = np.full((ny, nx), c)
    area = Lx * (Ly if ny > 1 else 1.0)
    assert abs(oracle_mod.mass(g, u) - c * area) < 1e-15 * nx * ny


def test_periodic_mass_is_the_integral_of_an_analytic_field(oracle_mod):
    """Periodic trapezoid sums of analytic periodic data converge spectrally:
    int_0^1 int_0^Ly exp(sin 2pi x) cos(2pi y/Ly)^2 = I_0(1) * Ly/2."""
    Ly = 0.8
    g = _grid(oracle_mod, 48, 40, 0, 1.0, Ly)
    u = _field(g, lambda x: np.exp(np.sin(2 * np.pi * x)), lambda y: np.cos(2 * np.pi * y / Ly) ** 2)
    exact = float(mp.besseli(0, 1)) * Ly / 2
    assert abs(oracle_mod.mass(g, u) - exact) < 1e-14


@pytest.mark.parametrize("shape", [(9, 1), (33, 17), (65, 20)])
def test_trapezoid_mass_of_an_exponential_is_closed_form(oracle_mod, shape):
    """Non-periodic ends: the trapezoid rule with end weights 1/2 sums
    exp(a x) over [0, L] to I * (a h / 2) coth(a h / 2) exactly (geometric
    series), I the integral; separable in 2D."""
    nx, ny = shape
    Lx, Ly, a, b = 1.0, 0.6, 1.7, -2.3
    g = _grid(oracle_mod, nx, ny, 1, Lx, Ly)
    u = _field(g, lambda x: np.exp(a * x), lambda y: np.exp(b * y))

    def trap(c, L, h):
        return (math.exp(c * L) - 1.0) / c * (c * h / 2) / math.tanh(c * h / 2)

    expect = trap(a, Lx, g.hx) * (trap(b, Ly, g.hy) if ny > 1 else 1.0)
    assert abs(oracle_mod.mass(g, u) - expect) < 1e-14 * abs(expect)


def test_neumann_mass_converges_with_the_euler_maclaurin_term(oracle_mod):
    """(T - I) / h^2 -> (f'(L) - f'(0)) / 12 for the trapezoid rule, so the
    mass of a smooth non-periodic field is second order with that constant."""
    f = lambda x: np.tanh(4.0 * (x - 0.3))  # noqa: E731
    fp = lambda x: 4.0 / np.cosh(4.0 * (x - 0.3)) ** 2  # noqa: E731
    exact = (math.log(math.cosh(4.0 * 0.7)) - math.log(math.cosh(4.0 * 0.3))) / 4.0
    ratios = []
    for n in (65, 129, 257):
        g = _grid(oracle_mod, n, 1, 1)
        ratios.append((oracle_mod.mass(g, _field(g, f)) - exact) / g.hx ** 2)
    lead = (fp(1.0) - fp(0.0)) / 12.0
    assert abs(ratios[-1] - lead) < 1e-3 * abs(lead)
    assert abs(ratios[-1] - lead) < abs(ratios[0] - lead)


# ---------------------------------------------------------------- energy ----
@pytest.mark.parametrize("bc", [0, 1, 2])
def test_energy_of_a_constant_is_potential_times_area(oracle_mod, bc):
    g = _grid(oracle_mod, 21, 14, bc, 0.9, 1.1)
    c = 0.41
    u = np.full((14, 21), c)
    expect = 0.25 * (c * c - 1) ** 2 * 0.9 * 1.1
    assert abs(oracle_mod.energy(g, 0.3, u) - expect) < 1e-13 * expect


@pytest.mark.parametrize("nx,k", [(16, 1), (40, 3), (64, 5)])
def test_periodic_1d_energy_of_a_mode_is_closed_form(oracle_mod, nx, k):
    """u = c + A cos(2 pi k x / L) on N periodic nodes: the forward-difference
    gradient sums to 2 A^2 sin^2(pi k / N) L / h^2, the potential's trapezoid
    sum is exact (trigonometric degree 4k < N) and equals L times the mean of
    1/4 (u^2 - 1)^2 over a period."""
    L, c, A, eps = 2 * np.pi, 0.2, 0.7, 0.13
    g = _grid(oracle_mod, nx, 1, 0, L)
    u = _field(g, lambda x: c + A * np.cos(2 * np.pi * k * x / L))
    h = g.hx
    grad = 2 * A * A * math.sin(math.pi * k / nx) ** 2 * L / h ** 2
    expect = 0.5 * eps * eps * grad + L * _mean_quartic(c, A)
    assert abs(oracle_mod.energy(g, eps, u) - expect) < 1e-13 * expect


@pytest.mark.parametrize("nx,ny,k,l", [(24, 20, 2, 1), (48, 36, 3, 4)])
def test_periodic_2d_energy_of_a_mode_is_closed_form(oracle_mod, nx, ny, k, l):
    """u = A cos(2 pi k x / Lx) cos(2 pi l y / Ly): gradient energy
    eps^2/2 * A^2 [sin^2(pi k/Nx) Ly Lx / hx^2 + sin^2(pi l/Ny) Lx Ly / hy^2],
    the potential's sum the exact mean of 1/4 (u^2 - 1)^2 times the area."""
    Lx, Ly, A, eps = 1.0, 0.75, 0.9, 0.05
    g = _grid(oracle_mod, nx, ny, 0, Lx, Ly)
    u = _field(g, lambda x: A * np.cos(2 * np.pi * k * x / Lx), lambda y: np.cos(2 * np.pi * l * y / Ly))
    gx = A * A * math.sin(math.pi * k / nx) ** 2 * Lx * Ly / g.hx ** 2
    gy = A * A * math.sin(math.pi * l / ny) ** 2 * Lx * Ly / g.hy ** 2
    mp.mp.dps = 30
    pot = mp.quad(lambda s, t: 0.25 * ((A * mp.cos(s) * mp.cos(t)) ** 2 - 1) ** 2, [0, 2 * mp.pi], [0, 2 * mp.pi])
    pot = float(pot) / (4 * math.pi ** 2) * Lx * Ly
    expect = 0.5 * eps * eps * (gx + gy) + pot
    assert abs(oracle_mod.energy(g, eps, u) - expect) < 1e-13 * expect


@pytest.mark.parametrize("bc", [1, 2])
@pytest.mark.parametrize("n,k", [(17, 1), (33, 3)])
def test_nonperiodic_energy_of_a_cosine_mode_is_closed_form(oracle_mod, bc, n, k):
    """u = c + A cos(pi k x / L) on n nodes including both ends (h = L/(n-1)):
    u_{i+1} - u_i = -2 A sin(pi k h / 2L) sin(pi k (x_i + h/2) / L), and the
    midpoint sum of sin^2 over the n-1 cells is (n-1)/2, so the gradient term
    is eps^2/2 * 2 A^2 sin^2(pi k h / 2L) L / h^2 with NO end weights; the
    trapezoid sum of the potential is exact (the even extension is periodic)."""
    L, c, A, eps = 1.0, -0.1, 0.8, 0.07
    g = _grid(oracle_mod, n, 1, bc, L)
    u = _field(g, lambda x: c + A * np.cos(np.pi * k * x / L))
    h = g.hx
    grad = 2 * A * A * math.sin(math.pi * k * h / (2 * L)) ** 2 * L / h ** 2
    expect = 0.5 * eps * eps * grad + L * _mean_quartic(c, A)
    assert abs(oracle_mod.energy(g, eps, u) - expect) < 1e-13 * expect


def test_neumann_2d_energy_of_a_cosine_mode_is_closed_form(oracle_mod):
    """u = A cos(pi k x) cos(pi l y) on [0,1]x[0,Ly] with both ends as nodes:
    each axis' difference term carries the trapezoid weight of the OTHER axis
    only, whose sum of cos^2 is exactly half the length."""
    nx, ny, k, l, Ly, A, eps = 25, 19, 2, 3, 0.9, 0.6, 0.04
    g = _grid(oracle_mod, nx, ny, 1, 1.0, Ly)
    u = _field(g, lambda x: A * np.cos(np.pi * k * x), lambda y: np.cos(np.pi * l * y / Ly))
    gx = 2 * A * A * math.sin(math.pi * k * g.hx / 2) ** 2 / g.hx ** 2 * (Ly / 2)
    gy = 2 * A * A * math.sin(math.pi * l * g.hy / (2 * Ly)) ** 2 * Ly / g.hy ** 2 * 0.5
    mp.mp.dps = 30
    pot = mp.quad(lambda s, t: 0.25 * ((A * mp.cos(s) * mp.cos(t)) ** 2 - 1) ** 2, [0, mp.pi], [0, mp.pi])
    pot = float(pot) / mp.pi ** 2 * Ly
    expect = 0.5 * eps * eps * (gx + gy) + float(pot)
    assert abs(oracle_mod.energy(g, eps, u) - expect) < 1e-13 * expect


def test_neumann_energy_of_an_interface_converges_at_second_order(oracle_mod):
    """A tanh interface on a Neumann square: the discrete energy reaches the
    integral of eq. EnergyFunctional (30-digit quadrature) at order 2."""
    eps, w = 0.05, 0.08
    prof = lambda x: np.tanh((x - 0.37) / w)  # noqa: E731
    mp.mp.dps = 30
    ex = mp.quad(lambda x: 0.5 * eps ** 2 * (1 / (w * mp.cosh((x - 0.37) / w) ** 2)) ** 2
                 + 0.25 * (mp.tanh((x - 0.37) / w) ** 2 - 1) ** 2, [0, 0.37, 1])
    exact = float(ex) * 0.5  # uniform along y on [0, 0.5]
    errs = []
    for n in (65, 129, 257):
        g = _grid(oracle_mod, n, 9, 1, 1.0, 0.5)
        errs.append(abs(oracle_mod.energy(g, eps, _field(g, prof)) - exact))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 2.0) < 0.15), orders
    assert errs[-1] < 1e-3 * exact


# --------------------------------------------------------- vector model ----
def test_vector_energy_at_the_pure_phases_and_the_origin(oracle_mod):
    """W vanishes at the cube roots of unity and equals 1 at the origin
    (|0 - z_i| = 1): a constant field's energy is W times the area."""
    g = _grid(oracle_mod, 12, 10, 1, 0.5, 0.8)
    for j in range(3):
        z = np.exp(2j * np.pi * j / 3)
        u = np.stack([np.full((10, 12), z.real), np.full((10, 12), z.imag)])
        assert abs(oracle_mod.vch_energy(g, 0.1, u)) < 1e-14
    u = np.zeros((2, 10, 12))
    assert abs(oracle_mod.vch_energy(g, 0.1, u) - 0.4) < 1e-15


def test_vector_energy_of_modes_is_the_integral(oracle_mod):
    """u1 = a cos(2 pi x), u2 = b sin(2 pi y) (periodic): the gradient terms of
    the two components add (each the scalar closed form), and the trapezoid
    sum of W (a trigonometric polynomial of degree 6 per axis, below the grid's
    aliasing limit) equals its integral, here in 30 digits."""
    nx, ny, a, b, eps = 32, 28, 0.6, 0.5, 0.09
    g = _grid(oracle_mod, nx, ny, 0)
    x, y = g.nodes_x(), g.nodes_y()
    u1 = np.broadcast_to(a * np.cos(2 * np.pi * x)[None, :], (ny, nx))
    u2 = np.broadcast_to(b * np.sin(2 * np.pi * y)[:, None], (ny, nx))
    u = np.stack([u1, u2]).copy()
    grad = 2 * a * a * math.sin(math.pi / nx) ** 2 / g.hx ** 2 + 2 * b * b * math.sin(math.pi / ny) ** 2 / g.hy ** 2
    mp.mp.dps = 30

    def W(s, t):
        w = mp.mpc(a * mp.cos(s), b * mp.sin(t))
        return abs(w ** 3 - 1) ** 2
    pot = float(mp.quad(W, [0, 2 * mp.pi], [0, 2 * mp.pi])) / (4 * math.pi ** 2)
    expect = 0.5 * eps * eps * grad + pot
    assert abs(oracle_mod.vch_energy(g, eps, u) - expect) < 1e-12 * expect


def test_vector_energy_neumann_end_weights(oracle_mod):
    """Neumann: a field along x only, u = (t(x), 0) with t = 0.3 + 0.4 cos(pi x):
    W = (t^3 - 1)^2 on the real axis; trapezoid end weights make the sum exact
    for this even-extension trigonometric polynomial (degree 6 < 2(n-1))."""
    n, eps = 21, 0.11
    g = _grid(oracle_mod, n, 7, 1, 1.0, 0.6)
    t = lambda x: 0.3 + 0.4 * np.cos(np.pi * x)  # noqa: E731
    u = np.stack([_field(g, t), np.zeros((7, n))])
    mp.mp.dps = 30
    pot = float(mp.quad(lambda x: ((0.3 + 0.4 * mp.cos(mp.pi * x)) ** 3 - 1) ** 2, [0, 1])) * 0.6
    grad = 2 * 0.16 * math.sin(math.pi * g.hx / 2) ** 2 / g.hx ** 2 * 0.6
    expect = 0.5 * eps * eps * grad + pot
    assert abs(oracle_mod.vch_energy(g, eps, u) - expect) < 1e-13 * expect
