"""FP64 CPU oracle of the MOL^T Cahn-Hilliard method (arXiv:1611.04214).

TEST INFRASTRUCTURE ONLY: the plain, slow reference the GPU library is checked
against.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it.  It shares no code with the GPU library; the two meet
only through the seeded input generators.

The arithmetic lives in ``molt_oracle.c`` (plain C, FP64, OpenMP over lines);
this module builds it with gcc and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "molt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_PERIODIC, BC_NEUMANN, BC_DIRICHLET = 0, 1, 2
BE, BDF2, BDF3 = 0, 1, 2
INIT_PREV, INIT_LINEAR = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double),
                ("y0", ctypes.c_double), ("y1", ctypes.c_double),
                ("bc", ctypes.c_int), ("M", ctypes.c_int)]


class _Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("dt", ctypes.c_double), ("tol", ctypes.c_double),
                ("sigma0", ctypes.c_double), ("stepper", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("init", ctypes.c_int), ("fixed_iters", ctypes.c_int),
                ("reaction", ctypes.c_int), ("react_k", ctypes.c_double), ("omega", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("residual", ctypes.c_double),
                ("mass", ctypes.c_double), ("energy", ctypes.c_double),
                ("s1", ctypes.c_double), ("s2", ctypes.c_double), ("sigma", ctypes.c_double),
                ("mass2", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_pqr.argtypes = [ctypes.c_double, dp, dp, dp]
        lib.oracle_weights.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        lib.oracle_weights_window.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, dp]
        lib.oracle_sweep.argtypes = [ctypes.POINTER(_Grid), ctypes.c_int, ctypes.c_double, dp, dp]
        lib.oracle_step.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Params), dp, dp,
                                    ctypes.POINTER(_Info)]
        lib.oracle_solve.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Params), dp,
                                     ctypes.c_int, ctypes.POINTER(_Info)]
        lib.oracle_mass.argtypes = [ctypes.POINTER(_Grid), dp]
        lib.oracle_mass.restype = ctypes.c_double
        lib.oracle_energy.argtypes = [ctypes.POINTER(_Grid), ctypes.c_double, dp]
        lib.oracle_energy.restype = ctypes.c_double
        lib.oracle_stepper_params.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_double, dp]
        lib.oracle_bdf3_step.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Params), dp, dp, dp,
                                         ctypes.POINTER(_Info)]
        lib.oracle_sdirk2_step.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Params), dp,
                                           ctypes.POINTER(_Info)]
        lib.oracle_vch_W.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.oracle_vch_W.restype = ctypes.c_double
        lib.oracle_vch_gradW.argtypes = [ctypes.c_double, ctypes.c_double, dp]
        lib.oracle_vch_energy.argtypes = [ctypes.POINTER(_Grid), ctypes.c_double, dp]
        lib.oracle_vch_energy.restype = ctypes.c_double
        lib.oracle_vch_step.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Params), dp, dp,
                                        ctypes.POINTER(_Info)]
        lib.oracle_vch_solve.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Params), dp,
                                         ctypes.c_int, ctypes.POINTER(_Info)]
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Grid:
    nx: int
    ny: int = 1
    x0: float = 0.0
    x1: float = 2 * np.pi
    y0: float = 0.0
    y1: float = 2 * np.pi
    bc: int = BC_PERIODIC
    M: int = 4

    def c(self) -> _Grid:
        return _Grid(self.nx, self.ny, self.x0, self.x1, self.y0, self.y1, self.bc, self.M)

    @property
    def hx(self) -> float:
        return (self.x1 - self.x0) / (self.nx if self.bc == BC_PERIODIC else self.nx - 1)

    @property
    def hy(self) -> float:
        if self.ny == 1:
            return 1.0
        return (self.y1 - self.y0) / (self.ny if self.bc == BC_PERIODIC else self.ny - 1)

    def nodes_x(self) -> np.ndarray:
        return self.x0 + self.hx * np.arange(self.nx)

    def nodes_y(self) -> np.ndarray:
        return self.y0 + self.hy * np.arange(self.ny)


@dataclass
class Params:
    eps: float
    dt: float
    tol: float = 1e-10
    stepper: int = BE
    max_iter: int = 300
    init: int = INIT_PREV
    fixed_iters: int = 0
    sigma0: float = 2.0
    reaction: int = 0          # 0: Cahn-Hilliard cubic; 1: linear f(v) = react_k*v (test hook)
    react_k: float = 0.0
    omega: float = 1.0         # BDF2 step ratio dt_n / dt_{n-1} (variable steps)

    def c(self) -> _Params:
        return _Params(self.eps, self.dt, self.tol, self.sigma0, self.stepper, self.max_iter,
                       self.init, self.fixed_iters, self.reaction, self.react_k, self.omega)


@dataclass
class Info:
    iters: int
    residual: float
    mass: float
    energy: float
    s1: float
    s2: float
    sigma: float
    mass2: float = 0.0


def _info(i: _Info) -> Info:
    return Info(i.iters, i.residual, i.mass, i.energy, i.s1, i.s2, i.sigma, i.mass2)


def pqr(nu: float):
    """The printed M=2 weights P, Q, R (Sec. 3.2)."""
    lib = _load()
    P, Q, R = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib.oracle_pqr(nu, ctypes.byref(P), ctypes.byref(Q), ctypes.byref(R))
    return P.value, Q.value, R.value


def weights(M: int, nu: float, r: int | None = None):
    """Cell weights (wl, wr) of window position r (default: centred)."""
    lib = _load()
    wl = np.zeros(M + 1)
    wr = np.zeros(M + 1)
    if r is None:
        rc = lib.oracle_weights(M, nu, _dp(wl), _dp(wr))
    else:
        rc = lib.oracle_weights_window(M, nu, r, _dp(wl), _dp(wr))
    if rc != 0:
        raise ValueError("bad weight arguments")
    return wl, wr


def sweep(grid: Grid, axis: int, alpha: float, field: np.ndarray) -> np.ndarray:
    """Apply L^{-1} = (I - d^2/alpha^2)^{-1} line by line along axis (0 = x, 1 = y)."""
    lib = _load()
    f = np.ascontiguousarray(field, dtype=np.float64).reshape(grid.ny, grid.nx)
    out = np.empty_like(f)
    rc = lib.oracle_sweep(ctypes.byref(grid.c()), axis, alpha, _dp(f), _dp(out))
    if rc != 0:
        raise ValueError("oracle_sweep: bad arguments")
    return out.reshape(np.shape(field)) if np.ndim(field) == 2 else out.reshape(-1)


def step(grid: Grid, params: Params, u: np.ndarray, u_prev: np.ndarray | None = None):
    """One time step; returns (u_next, Info).  u_prev=None gives a BE step."""
    lib = _load()
    uu = np.ascontiguousarray(u, dtype=np.float64).copy()
    up = None if u_prev is None else np.ascontiguousarray(u_prev, dtype=np.float64)
    info = _Info()
    rc = lib.oracle_step(ctypes.byref(grid.c()), ctypes.byref(params.c()), _dp(uu),
                         None if up is None else _dp(up), ctypes.byref(info))
    if rc < 0:
        raise ValueError("oracle_step failed (%d)" % rc)
    return uu, _info(info)


def bdf3_step(grid: Grid, params: Params, u: np.ndarray, u_prev: np.ndarray, u_prev2: np.ndarray):
    """One BDF3 step (eq. BDF3) from u^n, u^{n-1}, u^{n-2}; returns (u_next, Info)."""
    lib = _load()
    uu = np.ascontiguousarray(u, dtype=np.float64).copy()
    a = np.ascontiguousarray(u_prev, dtype=np.float64)
    b = np.ascontiguousarray(u_prev2, dtype=np.float64)
    info = _Info()
    rc = lib.oracle_bdf3_step(ctypes.byref(grid.c()), ctypes.byref(params.c()), _dp(uu), _dp(a), _dp(b),
                              ctypes.byref(info))
    if rc < 0:
        raise ValueError("oracle_bdf3_step failed (%d)" % rc)
    return uu, _info(info)


def sdirk2_step(grid: Grid, params: Params, u: np.ndarray):
    """One SDIRK2 step (Sec. 4.2) as two BE stages of eta*dt; returns (u_next, Info)."""
    lib = _load()
    uu = np.ascontiguousarray(u, dtype=np.float64).copy()
    info = _Info()
    rc = lib.oracle_sdirk2_step(ctypes.byref(grid.c()), ctypes.byref(params.c()), _dp(uu), ctypes.byref(info))
    if rc < 0:
        raise ValueError("oracle_sdirk2_step failed (%d)" % rc)
    return uu, _info(info)


def solve(grid: Grid, params: Params, u: np.ndarray, nsteps: int):
    """nsteps steps (BDF2: BE first step).  Returns (u_final, [Info])."""
    lib = _load()
    uu = np.ascontiguousarray(u, dtype=np.float64).copy()
    infos = (_Info * max(nsteps, 1))()
    rc = lib.oracle_solve(ctypes.byref(grid.c()), ctypes.byref(params.c()), _dp(uu), nsteps, infos)
    if rc < 0:
        raise ValueError("oracle_solve failed (%d)" % rc)
    return uu, [_info(infos[i]) for i in range(nsteps)]


def set_threads(n: int) -> int:
    """Threads of the oracle's OpenMP loops over lines (for timing it on one
    core or on all cores); returns the count now in effect."""
    _load()
    gomp = ctypes.CDLL("libgomp.so.1")
    gomp.omp_set_num_threads(int(n))
    return int(gomp.omp_get_max_threads())


def mass(grid: Grid, u: np.ndarray) -> float:
    lib = _load()
    uu = np.ascontiguousarray(u, dtype=np.float64)
    return lib.oracle_mass(ctypes.byref(grid.c()), _dp(uu))


def energy(grid: Grid, eps: float, u: np.ndarray) -> float:
    lib = _load()
    uu = np.ascontiguousarray(u, dtype=np.float64)
    return lib.oracle_energy(ctypes.byref(grid.c()), eps, _dp(uu))


def stepper_params(eps: float, dt: float, stepper: int, first: bool, sigma0: float = 2.0):
    """(s1, s2, sigma) of the factored operator (I - s1 Lap)(I - s2 Lap)."""
    lib = _load()
    out = np.zeros(3)
    lib.oracle_stepper_params(eps, dt, stepper, 1 if first else 0, sigma0, _dp(out))
    return float(out[0]), float(out[1]), float(out[2])


# ------------------------------------------------------------- vector model --
#: sigma0 of the vector model: the Hessian of W at its minima is 18 I (Sec. 5.2)
VCH_SIGMA0 = 18.0


def vch_W(u1: float, u2: float) -> float:
    """W(u) = prod |u - z_i|^2 (eq. CH_vector_reaction)."""
    return _load().oracle_vch_W(u1, u2)


def vch_gradW(u1: float, u2: float) -> np.ndarray:
    g = np.zeros(2)
    _load().oracle_vch_gradW(u1, u2, _dp(g))
    return g


def vch_energy(grid: Grid, eps: float, u: np.ndarray) -> float:
    """Energy of eq. EnergyFunctional_vector; u is (2, ny, nx) or component-major flat."""
    uu = np.ascontiguousarray(u, dtype=np.float64)
    return _load().oracle_vch_energy(ctypes.byref(grid.c()), eps, _dp(uu))


def vch_step(grid: Grid, params: Params, u: np.ndarray, u_prev: np.ndarray | None = None):
    """One vector-model step; u (2, ny, nx).  Returns (u_next, Info)."""
    lib = _load()
    uu = np.ascontiguousarray(u, dtype=np.float64).copy()
    up = None if u_prev is None else np.ascontiguousarray(u_prev, dtype=np.float64)
    info = _Info()
    rc = lib.oracle_vch_step(ctypes.byref(grid.c()), ctypes.byref(params.c()), _dp(uu),
                             None if up is None else _dp(up), ctypes.byref(info))
    if rc < 0:
        raise ValueError("oracle_vch_step failed (%d)" % rc)
    return uu, _info(info)


def vch_solve(grid: Grid, params: Params, u: np.ndarray, nsteps: int):
    """nsteps vector-model steps (BDF2: BE first step).  Returns (u_final, [Info])."""
    lib = _load()
    uu = np.ascontiguousarray(u, dtype=np.float64).copy()
    infos = (_Info * max(nsteps, 1))()
    rc = lib.oracle_vch_solve(ctypes.byref(grid.c()), ctypes.byref(params.c()), _dp(uu), nsteps, infos)
    if rc < 0:
        raise ValueError("oracle_vch_solve failed (%d)" % rc)
    return uu, [_info(infos[i]) for i in range(nsteps)]


# --------------------------------------------------------- adaptive steps --
@dataclass
class AdaptParams:
    """Algorithm 1 (Sec. 6): lte_tol is sigma_tol, nmaxit is N_maxit (each
    solve's iteration cap), theta and gamma the safety factors."""
    t_end: float
    dt0: float
    lte_tol: float
    nmaxit: int = 600
    theta: float = 0.8
    gamma: float = 1.3
    dt_min: float = 0.0
    dt_max: float = float("inf")
    max_attempts: int = 1000000


def adapt_decision(eta: float, tol: float, nit: int, nmaxit: int, theta: float, gamma: float):
    """Step-size control of Algorithm 1: (accepted, factor for the next trial step).
    eta <= tol: accepted unless nit >= nmaxit; the factor is min(theta sqrt(tol/eta),
    gamma) when nit/nmaxit < 0.7, min(theta sqrt(tol/eta), 1) below 1, and 1/gamma
    for a failed fixed point.  eta > tol: rejected, factor 1/gamma if eta/tol > 2,
    else theta sqrt(tol/eta)."""
    grow = theta * np.sqrt(tol / eta) if eta > 0 else float("inf")
    if eta <= tol:
        r = nit / nmaxit
        if r < 0.7:
            return True, min(grow, gamma)
        if r < 1.0:
            return True, min(grow, 1.0)
        return False, 1.0 / gamma
    if eta / tol > 2.0:
        return False, 1.0 / gamma
    return False, grow


def adaptive_solve(grid: Grid, params: Params, u0: np.ndarray, ap: AdaptParams, vch: bool = False,
                   stop=None):
    """Adaptive BE-BDF2 time stepping (Algorithm 1): each attempt solves a BE
    step and a variable-step BDF2 step from the same state; eta = max|u_BE -
    u_BDF2| and the BDF2 solution is kept (reading).  The first step has no
    history: it uses the printed Richardson estimate eta = |u_dt - u_dt/2|/2 of
    BE and keeps the two half steps.  `stop(t, u)` may end the run early.
    Returns (u, records) with records (t, dt, eta, iters, accepted)."""
    stepf = vch_step if vch else step
    u = np.ascontiguousarray(u0, dtype=np.float64).copy()
    uprev, dtprev = None, None
    t, dt = 0.0, ap.dt0
    recs = []
    base = dict(eps=params.eps, tol=params.tol, max_iter=ap.nmaxit, init=params.init, sigma0=params.sigma0,
                reaction=params.reaction, react_k=params.react_k)
    for _ in range(ap.max_attempts):
        if t >= ap.t_end * (1 - 1e-14):
            break
        dt = min(dt, ap.t_end - t, ap.dt_max)
        if dt < ap.dt_min:
            raise RuntimeError("time step fell below dt_min")
        if uprev is None:
            full, i1 = stepf(grid, Params(dt=dt, stepper=BE, **base), u)
            half1, i2 = stepf(grid, Params(dt=dt / 2, stepper=BE, **base), u)
            cand, i3 = stepf(grid, Params(dt=dt / 2, stepper=BE, **base), half1)
            eta = 0.5 * float(np.abs(full - cand).max())
            nit = max(i1.iters, i2.iters, i3.iters)
        else:
            be, i1 = stepf(grid, Params(dt=dt, stepper=BE, **base), u)
            cand, i2 = stepf(grid, Params(dt=dt, stepper=BDF2, omega=dt / dtprev, **base), u, uprev)
            eta = float(np.abs(be - cand).max())
            nit = max(i1.iters, i2.iters)
        ok, fac = adapt_decision(eta, ap.lte_tol, nit, ap.nmaxit, ap.theta, ap.gamma)
        recs.append((t, dt, eta, nit, ok))
        if ok:
            uprev, u = u, cand
            t += dt
            dtprev = dt
            if stop is not None and stop(t, u):
                break
        dt *= fac
    return u, recs
