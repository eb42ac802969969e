"""Seeded synthetic inputs: counter-based SplitMix64 streams.

This module holds random-number generation and the initial-condition recipes
only, none of the solver's arithmetic.  It is the one module that both the GPU
path and the FP64 oracle's tests draw inputs from, so that both see the same
array.

SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): state_i = seed + (i+1)*0x9E3779B97F4A7C15, then the
64-bit finalizer.  Uniforms take the top 53 bits; normals use Box-Muller on two
independent streams.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

#: Base seed of every workload stream (the arXiv number of the paper).
BASE_SEED = 161104214


def splitmix64(seed: int, n: int, stream: int = 0) -> np.ndarray:
    """n raw 64-bit outputs of the counter-based SplitMix64 stream (seed, stream)."""
    with np.errstate(over="ignore"):
        base = np.uint64((seed * 0x100000001B3 + stream * 0xD1B54A32D192ED03) % (1 << 64))
        z = base + (np.arange(1, n + 1, dtype=np.uint64) * _GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, n: int, stream: int = 0) -> np.ndarray:
    """n doubles uniform on [0, 1) (53-bit)."""
    return (splitmix64(seed, n, stream) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, n: int, stream: int = 0) -> np.ndarray:
    """n standard normals (Box-Muller on streams 2*stream and 2*stream+1)."""
    u1 = uniform(seed, n, 2 * stream)
    u2 = uniform(seed, n, 2 * stream + 1)
    u1 = np.where(u1 <= 0.0, 2.0 ** -53, u1)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


# --------------------------------------------------------------------------
# Initial conditions of the workloads (u, the paper's variable).
# --------------------------------------------------------------------------
def u0_uniform_noise(seed: int, ny: int, nx: int, amp: float, mean: float = 0.0,
                     zero_mean: bool = False) -> np.ndarray:
    """mean + amp*U(-1,1) i.i.d. per node; zero_mean subtracts the sample mean of the noise."""
    r = amp * (2.0 * uniform(seed, ny * nx) - 1.0)
    if zero_mean:
        r = r - r.mean()
    return (mean + r).reshape(ny, nx) if ny > 1 else (mean + r)


def u0_normal_noise(seed: int, ny: int, nx: int, mean: float, amp: float) -> np.ndarray:
    """mean + amp*N(0,1) i.i.d. per node (the off-critical quench)."""
    r = mean + amp * normal(seed, ny * nx)
    return r.reshape(ny, nx) if ny > 1 else r


def u0_table1(x: np.ndarray) -> np.ndarray:
    """1D initial condition of the paper's temporal refinement study (Sec. 4.4)."""
    return np.cos(2.0 * x) + 0.01 * np.exp(np.cos(x + 0.1))


def u0_table4(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """2D benchmark initial condition of Sec. 5.1 on [0,2pi]^2 (rows = y)."""
    X, Y = np.meshgrid(x, y)
    return 2.0 * np.exp(np.sin(X) + np.sin(Y) - 2.0) + 2.2 * np.exp(-np.sin(X) - np.sin(Y) - 2.0) - 1.0


# Workload recipes (seeded): each returns (description dict, u0).
WORKLOADS = {
    "ch1d_be_n256": dict(dim=1, n=256, bc="periodic", L=2 * np.pi, eps=0.05, dt=1e-3, stepper="BE",
                         tol=1e-10, steps=200, M=4, precision="f64"),
    "ch2d_neumann_bdf2_512": dict(dim=2, n=512, bc="neumann", L=1.0, eps=0.01, dt=5e-5, stepper="BDF2",
                                  tol=1e-10, steps=2000, M=4, precision="f64"),
    "ch2d_periodic_bdf2_4096": dict(dim=2, n=4096, bc="periodic", L=1.0, eps=0.005, dt=1e-5,
                                    stepper="BDF2", tol=1e-8, steps=500, M=4, precision="f32"),
}


def workload_u0(name: str, n: int | None = None) -> np.ndarray:
    """Initial field of a named workload (optionally on an n-point side instead)."""
    w = WORKLOADS[name]
    side = n or w["n"]
    idx = list(WORKLOADS).index(name)
    seed = BASE_SEED + idx + 1
    if name == "ch1d_be_n256":
        return u0_uniform_noise(seed, 1, side, 0.1, zero_mean=True)
    if name == "ch2d_neumann_bdf2_512":
        return u0_uniform_noise(seed, side, side, 0.05)
    if name == "ch2d_periodic_bdf2_4096":
        return u0_normal_noise(seed, side, side, 0.3, 0.05)
    raise KeyError(name)


# Batched workload: independent 2D instances with uneven sizes and parameters.
#: seed of the batched workload's draws (fourth workload recipe)
BATCH_SEED = BASE_SEED + 4


def batch_instances(count: int = 256, seed: int = BATCH_SEED, steps: int = 100) -> list:
    """Seeded instance draws: side n = round(exp(U(ln 64, ln 1024))), eps ~ U[0.005, 0.05],
    dt ~ U[1e-6, 1e-4], boundary periodic/Neumann and stepper BE/BDF2 each with
    probability 1/2, domain [0,1]^2, M = 4, tolerance 1e-8, `steps` steps each."""
    un, ue, ut = uniform(seed, count, 0), uniform(seed, count, 1), uniform(seed, count, 2)
    ub, us = uniform(seed, count, 3), uniform(seed, count, 4)
    lo, hi = np.log(64.0), np.log(1024.0)
    out = []
    for i in range(count):
        out.append(dict(n=int(round(float(np.exp(lo + un[i] * (hi - lo))))),
                        eps=0.005 + 0.045 * float(ue[i]), dt=1e-6 + (1e-4 - 1e-6) * float(ut[i]),
                        bc="periodic" if ub[i] < 0.5 else "neumann",
                        stepper="BE" if us[i] < 0.5 else "BDF2",
                        steps=steps, M=4, L=1.0, tol=1e-8, seed=seed, stream=16 + i))
    return out


def instance_u0(inst: dict) -> np.ndarray:
    """0.05 U(-1,1) i.i.d. per node on the instance's own stream (n x n)."""
    n = inst["n"]
    return (0.05 * (2.0 * uniform(inst["seed"], n * n, inst["stream"]) - 1.0)).reshape(n, n)


# Vector (three-phase) model: fractions c_i >= 0, sum 1, mapped to
# u = sum_i c_i z_i with z_i the cube roots of unity in the (u1, u2) plane.
VCH_Z = np.array([[1.0, 0.0], [-0.5, np.sqrt(3.0) / 2.0], [-0.5, -np.sqrt(3.0) / 2.0]])


def u0_vch(seed: int, ny: int, nx: int, stream: int = 0) -> np.ndarray:
    """Fractions c = 0.9 (1/3, 1/3, 1/3) + 0.1 Dirichlet(1,1,1) per node (the
    Dirichlet draw as normalized exponentials of three uniform streams); returns
    u as (2, ny, nx), component-major."""
    n = ny * nx
    e = np.stack([-np.log(np.maximum(uniform(seed, n, 3 * stream + k), 2.0 ** -53)) for k in range(3)])
    c = 0.9 / 3.0 + 0.1 * e / e.sum(axis=0)
    u = VCH_Z.T @ c
    return u.reshape(2, ny, nx)


def with_walls(u: np.ndarray, value) -> np.ndarray:
    """A copy of u with every wall node (first/last row and column; both ends
    of a 1D line) set to `value` (a scalar, or one value per component for a
    (2, ny, nx) vector field): inputs for Dirichlet walls."""
    w = np.array(u, dtype=np.float64, copy=True)
    comps = [w] if w.ndim < 3 else [w[k] for k in range(w.shape[0])]
    vals = [value] if w.ndim < 3 else list(value)
    for f, v in zip(comps, vals):
        if f.ndim == 1 or f.shape[0] == 1:  # a line: its two ends
            f.reshape(-1)[[0, -1]] = v
        else:
            f[0, :] = f[-1, :] = v
            f[:, 0] = f[:, -1] = v
    return w


# Served workload: Poisson arrivals of vector-model requests.
#: seed of the served workload's draws (fifth workload recipe)
SERVE_SEED = BASE_SEED + 5


def serve_requests(count: int, rate: float, seed: int = SERVE_SEED, n_min: int = 128, n_max: int = 2048,
                   steps_min: int = 10, steps_max: int = 500) -> list:
    """`count` requests with exponential inter-arrival gaps of mean 1/rate (s):
    side n = round(exp(U(ln n_min, ln n_max))), steps uniform on
    {steps_min..steps_max}, eps ~ U[0.005, 0.05], dt ~ U[1e-6, 1e-4], periodic
    or Neumann and BE or BDF2 each with probability 1/2, domain [0,1]^2, M = 4,
    tolerance 1e-8; the initial fractions come from u0_vch on stream 100 + i."""
    gaps = -np.log(np.maximum(uniform(seed, count, 0), 2.0 ** -53)) / rate
    un, us = uniform(seed, count, 1), uniform(seed, count, 2)
    ue, ut = uniform(seed, count, 3), uniform(seed, count, 4)
    ub, uq = uniform(seed, count, 5), uniform(seed, count, 6)
    lo, hi = np.log(float(n_min)), np.log(float(n_max))
    t = np.cumsum(gaps)
    out = []
    for i in range(count):
        out.append(dict(id=i, arrival=float(t[i]), n=int(round(float(np.exp(lo + un[i] * (hi - lo))))),
                        steps=steps_min + int(us[i] * (steps_max - steps_min + 1)),
                        eps=0.005 + 0.045 * float(ue[i]), dt=1e-6 + (1e-4 - 1e-6) * float(ut[i]),
                        bc="periodic" if ub[i] < 0.5 else "neumann",
                        stepper="BE" if uq[i] < 0.5 else "BDF2", M=4, L=1.0, tol=1e-8,
                        seed=seed, stream=100 + i))
    return out
