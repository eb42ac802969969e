"""ctypes binding of libmolt (C-ABI in include/molt.h).

Argument marshalling only: every step of the solver runs in the HIP library.
The functions keep the C names; device buffers are passed as integer device
addresses (e.g. ``tensor.data_ptr()``) and streams as integer handles
(``torch.cuda.current_stream().cuda_stream``).  A missing or unloadable
library raises immediately -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
#: the in-tree library; MOLT_LIB may name another build of the same sources
LIB_PATH = os.environ.get("MOLT_LIB", os.path.join(HERE, "libmolt.so"))

MOLT_OK, MOLT_NOT_CONVERGED = 0, 1
MOLT_EINVAL, MOLT_EUNSUPPORTED, MOLT_EHIP, MOLT_EWORKSPACE = -1, -2, -3, -4
MOLT_BC_PERIODIC, MOLT_BC_NEUMANN, MOLT_BC_DIRICHLET = 0, 1, 2
MOLT_BE, MOLT_BDF2, MOLT_BDF3 = 0, 1, 2
MOLT_INIT_PREV, MOLT_INIT_LINEAR = 0, 1
MOLT_MODEL_CH, MOLT_MODEL_VCH = 0, 1
#: sigma0 of the vector model (the Hessian of W at its minima is 18 I)
VCH_SIGMA0 = 18.0
MOLT_F64, MOLT_F32 = 0, 1

#: every symbol include/molt.h declares
EXPORTS = ("mol_t_helmholtz_sweep", "molt_sweep_workspace_bytes", "ch_workspace_bytes", "ch_step",
           "ch_solve", "ch_adaptive_workspace_bytes", "ch_solve_adaptive", "ch_batch_workspace_bytes",
           "ch_solve_batch", "molt_tune_get", "molt_tune_set",
           "molt_autotune_workspace_bytes", "molt_autotune", "molt_server_footprint", "molt_server_bytes",
           "molt_server_create", "molt_server_submit", "molt_server_run", "molt_server_poll",
           "molt_server_destroy", "molt_strerror", "molt_last_error", "molt_profile", "molt_profile_only",
           "molt_profile_read",
           "molt_set_option", "mol_t_helmholtz_sweep_noalloc", "molt_noalloc_scratch_bytes")
MOLT_TUNE_CLASSES = 7
MOLT_OPT_BATCH_TICKS, MOLT_OPT_BATCH_GRAPH, MOLT_OPT_BATCH_LEAN, MOLT_OPT_STEP_GRAPH = 2, 3, 5, 6

KERNEL_FAMILIES = ("xpass", "ytot", "ycomb", "yfin", "pointwise", "other")
PROGRAMS = ("sweep", "rhs", "P1", "P2", "P3", "P4", "P1v", "P2v")


#: kinds of FP64 launches are offset by this (their names start with "f64_")
PROF_F64 = 48


def kind_name(kind: int) -> str:
    f, p = divmod(kind % PROF_F64, 8)
    return ("f64_" if kind >= PROF_F64 else "") + f"{KERNEL_FAMILIES[f]}_{PROGRAMS[p] if p < len(PROGRAMS) else p}"


def kind_of(name: str) -> int:
    """Inverse of kind_name."""
    off = 0
    if name.startswith("f64_"):
        off, name = PROF_F64, name[4:]
    fam, prog = name.split("_", 1)
    return off + KERNEL_FAMILIES.index(fam) * 8 + PROGRAMS.index(prog)


class molt_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double),
                ("y0", ctypes.c_double), ("y1", ctypes.c_double),
                ("bc", ctypes.c_int32), ("order_M", ctypes.c_int32)]


class molt_ch_params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("dt", ctypes.c_double), ("tol", ctypes.c_double),
                ("sigma0", ctypes.c_double), ("stepper", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("init", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("fixed_iters", ctypes.c_int32), ("have_prev", ctypes.c_int32),
                ("model", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class molt_step_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("residual", ctypes.c_double), ("mass", ctypes.c_double), ("energy", ctypes.c_double),
                ("s1", ctypes.c_double), ("s2", ctypes.c_double), ("sigma", ctypes.c_double),
                ("mass2", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class molt_adapt_params(ctypes.Structure):
    _fields_ = [("t_end", ctypes.c_double), ("dt0", ctypes.c_double), ("lte_tol", ctypes.c_double),
                ("theta", ctypes.c_double), ("gamma", ctypes.c_double), ("dt_min", ctypes.c_double),
                ("dt_max", ctypes.c_double), ("nmaxit", ctypes.c_int32), ("max_attempts", ctypes.c_int32)]


class molt_adapt_record(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt", ctypes.c_double), ("eta", ctypes.c_double),
                ("iters", ctypes.c_int32), ("accepted", ctypes.c_int32), ("energy", ctypes.c_double)]


class molt_instance(ctypes.Structure):
    _fields_ = [("grid", molt_grid), ("params", molt_ch_params), ("d_u", ctypes.c_void_p),
                ("nsteps", ctypes.c_int64)]


class molt_result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("iters", ctypes.c_int64), ("last", molt_step_info)]


class molt_prof_entry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Open libmolt.so (raises OSError if it is missing: build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"libmolt.so not found at {path}; run `python -m paper_1611_04214_amd.build`")
    lib = ctypes.CDLL(path)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    G, P = ctypes.POINTER(molt_grid), ctypes.POINTER(molt_ch_params)
    lib.mol_t_helmholtz_sweep.argtypes = [G, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, vp, vp,
                                          ctypes.c_int64, vp, sz, vp]
    lib.mol_t_helmholtz_sweep.restype = ctypes.c_int32
    lib.molt_sweep_workspace_bytes.argtypes = [G, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64]
    lib.molt_sweep_workspace_bytes.restype = sz
    lib.mol_t_helmholtz_sweep_noalloc.argtypes = [G, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, vp, vp,
                                                  ctypes.c_int64, vp]
    lib.mol_t_helmholtz_sweep_noalloc.restype = ctypes.c_int32
    lib.molt_noalloc_scratch_bytes.argtypes = []
    lib.molt_noalloc_scratch_bytes.restype = sz
    lib.ch_workspace_bytes.argtypes = [G, P]
    lib.ch_workspace_bytes.restype = sz
    lib.ch_step.argtypes = [G, P, vp, vp, vp, sz, ctypes.POINTER(molt_step_info), vp]
    lib.ch_step.restype = ctypes.c_int32
    lib.ch_solve.argtypes = [G, P, vp, ctypes.c_int64, vp, sz, ctypes.POINTER(molt_step_info), vp]
    lib.ch_solve.restype = ctypes.c_int32
    lib.ch_adaptive_workspace_bytes.argtypes = [G, P]
    lib.ch_adaptive_workspace_bytes.restype = sz
    lib.ch_solve_adaptive.argtypes = [G, P, ctypes.POINTER(molt_adapt_params), vp, vp, sz,
                                      ctypes.POINTER(molt_adapt_record), ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), vp]
    lib.ch_solve_adaptive.restype = ctypes.c_int32
    I = ctypes.POINTER(molt_instance)
    lib.ch_batch_workspace_bytes.argtypes = [I, ctypes.c_int32]
    lib.ch_batch_workspace_bytes.restype = sz
    lib.ch_solve_batch.argtypes = [I, ctypes.c_int32, vp, sz, ctypes.POINTER(molt_step_info), vp]
    lib.ch_solve_batch.restype = ctypes.c_int32
    i32, pi32 = ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)
    lib.molt_tune_get.argtypes = [i32, i32, pi32, pi32]
    lib.molt_tune_get.restype = i32
    lib.molt_tune_set.argtypes = [i32, i32, i32, i32]
    lib.molt_tune_set.restype = i32
    lib.molt_autotune_workspace_bytes.argtypes = [i32, i32]
    lib.molt_autotune_workspace_bytes.restype = sz
    lib.molt_autotune.argtypes = [i32, i32, vp, sz, vp]
    lib.molt_autotune.restype = i32
    lib.molt_server_footprint.argtypes = [I]
    lib.molt_server_footprint.restype = sz
    lib.molt_server_bytes.argtypes = [i32, i32, sz]
    lib.molt_server_bytes.restype = sz
    lib.molt_server_create.argtypes = [i32, i32, vp, sz, vp, ctypes.POINTER(vp)]
    lib.molt_server_create.restype = i32
    lib.molt_server_submit.argtypes = [vp, I, ctypes.c_int64]
    lib.molt_server_submit.restype = i32
    lib.molt_server_run.argtypes = [vp, i32, pi32, pi32]
    lib.molt_server_run.restype = i32
    lib.molt_server_poll.argtypes = [vp, ctypes.POINTER(molt_result), i32]
    lib.molt_server_poll.restype = i32
    lib.molt_server_destroy.argtypes = [vp]
    lib.molt_server_destroy.restype = i32
    lib.molt_strerror.argtypes = [ctypes.c_int32]
    lib.molt_strerror.restype = ctypes.c_char_p
    lib.molt_last_error.argtypes = []
    lib.molt_last_error.restype = ctypes.c_char_p
    lib.molt_set_option.argtypes = [ctypes.c_int32, ctypes.c_int64]
    lib.molt_set_option.restype = ctypes.c_int32
    lib.molt_profile.argtypes = [ctypes.c_int32]
    lib.molt_profile.restype = ctypes.c_int32
    lib.molt_profile_only.argtypes = [ctypes.c_int32]
    lib.molt_profile_only.restype = ctypes.c_int32
    lib.molt_profile_read.argtypes = [ctypes.POINTER(molt_prof_entry), ctypes.c_int32]
    lib.molt_profile_read.restype = ctypes.c_int32
    _lib = lib
    return lib


class MoltError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str | None = None):
        lib = load()
        if detail is None:
            detail = lib.molt_last_error().decode()
        super().__init__(f"{where}: {lib.molt_strerror(status).decode()} ({status}): {detail}")
        self.status = status


def _check_tensor(t, where: str, what: str, precision: int, numel: int | None, multiple_of: int | None = None):
    """Raise MoltError (MOLT_EINVAL) unless t is a contiguous device tensor of
    the element type the precision names (float64 for MOLT_F64, float32 for
    MOLT_F32) holding exactly numel elements (or a positive multiple of
    multiple_of): the library takes a bare address and would otherwise read or
    write outside the tensor."""
    import torch
    want = {MOLT_F64: torch.float64, MOLT_F32: torch.float32}.get(precision)
    if want is None:
        raise MoltError(MOLT_EINVAL, where, f"unknown precision {precision}")
    if not isinstance(t, torch.Tensor):
        raise MoltError(MOLT_EINVAL, where, f"{what} must be a torch tensor")
    if t.dtype != want:
        raise MoltError(MOLT_EINVAL, where, f"{what} is {t.dtype}, the precision needs {want}")
    if not t.is_contiguous():
        raise MoltError(MOLT_EINVAL, where, f"{what} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise MoltError(MOLT_EINVAL, where, f"{what} holds {t.numel()} elements, the call needs {numel}")
    if multiple_of is not None and (t.numel() == 0 or t.numel() % multiple_of != 0):
        raise MoltError(MOLT_EINVAL, where,
                        f"{what} holds {t.numel()} elements, not a positive multiple of {multiple_of}")


def _check_device(where: str, *named) -> None:
    """Every (name, tensor) on one HIP device (after the type and size checks)."""
    dev = None
    for what, t in named:
        if not t.is_cuda:
            raise MoltError(MOLT_EINVAL, where, f"{what} must be on a HIP device")
        if dev is not None and t.device != dev:
            raise MoltError(MOLT_EINVAL, where, f"{what} is on another device")
        dev = t.device


def _field_elems(grid: molt_grid, params: molt_ch_params) -> int:
    """Elements of one field of this problem (both components for the vector model)."""
    return grid.nx * grid.ny * (2 if params.model == MOLT_MODEL_VCH else 1)


def _check_workspace(work, need: int, where: str, device) -> None:
    import torch
    if not isinstance(work, torch.Tensor) or not work.is_contiguous() or work.device != device:
        raise MoltError(MOLT_EINVAL, where, "the workspace must be a contiguous tensor on the field's device")
    if work.numel() * work.element_size() < need:
        raise MoltError(MOLT_EWORKSPACE, where, f"workspace of {work.numel() * work.element_size()} bytes, "
                                                f"the call needs {need}")


def _check(status: int, where: str, allow_not_converged: bool = True) -> int:
    if status < 0 or (status == MOLT_NOT_CONVERGED and not allow_not_converged):
        raise MoltError(status, where)
    return status


# ---------------------------------------------------------------- raw C-ABI --
def mol_t_helmholtz_sweep(grid: molt_grid, axis: int, alpha: float, precision: int, d_in: int, d_out: int,
                          batch: int, d_work: int, work_bytes: int, stream: int = 0) -> int:
    return load().mol_t_helmholtz_sweep(ctypes.byref(grid), axis, alpha, precision, d_in, d_out, batch,
                                        d_work or None, work_bytes, stream or None)


def molt_sweep_workspace_bytes(grid: molt_grid, axis: int, precision: int, batch: int) -> int:
    return load().molt_sweep_workspace_bytes(ctypes.byref(grid), axis, precision, batch)


def mol_t_helmholtz_sweep_noalloc(grid: molt_grid, axis: int, alpha: float, precision: int, d_in: int, d_out: int,
                                  batch: int, stream: int = 0) -> int:
    return load().mol_t_helmholtz_sweep_noalloc(ctypes.byref(grid), axis, alpha, precision, d_in, d_out, batch,
                                                stream or None)


def molt_noalloc_scratch_bytes() -> int:
    return load().molt_noalloc_scratch_bytes()


def ch_workspace_bytes(grid: molt_grid, params: molt_ch_params) -> int:
    return load().ch_workspace_bytes(ctypes.byref(grid), ctypes.byref(params))


def ch_step(grid: molt_grid, params: molt_ch_params, d_u: int, d_u_prev: int, d_work: int, work_bytes: int,
            info: molt_step_info | None = None, stream: int = 0) -> int:
    return load().ch_step(ctypes.byref(grid), ctypes.byref(params), d_u, d_u_prev or None, d_work or None,
                          work_bytes, ctypes.byref(info) if info is not None else None, stream or None)


def ch_solve(grid: molt_grid, params: molt_ch_params, d_u: int, nsteps: int, d_work: int, work_bytes: int,
             per_step=None, stream: int = 0) -> int:
    return load().ch_solve(ctypes.byref(grid), ctypes.byref(params), d_u, nsteps, d_work or None, work_bytes,
                           per_step, stream or None)


def ch_adaptive_workspace_bytes(grid: molt_grid, params: molt_ch_params) -> int:
    return load().ch_adaptive_workspace_bytes(ctypes.byref(grid), ctypes.byref(params))


def ch_solve_adaptive(grid, params, adapt, d_u: int, d_work: int, work_bytes: int, rec=None, max_rec: int = 0,
                      nrec=None, t_final=None, stream: int = 0) -> int:
    return load().ch_solve_adaptive(ctypes.byref(grid), ctypes.byref(params), ctypes.byref(adapt), d_u,
                                    d_work or None, work_bytes, rec, max_rec, nrec, t_final, stream or None)


def make_adapt(t_end: float, dt0: float, lte_tol: float, nmaxit: int = 600, theta: float = 0.8,
               gamma: float = 1.3, dt_min: float = 0.0, dt_max: float = 1e300,
               max_attempts: int = 1000000) -> molt_adapt_params:
    return molt_adapt_params(t_end, dt0, lte_tol, theta, gamma, dt_min, dt_max, nmaxit, max_attempts)


def solve_adaptive(u, grid: molt_grid, params: molt_ch_params, adapt: molt_adapt_params, max_rec: int = 100000):
    """ch_solve_adaptive in place on u; returns (status, [molt_adapt_record], t_final)."""
    import torch
    _check_tensor(u, "ch_solve_adaptive", "u", params.precision, _field_elems(grid, params))
    _check_device("ch_solve_adaptive", ("u", u))
    need = ch_adaptive_workspace_bytes(grid, params)
    if need == 0:
        raise MoltError(MOLT_EINVAL, "ch_adaptive_workspace_bytes")
    work = workspace(need, u.device)
    rec = (molt_adapt_record * max_rec)()
    n, tf = ctypes.c_int32(), ctypes.c_double()
    st = _check(ch_solve_adaptive(grid, params, adapt, u.data_ptr(), work.data_ptr(), work.numel(), rec, max_rec,
                                  ctypes.byref(n), ctypes.byref(tf), _stream(torch)), "ch_solve_adaptive")
    return st, [rec[i] for i in range(min(n.value, max_rec))], tf.value


def ch_batch_workspace_bytes(inst, count: int) -> int:
    return load().ch_batch_workspace_bytes(inst, count)


def ch_solve_batch(inst, count: int, d_work: int, work_bytes: int, per_step=None, stream: int = 0) -> int:
    return load().ch_solve_batch(inst, count, d_work or None, work_bytes, per_step, stream or None)


def molt_tune_get(precision: int, size_class: int):
    """(kx, ky) of one line-length class."""
    kx, ky = ctypes.c_int32(), ctypes.c_int32()
    _check(load().molt_tune_get(precision, size_class, ctypes.byref(kx), ctypes.byref(ky)), "molt_tune_get")
    return kx.value, ky.value


def molt_tune_set(precision: int, size_class: int, kx: int, ky: int) -> int:
    return load().molt_tune_set(precision, size_class, kx, ky)


def molt_autotune_workspace_bytes(precision: int, max_n: int) -> int:
    return load().molt_autotune_workspace_bytes(precision, max_n)


def molt_autotune(precision: int, max_n: int, d_work: int, work_bytes: int, stream: int = 0) -> int:
    return load().molt_autotune(precision, max_n, d_work or None, work_bytes, stream or None)


def tune_table(precision: int):
    """The whole shape table of one precision: [(kx, ky)] by size class."""
    return [molt_tune_get(precision, c) for c in range(MOLT_TUNE_CLASSES)]


def autotune(precision: int, max_n: int):
    """molt_autotune with a temporary workspace; returns the new table."""
    import torch
    need = molt_autotune_workspace_bytes(precision, max_n)
    if need == 0:
        raise MoltError(MOLT_EINVAL, "molt_autotune_workspace_bytes")
    work = workspace(need)
    _check(molt_autotune(precision, max_n, work.data_ptr(), work.numel(), _stream(torch)), "molt_autotune")
    return tune_table(precision)


def molt_strerror(status: int) -> str:
    return load().molt_strerror(status).decode()


def molt_last_error() -> str:
    return load().molt_last_error().decode()


def molt_set_option(option: int, value: int) -> int:
    return load().molt_set_option(option, value)


def molt_profile(enable: int) -> int:
    return load().molt_profile(enable)


def molt_profile_only(kind: int) -> int:
    return load().molt_profile_only(kind)


def molt_profile_read(max_entries: int = 96) -> dict:
    """{kind name: (launches, total_ms)} of the kernels timed since molt_profile(1)."""
    buf = (molt_prof_entry * max_entries)()
    m = load().molt_profile_read(buf, max_entries)
    if m < 0:
        raise MoltError(m, "molt_profile_read")
    return {kind_name(buf[i].kind): (buf[i].launches, buf[i].total_ms) for i in range(m)}


# ------------------------------------------------- torch-tensor conveniences --
def make_grid(nx: int, ny: int = 1, x0: float = 0.0, x1: float = 1.0, y0: float = 0.0, y1: float = 1.0,
              bc: int = MOLT_BC_PERIODIC, M: int = 4) -> molt_grid:
    return molt_grid(nx, ny, x0, x1, y0, y1, bc, M)


def make_params(eps: float, dt: float, tol: float = 1e-10, stepper: int = MOLT_BE, max_iter: int = 300,
                init: int = MOLT_INIT_PREV, precision: int = MOLT_F64, fixed_iters: int = 0,
                have_prev: int = 0, sigma0: float | None = None, model: int = MOLT_MODEL_CH) -> molt_ch_params:
    """Step parameters; sigma0 defaults to 2 (Cahn-Hilliard) or 18 (vector model)."""
    if sigma0 is None:
        sigma0 = VCH_SIGMA0 if model == MOLT_MODEL_VCH else 2.0
    return molt_ch_params(eps, dt, tol, sigma0, stepper, max_iter, init, precision, fixed_iters, have_prev,
                          model, 0)


def _stream(torch):
    return torch.cuda.current_stream().cuda_stream


def workspace(nbytes: int, device="cuda"):
    """A caller-owned device workspace (uint8 tensor) of nbytes."""
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def sweep(field, grid: molt_grid, axis: int, alpha: float, out=None, work=None):
    """L^{-1} along axis of a (batch, ny, nx) / (ny, nx) / (nx,) device tensor."""
    import torch
    where = "mol_t_helmholtz_sweep"
    if field.dtype not in (torch.float64, torch.float32):
        raise MoltError(MOLT_EINVAL, where, f"field is {field.dtype}; float64 or float32 only")
    prec = MOLT_F64 if field.dtype == torch.float64 else MOLT_F32
    f = field.contiguous()
    _check_tensor(f, where, "field", prec, None, multiple_of=grid.nx * grid.ny)
    batch = f.numel() // (grid.nx * grid.ny)
    out = torch.empty_like(f) if out is None else out
    _check_tensor(out, where, "out", prec, f.numel())
    _check_device(where, ("field", f), ("out", out))
    need = molt_sweep_workspace_bytes(grid, axis, prec, batch)
    if need == 0:
        raise MoltError(MOLT_EINVAL, "molt_sweep_workspace_bytes")
    if work is None:
        work = workspace(need, f.device)
    _check_workspace(work, need, where, f.device)
    _check(mol_t_helmholtz_sweep(grid, axis, alpha, prec, f.data_ptr(), out.data_ptr(), batch, work.data_ptr(),
                                 work.numel(), _stream(torch)), "mol_t_helmholtz_sweep")
    return out


def step(u, grid: molt_grid, params: molt_ch_params, u_prev=None, work=None) -> molt_step_info:
    """One ch_step in place on the device tensor u (u_prev: BDF2 history, rotated in place)."""
    import torch
    ne = _field_elems(grid, params)
    _check_tensor(u, "ch_step", "u", params.precision, ne)
    if u_prev is not None:
        _check_tensor(u_prev, "ch_step", "u_prev", params.precision,
                      ne * (2 if params.stepper == MOLT_BDF3 else 1))
    _check_device("ch_step", ("u", u), *([] if u_prev is None else [("u_prev", u_prev)]))
    need = ch_workspace_bytes(grid, params)
    if need == 0:
        raise MoltError(MOLT_EINVAL, "ch_workspace_bytes")
    if work is None:
        work = workspace(need, u.device)
    _check_workspace(work, need, "ch_step", u.device)
    info = molt_step_info()
    _check(ch_step(grid, params, u.data_ptr(), 0 if u_prev is None else u_prev.data_ptr(), work.data_ptr(),
                   work.numel(), info, _stream(torch)), "ch_step")
    return info


def solve(u, grid: molt_grid, params: molt_ch_params, nsteps: int, work=None):
    """ch_solve in place on u; returns (status, [molt_step_info])."""
    import torch
    _check_tensor(u, "ch_solve", "u", params.precision, _field_elems(grid, params))
    _check_device("ch_solve", ("u", u))
    need = ch_workspace_bytes(grid, params)
    if need == 0:
        raise MoltError(MOLT_EINVAL, "ch_workspace_bytes")
    if work is None:
        work = workspace(need, u.device)
    _check_workspace(work, need, "ch_solve", u.device)
    infos = (molt_step_info * max(nsteps, 1))()
    st = _check(ch_solve(grid, params, u.data_ptr(), nsteps, work.data_ptr(), work.numel(), infos,
                         _stream(torch)), "ch_solve")
    return st, [infos[i] for i in range(nsteps)]


def make_instances(specs) -> "ctypes.Array":
    """molt_instance array from (grid, params, device tensor, nsteps) tuples."""
    arr = (molt_instance * len(specs))()
    for i, (g, p, u, ns) in enumerate(specs):
        arr[i].grid = g
        arr[i].params = p
        arr[i].d_u = u.data_ptr()
        arr[i].nsteps = ns
    return arr


def solve_batch(specs, work=None, stream=None):
    """ch_solve_batch over (grid, params, device tensor, nsteps) tuples, in place on
    the tensors; returns (status, per-instance lists of molt_step_info)."""
    import torch
    if not specs:
        raise MoltError(MOLT_EINVAL, "ch_solve_batch", "no instances")
    dev = specs[0][2].device
    for i, (g, p, u, _) in enumerate(specs):
        _check_tensor(u, "ch_solve_batch", f"instance {i}'s field", p.precision, _field_elems(g, p))
    _check_device("ch_solve_batch", *[(f"instance {i}'s field", sp[2]) for i, sp in enumerate(specs)])
    inst = make_instances(specs)
    need = ch_batch_workspace_bytes(inst, len(specs))
    if need == 0:
        raise MoltError(MOLT_EINVAL, "ch_batch_workspace_bytes")
    if work is None:
        work = workspace(need, dev)
    _check_workspace(work, need, "ch_solve_batch", dev)
    nrec = sum(int(s[3]) for s in specs)
    recs = (molt_step_info * max(nrec, 1))()
    st = _check(ch_solve_batch(inst, len(specs), work.data_ptr(), work.numel(), recs,
                               _stream(torch) if stream is None else stream), "ch_solve_batch")
    out, k = [], 0
    for s in specs:
        out.append([recs[k + j] for j in range(int(s[3]))])
        k += int(s[3])
    return st, out


# ------------------------------------------------------------------ serving --
def molt_server_footprint(inst) -> int:
    return load().molt_server_footprint(ctypes.byref(inst))


def molt_server_bytes(precision: int, max_slots: int, pool_bytes: int) -> int:
    return load().molt_server_bytes(precision, max_slots, pool_bytes)


class Server:
    """A resident continuous-batching server (molt_server_*) on one stream.

    Requests are (grid, params, device tensor, nsteps); the tensor is solved in
    place and kept referenced here until its result is polled."""

    def __init__(self, precision: int, max_slots: int, pool_bytes: int, stream=None):
        import torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        need = molt_server_bytes(precision, max_slots, pool_bytes)
        if need == 0:
            raise MoltError(MOLT_EINVAL, "molt_server_bytes")
        self.work = workspace(need)
        self._h = ctypes.c_void_p()
        _check(load().molt_server_create(precision, max_slots, self.work.data_ptr(), self.work.numel(),
                                         self.stream.cuda_stream, ctypes.byref(self._h)), "molt_server_create")
        self._live = {}

    def submit(self, grid: molt_grid, params: molt_ch_params, u, nsteps: int, rid: int) -> None:
        _check_tensor(u, "molt_server_submit", "u", params.precision, _field_elems(grid, params))
        _check_device("molt_server_submit", ("the server's workspace", self.work), ("u", u))
        inst = molt_instance(grid, params, u.data_ptr(), nsteps)
        _check(load().molt_server_submit(self._h, ctypes.byref(inst), rid), "molt_server_submit")
        self._live[rid] = u

    def run(self, rounds: int = 1):
        """Admit what fits and queue `rounds` rounds; returns (admitted, queued)."""
        a, q = ctypes.c_int32(), ctypes.c_int32()
        _check(load().molt_server_run(self._h, rounds, ctypes.byref(a), ctypes.byref(q)), "molt_server_run")
        return a.value, q.value

    def poll(self, max_results: int = 256) -> list:
        buf = (molt_result * max_results)()
        m = load().molt_server_poll(self._h, buf, max_results)
        if m < 0:
            raise MoltError(m, "molt_server_poll")
        out = [buf[i] for i in range(m)]
        for r in out:
            self._live.pop(r.id, None)
        return out

    def close(self) -> None:
        if self._h:
            load().molt_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
