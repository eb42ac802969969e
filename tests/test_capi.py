"""The C-ABI library loads and exports what include/molt.h declares; host-only
argument checks and workspace queries (no device work is launched here)."""
import ctypes
import os
import re

import pytest

from paper_1611_04214_amd import molt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "molt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", src))
    return sorted(n for n in names if n not in {"defined", "sizeof"})


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(molt.LIB_PATH):
        pytest.fail("libmolt.so is not built (run __graft_entry__.build())")
    return molt.load()


def test_every_declared_symbol_is_exported(lib):
    decl = _declared()
    assert set(decl) == set(molt.EXPORTS), decl
    for name in decl:
        assert hasattr(lib, name), name


def test_struct_layouts_match_header():
    # natural C alignment of the header's structs
    assert ctypes.sizeof(molt.molt_grid) == 48
    assert ctypes.sizeof(molt.molt_ch_params) == 64
    assert ctypes.sizeof(molt.molt_step_info) == 64
    assert ctypes.sizeof(molt.molt_instance) == 128
    assert ctypes.sizeof(molt.molt_result) == 88
    assert ctypes.sizeof(molt.molt_adapt_params) == 64
    assert ctypes.sizeof(molt.molt_adapt_record) == 40


def test_strerror_names_every_status(lib):
    for code in (0, 1, -1, -2, -3, -4):
        assert molt.molt_strerror(code) not in ("", "unknown status")
    assert molt.molt_strerror(99) == "unknown status"


def test_workspace_queries(lib):
    g = molt.make_grid(64, 48, bc=molt.MOLT_BC_NEUMANN, M=4)
    p = molt.make_params(0.02, 1e-4, precision=molt.MOLT_F32)
    w32 = molt.ch_workspace_bytes(g, p)
    p.precision = molt.MOLT_F64
    w64 = molt.ch_workspace_bytes(g, p)
    # an FP32 problem also carries the FP64 shadow of its R phase and FP64 iterations
    assert w32 > 10 * 64 * 48 * 4 and w64 > 10 * 64 * 48 * 8 and w32 > w64
    # BDF3 keeps a second history and the SDIRK2 stage value: two fields more
    p.stepper = molt.MOLT_BDF3
    assert molt.ch_workspace_bytes(g, p) >= w64 + 2 * 64 * 48 * 8
    assert molt.molt_sweep_workspace_bytes(g, 0, molt.MOLT_F32, 1) > 0
    assert molt.molt_sweep_workspace_bytes(g, 1, molt.MOLT_F32, 3) > 3 * 64 * 48 * 4


@pytest.mark.parametrize("change,code", [
    (dict(nx=4), molt.MOLT_EINVAL),          # fewer than M+1 nodes
    (dict(order_M=3), molt.MOLT_EINVAL),
    (dict(bc=7), molt.MOLT_EINVAL),
    (dict(x1=0.0), molt.MOLT_EINVAL),
    (dict(nx=20000), molt.MOLT_EUNSUPPORTED),
])
def test_bad_grids_are_rejected_before_any_device_work(lib, change, code):
    g = molt.make_grid(32, 32, M=4)
    for k, v in change.items():
        setattr(g, k, v)
    p = molt.make_params(0.05, 1e-3)
    assert molt.ch_workspace_bytes(g, p) == 0
    rc = molt.ch_step(g, p, 1, 0, 1, 1 << 30)
    assert rc == code, (rc, molt.molt_last_error())
    assert molt.molt_last_error() != ""


@pytest.mark.parametrize("change", [dict(eps=0.0), dict(dt=-1.0), dict(stepper=5), dict(init=9),
                                    dict(max_iter=0), dict(fixed_iters=-2), dict(precision=3)])
def test_bad_params_are_rejected(lib, change):
    g = molt.make_grid(32, 32, M=4)
    p = molt.make_params(0.05, 1e-3)
    for k, v in change.items():
        setattr(p, k, v)
    assert molt.ch_step(g, p, 1, 0, 1, 1 << 30) == molt.MOLT_EINVAL


def test_vector_model_with_bdf3_is_unsupported(lib):
    g = molt.make_grid(32, 32, M=4)
    p = molt.make_params(0.05, 1e-5, stepper=molt.MOLT_BDF3, model=molt.MOLT_MODEL_VCH)
    assert molt.ch_workspace_bytes(g, p) == 0
    assert molt.ch_step(g, p, 1, 0, 1, 1 << 30) == molt.MOLT_EUNSUPPORTED
    # the adaptive driver ignores the stepper
    assert molt.ch_adaptive_workspace_bytes(g, p) > 0


def test_small_workspace_is_rejected(lib):
    g = molt.make_grid(32, 32, M=4)
    p = molt.make_params(0.05, 1e-3)
    need = molt.ch_workspace_bytes(g, p)
    assert molt.ch_step(g, p, 1, 0, 1, need - 1) == molt.MOLT_EWORKSPACE
    assert molt.ch_solve(g, p, 1, 3, 1, need - 1) == molt.MOLT_EWORKSPACE


def test_sweep_argument_checks(lib):
    g = molt.make_grid(32, 16, M=4)
    assert molt.mol_t_helmholtz_sweep(g, 2, 1.0, 0, 1, 1, 1, 0, 0) == molt.MOLT_EINVAL
    assert molt.mol_t_helmholtz_sweep(g, 0, -1.0, 0, 1, 1, 1, 0, 0) == molt.MOLT_EINVAL
    assert molt.mol_t_helmholtz_sweep(g, 0, 1.0, 0, 0, 1, 1, 0, 0) == molt.MOLT_EINVAL
    assert molt.mol_t_helmholtz_sweep(g, 1, 1.0, 0, 1, 1, 1, 0, 0) == molt.MOLT_EWORKSPACE


def _inst(specs):
    arr = (molt.molt_instance * len(specs))()
    for i, (g, p, ns) in enumerate(specs):
        arr[i].grid, arr[i].params, arr[i].d_u, arr[i].nsteps = g, p, 4096 * (i + 1), ns
    return arr


def test_batch_workspace_query(lib):
    p = molt.make_params(0.02, 1e-5, precision=molt.MOLT_F32, stepper=molt.MOLT_BDF2)
    gs = [molt.make_grid(n, n + 3, bc=bc, M=4) for n, bc in ((64, 0), (100, 1), (300, 0))]
    one = [molt.ch_workspace_bytes(g, p) for g in gs]
    arr = _inst([(g, p, 5) for g in gs])
    need = molt.ch_batch_workspace_bytes(arr, 3)
    assert need >= sum(one)
    # a batch of one needs the instance's workspace plus its descriptors and maps only
    assert molt.ch_batch_workspace_bytes(_inst([(gs[0], p, 5)]), 1) < one[0] + (1 << 16)


@pytest.mark.parametrize("case", ["count0", "mixed_precision", "one_d", "dirichlet", "null_field",
                                  "negative_steps", "bad_params", "bdf3"])
def test_batch_argument_checks(lib, case):
    p = molt.make_params(0.02, 1e-5, precision=molt.MOLT_F32)
    g = molt.make_grid(64, 64, bc=molt.MOLT_BC_PERIODIC, M=4)
    specs = [(g, p, 3), (molt.make_grid(80, 72, bc=molt.MOLT_BC_NEUMANN, M=4), p, 2)]
    count = 2
    arr = _inst(specs)
    if case == "count0":
        count = 0
    elif case == "mixed_precision":
        arr[1].params.precision = molt.MOLT_F64
    elif case == "one_d":
        arr[1].grid.ny = 1
    elif case == "dirichlet":
        arr[0].grid.bc = molt.MOLT_BC_DIRICHLET
    elif case == "null_field":
        arr[1].d_u = None
    elif case == "negative_steps":
        arr[0].nsteps = -1
    elif case == "bad_params":
        arr[1].params.eps = -1.0
    elif case == "bdf3":
        arr[0].params.stepper = molt.MOLT_BDF3
    assert molt.ch_batch_workspace_bytes(arr, count) == 0
    rc = molt.ch_solve_batch(arr, count, 1, 1 << 40)
    assert rc in (molt.MOLT_EINVAL, molt.MOLT_EUNSUPPORTED), rc
    assert molt.molt_last_error() != ""


def test_batch_small_workspace_is_rejected(lib):
    p = molt.make_params(0.02, 1e-5, precision=molt.MOLT_F32)
    arr = _inst([(molt.make_grid(64, 64, M=4), p, 3)])
    need = molt.ch_batch_workspace_bytes(arr, 1)
    assert molt.ch_solve_batch(arr, 1, 1, need - 1) == molt.MOLT_EWORKSPACE


def test_batch_options(lib):
    assert molt.molt_set_option(molt.MOLT_OPT_BATCH_TICKS, 0) == molt.MOLT_EINVAL
    assert molt.molt_set_option(molt.MOLT_OPT_BATCH_TICKS, 8) == molt.MOLT_OK
    assert molt.molt_set_option(molt.MOLT_OPT_BATCH_GRAPH, 2) == molt.MOLT_EINVAL
    assert molt.molt_set_option(molt.MOLT_OPT_BATCH_GRAPH, 1) == molt.MOLT_OK
    assert molt.molt_set_option(molt.MOLT_OPT_BATCH_LEAN, -1) == molt.MOLT_EINVAL
    assert molt.molt_set_option(molt.MOLT_OPT_BATCH_LEAN, 2) == molt.MOLT_OK
    assert molt.molt_set_option(molt.MOLT_OPT_STEP_GRAPH, 2) == molt.MOLT_EINVAL
    assert molt.molt_set_option(molt.MOLT_OPT_STEP_GRAPH, 0) == molt.MOLT_OK
    assert molt.molt_set_option(molt.MOLT_OPT_STEP_GRAPH, 1) == molt.MOLT_OK
    assert molt.molt_set_option(99, 1) == molt.MOLT_EINVAL
    assert molt.molt_profile_only(95) == molt.MOLT_OK  # FP64 launches: kinds 48..95
    assert molt.molt_profile_only(96) == molt.MOLT_EINVAL
    assert molt.molt_profile_only(-1) == molt.MOLT_OK


def test_tune_table_defaults_and_validation(lib):
    # defaults: the smallest kx that fits a line in one 256-thread block, but 16 in
    # 512-thread rows for FP32 lines of 8192 (kx 32 spills); ky 16 (FP32) / 8 (FP64)
    assert molt.tune_table(molt.MOLT_F32) == [(4, 16), (4, 16), (4, 16), (4, 16), (8, 16), (16, 16), (16, 16)]
    assert molt.tune_table(molt.MOLT_F64) == [(4, 8), (4, 8), (4, 8), (4, 8), (8, 8), (16, 8), (16, 8)]
    assert molt.molt_tune_set(molt.MOLT_F32, 4, 4, 16) == molt.MOLT_EINVAL   # 2048 nodes need kx >= 8
    assert molt.molt_tune_set(molt.MOLT_F32, 5, 4, 16) == molt.MOLT_EINVAL   # 4096 nodes: kx >= 8 (512 threads)
    assert molt.molt_tune_set(molt.MOLT_F32, 5, 8, 16) == molt.MOLT_OK       # rows of 512 threads
    assert molt.molt_tune_set(molt.MOLT_F32, 5, 16, 16) == molt.MOLT_OK
    assert molt.molt_tune_set(molt.MOLT_F64, 0, 32, 8) == molt.MOLT_EINVAL   # kx 32 is FP32 only
    assert molt.molt_tune_set(molt.MOLT_F64, 0, 4, 16) == molt.MOLT_EINVAL   # ky 16 is FP32 only
    assert molt.molt_tune_set(molt.MOLT_F32, 7, 4, 4) == molt.MOLT_EINVAL
    assert molt.molt_tune_set(molt.MOLT_F32, 2, 8, 4) == molt.MOLT_OK
    assert molt.molt_tune_get(molt.MOLT_F32, 2) == (8, 4)
    assert molt.molt_tune_set(molt.MOLT_F32, 2, 4, 16) == molt.MOLT_OK
    assert molt.molt_autotune_workspace_bytes(molt.MOLT_F64, 8192) == 0
    assert molt.molt_autotune_workspace_bytes(molt.MOLT_F32, 100) == 0
    assert molt.molt_autotune_workspace_bytes(molt.MOLT_F32, 1024) > 7 * 1024 * 1024 * 4
    assert molt.molt_autotune(molt.MOLT_F32, 1024, 1, 10) == molt.MOLT_EWORKSPACE


def test_server_queries_and_argument_checks(lib):
    p = molt.make_params(0.02, 1e-5, precision=molt.MOLT_F32, model=molt.MOLT_MODEL_VCH, stepper=molt.MOLT_BDF2)
    inst = molt.molt_instance(molt.make_grid(128, 128, M=4), p, 4096, 20)
    fp = molt.molt_server_footprint(inst)
    p1 = molt.make_params(0.02, 1e-5, precision=molt.MOLT_F32, stepper=molt.MOLT_BDF2)
    one = molt.ch_workspace_bytes(molt.make_grid(128, 128, M=4), p1)
    assert fp > 2 * 10 * 128 * 128 * 4 and fp > one  # two components, records
    assert molt.molt_server_bytes(molt.MOLT_F32, 16, 1 << 20) > 1 << 20
    assert molt.molt_server_bytes(molt.MOLT_F32, 0, 1 << 20) == 0
    h = ctypes.c_void_p()
    # a server needs a stream; a NULL stream or a tiny workspace is rejected before any device work
    assert lib.molt_server_create(molt.MOLT_F32, 4, 4096, 1 << 30, None, ctypes.byref(h)) == molt.MOLT_EINVAL
    assert lib.molt_server_create(molt.MOLT_F32, 4, 4096, 100, 1, ctypes.byref(h)) == molt.MOLT_EWORKSPACE
    assert lib.molt_server_submit(None, ctypes.byref(inst), 1) == molt.MOLT_EINVAL
    assert lib.molt_server_run(None, 1, None, None) == molt.MOLT_EINVAL
    assert lib.molt_server_destroy(None) == molt.MOLT_OK


@pytest.mark.parametrize("change", [dict(t_end=0.0), dict(dt0=-1.0), dict(lte_tol=0.0), dict(gamma=1.0),
                                    dict(nmaxit=0), dict(max_attempts=0)])
def test_adaptive_argument_checks(lib, change):
    g = molt.make_grid(32, 32, M=4)
    p = molt.make_params(0.05, 1e-3)
    assert molt.ch_adaptive_workspace_bytes(g, p) > molt.ch_workspace_bytes(g, p)
    ap = molt.make_adapt(1.0, 1e-3, 1e-3)
    for k, v in change.items():
        setattr(ap, k, v)
    assert molt.ch_solve_adaptive(g, p, ap, 1, 1, 1 << 30) == molt.MOLT_EINVAL


def test_noalloc_sweep_refuses_what_its_scratch_cannot_hold(lib):
    """Checked on the host before any device call: an in-place y sweep needs the
    workspace variant, and a y sweep larger than the static scratch is refused
    with the size it would need."""
    assert molt.molt_noalloc_scratch_bytes() == 16 * 1024 * 1024
    g = molt.make_grid(4096, 4096)
    fake_in, fake_out = 0x10000, 0x20000
    rc = molt.mol_t_helmholtz_sweep_noalloc(g, 1, 100.0, molt.MOLT_F32, fake_in, fake_in, 1, 0)
    assert rc == molt.MOLT_EINVAL and "in-place" in molt.molt_last_error()
    rc = molt.mol_t_helmholtz_sweep_noalloc(g, 1, 100.0, molt.MOLT_F64, fake_in, fake_out, 64, 0)
    assert rc == molt.MOLT_EUNSUPPORTED and "scratch" in molt.molt_last_error()
    rc = molt.mol_t_helmholtz_sweep_noalloc(g, 2, 100.0, molt.MOLT_F32, fake_in, fake_out, 1, 0)
    assert rc == molt.MOLT_EINVAL
