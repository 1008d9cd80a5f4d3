"""ctypes binding of the C ABI declared in include/pp.h.

Argument marshalling only: every step of a solve runs in the HIP library
``libpp_hip.so``.  If the library has not been built the import fails; there is
no fallback of any kind.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpp_hip.so")

PP_OK = 0
PP_ERR_ARG = -1
PP_ERR_DOMAIN = -2
PP_ERR_NOMEM = -3
PP_ERR_DEVICE = -4
PP_ERR_LIMIT = -5

PP_FP64 = 0
PP_MIXED = 1
PP_SELF_SKIP = 0
PP_SELF_CELLAVG = 1
PP_METHOD_FMM = 0
PP_METHOD_TREECODE = 1

ARRAYS = dict(
    SRC_KEY=0, SRC_INDEX=1, TGT_KEY=2, TGT_PERM=3, CELL_LEVEL=4, CELL_IX=5, CELL_IY=6, CELL_SB=7, CELL_SE=8,
    CELL_TB=9, CELL_TE=10, CELL_CHILD=11, CELL_NCHILD=12, CELL_PARENT=13, M2L_OFF=14, M2L_CNT=15, M2L_SRC=16,
    P2P_OFF=17, P2P_CNT=18, P2P_SRC=19, MULTIPOLE=20, LOCAL=21, FAR=22, NEAR=23, LEAF_WNEAR=24, TGT_LEAF=25,
)
DOUBLE_ARRAYS = {"MULTIPOLE", "LOCAL", "FAR", "NEAR", "LEAF_WNEAR"}
UNSIGNED_ARRAYS = {"SRC_KEY", "TGT_KEY", "SRC_INDEX"}

#: C symbols the header declares (checked by the CPU test suite)
EXPORTED = ("pp_create", "pp_destroy", "pp_solve_grid", "pp_solve_grid_noalloc", "pp_solve_grid_resident",
            "pp_solve_grid_batch", "pp_direct_grid", "pp_solve_points", "pp_direct_points",
            "pp_surface_forces", "pp_pressure_source", "pp_viscous_forces", "pp_get_stats", "pp_set_profiling", "pp_debug_copy", "pp_status_string", "pp_last_error",
            "pp_server_create", "pp_server_submit", "pp_server_wait", "pp_server_cancel", "pp_server_destroy",
            "pp_server_last_error", "pp_server_device_bytes", "pp_footprint_estimate")
PP_ERR_TIMEOUT = -6
PP_ERR_CANCELLED = -7
PP_ERR_BUSY = -8


class pp_params(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("theta", ctypes.c_double), ("leaf_max", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("self_mode", ctypes.c_int32), ("method", ctypes.c_int32)]


class pp_stats(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("ncells", ctypes.c_int32), ("nsrc_leaves", ctypes.c_int32),
                ("ntgt_leaves", ctypes.c_int32), ("nsources", ctypes.c_int64), ("ntargets", ctypes.c_int64),
                ("n_m2l", ctypes.c_int64), ("n_p2p_lists", ctypes.c_int64), ("n_p2p_pairs", ctypes.c_int64),
                ("ms_total", ctypes.c_double), ("ms_phase", ctypes.c_double * 12)]


class pp_force(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_double), ("fy", ctypes.c_double), ("drag", ctypes.c_double), ("cd", ctypes.c_double)]


class pp_server_cfg(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_slots", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_uint64),
                ("work_budget_points", ctypes.c_uint64), ("max_batch", ctypes.c_int32)]


class pp_request(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("h", ctypes.c_double), ("f", ctypes.c_void_p), ("m", ctypes.c_int64), ("tx", ctypes.c_void_p),
                ("ty", ctypes.c_void_p), ("params", pp_params), ("p_out", ctypes.c_void_p)]


class pp_ticket_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("slot", ctypes.c_int32), ("queue_us", ctypes.c_double),
                ("run_us", ctypes.c_double), ("total_us", ctypes.c_double), ("start_us", ctypes.c_double),
                ("end_us", ctypes.c_double)]


PHASES = ("ingest", "sort", "tree", "lists", "pack", "p2m", "m2m", "m2l", "l2l", "l2p", "p2p", "finalize")


class LibraryMissing(ImportError):
    pass


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library and declare the C signatures."""
    if not os.path.exists(path):
        raise LibraryMissing(f"{path} is not built; run `python -m paper_1610_04398_amd.build` "
                             "(the library has no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.pp_create.argtypes = [i32, ctypes.c_uint64, ctypes.POINTER(vp)]
    lib.pp_create.restype = i32
    lib.pp_destroy.argtypes = [vp]
    lib.pp_destroy.restype = None
    solve_args = [vp, i32, i32, f64, f64, f64, vp, i64, vp, vp, ctypes.POINTER(pp_params), vp, vp]
    lib.pp_solve_grid.argtypes = solve_args
    lib.pp_solve_grid.restype = i32
    lib.pp_solve_grid_noalloc.argtypes = solve_args
    lib.pp_solve_grid_noalloc.restype = i32
    lib.pp_solve_grid_resident.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.pp_solve_grid_resident.restype = i32
    lib.pp_solve_grid_batch.argtypes = [vp, i32, i32, i32, f64, f64, f64, vp, vp, vp, vp, ctypes.POINTER(pp_params),
                                        vp, vp]
    lib.pp_solve_grid_batch.restype = i32
    lib.pp_direct_grid.argtypes = solve_args
    lib.pp_direct_grid.restype = i32
    points_args = [vp, i64, vp, vp, vp, i64, vp, vp, ctypes.POINTER(pp_params), vp, vp]
    lib.pp_solve_points.argtypes = points_args
    lib.pp_solve_points.restype = i32
    lib.pp_direct_points.argtypes = points_args
    lib.pp_direct_points.restype = i32
    lib.pp_surface_forces.argtypes = [vp, i64, vp, vp, vp, vp, i32, vp, f64, f64, f64, f64, vp, vp, vp, vp]
    lib.pp_surface_forces.restype = i32
    lib.pp_pressure_source.argtypes = [vp, i32, i32, f64, vp, vp, f64, f64, vp, vp, vp, vp, vp]
    lib.pp_pressure_source.restype = i32
    lib.pp_viscous_forces.argtypes = [vp, i32, i32, f64, f64, f64, vp, vp, i64, vp, vp, vp, vp, vp, i32, vp, f64, f64,
                                      f64, f64, f64, vp, vp, vp, vp]
    lib.pp_viscous_forces.restype = i32
    lib.pp_get_stats.argtypes = [vp, ctypes.POINTER(pp_stats)]
    lib.pp_get_stats.restype = i32
    lib.pp_set_profiling.argtypes = [vp, i32]
    lib.pp_set_profiling.restype = i32
    lib.pp_debug_copy.argtypes = [vp, i32, vp, i64, ctypes.POINTER(i64)]
    lib.pp_debug_copy.restype = i32
    lib.pp_server_create.argtypes = [ctypes.POINTER(pp_server_cfg), ctypes.POINTER(vp)]
    lib.pp_server_create.restype = i32
    lib.pp_server_submit.argtypes = [vp, ctypes.POINTER(pp_request), ctypes.POINTER(ctypes.c_uint64)]
    lib.pp_server_submit.restype = i32
    lib.pp_server_wait.argtypes = [vp, ctypes.c_uint64, i64, ctypes.POINTER(pp_ticket_info)]
    lib.pp_server_wait.restype = i32
    lib.pp_server_cancel.argtypes = [vp, ctypes.c_uint64]
    lib.pp_server_cancel.restype = i32
    lib.pp_server_destroy.argtypes = [vp]
    lib.pp_server_destroy.restype = i32
    lib.pp_server_last_error.argtypes = [vp]
    lib.pp_server_last_error.restype = ctypes.c_char_p
    lib.pp_server_device_bytes.argtypes = [vp]
    lib.pp_server_device_bytes.restype = ctypes.c_uint64
    lib.pp_footprint_estimate.argtypes = [i32, i32, i64, i32, i32]
    lib.pp_footprint_estimate.restype = ctypes.c_uint64
    lib.pp_status_string.argtypes = [i32]
    lib.pp_status_string.restype = ctypes.c_char_p
    lib.pp_last_error.argtypes = [vp]
    lib.pp_last_error.restype = ctypes.c_char_p
    return lib


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def pp_create(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    h = ctypes.c_void_p()
    st = lib().pp_create(device, hbm_budget_bytes, ctypes.byref(h))
    if st != PP_OK:
        raise PPError(st, "pp_create failed")
    return h.value


def pp_destroy(ctx: int) -> None:
    lib().pp_destroy(ctx)


def pp_solve_grid(ctx, nx, ny, x0, y0, h, f_ptr, m, tx_ptr, ty_ptr, params: pp_params, out_ptr, stream) -> int:
    return lib().pp_solve_grid(ctx, nx, ny, x0, y0, h, f_ptr, m, tx_ptr, ty_ptr, ctypes.byref(params), out_ptr,
                               stream)


def pp_solve_grid_noalloc(ctx, nx, ny, x0, y0, h, f_ptr, m, tx_ptr, ty_ptr, params: pp_params, out_ptr,
                          stream) -> int:
    return lib().pp_solve_grid_noalloc(ctx, nx, ny, x0, y0, h, f_ptr, m, tx_ptr, ty_ptr, ctypes.byref(params),
                                       out_ptr, stream)


def pp_solve_grid_resident(ctx, f_ptr, tx_ptr, ty_ptr, out_ptr, stream) -> int:
    return lib().pp_solve_grid_resident(ctx, f_ptr, tx_ptr, ty_ptr, out_ptr, stream)


def pp_solve_grid_batch(ctx, nx, ny, x0, y0, h, f_ptrs, ms, tx_ptrs, ty_ptrs, params: pp_params, out_ptrs,
                        stream) -> int:
    """Pointer lists become the C arrays of pointers and counts."""
    n = len(f_ptrs)
    arr = lambda v: (ctypes.c_void_p * n)(*v)
    return lib().pp_solve_grid_batch(ctx, n, nx, ny, x0, y0, h, arr(f_ptrs), (ctypes.c_int64 * n)(*ms),
                                     arr(tx_ptrs), arr(ty_ptrs), ctypes.byref(params), arr(out_ptrs), stream)


def pp_direct_grid(ctx, nx, ny, x0, y0, h, f_ptr, m, tx_ptr, ty_ptr, params: pp_params, out_ptr, stream) -> int:
    return lib().pp_direct_grid(ctx, nx, ny, x0, y0, h, f_ptr, m, tx_ptr, ty_ptr, ctypes.byref(params), out_ptr,
                                stream)


def pp_solve_points(ctx, n, sx_ptr, sy_ptr, w_ptr, m, tx_ptr, ty_ptr, params: pp_params, out_ptr, stream) -> int:
    return lib().pp_solve_points(ctx, n, sx_ptr, sy_ptr, w_ptr, m, tx_ptr, ty_ptr, ctypes.byref(params), out_ptr,
                                 stream)


def pp_direct_points(ctx, n, sx_ptr, sy_ptr, w_ptr, m, tx_ptr, ty_ptr, params: pp_params, out_ptr, stream) -> int:
    return lib().pp_direct_points(ctx, n, sx_ptr, sy_ptr, w_ptr, m, tx_ptr, ty_ptr, ctypes.byref(params), out_ptr,
                                  stream)


def pp_surface_forces(ctx, m, p_ptr, nx_ptr, ny_ptr, ds_ptr, nseg, seg_ptr, ux, uy, rho, area, dfx_ptr, dfy_ptr,
                      out_ptr, stream) -> int:
    return lib().pp_surface_forces(ctx, m, p_ptr, nx_ptr, ny_ptr, ds_ptr, nseg, seg_ptr, ux, uy, rho, area, dfx_ptr,
                                   dfy_ptr, out_ptr, stream)


def pp_pressure_source(ctx, nx, ny, h, u_ptr, v_ptr, rho, lam, chi_ptr, us_ptr, vs_ptr, f_ptr, stream) -> int:
    return lib().pp_pressure_source(ctx, nx, ny, h, u_ptr, v_ptr, rho, lam, chi_ptr, us_ptr, vs_ptr, f_ptr, stream)


def pp_viscous_forces(ctx, nx, ny, x0, y0, h, u_ptr, v_ptr, m, lx_ptr, ly_ptr, nx_ptr, ny_ptr, ds_ptr, nseg, seg_ptr,
                      mu, ux, uy, rho, area, dfx_ptr, dfy_ptr, out_ptr, stream) -> int:
    return lib().pp_viscous_forces(ctx, nx, ny, x0, y0, h, u_ptr, v_ptr, m, lx_ptr, ly_ptr, nx_ptr, ny_ptr, ds_ptr,
                                   nseg, seg_ptr, mu, ux, uy, rho, area, dfx_ptr, dfy_ptr, out_ptr, stream)


def pp_get_stats(ctx) -> pp_stats:
    s = pp_stats()
    st = lib().pp_get_stats(ctx, ctypes.byref(s))
    if st != PP_OK:
        raise PPError(st, "pp_get_stats failed")
    return s


def pp_set_profiling(ctx, on: int) -> int:
    return lib().pp_set_profiling(ctx, int(on))


def pp_debug_copy(ctx, what: int, dst_ptr, capacity: int) -> tuple[int, int]:
    n = ctypes.c_int64(0)
    st = lib().pp_debug_copy(ctx, what, dst_ptr, capacity, ctypes.byref(n))
    return st, n.value


def pp_status_string(st: int) -> str:
    return lib().pp_status_string(st).decode()


def pp_last_error(ctx) -> str:
    return lib().pp_last_error(ctx).decode()


def pp_server_create(device: int = 0, max_slots: int = 4, hbm_budget_bytes: int = 0,
                     work_budget_points: int = 0, max_batch: int = 0) -> int:
    cfg = pp_server_cfg(device, max_slots, hbm_budget_bytes, work_budget_points, max_batch)
    h = ctypes.c_void_p()
    st = lib().pp_server_create(ctypes.byref(cfg), ctypes.byref(h))
    if st != PP_OK:
        raise PPError(st, "pp_server_create failed")
    return h.value


def pp_server_submit(server, req: pp_request) -> int:
    t = ctypes.c_uint64(0)
    st = lib().pp_server_submit(server, ctypes.byref(req), ctypes.byref(t))
    if st != PP_OK:
        raise PPError(st, "pp_server_submit failed")
    return t.value


def pp_server_wait(server, ticket: int, timeout_us: int = -1) -> tuple[int, pp_ticket_info]:
    info = pp_ticket_info()
    st = lib().pp_server_wait(server, ticket, timeout_us, ctypes.byref(info))
    return st, info


def pp_server_cancel(server, ticket: int) -> int:
    return lib().pp_server_cancel(server, ticket)


def pp_server_destroy(server) -> int:
    return lib().pp_server_destroy(server)


def pp_server_last_error(server) -> str:
    return lib().pp_server_last_error(server).decode()


def pp_server_device_bytes(server) -> int:
    return int(lib().pp_server_device_bytes(server))


def pp_footprint_estimate(nx: int, ny: int, m: int, p: int, leaf_max: int) -> int:
    return int(lib().pp_footprint_estimate(nx, ny, m, p, leaf_max))


class PPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status
