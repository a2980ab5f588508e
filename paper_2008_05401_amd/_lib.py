"""ctypes binding of libcrbm.so: argument marshalling only, same names as the
C ABI in include/crbm.h.  Every computation runs in the library's HIP kernels;
if the library is missing this module raises instead of falling back."""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcrbm.so")

CRBM_OK, CRBM_EINVAL, CRBM_EBUDGET, CRBM_EHIP, CRBM_EUNSUPPORTED = 0, -1, -2, -3, -4
CRBM_ISING, CRBM_KITAEV, CRBM_GIBBS = 0, 1, 2


class CRBMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"crbm status {status}: {msg}")
        self.status = status


class crbm_params(ct.Structure):
    _fields_ = [("K", ct.c_int32), ("C", ct.c_int32), ("Lw", ct.c_int32),
                ("W", ct.c_void_p), ("hbias", ct.c_void_p), ("vbias", ct.c_void_p),
                ("open_cols", ct.c_int32), ("n_edge", ct.c_int32), ("dense", ct.c_int32)]


class crbm_batch_desc(ct.Structure):
    _fields_ = [("target", ct.c_int32), ("L", ct.c_int32), ("n_chains", ct.c_int32),
                ("gibbs_k", ct.c_int32), ("burnin_sweeps", ct.c_int32), ("init_state", ct.c_int32),
                ("chain_offset", ct.c_uint32), ("boundary", ct.c_int32), ("seed", ct.c_uint64),
                ("J", ct.c_double * 3), ("T", ct.c_void_p), ("state", ct.c_void_p),
                ("rbm_state", ct.c_void_p), ("workspace", ct.c_void_p), ("workspace_bytes", ct.c_size_t),
                ("mh_band_min", ct.c_double)]


# crbm_chain_stats
STATS_DTYPE = np.dtype([
    ("sweeps", "<i8"), ("n_acc", "<i8"), ("n_meas", "<i8"), ("n_recheck", "<i8"),
    ("sumE", "<i8"), ("sumE2", "<i8"), ("sumM", "<i8"), ("sumAbsM", "<i8"), ("sumM2", "<i8"),
    ("E", "<i8"), ("F", "<f8"), ("S", "<f8"), ("Ef", "<f8"), ("Cf", "<f8"),
    ("kE", "<f8"), ("kE2", "<f8"), ("kCf", "<f8"), ("F_bound", "<f8"), ("n_swap", "<i8"), ("S_bound", "<f8"),
])
assert STATS_DTYPE.itemsize == 160

EXPORTS = ["crbm_workspace_size", "crbm_init", "crbm_propose_accept", "crbm_propose_accept_many",
           "crbm_graph_create", "crbm_graph_launch", "crbm_graph_destroy",
           "crbm_tempering_swap", "crbm_set_trace", "crbm_autocorr",
           "crbm_read_stats", "crbm_sweeps_done", "crbm_destroy", "crbm_free_energy", "target_energy",
           "crbm_grad_workspace_size", "crbm_grad", "crbm_grad_static", "crbm_set_tuning", "crbm_clear_tuning", "crbm_last_error",
           "crbm_version"]

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with paper_2008_05401_amd.build.build()")
    L = ct.CDLL(path)
    vp, P = ct.c_void_p, ct.POINTER
    L.crbm_workspace_size.argtypes = [P(crbm_params), P(crbm_batch_desc)]
    L.crbm_workspace_size.restype = ct.c_size_t
    L.crbm_init.argtypes = [P(vp), P(crbm_params), P(crbm_batch_desc), vp]
    L.crbm_propose_accept.argtypes = [vp, ct.c_int32]
    L.crbm_propose_accept_many.argtypes = [P(vp), ct.c_int32, ct.c_int32]
    L.crbm_graph_create.argtypes = [P(vp), P(vp), ct.c_int32, ct.c_int32, ct.c_int32]
    L.crbm_graph_launch.argtypes = [vp]
    L.crbm_graph_destroy.argtypes = [vp]
    L.crbm_tempering_swap.argtypes = [vp, ct.c_int32, ct.c_int32]
    L.crbm_set_trace.argtypes = [vp, vp, ct.c_int32]
    L.crbm_autocorr.argtypes = [vp, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_double, vp, vp, vp, vp]
    L.crbm_read_stats.argtypes = [vp, vp, ct.c_int32]
    L.crbm_sweeps_done.argtypes = [vp]
    L.crbm_sweeps_done.restype = ct.c_int64
    L.crbm_destroy.argtypes = [vp]
    L.crbm_free_energy.argtypes = [P(crbm_params), vp, ct.c_int32, ct.c_int32, vp, vp]
    L.target_energy.argtypes = [ct.c_int32, vp, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32, P(ct.c_double), vp, vp,
                                vp, vp]
    L.crbm_grad_workspace_size.argtypes = [P(crbm_params), ct.c_int32]
    L.crbm_grad_workspace_size.restype = ct.c_size_t
    L.crbm_grad.argtypes = [P(crbm_params), vp, ct.c_int32, ct.c_int32, vp, vp, vp, vp, vp, ct.c_size_t, vp]
    L.crbm_grad_static.argtypes = [P(crbm_params), vp, ct.c_int32, ct.c_int32, vp, vp, vp, vp, vp]
    L.crbm_set_tuning.argtypes = [ct.c_int32] * 5
    L.crbm_set_tuning.restype = ct.c_int
    L.crbm_clear_tuning.argtypes = []
    L.crbm_clear_tuning.restype = ct.c_int
    L.crbm_last_error.restype = ct.c_char_p
    L.crbm_version.restype = ct.c_char_p
    for name in ("crbm_init", "crbm_propose_accept", "crbm_propose_accept_many", "crbm_tempering_swap",
                 "crbm_graph_create", "crbm_graph_launch", "crbm_graph_destroy",
                 "crbm_set_trace", "crbm_autocorr",
                 "crbm_read_stats",
                 "crbm_destroy", "crbm_free_energy", "target_energy", "crbm_grad", "crbm_grad_static"):
        getattr(L, name).restype = ct.c_int
    _lib = L
    return L


def check(status: int):
    if status != CRBM_OK:
        raise CRBMError(status, load().crbm_last_error().decode())
    return status


def crbm_workspace_size(params, desc) -> int:
    return int(load().crbm_workspace_size(ct.byref(params), ct.byref(desc)))


def crbm_init(params, desc, stream) -> int:
    ctx = ct.c_void_p()
    check(load().crbm_init(ct.byref(ctx), ct.byref(params), ct.byref(desc), stream))
    return ctx.value


def crbm_propose_accept(ctx, n_sweeps: int):
    check(load().crbm_propose_accept(ctx, int(n_sweeps)))


def crbm_propose_accept_many(ctxs, n_sweeps: int):
    arr = (ct.c_void_p * len(ctxs))(*ctxs)
    check(load().crbm_propose_accept_many(arr, len(ctxs), int(n_sweeps)))


def crbm_graph_create(ctxs, n_blocks: int, sweeps_per_block: int) -> int:
    arr = (ct.c_void_p * len(ctxs))(*ctxs)
    g = ct.c_void_p()
    check(load().crbm_graph_create(ct.byref(g), arr, len(ctxs), int(n_blocks), int(sweeps_per_block)))
    return g.value


def crbm_graph_launch(graph):
    check(load().crbm_graph_launch(graph))


def crbm_graph_destroy(graph):
    check(load().crbm_graph_destroy(graph))


def crbm_tempering_swap(ctx, n_ladders: int, round_: int):
    check(load().crbm_tempering_swap(ctx, int(n_ladders), int(round_)))


def crbm_set_trace(ctx, trace_ptr, trace_len: int):
    check(load().crbm_set_trace(ctx, trace_ptr, int(trace_len)))


def crbm_autocorr(trace_ptr, n: int, length: int, start: int, max_lag: int, c_window: float, out_ptr, tau_ptr,
                  window_ptr, stream):
    check(load().crbm_autocorr(trace_ptr, int(n), int(length), int(start), int(max_lag), float(c_window), out_ptr,
                               tau_ptr, window_ptr, stream))


def crbm_read_stats(ctx, out_ptr: int, on_device: bool):
    check(load().crbm_read_stats(ctx, out_ptr, 1 if on_device else 0))


def crbm_sweeps_done(ctx) -> int:
    return int(load().crbm_sweeps_done(ctx))


def crbm_destroy(ctx):
    check(load().crbm_destroy(ctx))


def crbm_free_energy(params, x_ptr, B, L, F_ptr, stream):
    check(load().crbm_free_energy(ct.byref(params), x_ptr, B, L, F_ptr, stream))


def target_energy(target, x_ptr, B, C, L, boundary, J, T_ptr, E_ptr, S_ptr, stream):
    Jv = (ct.c_double * 3)(*J)
    check(load().target_energy(target, x_ptr, B, C, L, int(boundary), Jv, T_ptr, E_ptr, S_ptr, stream))


def crbm_grad_workspace_size(params, B) -> int:
    return int(load().crbm_grad_workspace_size(ct.byref(params), B))


def crbm_grad(params, x_ptr, B, L, gF_ptr, dW_ptr, dhb_ptr, dvb_ptr, ws_ptr, ws_bytes, stream):
    check(load().crbm_grad(ct.byref(params), x_ptr, B, L, gF_ptr, dW_ptr, dhb_ptr, dvb_ptr, ws_ptr, ws_bytes, stream))


def crbm_grad_static(params, x_ptr, B, L, gF_ptr, dW_ptr, dhb_ptr, dvb_ptr, stream):
    check(load().crbm_grad_static(ct.byref(params), x_ptr, B, L, gF_ptr, dW_ptr, dhb_ptr, dvb_ptr, stream))


def crbm_set_tuning(L, K, Lw, rows, threads):
    check(load().crbm_set_tuning(int(L), int(K), int(Lw), int(rows), int(threads)))


def crbm_clear_tuning():
    check(load().crbm_clear_tuning())


def crbm_last_error() -> str:
    return load().crbm_last_error().decode()


def crbm_version() -> str:
    return load().crbm_version().decode()
