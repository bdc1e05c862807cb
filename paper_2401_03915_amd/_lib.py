"""ctypes binding of libtls.so (include/tls.h): argument marshalling only.

Every computation happens in the HIP library; this module only converts
PyTorch device tensors to pointers and C structs to Python values. It fails
loudly (ImportError / OSError) when the library has not been built.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtls.so")

TLS_OK, TLS_E_ARG, TLS_E_NOT_SPD, TLS_E_SINGULAR, TLS_E_NOCONV, TLS_E_NOMEM, TLS_E_HIP, TLS_E_STATE = range(8)
STATUS_NAMES = {0: "TLS_OK", 1: "TLS_E_ARG", 2: "TLS_E_NOT_SPD", 3: "TLS_E_SINGULAR", 4: "TLS_E_NOCONV",
                5: "TLS_E_NOMEM", 6: "TLS_E_HIP", 7: "TLS_E_STATE"}

# Names declared in include/tls.h (checked by the tests against the header).
EXPORTED = ["tls_default_options", "tls_setup", "tls_apply", "tls_spmv", "tls_solve", "tls_info", "tls_export",
            "tls_local_solve", "tls_export_zblocks", "tls_gnn_forward", "tls_gnn_loss_grad", "tls_last_error",
            "tls_destroy", "tls_trim", "tls_solve_noalloc"]

GNN_LAYERS = 4
GNN_FEATURES = 12
GNN_HIDDEN = 32


def gnn_n_weights(c_out: int) -> int:
    """TLS_GNN_NWEIGHTS(c_out) of include/tls.h."""
    return (2 * GNN_FEATURES * GNN_HIDDEN + GNN_HIDDEN
            + (GNN_LAYERS - 1) * (2 * GNN_HIDDEN * GNN_HIDDEN + GNN_HIDDEN) + GNN_HIDDEN * c_out)


class TlsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class tls_options(C.Structure):
    _fields_ = [
        ("precision", C.c_int32),
        ("matrix_kind", C.c_int32),
        ("nev1", C.c_int32),
        ("tau", C.c_double),
        ("nu", C.c_double),
        ("restart", C.c_int32),
        ("maxit", C.c_int32),
        ("eig_maxit", C.c_int32),
        ("eig_tol", C.c_double),
        ("eig_oversample", C.c_int32),
        ("seed", C.c_uint64),
        ("use_graph", C.c_int32),
        ("flexible", C.c_int32),
        ("jacobi_scale", C.c_int32),
        ("profile", C.c_int32),
        ("solve_wgs", C.c_int32),
        ("solve_order", C.c_int32),
        ("autotune", C.c_int32),
        ("tune_cache", C.c_char_p),
        ("gnn_weights", C.c_void_p),
        ("gnn_c_out", C.c_int32),
        ("gnn_train", C.c_int32),
        ("composition", C.c_int32),
        ("local_inverse", C.c_int32),
        ("local_refine", C.c_int32),
        ("solve_rows", C.c_int32),
        ("stream", C.c_void_p),
    ]


class tls_info_t(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("n_parts", C.c_int32),
        ("n_coarse", C.c_int32),
        ("gc", C.c_double),
        ("oc", C.c_double),
        ("local_sum_m", C.c_int64),
        ("local_sum_m2", C.c_int64),
        ("factor_bytes", C.c_int64),
        ("max_m", C.c_int32),
        ("min_m", C.c_int32),
        ("t_setup", C.c_double * 8),
        ("t_solve", C.c_double),
        ("iters", C.c_int32),
        ("relres", C.c_double),
        ("eig_resid_max", C.c_double),
        ("eig_iters_max", C.c_int32),
        ("eig_iters_mean", C.c_double),
        ("n_res_history", C.c_int32),
        ("n_profiled", C.c_int32),
        ("t_local_solve_ms", C.c_double),
        ("t_apply_ms", C.c_double),
        ("t_local_fwd_ms", C.c_double),
        ("solve_wgs", C.c_int32),
        ("solve_order", C.c_int32),
        ("tuned", C.c_int32),
        ("res_history", C.POINTER(C.c_double)),
        ("local_inverse", C.c_int32),
        ("t_inverse_ms", C.c_double),
        ("wait_timeout", C.c_int32),
        ("local_refine", C.c_int32),
        ("symv_block", C.c_int32),
        ("factor_panel", C.c_int32),
        ("factor_flops", C.c_double),
        ("inverse_flops", C.c_double),
        ("solve_tiles_fwd", C.c_int64),
        ("solve_tiles_bwd", C.c_int64),
        ("lower_tiles", C.c_int64),
        ("solve_rows", C.c_int32),
        ("solve_order_bwd", C.c_int32),
    ]


_lib = None


def lib() -> C.CDLL:
    """Load libtls.so once (raises OSError if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError(f"{LIB_PATH} is missing: build it with paper_2401_03915_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
        L.tls_default_options.argtypes = [C.POINTER(tls_options)]
        L.tls_default_options.restype = None
        L.tls_setup.argtypes = [i32, i32, vp, vp, vp, vp, i32, i32, i32, C.POINTER(tls_options), C.POINTER(vp)]
        L.tls_setup.restype = C.c_int
        L.tls_apply.argtypes = [vp, vp, vp]
        L.tls_apply.restype = C.c_int
        L.tls_spmv.argtypes = [vp, vp, vp]
        L.tls_spmv.restype = C.c_int
        L.tls_solve.argtypes = [vp, vp, vp, dbl, C.POINTER(i32), C.POINTER(dbl)]
        L.tls_solve.restype = C.c_int
        L.tls_solve_noalloc.argtypes = [vp, vp, vp, dbl, C.POINTER(i32), C.POINTER(dbl)]
        L.tls_solve_noalloc.restype = C.c_int
        L.tls_info.argtypes = [vp, C.POINTER(tls_info_t)]
        L.tls_info.restype = C.c_int
        L.tls_export.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.tls_export.restype = C.c_int
        L.tls_local_solve.argtypes = [vp, i32, vp, vp]
        L.tls_local_solve.restype = C.c_int
        L.tls_export_zblocks.argtypes = [vp, vp]
        L.tls_export_zblocks.restype = C.c_int
        L.tls_gnn_forward.argtypes = [vp, vp, i32, vp]
        L.tls_gnn_forward.restype = C.c_int
        L.tls_gnn_loss_grad.argtypes = [vp, vp, i32, vp, C.POINTER(C.c_double)]
        L.tls_gnn_loss_grad.restype = C.c_int
        L.tls_last_error.argtypes = [vp]
        L.tls_last_error.restype = C.c_char_p
        L.tls_destroy.argtypes = [vp]
        L.tls_destroy.restype = None
        L.tls_trim.argtypes = []
        L.tls_trim.restype = None
        _lib = L
    return _lib


def last_error(ctx=None) -> str:
    s = lib().tls_last_error(ctx)
    return s.decode() if s else ""


def check(status: int, ctx=None, allow=()) -> int:
    if status != TLS_OK and status not in allow:
        raise TlsError(status, last_error(ctx))
    return status


def tls_default_options() -> tls_options:
    o = tls_options()
    lib().tls_default_options(C.byref(o))
    return o


def tls_setup(n, nnz, row_ptr, col_idx, val, part, n_parts, overlap, nev, opt: tls_options | None):
    """Pointers are integers (device addresses). Returns the context handle."""
    out = C.c_void_p()
    st = lib().tls_setup(n, nnz, row_ptr, col_idx, val, part, n_parts, overlap, nev,
                         C.byref(opt) if opt is not None else None, C.byref(out))
    check(st, None)
    return out.value


def tls_apply(ctx, r_ptr, z_ptr):
    return check(lib().tls_apply(ctx, r_ptr, z_ptr), ctx)


def tls_spmv(ctx, x_ptr, y_ptr):
    return check(lib().tls_spmv(ctx, x_ptr, y_ptr), ctx)


def tls_solve(ctx, b_ptr, x_ptr, tol):
    it = C.c_int32(0)
    rr = C.c_double(0.0)
    st = lib().tls_solve(ctx, b_ptr, x_ptr, tol, C.byref(it), C.byref(rr))
    check(st, ctx, allow=(TLS_E_NOCONV,))
    return st, it.value, rr.value


def tls_solve_noalloc(ctx, b_ptr, x_ptr, tol, allow=(TLS_E_NOCONV,)):
    it = C.c_int32(0)
    rr = C.c_double(0.0)
    st = lib().tls_solve_noalloc(ctx, b_ptr, x_ptr, tol, C.byref(it), C.byref(rr))
    check(st, ctx, allow=allow)
    return st, it.value, rr.value


def tls_info(ctx) -> dict:
    inf = tls_info_t()
    check(lib().tls_info(ctx, C.byref(inf)), ctx)
    d = {name: getattr(inf, name) for name, _ in tls_info_t._fields_ if name not in ("t_setup", "res_history")}
    d["t_setup"] = list(inf.t_setup)
    d["res_history"] = [inf.res_history[k] for k in range(inf.n_res_history)] if inf.n_res_history else []
    return d


def tls_export(ctx, **bufs):
    """bufs: numpy arrays (or None) for sub_ptr, sub_idx, layer_ptr, zcol_ptr, eigvals, zsrc, Z, A0."""
    def p(a):
        return None if a is None else a.ctypes.data
    check(lib().tls_export(ctx, p(bufs.get("sub_ptr")), p(bufs.get("sub_idx")), p(bufs.get("layer_ptr")),
                           p(bufs.get("zcol_ptr")), p(bufs.get("eigvals")), p(bufs.get("zsrc")), p(bufs.get("Z")),
                           p(bufs.get("A0"))),
          ctx)


def tls_local_solve(ctx, i, b, x):
    return check(lib().tls_local_solve(ctx, i, b.ctypes.data, x.ctypes.data), ctx)


def tls_export_zblocks(ctx, blocks):
    """blocks: float64 numpy of sum_i #I_i k_i entries, filled."""
    assert blocks.dtype == np.float64 and blocks.flags.c_contiguous
    return check(lib().tls_export_zblocks(ctx, blocks.ctypes.data), ctx)


def tls_gnn_forward(ctx, weights, c_out, X):
    """weights: float32 numpy (gnn_n_weights(c_out)); X: float32 numpy (sum m_i, c_out), filled."""
    assert weights.dtype == np.float32 and X.dtype == np.float32 and X.flags.c_contiguous
    assert weights.size == gnn_n_weights(c_out)
    return check(lib().tls_gnn_forward(ctx, weights.ctypes.data, c_out, X.ctypes.data), ctx)


def tls_gnn_loss_grad(ctx, weights, c_out, grad):
    """Returns the loss; grad (float32 numpy, same size as weights) is filled."""
    assert weights.dtype == np.float32 and grad.dtype == np.float32
    assert weights.size == gnn_n_weights(c_out) and grad.size == weights.size
    loss = C.c_double(0.0)
    check(lib().tls_gnn_loss_grad(ctx, weights.ctypes.data, c_out, grad.ctypes.data, C.byref(loss)), ctx)
    return loss.value


def tls_destroy(ctx):
    if ctx:
        lib().tls_destroy(ctx)


def tls_trim():
    """Hand the device blocks the library keeps for reuse back to the driver."""
    lib().tls_trim()
