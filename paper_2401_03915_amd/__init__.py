"""MI355X two-level additive Schwarz preconditioner (HIP for gfx950).

The method is the fully algebraic two-level Schwarz preconditioner of
Al Daas, Jolivet, Nataf and Tournier (arXiv 2401.03915). All of its steps run
in the HIP library ``libtls.so`` behind the C ABI of ``include/tls.h``; this
package only moves PyTorch device tensors across that boundary.

``Preconditioner`` is a convenience wrapper: it uploads a SciPy CSR matrix
and a partition with PyTorch, calls ``tls_setup``, and exposes ``apply``,
``solve``, ``spmv``, ``info`` and ``export``.
"""

from __future__ import annotations

import numpy as np

from . import _lib
from ._lib import (TlsError, gnn_n_weights, tls_apply, tls_default_options, tls_destroy,  # noqa: F401
                   tls_export, tls_export_zblocks, tls_gnn_forward, tls_gnn_loss_grad, tls_info, tls_local_solve,
                   tls_setup, tls_solve, tls_spmv, tls_trim)

__all__ = ["Preconditioner", "TlsError", "tls_default_options", "tls_setup", "tls_apply", "tls_spmv", "tls_solve",
           "tls_info", "tls_export", "tls_export_zblocks", "tls_local_solve", "tls_gnn_forward",
           "tls_gnn_loss_grad", "tls_destroy", "tls_trim",
           "gnn_n_weights"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2401_03915_amd needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


class Preconditioner:
    """Two-level Schwarz preconditioner of a CSR matrix on ``device``.

    Options are the fields of ``tls_options`` (precision, matrix_kind, nev1,
    tau, nu, restart, maxit, eig_maxit, eig_tol, eig_oversample, seed,
    use_graph, flexible, jacobi_scale, gnn_train, ...). ``gnn_weights`` takes a
    float32 array of trained warm-start weights (its ``gnn_c_out`` is
    inferred from the length). ``stream`` may be a torch.cuda.Stream on which
    all library work is ordered.
    """

    def __init__(self, A, part, overlap: int, nev: int, device: str = "cuda:0", stream=None, **options):
        torch = _torch()
        self.device = torch.device(device)
        A = A.tocsr()
        self.n = A.shape[0]
        self.nnz = A.nnz
        self.n_parts = int(np.max(part)) + 1
        self.overlap = overlap
        self.nev = nev
        dev = self.device
        self._rp = torch.as_tensor(np.asarray(A.indptr, dtype=np.int32), device=dev)
        self._ci = torch.as_tensor(np.asarray(A.indices, dtype=np.int32), device=dev)
        self._val = torch.as_tensor(np.asarray(A.data, dtype=np.float64), device=dev)
        self._part = torch.as_tensor(np.asarray(part, dtype=np.int32), device=dev)
        opt = tls_default_options()
        w = options.pop("gnn_weights", None)
        for k, v in options.items():
            if not hasattr(opt, k) or k == "stream":
                raise TypeError(f"unknown option {k}")
            setattr(opt, k, v)
        self._gnn_w = None
        if w is not None:
            self._gnn_w = np.ascontiguousarray(w, dtype=np.float32)
            c_out = (self._gnn_w.size - gnn_n_weights(0)) // _lib.GNN_HIDDEN
            if gnn_n_weights(c_out) != self._gnn_w.size:
                raise ValueError("gnn_weights has a length that no c_out matches")
            opt.gnn_weights = self._gnn_w.ctypes.data
            opt.gnn_c_out = c_out
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        # 0 (the legacy default stream) lets the library create a blocking stream
        opt.stream = stream.cuda_stream or None
        torch.cuda.synchronize(dev)
        self.ctx = tls_setup(self.n, self.nnz, self._rp.data_ptr(), self._ci.data_ptr(), self._val.data_ptr(),
                             self._part.data_ptr(), self.n_parts, overlap, nev, opt)
        self.options = opt

    # -- device-side calls -------------------------------------------------
    def apply(self, r, z=None):
        """z = M^{-1} r for a float64 device tensor r (asynchronous on the stream)."""
        torch = _torch()
        if z is None:
            z = torch.empty_like(r)
        tls_apply(self.ctx, r.data_ptr(), z.data_ptr())
        return z

    def spmv(self, x, y=None):
        torch = _torch()
        if y is None:
            y = torch.empty_like(x)
        tls_spmv(self.ctx, x.data_ptr(), y.data_ptr())
        return y

    def solve(self, b, tol: float = 1e-8, x=None):
        """Returns (x, iterations, true relative residual, status)."""
        torch = _torch()
        if x is None:
            x = torch.empty_like(b)
        st, it, rr = tls_solve(self.ctx, b.data_ptr(), x.data_ptr(), tol)
        return x, it, rr, st

    def info(self) -> dict:
        return tls_info(self.ctx)

    def export(self, Z: bool = False, A0: bool = False) -> dict:
        inf = self.info()
        N, nC = self.n_parts, inf["n_coarse"]
        out = {
            "sub_ptr": np.zeros(N + 1, dtype=np.int32),
            "layer_ptr": np.zeros(N * (self.overlap + 2), dtype=np.int32),
            "zcol_ptr": np.zeros(N + 1, dtype=np.int32),
            "eigvals": np.zeros(max(nC, 1)),
            "zsrc": np.zeros(max(nC, 1), dtype=np.int32),
        }
        tls_export(self.ctx, sub_ptr=out["sub_ptr"])
        out["sub_idx"] = np.zeros(int(out["sub_ptr"][-1]), dtype=np.int32)
        if Z:
            out["Z"] = np.zeros((nC, self.n))  # row a = coarse column a
        if A0:
            out["A0"] = np.zeros((nC, nC))
        tls_export(self.ctx, sub_ptr=out["sub_ptr"], sub_idx=out["sub_idx"], layer_ptr=out["layer_ptr"],
                   zcol_ptr=out["zcol_ptr"], eigvals=out["eigvals"], zsrc=out["zsrc"], Z=out.get("Z"),
                   A0=out.get("A0"))
        out["eigvals"] = out["eigvals"][:nC]
        out["zsrc"] = out["zsrc"][:nC]
        if Z:
            out["Z"] = out["Z"].T.copy()  # n x nC
        if A0:
            out["A0"] = out["A0"].T.copy()  # the C side writes column-major
        return out

    def z_sparse(self, ex=None):
        """The coarse basis as a SciPy CSR matrix (n x n_C) from its compact blocks."""
        import scipy.sparse as sp
        if ex is None:
            ex = self.export()
        zc, spt, lp = ex["zcol_ptr"], ex["sub_ptr"], ex["layer_ptr"]
        stride = self.overlap + 2
        nI = np.array([lp[i * stride + 1] - lp[i * stride] for i in range(self.n_parts)])
        k = np.diff(zc)
        blocks = np.zeros(int((nI * k).sum()), dtype=np.float64)
        tls_export_zblocks(self.ctx, blocks)
        rows, cols, vals = [], [], []
        off = 0
        for i in range(self.n_parts):
            if k[i] == 0:
                continue
            B = blocks[off:off + nI[i] * k[i]].reshape(k[i], nI[i]).T  # column-major nI x k
            off += nI[i] * k[i]
            idx = ex["sub_idx"][spt[i]:spt[i] + nI[i]]
            rr, cc = np.meshgrid(idx, np.arange(zc[i], zc[i + 1]), indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(B.ravel())
        if not rows:
            return sp.csr_matrix((self.n, 0))
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.n, int(zc[-1])))

    def gnn_forward(self, weights: np.ndarray, c_out: int) -> np.ndarray:
        """Network output on every local graph: (sum #Omega_i) x c_out, rows in sub_idx order."""
        total = int(self.export()["sub_ptr"][-1])
        X = np.zeros((total, c_out), dtype=np.float32)
        tls_gnn_forward(self.ctx, np.ascontiguousarray(weights, dtype=np.float32), c_out, X)
        return X

    def gnn_loss_grad(self, weights: np.ndarray, c_out: int):
        """(loss, gradient) of the warm-start network against this context's targets."""
        w = np.ascontiguousarray(weights, dtype=np.float32)
        g = np.zeros_like(w)
        loss = tls_gnn_loss_grad(self.ctx, w, c_out, g)
        return loss, g

    def local_solve(self, i: int, b: np.ndarray) -> np.ndarray:
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b)
        tls_local_solve(self.ctx, i, b, x)
        return x

    def close(self):
        if getattr(self, "ctx", None):
            tls_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
