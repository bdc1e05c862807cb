"""The FP64 oracle with its per-subdomain work spread over worker processes.

Test infrastructure only, like the rest of ``oracle``. The arithmetic is
that of ``schwarz.setup`` and ``schwarz.apply`` (overlap layers, Section 2.1;
A_ii = R_i A R_i^T and their sparse LU, Section 2.3; the coarse blocks of
eq. coarse_space_2 or Section 6; A_00 = Z^T A Z, Section 4.1; the two-level
apply of the Remark in Section 4.3 and the RAS + deflated form of
Section 7.2); only where it runs changes. Each worker process (forked, so it
shares the parent's copy of A) owns a fixed set of subdomains: it builds
their index sets, local matrices and LU factors once, computes their coarse
blocks when no basis is given, and for each apply returns the sum over its
subdomains of R_i^T A_ii^{-1} R_i r (or with D_i, eq. onelevelras). The
parent adds the workers' sums in worker order, so a result does not depend
on timing, and does the coarse correction and the Krylov iteration. It
differs from the serial oracle only in the order in which the one-level
contributions are added (rounding level), which tests/test_oracle_pool.py
checks.

The coarse basis is held as a sparse n x n_C matrix (Z is zero outside the
rows I_i of each subdomain's block), so the configurations of the benchmark
(n up to 2.1M, n_C up to 12,288) fit in host memory.
"""

from __future__ import annotations

import mmap
import multiprocessing as mp
import os

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import krylov, schwarz

# inherited by the forked workers (never pickled)
_JOB: dict = {}


def _worker(conn, w, ids):
    # one BLAS thread per worker: the workers already use every core
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:  # pragma: no cover
        pass
    j = _JOB
    A, part, delta = j["A"], j["part"], j["delta"]
    r, zw = j["r"], j["z"][w]
    G = schwarz.sym_pattern(A)
    subs, lus, out = [], [], []
    for i in ids:
        s = schwarz.overlap(A, part, i, delta, G)
        Aii = schwarz.local_matrix(A, s)
        subs.append(s)
        lus.append(spla.splu(Aii.tocsc()))
        blk = None
        if j["blocks"]:
            blk = schwarz.coarse_block(Aii, s, j["nev"], j["nev1"], j["spd"], j["tau"], j["nu"], j["dense"])
        out.append((i, s.idx, s.n_interior, list(s.layer_sizes), blk))
    touched = np.unique(np.concatenate([s.idx for s in subs])) if subs else np.zeros(0, dtype=np.int64)
    conn.send((out, touched))
    while True:
        restricted = conn.recv()
        if restricted is None:
            break
        # this worker's sum, written to its own row of the shared array
        zw[touched] = 0.0
        for s, lu in zip(subs, lus):
            zi = lu.solve(r[s.idx])
            if restricted:
                zi = zi * s.D()
            zw[s.idx] += zi  # indices are distinct within one subdomain
        conn.send(True)
    conn.close()


def _shared(count: int) -> np.ndarray:
    """float64 array in anonymous shared memory (shared with forked workers)."""
    buf = mmap.mmap(-1, max(count, 1) * 8)
    return np.frombuffer(buf, dtype=np.float64, count=count)


def default_workers() -> int:
    """Worker processes: the host's cores, at most 16 (the CPU share of one
    GPU on the benchmark machines)."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        cores = os.cpu_count() or 1
    return max(1, min(16, cores))


class Pool:
    """``schwarz.setup`` + ``apply`` + ``solve`` over worker processes.

    ``Z`` (dense or sparse, n x n_C) imports a coarse basis instead of
    computing it; ``with_basis`` swaps the basis later without refactoring
    the local matrices. Use as a context manager or call ``close``."""

    def __init__(self, A, part, overlap_layers: int, nev: int, *, nev1: int = 0, spd: bool = True,
                 tau=None, nu=None, dense=None, Z=None, workers: int | None = None):
        A = sp.csr_matrix(A, dtype=np.float64)
        part = np.asarray(part)
        if overlap_layers == 0 and nev > 0:
            raise ValueError("overlap 0 leaves Gamma_{i,delta} empty: no coarse space can be built")
        self.A, self.spd, self.n = A, spd, A.shape[0]
        N = int(part.max()) + 1
        self.n_parts = N
        self.workers = min(workers or default_workers(), N)
        # subdomains dealt out by size (largest first, round robin) to even the load
        sizes = np.bincount(part, minlength=N)
        order = np.argsort(-sizes, kind="stable")
        ids = [order[w::self.workers].tolist() for w in range(self.workers)]
        # r and the workers' partial sums live in shared memory; the pipes
        # carry only the set-up results and one flag per apply
        self._r = _shared(self.n)
        self._z = _shared(self.workers * self.n).reshape(self.workers, self.n)
        _JOB.clear()
        _JOB.update(A=A, part=part, delta=overlap_layers, nev=nev, nev1=nev1, spd=spd, tau=tau, nu=nu,
                    dense=dense, blocks=Z is None, r=self._r, z=self._z)
        ctx = mp.get_context("fork")
        self._conns, self._procs = [], []
        for w in range(self.workers):
            a, b = ctx.Pipe()
            p = ctx.Process(target=_worker, args=(b, w, ids[w]), daemon=True)
            p.start()
            b.close()
            self._conns.append(a)
            self._procs.append(p)
        got = {}
        self._touched = []
        for c in self._conns:
            out, touched = c.recv()
            self._touched.append(touched)
            for i, idx, nI, layers, blk in out:
                got[i] = (schwarz.Subdomain(idx, nI, layers), blk)
        _JOB.clear()
        self.subs = [got[i][0] for i in range(N)]
        self.eig = []
        if Z is None:
            cols, rows, vals, c0 = [], [], [], 0
            for i in range(N):
                Zi, e, _ = got[i][1]
                self.eig.append(e)
                s = self.subs[i]
                k = Zi.shape[1]
                if k:
                    rr, cc = np.meshgrid(s.idx[:s.n_interior], np.arange(c0, c0 + k), indexing="ij")
                    rows.append(rr.ravel())
                    cols.append(cc.ravel())
                    vals.append(Zi.ravel())
                c0 += k
            if c0:
                Z = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                  shape=(self.n, c0))
            else:
                Z = sp.csc_matrix((self.n, 0))
        self.with_basis(Z)

    def with_basis(self, Z):
        """Coarse basis Z (n x n_C, dense or sparse): A_00 = Z^T A Z in FP64
        and its Cholesky (SPD) or LU with partial pivoting (general)."""
        Z = sp.csc_matrix(Z)
        self.Z = Z
        self.n_coarse = Z.shape[1]
        if self.n_coarse:
            A0 = (Z.T @ (self.A @ Z)).toarray()
            self.A0 = A0
            self._fac = ("chol", sla.cho_factor(A0, lower=True)) if self.spd else ("lu", sla.lu_factor(A0))
        else:
            self.A0 = np.zeros((0, 0))
            self._fac = None
        return self

    # -- the preconditioner ---------------------------------------------------
    def one_level(self, r: np.ndarray, restricted: bool = False) -> np.ndarray:
        """sum_i R_i^T A_ii^{-1} R_i r (eq. onelevelasm), or with D_i
        (eq. onelevelras)."""
        self._r[:] = r
        for c in self._conns:
            c.send(bool(restricted))
        for c in self._conns:
            c.recv()
        z = np.zeros(self.n)
        for w, t in enumerate(self._touched):
            z[t] += self._z[w, t]
        return z

    def coarse_correction(self, r: np.ndarray) -> np.ndarray:
        """Q r = Z A_00^{-1} Z^T r (Section 4.1)."""
        if not self.n_coarse:
            return np.zeros(self.n)
        y = self.Z.T @ r
        kind, f = self._fac
        y0 = sla.cho_solve(f, y) if kind == "chol" else sla.lu_solve(f, y)
        return self.Z @ y0

    def apply(self, r: np.ndarray, composition: str = "additive") -> np.ndarray:
        """The two-level preconditioner, as ``schwarz.apply``."""
        if composition == "additive":
            z = self.one_level(r)
            if self.n_coarse:
                z += self.coarse_correction(r)
            return z
        if composition != "ras_deflated":
            raise ValueError(f"composition must be one of {schwarz.COMPOSITIONS}")
        if not self.n_coarse:
            return self.one_level(r, restricted=True)
        t = self.coarse_correction(r)
        return t + self.one_level(r - self.A @ t, restricted=True)

    def solve(self, b, tol: float = 1e-8, maxit: int | None = None, restart: int = 30,
              composition: str = "additive"):
        """As ``schwarz.solve``: PCG for SPD A with the additive composition,
        right-preconditioned FGMRES(restart) otherwise; x0 = 0."""
        Amv = lambda v: self.A @ v  # noqa: E731
        Mv = lambda v: self.apply(v, composition)  # noqa: E731
        if self.spd and composition == "additive":
            return krylov.pcg(Amv, Mv, b, tol, maxit or 1000)
        return krylov.fgmres(Amv, Mv, b, tol, restart, maxit or 3000)

    def close(self):
        for c in self._conns:
            try:
                c.send(None)
                c.close()
            except (OSError, BrokenPipeError):
                pass
        for p in self._procs:
            p.join(timeout=10)
            if p.is_alive():
                p.kill()
        self._conns, self._procs = [], []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        if getattr(self, "_procs", None):
            self.close()
