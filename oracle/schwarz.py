"""FP64 oracle: the two-level additive Schwarz preconditioner, step by step.

Test infrastructure only (see the package docstring). Notation follows the
paper: I_i is the nonoverlapping set of subdomain i, Gamma_{i,1:delta} the
unknowns reached from I_i through at most delta edges of graph(A + A^T),
Omega_i = [I_i, Gamma_{i,1}, ..., Gamma_{i,delta}], Omega' = Omega_{i,1:delta-1}
(I_i followed by the first delta-1 layers) and Gamma = Gamma_{i,delta}.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import krylov

# Dense eigen/SVD paths are used up to this local size, ARPACK beyond it.
DENSE_LIMIT = 1600


# --------------------------------------------------------------------------
# Section 2.1: overlapping subdomains, restriction and partition of unity
# --------------------------------------------------------------------------

@dataclass
class Subdomain:
    """Ordered index set of Omega_i = [I_i, Gamma_{i,1}, ..., Gamma_{i,delta}]
    (Section 2.1). ``idx`` is R_i as an index list; D_i is 1 on the first
    ``n_interior`` positions and 0 elsewhere."""

    idx: np.ndarray
    n_interior: int
    layer_sizes: list = field(default_factory=list)

    @property
    def size(self) -> int:
        return int(self.idx.size)

    @property
    def n_prime(self) -> int:
        """#Omega_{i,1:delta-1}: interior plus all layers but the last."""
        return self.n_interior + int(sum(self.layer_sizes[:-1])) if self.layer_sizes else self.n_interior

    @property
    def n_gamma(self) -> int:
        """#Gamma_{i,delta}: the last layer."""
        return int(self.layer_sizes[-1]) if self.layer_sizes else 0

    def D(self) -> np.ndarray:
        """Boolean partition-of-unity diagonal (Section 2.1)."""
        d = np.zeros(self.size)
        d[: self.n_interior] = 1.0
        return d


def sym_pattern(A: sp.spmatrix) -> sp.csr_matrix:
    """Sparsity graph of A + A^T as a 0/1 CSR matrix (Section 2.1)."""
    P = (abs(A) + abs(A).T).tocsr()
    P.data[:] = 1.0
    return P


def overlap(A: sp.spmatrix, part: np.ndarray, i: int, delta: int, G: sp.csr_matrix | None = None) -> Subdomain:
    """Omega_{i,1:delta} by breadth-first layers on graph(A + A^T)
    (Section 2.1): layer l holds the nodes not in I_i and not in an earlier
    layer that are adjacent to layer l-1 (layer 0 = I_i). Within I_i and
    within each layer, nodes are in ascending global order (the paper leaves
    that order free; the worked example of Section 2.1 uses it). ``G`` may
    pass sym_pattern(A) when it is already formed."""
    G = sym_pattern(A) if G is None else G
    n = A.shape[0]
    interior = np.flatnonzero(part == i)
    seen = np.zeros(n, dtype=bool)
    seen[interior] = True
    frontier = interior
    layers = []
    for _ in range(delta):
        if frontier.size == 0:
            layers.append(np.zeros(0, dtype=np.int64))
            continue
        reach = np.unique(G[frontier].indices)
        new = reach[~seen[reach]]
        seen[new] = True
        layers.append(new)
        frontier = new
    idx = np.concatenate([interior] + layers) if layers else interior
    return Subdomain(idx.astype(np.int64), int(interior.size), [int(l.size) for l in layers])


def restriction(sub: Subdomain, n: int) -> sp.csr_matrix:
    """R_i as a sparse 0/1 matrix of shape (#Omega_i, n) (Section 2.1)."""
    m = sub.size
    return sp.csr_matrix((np.ones(m), (np.arange(m), sub.idx)), shape=(m, n))


def local_matrix(A: sp.spmatrix, sub: Subdomain) -> sp.csr_matrix:
    """A_ii = R_i A R_i^T (Section 2.3)."""
    A = A.tocsr()
    return A[sub.idx][:, sub.idx].tocsr()


# --------------------------------------------------------------------------
# Section 3.2: local harmonic operator
# --------------------------------------------------------------------------

def harmonic_block(Aii: sp.spmatrix, sub: Subdomain) -> np.ndarray:
    """E = -A_{Omega',Omega'}^{-1} A_{Omega',Gamma}, the upper block of
    Pi_i restricted to its Gamma columns (eq. HOp), computed with a sparse LU
    solve. Shape (#Omega', #Gamma)."""
    npr, ng = sub.n_prime, sub.n_gamma
    if ng == 0:
        return np.zeros((npr, 0))
    Aii = Aii.tocsc()
    App = Aii[:npr, :npr].tocsc()
    ApG = Aii[:npr, npr:].toarray()
    return -spla.splu(App).solve(ApG)


def harmonic_operator(Aii: sp.spmatrix, sub: Subdomain) -> np.ndarray:
    """Dense Pi_i (eq. HOp): Pi_i v = [E v_Gamma ; v_Gamma]."""
    m, npr = sub.size, sub.n_prime
    Pi = np.zeros((m, m))
    E = harmonic_block(Aii, sub)
    Pi[:npr, npr:] = E
    Pi[npr:, npr:] = np.eye(m - npr)
    return Pi


# --------------------------------------------------------------------------
# Section 3.3 and Proposition gevpsvd: the two local eigenproblems
# --------------------------------------------------------------------------

def _top_pairs(vals: np.ndarray, vecs: np.ndarray, k: int, floor_rel: float = 1e-12,
               threshold: float | None = None):
    order = np.argsort(vals)[::-1]
    vals, vecs = vals[order], vecs[:, order]
    if vals.size == 0:
        return vals, vecs
    vmax = max(vals[0], 0.0)
    keep = vals > floor_rel * vmax if vmax > 0 else np.zeros(vals.size, dtype=bool)
    if threshold is not None:
        keep &= vals > threshold
    vals, vecs = vals[keep], vecs[:, keep]
    return vals[:k], vecs[:, :k]


def gevp2(Aii: sp.spmatrix, sub: Subdomain, k: int, tau2: float | None = None,
          dense: bool | None = None):
    """Largest eigenpairs of Pi_i^T D_i A_ii D_i Pi_i w = lambda^2 A_ii w
    (eq. gevpsvd), A_ii-normalized. Returns (lambda^2 descending, W) with at
    most k pairs; pairs with lambda^2 <= 1e-12 * max lambda^2 are dropped
    (they give D_i Pi_i w = 0), and with ``tau2`` only lambda^2 > tau2 is
    kept. Small subdomains use a dense symmetric-definite solver on the full
    pencil; larger ones use ARPACK in generalized mode with the operator
    applied through sparse LU solves."""
    m = sub.size
    if sub.n_gamma == 0 or k == 0:
        return np.zeros(0), np.zeros((m, 0))
    dense = (m <= DENSE_LIMIT) if dense is None else dense
    D = sub.D()
    if dense:
        Ad = Aii.toarray()
        Pi = harmonic_operator(Aii, sub)
        lhs = Pi.T @ (D[:, None] * Ad * D[None, :]) @ Pi
        lhs = 0.5 * (lhs + lhs.T)
        vals, vecs = sla.eigh(lhs, Ad)
        return _top_pairs(vals, vecs, k, threshold=tau2)
    npr = sub.n_prime
    Aii = Aii.tocsc()
    lu_p = spla.splu(Aii[:npr, :npr].tocsc())
    ApG = Aii[:npr, npr:].tocsc()
    AGp = Aii[npr:, :npr].tocsc()
    lu_a = spla.splu(Aii)

    def pi(v):
        out = np.empty(m)
        out[npr:] = v[npr:]
        out[:npr] = -lu_p.solve(ApG @ v[npr:])
        return out

    def pi_t(u):
        out = np.zeros(m)
        out[npr:] = u[npr:] - AGp @ lu_p.solve(u[:npr], trans="T")
        return out

    def op(v):
        return pi_t(D * (Aii @ (D * pi(v))))

    Aop = spla.LinearOperator((m, m), matvec=op, dtype=np.float64)
    Mop = spla.LinearOperator((m, m), matvec=lambda v: Aii @ v, dtype=np.float64)
    Minv = spla.LinearOperator((m, m), matvec=lambda v: lu_a.solve(v), dtype=np.float64)
    kk = min(k, sub.n_gamma, m - 2)
    vals, vecs = spla.eigsh(Aop, k=kk, M=Mop, Minv=Minv, which="LA", tol=1e-12,
                            ncv=min(m - 1, max(2 * kk + 1, kk + 20)), maxiter=20000)
    # A_ii-normalize
    for j in range(vecs.shape[1]):
        vecs[:, j] /= np.sqrt(vecs[:, j] @ (Aii @ vecs[:, j]))
    return _top_pairs(vals, vecs, k, threshold=tau2)


def gevp1(Aii: sp.spmatrix, sub: Subdomain, k: int, nu: float = 1.0, dense: bool | None = None):
    """Largest eigenpairs of D_i A_ii D_i u = lambda A_ii u (eq. uppergevp)
    with lambda > nu, A_ii-normalized; at most k of them. Dense on small
    subdomains, ARPACK with a sparse LU of A_ii otherwise."""
    m = sub.size
    if k == 0:
        return np.zeros(0), np.zeros((m, 0))
    dense = (m <= DENSE_LIMIT) if dense is None else dense
    D = sub.D()
    if dense:
        Ad = Aii.toarray()
        vals, vecs = sla.eigh(D[:, None] * Ad * D[None, :], Ad)
        return _top_pairs(vals, vecs, k, floor_rel=0.0, threshold=nu)
    Aii = Aii.tocsc()
    lu_a = spla.splu(Aii)
    Aop = spla.LinearOperator((m, m), matvec=lambda v: D * (Aii @ (D * v)), dtype=np.float64)
    Mop = spla.LinearOperator((m, m), matvec=lambda v: Aii @ v, dtype=np.float64)
    Minv = spla.LinearOperator((m, m), matvec=lambda v: lu_a.solve(v), dtype=np.float64)
    kk = min(k, m - 2)
    vals, vecs = spla.eigsh(Aop, k=kk, M=Mop, Minv=Minv, which="LA", tol=1e-12,
                            ncv=min(m - 1, max(2 * kk + 1, kk + 20)), maxiter=20000)
    for j in range(vecs.shape[1]):
        vecs[:, j] /= np.sqrt(vecs[:, j] @ (Aii @ vecs[:, j]))
    return _top_pairs(vals, vecs, k, floor_rel=0.0, threshold=nu)


def svd_variant(Aii: sp.spmatrix, sub: Subdomain, k: int, tau: float | None = None):
    """Section 6 (general A): left singular vectors of D_i Pi_i in the
    Euclidean inner product. D_i Pi_i is zero outside rows I_i and columns
    Gamma_{i,delta}; its nonzero block is H = rows I_i of
    E = -A_{Omega',Omega'}^{-1} A_{Omega',Gamma}. Returns (sigma descending,
    left singular vectors padded to #Omega_i rows) for the k largest nonzero
    sigma (and sigma > tau when given)."""
    m, nI = sub.size, sub.n_interior
    if sub.n_gamma == 0 or k == 0:
        return np.zeros(0), np.zeros((m, 0))
    H = harmonic_block(Aii, sub)[:nI]
    U, s, _ = np.linalg.svd(H, full_matrices=False)
    smax = s[0] if s.size else 0.0
    keep = s > 1e-12 * smax if smax > 0 else np.zeros(s.size, dtype=bool)
    if tau is not None:
        keep &= s > tau
    s, U = s[keep][:k], U[:, keep][:, :k]
    out = np.zeros((m, s.size))
    out[:nI] = U
    return s, out


# --------------------------------------------------------------------------
# Setup, apply and solve (eq. coarse_space_2, Section 4.1, Remark in 4.4)
# --------------------------------------------------------------------------

@dataclass
class Handle:
    """Everything the oracle's two-level preconditioner holds."""

    A: sp.csr_matrix
    subs: list
    local_lu: list
    Z: np.ndarray              # n x n_C coarse basis (columns R_0^T)
    A0: np.ndarray             # Z^T A Z
    A0_fac: object
    spd: bool
    eig: list                  # per subdomain: kept eigenvalues (lambda^2 or sigma)
    eig1: list                 # per subdomain: kept GEVP1 eigenvalues
    n_coarse: int = 0

    @property
    def gc(self) -> float:
        return 1.0 + self.n_coarse / self.A.shape[0]

    @property
    def oc(self) -> float:
        nnz0 = int(np.count_nonzero(self.A0))
        return 1.0 + nnz0 / self.A.nnz


def coarse_block(Aii, sub: Subdomain, nev: int, nev1: int, spd: bool, tau=None, nu=None,
                 dense=None):
    """Columns D_i [Pi_i W_i^(1), Z_i] of eq. coarse_space_2 for one
    subdomain (general A: the left singular vectors of D_i Pi_i, Section 6),
    restricted to the rows I_i (D_i is zero elsewhere), then orthonormalized
    with an SVD dropping sigma <= 1e-10 sigma_max. Orthonormalizing does not
    change the span, hence not the coarse correction."""
    nI = sub.n_interior
    D = sub.D()
    cols = []
    if spd:
        lam2, W = gevp2(Aii, sub, nev, None if tau is None else tau * tau, dense)
        if W.shape[1]:
            # D_i Pi_i W: apply Pi_i through the sparse LU of A_{Omega',Omega'}
            E = harmonic_block(Aii, sub)
            npr = sub.n_prime
            PiW = np.vstack([E @ W[npr:], W[npr:]])
            cols.append((D[:, None] * PiW)[:nI])
        lam1, Zi = gevp1(Aii, sub, nev1, 1.0 if nu is None else nu, dense)
        if Zi.shape[1]:
            cols.append((D[:, None] * Zi)[:nI])
        eig = lam2
    else:
        s, Uleft = svd_variant(Aii, sub, nev, tau)
        if Uleft.shape[1]:
            cols.append(Uleft[:nI])
        eig, lam1 = s, np.zeros(0)
    if not cols:
        return np.zeros((nI, 0)), eig, lam1
    C = np.hstack(cols)
    U, s, _ = np.linalg.svd(C, full_matrices=False)
    keep = s > 1e-10 * s[0] if s.size and s[0] > 0 else np.zeros(s.size, dtype=bool)
    return U[:, keep], eig, lam1


def setup(A: sp.spmatrix, part: np.ndarray, overlap_layers: int, nev: int, *, nev1: int = 0,
          spd: bool = True, tau: float | None = None, nu: float | None = None,
          dense: bool | None = None, Z: np.ndarray | None = None) -> Handle:
    """Two-level setup: overlap (Section 2.1), local matrices (Section 2.3),
    coarse space eq. coarse_space_2 (or Section 6 for general A), Galerkin
    coarse operator A_00 = R_0 A R_0^T (Section 4.1) and its factorization.

    ``Z`` may be given (n x n_C) to build the coarse operator from an
    externally computed coarse basis instead."""
    A = sp.csr_matrix(A, dtype=np.float64)
    n = A.shape[0]
    n_parts = int(part.max()) + 1
    if overlap_layers == 0 and nev > 0:
        raise ValueError("overlap 0 leaves Gamma_{i,delta} empty: no coarse space can be built")
    subs, lus, eig, eig1, blocks = [], [], [], [], []
    G = sym_pattern(A)
    for i in range(n_parts):
        s = overlap(A, part, i, overlap_layers, G)
        Aii = local_matrix(A, s)
        subs.append(s)
        lus.append(spla.splu(Aii.tocsc()))
        if Z is None:
            Zi, e, e1 = coarse_block(Aii, s, nev, nev1, spd, tau, nu, dense)
            blocks.append(Zi)
            eig.append(e)
            eig1.append(e1)
    if Z is None:
        nC = sum(b.shape[1] for b in blocks)
        Z = np.zeros((n, nC))
        c = 0
        for s, b in zip(subs, blocks):
            Z[s.idx[: s.n_interior], c: c + b.shape[1]] = b
            c += b.shape[1]
    nC = Z.shape[1]
    A0 = Z.T @ (A @ Z) if nC else np.zeros((0, 0))
    if nC:
        fac = ("chol", sla.cho_factor(A0, lower=True)) if spd else ("lu", sla.lu_factor(A0))
    else:
        fac = None
    return Handle(A, subs, lus, Z, A0, fac, spd, eig, eig1, nC)


def coarse_solve(h: Handle, y: np.ndarray) -> np.ndarray:
    if h.A0_fac is None:
        return np.zeros(0)
    kind, f = h.A0_fac
    return sla.cho_solve(f, y) if kind == "chol" else sla.lu_solve(f, y)


def one_level(h: Handle, r: np.ndarray, *, restricted: bool = False) -> np.ndarray:
    """sum_i R_i^T A_ii^{-1} R_i r (eq. onelevelasm), or with the partition
    of unity D_i between the local solve and the prolongation,
    sum_i R_i^T D_i A_ii^{-1} R_i r (eq. onelevelras, restricted=True)."""
    z = np.zeros_like(r, dtype=np.float64)
    for s, lu in zip(h.subs, h.local_lu):
        zi = lu.solve(r[s.idx])
        if restricted:
            zi = zi * s.D()
        np.add.at(z, s.idx, zi)
    return z


def coarse_correction(h: Handle, r: np.ndarray) -> np.ndarray:
    """Q r = R_0^T A_00^{-1} R_0 r with R_0 = Z^T (Section 4.1)."""
    if not h.n_coarse:
        return np.zeros_like(r, dtype=np.float64)
    return h.Z @ coarse_solve(h, h.Z.T @ r)


COMPOSITIONS = ("additive", "ras_deflated")


def apply(h: Handle, r: np.ndarray, *, coarse: bool = True, restricted: bool = False,
          composition: str = "additive") -> np.ndarray:
    """The two-level preconditioner applied to r.

    composition="additive" (the theory's operator, Remark after Section 4.3):
        z = M_2^{-1} r = sum_i R_i^T A_ii^{-1} R_i r + Q r;
    ``restricted=True`` puts D_i into the one-level part (eq. onelevelras)
    of that sum.

    composition="ras_deflated" (what the experiments of Section 7.2 run,
    where the coarse correction is "deflated" by citation only; read as
    the standard deflated two-level form):
        z = Q r + M_RAS^{-1} (r - A Q r),
    with M_RAS^{-1} of eq. onelevelras. It is not symmetric, so it goes
    with (F)GMRES. Pinned by: M^{-1} A Z = Z (the coarse space is solved
    exactly), the one-level part equal to one step of the parallel Schwarz
    method (Efstathiou and Gander, 2003), N = 1 giving A^{-1}.

    ``coarse=False`` drops Q in either form."""
    if composition not in COMPOSITIONS:
        raise ValueError(f"composition must be one of {COMPOSITIONS}")
    use_q = coarse and h.n_coarse > 0
    if composition == "additive":
        z = one_level(h, r, restricted=restricted)
        if use_q:
            z += coarse_correction(h, r)
        return z
    if not use_q:
        return one_level(h, r, restricted=True)
    t = coarse_correction(h, r)
    return t + one_level(h, r - h.A @ t, restricted=True)


def solve(h: Handle, b: np.ndarray, tol: float = 1e-8, maxit: int | None = None, restart: int = 30,
          composition: str = "additive"):
    """x0 = 0; PCG for SPD A with the (symmetric) additive composition,
    right-preconditioned FGMRES(restart) otherwise, stopping on the
    unpreconditioned relative residual ||b - A x|| / ||b|| (Section 7.2).
    Returns (x, iterations, true relative residual)."""
    Amv = lambda v: h.A @ v  # noqa: E731
    Mv = lambda v: apply(h, v, composition=composition)  # noqa: E731
    if h.spd and composition == "additive":
        return krylov.pcg(Amv, Mv, b, tol, maxit or 1000)
    return krylov.fgmres(Amv, Mv, b, tol, restart, maxit or 3000)


def one_level_matrix(h: Handle) -> np.ndarray:
    """Dense sum_i R_i^T inv(A_ii) R_i with numpy's dense inverse (tiny
    inputs only): an independent route to eq. onelevelasm."""
    n = h.A.shape[0]
    M = np.zeros((n, n))
    for s in h.subs:
        Aii = local_matrix(h.A, s).toarray()
        M[np.ix_(s.idx, s.idx)] += np.linalg.inv(Aii)
    return M


def dense_preconditioner(h: Handle) -> np.ndarray:
    """Dense M_2^{-1} by applying the oracle to the identity (tiny inputs)."""
    n = h.A.shape[0]
    return np.column_stack([apply(h, e) for e in np.eye(n)])
