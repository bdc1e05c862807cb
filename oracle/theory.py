"""FP64 oracle: brute-force theory objects for tiny inputs (test
infrastructure only). Dense everything; use on grids of a few hundred
unknowns."""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .schwarz import Handle, Subdomain, harmonic_operator, local_matrix


def spsd_splitting_block(A, sub: Subdomain) -> np.ndarray:
    """Local SPSD splitting of Lemma spsd_splitting (eq. LSPSD), restricted
    to Omega_i (tilde A_ii), from its block formula: A_ii with the
    (Gamma_delta, Gamma_delta) block replaced by
    A_{Gd,G'} S_{G'}^{-1} A_{G',Gd}, S_{G'} the Schur complement of eq. S_G.
    The formula needs delta >= 2 (it assumes A_{I, Gamma_delta} = 0)."""
    Ad = local_matrix(A, sub).toarray()
    nI, npr = sub.n_interior, sub.n_prime
    if npr == nI:
        raise ValueError("the block formula of eq. LSPSD needs delta >= 2")
    I = slice(0, nI)
    G = slice(nI, npr)  # Gamma_{1:delta-1}
    Gd = slice(npr, sub.size)
    S = Ad[G, G] - Ad[G, I] @ np.linalg.solve(Ad[I, I], Ad[I, G])
    T = Ad.copy()
    T[Gd, Gd] = Ad[Gd, G] @ np.linalg.solve(S, Ad[G, Gd])
    return T


def spsd_splitting_projection(A, sub: Subdomain) -> np.ndarray:
    """tilde A_ii = (I - Pi_i)^T A_ii (I - Pi_i), eq.
    local_problem_local_spsd_splitting; valid for every delta >= 1."""
    Ad = local_matrix(A, sub).toarray()
    Pi = harmonic_operator(local_matrix(A, sub), sub)
    Q = np.eye(sub.size) - Pi
    return Q.T @ Ad @ Q


def overlap_colors(subs: list, n: int) -> int:
    """k_c of Lemma multiplicity: number of colors of a greedy coloring of
    the graph in which subdomains i != j are adjacent when Omega_i and
    Omega_j intersect (same-colored subdomains then never overlap)."""
    N = len(subs)
    member = [set(s.idx.tolist()) for s in subs]
    adj = [[j for j in range(N) if j != i and member[i] & member[j]] for i in range(N)]
    color = [-1] * N
    for i in range(N):
        used = {color[j] for j in adj[i] if color[j] >= 0}
        c = 0
        while c in used:
            c += 1
        color[i] = c
    return max(color) + 1 if N else 0


def lambda_star(A, subs: list) -> float:
    """Largest eigenvalue of sum_i R_i^T A_ii R_i u = lambda A u
    (eq. lambda_star), dense."""
    Ad = A.toarray()
    S = np.zeros_like(Ad)
    for s in subs:
        S[np.ix_(s.idx, s.idx)] += Ad[np.ix_(s.idx, s.idx)]
    return float(sla.eigh(S, Ad, eigvals_only=True)[-1])


def preconditioned_spectrum(h: Handle, Minv: np.ndarray) -> np.ndarray:
    """Eigenvalues of M^{-1} A for SPD A and SPD M^{-1}: the pencil
    (A, inv(M^{-1})) has the same spectrum, solved with a dense
    symmetric-definite eigensolver."""
    Ad = h.A.toarray()
    M = np.linalg.inv(0.5 * (Minv + Minv.T))
    return sla.eigh(Ad, 0.5 * (M + M.T), eigvals_only=True)


def bound_all_kept(kc: int, nu: float) -> float:
    """Theorem upper_bound_1: kappa <= (k_c+1)(2 + (2k_c+1) k_c nu)."""
    return (kc + 1) * (2 + (2 * kc + 1) * kc * nu)


def bound_truncated(kc: int, nu: float, tau: float, lam_star: float) -> float:
    """Theorem upper_bound_2:
    kappa <= (k_c+1)(2 + (2k_c+1) nu (k_c + lambda_* (2 tau + tau^2)))."""
    return (kc + 1) * (2 + (2 * kc + 1) * nu * (kc + lam_star * (2 * tau + tau * tau)))


def coarse_space_v1(A, subs: list, nu: float) -> np.ndarray:
    """Basis of eq. coarse_space (all harmonic columns kept): for each i the
    columns R_i^T D_i [E_i ; I] (E_i from eq. HOp) and R_i^T D_i Z_i with Z_i
    the GEVP1 vectors of eigenvalue > nu (eq. Z_i). Dense, tiny inputs."""
    from .schwarz import gevp1
    n = A.shape[0]
    cols = []
    for s in subs:
        Aii = local_matrix(A, s)
        Pi = harmonic_operator(Aii, s)
        D = s.D()
        blk = (D[:, None] * Pi)[:, s.n_prime:]
        _, Zi = gevp1(Aii, s, s.size, nu, dense=True)
        blk = np.hstack([blk, D[:, None] * Zi])
        full = np.zeros((n, blk.shape[1]))
        full[s.idx] = blk
        cols.append(full)
    C = np.hstack(cols)
    U, sv, _ = np.linalg.svd(C, full_matrices=False)
    return U[:, sv > 1e-10 * sv[0]]
