"""FP64 oracle: Krylov solvers with x0 = 0 (test infrastructure only).

Both stop when the unpreconditioned relative residual ||b - A x_k|| / ||b||
(the recurrence value) drops to ``tol`` and report the true residual at
exit, as the paper's experiments measure convergence (Section 7.2).
"""

from __future__ import annotations

import numpy as np


def pcg(A, M, b, tol=1e-8, maxit=1000):
    """Preconditioned conjugate gradients (Hestenes-Stiefel form), the
    method named for SPD systems in Section 1. ``A`` and ``M`` are callables
    (M applies the preconditioner). Returns (x, iterations, true relres)."""
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    if nb == 0.0:
        return x, 0, 0.0
    r = b.copy()
    z = M(r)
    p = z.copy()
    rz = r @ z
    it = 0
    for it in range(1, maxit + 1):
        q = A(p)
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) <= tol * nb:
            break
        z = M(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, np.linalg.norm(b - A(x)) / nb


def fgmres(A, M, b, tol=1e-8, restart=30, maxit=3000):
    """Right-preconditioned flexible GMRES(restart) with modified
    Gram-Schmidt; the small least-squares problem is solved directly at every
    step. Returns (x, iterations, true relres)."""
    nb = np.linalg.norm(b)
    n = b.size
    x = np.zeros_like(b)
    if nb == 0.0:
        return x, 0, 0.0
    it = 0
    r = b.copy()
    while it < maxit:
        beta = np.linalg.norm(r)
        if beta <= tol * nb:
            break
        V = np.zeros((n, restart + 1))
        Zs = np.zeros((n, restart))
        H = np.zeros((restart + 1, restart))
        V[:, 0] = r / beta
        e1 = np.zeros(restart + 1)
        e1[0] = beta
        j_done = 0
        y = np.zeros(0)
        for j in range(restart):
            it += 1
            Zs[:, j] = M(V[:, j])
            w = A(Zs[:, j])
            for i in range(j + 1):
                H[i, j] = V[:, i] @ w
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[:, j + 1] = w / H[j + 1, j]
            y, *_ = np.linalg.lstsq(H[: j + 2, : j + 1], e1[: j + 2], rcond=None)
            res = np.linalg.norm(e1[: j + 2] - H[: j + 2, : j + 1] @ y)
            j_done = j + 1
            if res <= tol * nb or H[j + 1, j] == 0 or it >= maxit:
                break
        x = x + Zs[:, :j_done] @ y
        r = b - A(x)
        if np.linalg.norm(r) <= tol * nb:
            break
    return x, it, np.linalg.norm(b - A(x)) / nb
