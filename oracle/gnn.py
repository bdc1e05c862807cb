"""Warm-start network for the local eigensolver: plain NumPy forward, loss
and backward in float64, one subdomain at a time.

TEST INFRASTRUCTURE ONLY (see the package docstring): the GPU library's
network kernels are checked against this.

The network is not part of the paper. It predicts a start block for the
subspace iteration that computes the dominant eigenvectors of
eq. gevpsvd; the method itself is unchanged by it (the paper's eigenvectors
are still computed to the same tolerance), so the network only has to be
a good guess. Definition, for the local matrix A_ii with Omega_i ordered
[I_i, Gamma_{i,1}, .., Gamma_{i,delta}] (Section 2.1):

* graph: nodes Omega_i; an edge (a, b), a != b, wherever (A_ii)_ab != 0,
  weighted e_ab = |a_ab| / sqrt(|a_aa| |a_bb|)  (E: m x m, zero diagonal);
* features (m x 4): [1, 1{a in I_i}, 1{a in Gamma_{i,delta}},
  log10(|a_aa| / mean_b |a_bb|)];
* four layers of width 32: H_l = tanh(E H_{l-1} Theta_l + H_{l-1} Phi_l + b_l),
  H_0 = features;
* output X = H_4 Omega (m x c_out).

Training loss for one subdomain, on the rows T = Gamma_{i,delta} (the only
rows the eigensolver's reduced problem sees), against an orthonormal basis
Q (#T x k) of the rows T of the top-k eq. gevpsvd eigenvectors:

    f = -(1/k) tr(G^{-1} X_T^T Q Q^T X_T),   G = X_T^T X_T,

which is -1 exactly when span(X_T) contains span(Q) and is unchanged by
X_T -> X_T R for any invertible R (it depends on span(X_T) only).

Weights are one flat vector: for l = 1..4, Theta_l (c_{l-1} x 32, row
major), Phi_l (c_{l-1} x 32), b_l (32); then Omega (32 x c_out); c_0 = 4.

Pinned by: central finite differences of the loss (gradient), the loss's
closed values (-1 on the target span, 0 on its orthogonal complement) and
its invariance under X_T -> X_T R, permutation equivariance of the forward
pass, and a three-node graph worked by hand (tests/test_oracle_gnn.py).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

LAYERS = 4
FEATURES = 4
HIDDEN = 32


def n_weights(c_out: int) -> int:
    """Length of the flat weight vector."""
    n = 0
    cin = FEATURES
    for _ in range(LAYERS):
        n += 2 * cin * HIDDEN + HIDDEN
        cin = HIDDEN
    return n + HIDDEN * c_out


def unpack(w: np.ndarray, c_out: int):
    """Flat weights -> ([(Theta, Phi, b)] * LAYERS, Omega)."""
    w = np.asarray(w, dtype=np.float64)
    assert w.size == n_weights(c_out)
    layers, o, cin = [], 0, FEATURES
    for _ in range(LAYERS):
        th = w[o:o + cin * HIDDEN].reshape(cin, HIDDEN)
        o += cin * HIDDEN
        ph = w[o:o + cin * HIDDEN].reshape(cin, HIDDEN)
        o += cin * HIDDEN
        b = w[o:o + HIDDEN]
        o += HIDDEN
        layers.append((th, ph, b))
        cin = HIDDEN
    om = w[o:o + HIDDEN * c_out].reshape(HIDDEN, c_out)
    return layers, om


def pack(layers, om) -> np.ndarray:
    parts = []
    for th, ph, b in layers:
        parts += [np.ravel(th), np.ravel(ph), np.ravel(b)]
    parts.append(np.ravel(om))
    return np.concatenate(parts)


def graph(Aii: sp.spmatrix) -> sp.csr_matrix:
    """E with e_ab = |a_ab| / sqrt(|a_aa| |a_bb|) off the diagonal."""
    A = sp.csr_matrix(Aii, dtype=np.float64)
    d = np.abs(A.diagonal())
    s = np.zeros_like(d)
    s[d > 0] = 1.0 / np.sqrt(d[d > 0])
    E = sp.diags(s) @ abs(A) @ sp.diags(s)
    E = E.tolil()
    E.setdiag(0.0)
    E = E.tocsr()
    E.eliminate_zeros()
    return E


def features(Aii: sp.spmatrix, n_interior: int, n_last: int) -> np.ndarray:
    """[1, in I_i, in Gamma_{i,delta}, log10(|a_aa| / mean |a_bb|)]."""
    m = Aii.shape[0]
    d = np.abs(np.asarray(Aii.diagonal(), dtype=np.float64))
    F = np.zeros((m, FEATURES))
    F[:, 0] = 1.0
    F[:n_interior, 1] = 1.0
    F[m - n_last:, 2] = 1.0
    mean = d.mean()
    F[:, 3] = np.log10(d / mean)
    return F


def forward(Aii: sp.spmatrix, n_interior: int, n_last: int, w: np.ndarray, c_out: int):
    """Returns (X, cache) with X = H_4 Omega."""
    layers, om = unpack(w, c_out)
    E = graph(Aii)
    H = [features(Aii, n_interior, n_last)]
    M = []
    for th, ph, b in layers:
        msg = E @ H[-1]
        M.append(msg)
        H.append(np.tanh(msg @ th + H[-1] @ ph + b[None, :]))
    X = H[-1] @ om
    return X, {"E": E, "H": H, "M": M, "layers": layers, "om": om}


def loss(X: np.ndarray, n_last: int, Q: np.ndarray):
    """f = -(1/k) tr(G^{-1} X_T^T Q Q^T X_T) and df/dX (zero outside rows T)."""
    m = X.shape[0]
    k = Q.shape[1]
    XT = X[m - n_last:]
    G = XT.T @ XT
    A1 = Q.T @ XT                     # k x c
    B = A1.T @ A1                     # X_T^T Q Q^T X_T
    Gi = np.linalg.inv(G)
    f = -np.trace(Gi @ B) / k
    # d tr(G^{-1} B) / dX_T = 2 (Q Q^T X_T G^{-1} - X_T G^{-1} B G^{-1})
    dXT = -(2.0 / k) * (Q @ (A1 @ Gi) - XT @ (Gi @ B @ Gi))
    dX = np.zeros_like(X)
    dX[m - n_last:] = dXT
    return f, dX


def backward(cache, dX: np.ndarray, c_out: int) -> np.ndarray:
    """Gradient of <dX, X> with respect to the flat weights."""
    E, H, M, layers, om = cache["E"], cache["H"], cache["M"], cache["layers"], cache["om"]
    d_om = H[-1].T @ dX
    dH = dX @ om.T
    grads = []
    for l in range(LAYERS - 1, -1, -1):
        th, ph, _ = layers[l]
        dZ = dH * (1.0 - H[l + 1] ** 2)
        d_th = M[l].T @ dZ
        d_ph = H[l].T @ dZ
        d_b = dZ.sum(axis=0)
        grads.append((d_th, d_ph, d_b))
        dM = dZ @ th.T
        dH = dZ @ ph.T + E.T @ dM
    grads.reverse()
    return pack(grads, d_om)


def loss_grad(Aii, n_interior: int, n_last: int, w: np.ndarray, c_out: int, Q: np.ndarray):
    """(loss, gradient) of one subdomain."""
    X, cache = forward(Aii, n_interior, n_last, w, c_out)
    f, dX = loss(X, n_last, Q)
    return f, backward(cache, dX, c_out)


def target_basis(W: np.ndarray, n_last: int) -> np.ndarray:
    """Orthonormal basis of the rows Gamma_{i,delta} of eigenvectors W."""
    WT = W[W.shape[0] - n_last:]
    Qm, _ = np.linalg.qr(WT)
    return Qm
