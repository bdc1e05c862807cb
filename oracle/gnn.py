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
* features (m x 12): [1, 1{a in I_i}, 1{a in Gamma_{i,delta}},
  log10(|a_aa| / mean_b |a_bb|), r_a0 .. r_a7], where the eight random
  channels r_aj = 2 u - 1 with u = (z >> 11) 2^-53, z the (8a + j + 1)-th
  output of SplitMix64 started from state 0 (Steele, Lea and Flood, 2014);
  they let the network turn noise into smooth, distinct columns, which
  structural features alone cannot (all nodes of a layer look alike);
* four layers of width 32: H_l = tanh(E H_{l-1} Theta_l + H_{l-1} Phi_l + b_l),
  H_0 = features;
* output X = H_4 Omega (m x c_out).

Training loss for one subdomain, on the rows T = Gamma_{i,delta} (the only
rows the eigensolver's reduced problem sees), against an orthonormal basis
Q (#T x k) of the rows T of the top-k eq. gevpsvd eigenvectors:

    f = -(1/k) tr(G_e^{-1} X_T^T Q Q^T X_T),
    G_e = X_T^T X_T + EPS (tr(X_T^T X_T) / c) I,   EPS = 1e-3,

the fraction of the target span that span(X_T) captures, regularized so
that nearly dependent columns do not blow up G^{-1}. It is -1/(1 + EPS)
when X_T = Q, 0 when X_T is orthogonal to Q, and unchanged by
X_T -> alpha X_T R for alpha != 0 and orthogonal R.

Weights are one flat vector: for l = 1..4, Theta_l (c_{l-1} x 32, row
major), Phi_l (c_{l-1} x 32), b_l (32); then Omega (32 x c_out); c_0 = 12.

Pinned by: central finite differences of the loss (gradient), the loss's
closed values and invariances, the published first outputs of SplitMix64,
permutation equivariance of the forward pass (features permuted along),
and a three-node graph worked by hand (tests/test_oracle_gnn.py).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

LAYERS = 4
STRUCT = 4            # structural input channels
RANDOM = 8            # random input channels
FEATURES = STRUCT + RANDOM
HIDDEN = 32
EPS = 1e-3            # loss regularization


def splitmix64(counter: np.ndarray) -> np.ndarray:
    """Output number counter + 1 of SplitMix64 started from state 0, as
    uint64 (published definition: state += 0x9E3779B97F4A7C15, then the
    xor-shift-multiply finalizer)."""
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (c + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def random_channels(m: int) -> np.ndarray:
    """m x RANDOM uniform values in [-1, 1): channel j of node a from
    counter RANDOM * a + j."""
    a = np.arange(m, dtype=np.uint64)[:, None] * np.uint64(RANDOM) + np.arange(RANDOM, dtype=np.uint64)[None, :]
    z = splitmix64(a)
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 * 2.0 - 1.0


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
    """[1, in I_i, in Gamma_{i,delta}, log10(|a_aa| / mean |a_bb|), random channels]."""
    m = Aii.shape[0]
    d = np.abs(np.asarray(Aii.diagonal(), dtype=np.float64))
    F = np.zeros((m, FEATURES))
    F[:, 0] = 1.0
    F[:n_interior, 1] = 1.0
    F[m - n_last:, 2] = 1.0
    mean = d.mean()
    F[:, 3] = np.log10(d / mean)
    F[:, STRUCT:] = random_channels(m)
    return F


def forward(Aii: sp.spmatrix, n_interior: int, n_last: int, w: np.ndarray, c_out: int, feats=None):
    """Returns (X, cache) with X = H_4 Omega (features from ``features``
    unless given)."""
    layers, om = unpack(w, c_out)
    E = graph(Aii)
    H = [features(Aii, n_interior, n_last) if feats is None else np.asarray(feats, dtype=np.float64)]
    M = []
    for th, ph, b in layers:
        msg = E @ H[-1]
        M.append(msg)
        H.append(np.tanh(msg @ th + H[-1] @ ph + b[None, :]))
    X = H[-1] @ om
    return X, {"E": E, "H": H, "M": M, "layers": layers, "om": om}


def loss(X: np.ndarray, n_last: int, Q: np.ndarray):
    """f = -(1/k) tr(G_e^{-1} X_T^T Q Q^T X_T) and df/dX (zero outside rows T)."""
    m = X.shape[0]
    k = Q.shape[1]
    XT = X[m - n_last:]
    c = XT.shape[1]
    G = XT.T @ XT
    Ge = G + EPS * (np.trace(G) / c) * np.eye(c)
    A1 = Q.T @ XT                     # k x c
    B = A1.T @ A1                     # X_T^T Q Q^T X_T
    Gi = np.linalg.inv(Ge)
    f = -np.trace(Gi @ B) / k
    # d tr(G_e^{-1} B) / dX_T = 2 (Q Q^T X_T G_e^{-1} - X_T G_e^{-1} B G_e^{-1})
    #                           - (2 EPS / c) tr(G_e^{-1} B G_e^{-1}) X_T
    T2 = Gi @ B @ Gi
    dXT = -(2.0 / k) * (Q @ (A1 @ Gi) - XT @ T2 - (EPS / c) * np.trace(T2) * XT)
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
