"""Pins of the warm-start network oracle (oracle/gnn.py): finite
differences, closed values of the loss, invariances and a three-node graph
worked by hand."""

import numpy as np
import scipy.sparse as sp

from oracle import gnn, schwarz
from workloads import box_partition_2d, poisson_2d


def _subdomain(delta=1):
    A = poisson_2d(12)
    part = box_partition_2d(12, 12, 2, 2)
    s = schwarz.overlap(A, part, 0, delta)
    Aii = schwarz.local_matrix(A, s)
    return Aii, s


def _weights(c_out, seed, scale=0.4):
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(gnn.n_weights(c_out))


def test_weight_count():
    # 4 layers: 2*12*32+32, then 3 x (2*32*32+32), then 32*c_out
    assert gnn.n_weights(40) == 800 + 3 * 2080 + 32 * 40
    w = _weights(5, 0)
    layers, om = gnn.unpack(w, 5)
    assert np.array_equal(gnn.pack(layers, om), w)


def test_three_node_graph_by_hand():
    A = sp.csr_matrix(np.array([[4.0, -1.0, 0.0], [-1.0, 9.0, -3.0], [0.0, -3.0, 16.0]]))
    E = gnn.graph(A).toarray()
    # e_01 = 1/sqrt(4*9) = 1/6, e_12 = 3/sqrt(9*16) = 1/4, zero diagonal
    assert np.allclose(E, [[0, 1 / 6, 0], [1 / 6, 0, 0.25], [0, 0.25, 0]], atol=1e-15)
    F = gnn.features(A, 1, 1)
    # mean diagonal 29/3: log10(12/29), log10(27/29), log10(48/29)
    assert np.allclose(F[:, 3], [-0.383216752, -0.031034234, 0.218843239], atol=1e-9)
    assert np.array_equal(F[:, :3], [[1, 1, 0], [1, 0, 0], [1, 0, 1]])
    assert np.all(np.abs(F[:, 4:]) <= 1.0)
    # one path through the network: feature "1" -> hidden 0 by Theta_1, then
    # Phi_l passes hidden 0 on, Omega reads it: X = tanh^4(row sums of E)
    layers, om = gnn.unpack(np.zeros(gnn.n_weights(2)), 2)
    layers[0][0][0, 0] = 1.0
    for l in range(1, 4):
        layers[l][1][0, 0] = 1.0
    om[0, 1] = 1.0
    X, _ = gnn.forward(A, 1, 1, gnn.pack(layers, om), 2, feats=np.hstack([F[:, :4], np.zeros((3, 8))]))
    rows = np.array([1 / 6, 1 / 6 + 0.25, 0.25])
    assert np.allclose(X[:, 0], 0.0)
    assert np.allclose(X[:, 1], np.tanh(np.tanh(np.tanh(np.tanh(rows)))), atol=1e-15)


def test_splitmix64_published_outputs():
    """First three outputs of SplitMix64 from state 0 (the published
    sequence) and the mapping to [-1, 1)."""
    z = gnn.splitmix64(np.arange(3))
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    r = gnn.random_channels(2)
    assert r.shape == (2, 8)
    assert abs(r[0, 0] - ((0xE220A8397B1DCDAF >> 11) * 2.0 ** -53 * 2 - 1)) < 1e-16
    assert abs(r[0, 2] - ((0x06C45D188009454F >> 11) * 2.0 ** -53 * 2 - 1)) < 1e-16


def test_loss_closed_values_and_span_invariance():
    rng = np.random.default_rng(3)
    m, nT, k = 30, 12, 4
    Q, _ = np.linalg.qr(rng.standard_normal((nT, k)))
    X = rng.standard_normal((m, k))
    X[m - nT:] = Q
    f, _ = gnn.loss(X, nT, Q)
    assert abs(f + 1.0 / (1.0 + gnn.EPS)) < 1e-13
    # columns orthogonal to span(Q)
    P = np.eye(nT) - Q @ Q.T
    X0 = rng.standard_normal((m, 3))
    X0[m - nT:] = P @ rng.standard_normal((nT, 3))
    f0, _ = gnn.loss(X0, nT, Q)
    assert abs(f0) < 1e-13
    # unchanged by X_T -> alpha X_T R with R orthogonal
    X = rng.standard_normal((m, 6))
    R, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    f1, _ = gnn.loss(X, nT, Q)
    f2, _ = gnn.loss(-2.5 * X @ R, nT, Q)
    assert abs(f1 - f2) < 1e-12 * abs(f1)
    assert -1.0 <= f1 <= 0.0
    # without regularization it would be the captured fraction of span(Q)
    XT = X[m - nT:]
    P = XT @ np.linalg.solve(XT.T @ XT, XT.T)
    frac = np.trace(Q.T @ P @ Q) / k
    assert abs(-f1 - frac) < 10 * gnn.EPS


def test_gradient_by_finite_differences():
    Aii, s = _subdomain(delta=2)
    nT = s.layer_sizes[-1]
    lam, W = schwarz.gevp2(Aii, s, 3, dense=True)
    Q = gnn.target_basis(W, nT)
    c_out = 6
    w = _weights(c_out, 1)
    f, g = gnn.loss_grad(Aii, s.n_interior, nT, w, c_out, Q)
    rng = np.random.default_rng(2)
    h = 1e-5  # unit directions: central-difference truncation ~1e-10, rounding ~1e-7
    for _ in range(6):
        v = rng.standard_normal(w.size)
        v /= np.linalg.norm(v)
        fp, _ = gnn.loss_grad(Aii, s.n_interior, nT, w + h * v, c_out, Q)
        fm, _ = gnn.loss_grad(Aii, s.n_interior, nT, w - h * v, c_out, Q)
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g @ v) <= 1e-6 * max(1.0, abs(fd)), (fd, g @ v)
    # each weight block is reached: single-coordinate differences
    layers, om = gnn.unpack(np.arange(w.size, dtype=float), c_out)
    probes = [int(layers[0][0][3, 5]), int(layers[2][1][7, 1]), int(layers[3][2][4]), int(om[9, 2])]
    for j in probes:
        e = np.zeros(w.size)
        e[j] = 1.0
        fp, _ = gnn.loss_grad(Aii, s.n_interior, nT, w + h * e, c_out, Q)
        fm, _ = gnn.loss_grad(Aii, s.n_interior, nT, w - h * e, c_out, Q)
        assert abs((fp - fm) / (2 * h) - g[j]) <= 1e-6 * max(1.0, abs(g[j]))


def test_forward_is_permutation_equivariant():
    """Relabelling nodes inside I_i, inside the middle layers and inside
    Gamma_{i,delta}, with their features, permutes the rows of X the same way."""
    Aii, s = _subdomain(delta=2)
    m, nI, nT = s.size, s.n_interior, s.layer_sizes[-1]
    rng = np.random.default_rng(5)
    perm = np.concatenate([rng.permutation(nI), nI + rng.permutation(m - nI - nT), m - nT + rng.permutation(nT)])
    P = sp.csr_matrix((np.ones(m), (np.arange(m), perm)), shape=(m, m))
    w = _weights(4, 7)
    F = gnn.features(Aii, nI, nT)
    X, _ = gnn.forward(Aii, nI, nT, w, 4)
    Xp, _ = gnn.forward((P @ Aii @ P.T).tocsr(), nI, nT, w, 4, feats=F[perm])
    assert np.allclose(Xp, X[perm], atol=1e-13)
