"""Pins of the FP64 oracle against what the paper and the mathematics fix
(CPU only). Each test names the passage it checks. None of them compares the
oracle with itself: the expected values come from the paper's printed
example, closed-form spectra, invariants, textbook routines on dense
matrices, or brute force on tiny grids."""

import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from oracle import krylov, schwarz, theory
from workloads import (box_partition_2d, convdiff_2d, fv_diffusion_2d, high_contrast_kappa_2d,
                       one_way_convection_2d, poisson_2d, rcb_partition, worked_example_7x7)


def _dense_pi_d(A, sub):
    """Dense D_i Pi_i assembled from numpy's dense inverse (independent of
    the oracle's sparse LU route)."""
    Ad = schwarz.local_matrix(A, sub).toarray()
    npr = sub.n_prime
    E = -np.linalg.inv(Ad[:npr, :npr]) @ Ad[:npr, npr:]
    Pi = np.zeros_like(Ad)
    Pi[:npr, npr:] = E
    Pi[npr:, npr:] = np.eye(sub.size - npr)
    return np.diag(sub.D()) @ Pi, Pi, Ad


def _small_hc(nx=16, seed=3):
    rng = np.random.default_rng(seed)
    kappa = high_contrast_kappa_2d(nx, nx, rng, n_channels=3, kmax=1e3)
    A = fv_diffusion_2d(kappa)
    part = rcb_partition((nx, nx), 2, rng)
    return A, part


# ----------------------------------------------------------------------------
# P1: the worked example of Section 2.1
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("delta", [1, 2])
def test_worked_example_index_sets(golden_dir, delta):
    g = json.load(open(os.path.join(golden_dir, "worked_example_7x7.json")))
    A, part = worked_example_7x7()
    assert np.array_equal(A.toarray(), np.array(g["A"], dtype=float))
    case = g[f"delta{delta}"]
    for i in range(2):
        s = schwarz.overlap(A, part, i, delta)
        assert (s.idx + 1).tolist() == case["Omega"][i]
        assert s.D().astype(int).tolist() == case["D"][i]
        assert schwarz.restriction(s, 7).toarray().astype(int).tolist() == case["R"][i]


def test_worked_example_local_matrix(golden_dir):
    """A_22 = R_2 A R_2^T for delta = 1 (Section 2.3) from the printed A and
    printed R_{2,1:1}."""
    g = json.load(open(os.path.join(golden_dir, "worked_example_7x7.json")))
    A, part = worked_example_7x7()
    R = np.array(g["delta1"]["R"][1], dtype=float)
    s = schwarz.overlap(A, part, 1, 1)
    expect = R @ np.array(g["A"], dtype=float) @ R.T
    assert np.array_equal(schwarz.local_matrix(A, s).toarray(), expect)
    assert expect.tolist() == [[11, 12, 0, 0, 10], [13, 14, 15, 0, 0], [0, 16, 17, 18, 0],
                               [0, 0, 19, 20, 0], [9, 0, 0, 0, 8]]


def test_overlap_layers_brute_force_distance():
    """Section 2.1: Gamma_{i,l} is the set of nodes at graph distance exactly
    l from I_i; checked against all-pairs shortest paths on a small RCB
    partition of an anisotropic pattern."""
    A, part = _small_hc(12, seed=5)
    G = schwarz.sym_pattern(A)
    dist = sp.csgraph.shortest_path(G, unweighted=True)
    for i in range(int(part.max()) + 1):
        s = schwarz.overlap(A, part, i, 3)
        d = dist[part == i].min(axis=0)
        start = s.n_interior
        for l, size in enumerate(s.layer_sizes, start=1):
            layer = s.idx[start:start + size]
            assert np.array_equal(np.sort(layer), np.flatnonzero(d == l))
            assert np.all(np.diff(layer) > 0)  # ascending within a layer
            start += size
        assert np.all(np.diff(s.idx[:s.n_interior]) > 0)


@pytest.mark.parametrize("delta", [1, 2, 3])
def test_overlap_layers_on_a_structurally_nonsymmetric_pattern(delta):
    """Section 2.1 grows the overlap on graph(A + A^T). On a matrix whose
    pattern is not symmetric (one-way upwind coupling in x), the layers must
    follow the edges of A and of A^T: checked against breadth-first
    distances on the boolean pattern (A != 0) | (A != 0)^T formed here, and
    shown to differ from the layers that A's own rows (or A^T's) would give,
    so that a search on one of the two patterns fails this test."""
    A = one_way_convection_2d(12, np.random.default_rng(7))
    part = box_partition_2d(12, 12, 3, 3)
    P = (A != 0).astype(np.int8)
    assert (P != P.T).nnz > 0
    U = ((P + P.T) > 0).astype(np.int8)
    d_sym = sp.csgraph.shortest_path(U, unweighted=True)
    d_row = sp.csgraph.shortest_path(P, unweighted=True, directed=True)
    d_col = sp.csgraph.shortest_path(P.T.tocsr(), unweighted=True, directed=True)
    differs_row = differs_col = False
    for i in range(int(part.max()) + 1):
        s = schwarz.overlap(A, part, i, delta)
        d = d_sym[part == i].min(axis=0)
        start = s.n_interior
        for l, size in enumerate(s.layer_sizes, start=1):
            layer = s.idx[start:start + size]
            assert np.array_equal(layer, np.flatnonzero(d == l))
            start += size
        assert np.array_equal(np.sort(s.idx), np.flatnonzero(d <= delta))
        differs_row |= not np.array_equal(np.sort(s.idx), np.flatnonzero(d_row[part == i].min(axis=0) <= delta))
        differs_col |= not np.array_equal(np.sort(s.idx), np.flatnonzero(d_col[part == i].min(axis=0) <= delta))
    assert differs_row and differs_col


# ----------------------------------------------------------------------------
# P2: partition of unity (Section 2.1)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("delta", [1, 2, 3])
def test_partition_of_unity(delta):
    A, part = _small_hc(16)
    n = A.shape[0]
    S = sp.csr_matrix((n, n))
    for i in range(int(part.max()) + 1):
        s = schwarz.overlap(A, part, i, delta)
        R = schwarz.restriction(s, n)
        S = S + R.T @ sp.diags(s.D()) @ R
    assert np.array_equal(S.toarray(), np.eye(n))


# ----------------------------------------------------------------------------
# P4: harmonic projection and SPSD splitting (Sections 3.1-3.2)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("delta", [1, 2, 3])
def test_harmonic_projection_identities(delta):
    A, part = _small_hc(16)
    for i in range(int(part.max()) + 1):
        s = schwarz.overlap(A, part, i, delta)
        Aii = schwarz.local_matrix(A, s)
        Pi = schwarz.harmonic_operator(Aii, s)
        Ad = Aii.toarray()
        scale = np.abs(Ad).max()
        # Lemma projection: Pi^2 = Pi and (I - Pi)^T A_ii Pi = 0
        assert np.abs(Pi @ Pi - Pi).max() <= 1e-10 * max(1.0, np.abs(Pi).max())
        Q = np.eye(s.size) - Pi
        assert np.abs(Q.T @ Ad @ Pi).max() <= 1e-10 * scale * max(1.0, np.abs(Pi).max())
        # dense-inverse route for Pi agrees
        _, Pi_dense, _ = _dense_pi_d(A, s)
        assert np.allclose(Pi, Pi_dense, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("delta", [1, 2])
def test_spsd_splitting(delta):
    """Lemma spsd_splitting: tilde A_i and A - tilde A_i are SPSD; for
    delta >= 2 the block formula eq. LSPSD equals (I-Pi)^T A_ii (I-Pi)
    (eq. local_problem_local_spsd_splitting)."""
    A, part = _small_hc(14, seed=7)
    n = A.shape[0]
    Ad = A.toarray()
    for i in range(int(part.max()) + 1):
        s = schwarz.overlap(A, part, i, delta)
        T = theory.spsd_splitting_projection(A, s)
        scale = np.abs(Ad).max()
        assert np.linalg.eigvalsh(0.5 * (T + T.T)).min() >= -1e-9 * scale
        full = np.zeros((n, n))
        full[np.ix_(s.idx, s.idx)] = T
        assert np.linalg.eigvalsh(Ad - 0.5 * (full + full.T)).min() >= -1e-9 * scale
        if delta >= 2:
            Tb = theory.spsd_splitting_block(A, s)
            assert np.allclose(T, Tb, rtol=1e-9, atol=1e-9 * scale)


# ----------------------------------------------------------------------------
# P5, P7: GEVP1 spectrum (Theorem after eq. uppergevp)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("delta", [1, 2])
def test_gevp1_spectrum_structure(delta):
    A = poisson_2d(16)
    part = box_partition_2d(16, 16, 2, 2)
    for i in range(4):
        s = schwarz.overlap(A, part, i, delta)
        Aii = schwarz.local_matrix(A, s)
        Ad = Aii.toarray()
        D = s.D()
        lam = sla.eigh(D[:, None] * Ad * D[None, :], Ad, eigvals_only=True)
        nI = s.n_interior
        n_gamma_all = s.size - nI
        A_GI = Ad[nI:, :nI]
        n_ones = nI - np.linalg.matrix_rank(A_GI)
        assert np.sum(np.abs(lam) < 1e-9) == n_gamma_all
        assert np.sum(np.abs(lam - 1) < 1e-9) == n_ones
        assert np.sum(lam > 1 + 1e-9) == nI - n_ones
        # the oracle's selection returns exactly the eigenvalues > 1
        vals, vecs = schwarz.gevp1(Aii, s, s.size, nu=1.0 + 1e-9)
        assert np.allclose(np.sort(vals), np.sort(lam[lam > 1 + 1e-9]), rtol=1e-9)
        assert np.allclose(vecs.T @ Ad @ vecs, np.eye(vals.size), atol=1e-8)


def test_delta1_gevp1_equals_one_plus_gevp2():
    """For delta = 1, GEVP1's eigenvalues above one are 1 + the nonzero
    eigenvalues of eq. gevpsvd (derived from the two pencils: for delta = 1
    Omega' = I_i so Pi_i^T D A D Pi_i and D A D differ by the harmonic
    correction on Gamma)."""
    A = poisson_2d(12)
    part = box_partition_2d(12, 12, 2, 2)
    s = schwarz.overlap(A, part, 0, 1)
    Aii = schwarz.local_matrix(A, s)
    l2, _ = schwarz.gevp2(Aii, s, s.size)
    l1, _ = schwarz.gevp1(Aii, s, s.size, nu=1.0 + 1e-9)
    assert l1.size == l2.size
    assert np.allclose(np.sort(l1), np.sort(1.0 + l2), rtol=1e-10)


# ----------------------------------------------------------------------------
# P6: GEVP2 (Proposition gevpsvd)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("delta", [1, 2])
def test_gevp2_against_dense_operator(delta):
    A, part = _small_hc(16)
    for i in range(int(part.max()) + 1):
        s = schwarz.overlap(A, part, i, delta)
        Aii = schwarz.local_matrix(A, s)
        DPi, Pi, Ad = _dense_pi_d(A, s)
        lhs = DPi.T @ Ad @ DPi
        ref = sla.eigh(0.5 * (lhs + lhs.T), Ad, eigvals_only=True)[::-1]
        # rank <= #Gamma_{i,delta}
        assert np.sum(ref > 1e-10 * ref[0]) <= s.n_gamma
        vals, W = schwarz.gevp2(Aii, s, 6)
        assert np.allclose(vals, ref[:vals.size], rtol=1e-9)
        assert np.allclose(W.T @ Ad @ W, np.eye(vals.size), atol=1e-8)
        # eigen-residual of the pencil
        res = lhs @ W - Ad @ W * vals[None, :]
        assert np.abs(res).max() <= 1e-8 * np.abs(Ad).max()
        # ARPACK route agrees with the dense route
        va, Wa = schwarz.gevp2(Aii, s, 6, dense=False)
        assert np.allclose(va, vals, rtol=1e-8)


def test_gevp2_splitting_identities():
    """eq. svdsplitting, eq. gevpsplitting1 and eq. gevpsplitting2 with
    tau^2 set between two kept eigenvalues."""
    A, part = _small_hc(16)
    s = schwarz.overlap(A, part, 1, 2)
    Aii = schwarz.local_matrix(A, s)
    DPi, Pi, Ad = _dense_pi_d(A, s)
    lhs = DPi.T @ Ad @ DPi
    lam, W = sla.eigh(0.5 * (lhs + lhs.T), Ad)
    lam, W = lam[::-1], W[:, ::-1]
    tau2 = 0.5 * (lam[3] + lam[4])
    vals, W1 = schwarz.gevp2(Aii, s, s.size, tau2=tau2)
    assert vals.size == 4
    W2 = W[:, 4:]
    Xi1 = DPi @ W1 @ W1.T @ Ad
    Xi2 = DPi @ W2 @ W2.T @ Ad
    assert np.allclose(Xi1 + Xi2, DPi, atol=1e-8 * max(1, np.abs(DPi).max()))
    assert np.abs(Xi2.T @ Ad @ Xi1).max() <= 1e-8 * np.abs(Ad).max()
    # v^T Xi2^T A Xi2 v <= tau^2 v^T A v  <=> lambda_max(Xi2^T A Xi2, A) <= tau^2
    top = sla.eigh(0.5 * (Xi2.T @ Ad @ Xi2 + (Xi2.T @ Ad @ Xi2).T), Ad, eigvals_only=True)[-1]
    assert top <= tau2 * (1 + 1e-8)


def test_gevp2_all_kept_span_is_range_of_DPi():
    """When every nonzero pair is kept, span(D_i Pi_i W^(1)) = range(D_i Pi_i)
    = span{D_i E e_j : j in Gamma_{i,delta}} (eq. coarse_space vs
    eq. coarse_space_2)."""
    A, part = _small_hc(16)
    s = schwarz.overlap(A, part, 2, 2)
    Aii = schwarz.local_matrix(A, s)
    DPi, _, _ = _dense_pi_d(A, s)
    Zi, eig, _ = schwarz.coarse_block(Aii, s, s.size, 0, True)
    B = DPi[:s.n_interior, s.n_prime:]
    U, sv, _ = np.linalg.svd(B, full_matrices=False)
    U = U[:, sv > 1e-10 * sv[0]]
    assert Zi.shape[1] == U.shape[1]
    # principal angles: both orthonormal, so singular values of U^T Zi are 1
    assert np.allclose(np.linalg.svd(U.T @ Zi, compute_uv=False), 1.0, atol=1e-8)


# ----------------------------------------------------------------------------
# P15: nonsymmetric variant (Section 6)
# ----------------------------------------------------------------------------

def test_svd_variant_against_dense_svd():
    rng = np.random.default_rng(2)
    A, _ = convdiff_2d(16, rng)
    part = box_partition_2d(16, 16, 2, 2)
    for i in range(4):
        s = schwarz.overlap(A, part, i, 2)
        Aii = schwarz.local_matrix(A, s)
        DPi, _, _ = _dense_pi_d(A, s)
        U, sv, _ = np.linalg.svd(DPi)
        sig, Ul = schwarz.svd_variant(Aii, s, 5)
        assert np.allclose(sig, sv[:5], rtol=1e-9)
        # same dominant left singular subspace (gaps are generic here)
        assert np.allclose(np.linalg.svd(U[:, :5].T @ Ul, compute_uv=False), 1.0, atol=1e-7)


# ----------------------------------------------------------------------------
# P8-P12: the two-level operator (eq. onelevelasm, Remark in Section 4.3)
# ----------------------------------------------------------------------------

def test_single_subdomain_is_exact_inverse():
    """N = 1: Gamma is empty, so no coarse space, and M^{-1} = A^{-1};
    PCG converges in one iteration."""
    A, _ = _small_hc(16)
    part = np.zeros(A.shape[0], dtype=np.int32)
    h = oracle.setup(A, part, 1, 8)
    assert h.n_coarse == 0
    b = np.random.default_rng(0).standard_normal(A.shape[0])
    assert np.allclose(oracle.apply(h, b), np.linalg.solve(A.toarray(), b), rtol=1e-10, atol=1e-12)
    x, it, rr = oracle.solve(h, b)
    assert it == 1 and rr <= 1e-10


def test_single_subdomain_general_fgmres_one_step():
    rng = np.random.default_rng(4)
    A, _ = convdiff_2d(12, rng)
    part = np.zeros(A.shape[0], dtype=np.int32)
    h = oracle.setup(A, part, 2, 4, spd=False)
    b = rng.standard_normal(A.shape[0])
    x, it, rr = oracle.solve(h, b)
    assert it == 1 and rr <= 1e-10


def test_nev0_is_one_level_asm():
    """nev = 0 leaves the one-level additive Schwarz operator of
    eq. onelevelasm, here compared with dense inverses of the blocks."""
    A, part = _small_hc(16)
    h = oracle.setup(A, part, 2, 0)
    M = schwarz.one_level_matrix(h)
    r = np.random.default_rng(1).standard_normal(A.shape[0])
    assert np.allclose(oracle.apply(h, r), M @ r, rtol=1e-10, atol=1e-12)


def test_two_level_against_dense_formula():
    """z = sum R_i^T A_ii^{-1} R_i r + Z (Z^T A Z)^{-1} Z^T r, with the
    coarse term from numpy's dense inverse."""
    A, part = _small_hc(16)
    h = oracle.setup(A, part, 2, 4)
    M = schwarz.one_level_matrix(h)
    Z = h.Z
    M = M + Z @ np.linalg.inv(Z.T @ A.toarray() @ Z) @ Z.T
    r = np.random.default_rng(1).standard_normal(A.shape[0])
    assert np.allclose(oracle.apply(h, r), M @ r, rtol=1e-9, atol=1e-12)


def test_apply_symmetric():
    A, part = _small_hc(16)
    h = oracle.setup(A, part, 2, 4)
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal((2, A.shape[0]))
    a, b = x @ oracle.apply(h, y), y @ oracle.apply(h, x)
    assert abs(a - b) <= 1e-13 * max(abs(a), 1.0) * 10


def test_basis_freedom():
    """Z -> Z G (G invertible) leaves Z (Z^T A Z)^{-1} Z^T unchanged."""
    A, part = _small_hc(16)
    h = oracle.setup(A, part, 2, 4)
    G = np.random.default_rng(0).standard_normal((h.n_coarse, h.n_coarse)) + 5 * np.eye(h.n_coarse)
    h2 = oracle.setup(A, part, 2, 4, Z=h.Z @ G)
    r = np.random.default_rng(1).standard_normal(A.shape[0])
    assert np.allclose(oracle.apply(h, r), oracle.apply(h2, r), rtol=1e-8, atol=1e-10)


def test_eigenvalue_decay_faster_with_more_layers():
    """Section 7 (Fig. 1): more overlap layers make the eq. gevpsvd
    eigenvalues decay faster, so a fixed tau keeps fewer vectors. 3D
    lognormal diffusion on 12^3 cells, 8 RCB parts, delta = 1, 3, 5."""
    from workloads import fv_diffusion_3d, lognormal_kappa_3d
    rng = np.random.default_rng(21)
    A = fv_diffusion_3d(lognormal_kappa_3d(12, rng)).tocsr()
    part = rcb_partition((12, 12, 12), 3, rng, (0.45, 0.55))
    med, counts = {}, {}
    for delta in (1, 3, 5):
        spec = []
        for i in range(8):
            s = schwarz.overlap(A, part, i, delta)
            lam, _ = schwarz.gevp2(schwarz.local_matrix(A, s), s, 16, dense=True)
            spec.append(lam)
        med[delta] = np.median(np.array([l / l[0] for l in spec]), axis=0)
        counts[delta] = sum(int(np.sum(l / l[0] > 1e-2)) for l in spec)
    for j in (6, 10, 15):
        assert med[1][j] > med[3][j] > med[5][j]
    assert counts[1] > counts[3] > counts[5]


def test_weak_scaling_two_level_iterations_stay_flat():
    """Section 7 (Table diffusion-3d): under weak scaling of the constant-
    coefficient 3D Poisson problem (fixed unknowns per subdomain, N grows)
    the two-level PCG iteration count stays nearly flat while the one-level
    count keeps growing; the condition-number bound of the two-level method
    depends on N only through lambda_*. 250 unknowns per part, delta = 1,
    8 eq. gevpsvd vectors per subdomain, rtol 1e-10, N = 4, 16, 64."""
    from workloads import weak_scaling_poisson_3d
    two, one = {}, {}
    for N in (4, 16, 64):
        p = weak_scaling_poisson_3d(N, per_part=250)
        for nev, out in ((8, two), (0, one)):
            h = schwarz.setup(p.A, p.part, 1, nev)
            x, it, rr = schwarz.solve(h, p.b, 1e-10)
            assert rr <= 1e-10
            out[N] = it
    assert two[64] <= 1.35 * two[4]
    assert one[64] >= 1.6 * one[4]
    assert two[64] <= 0.75 * one[64]


def test_saddle_point_section6_basis():
    """Section 6 on a symmetric indefinite saddle-point matrix (the MAC
    lid-driven cavity, velocities numbered first, stabilized pressure
    block). The matrix has one positive eigenvalue per velocity and one
    negative per pressure unknown; N = 1 is exact (one FGMRES step); on
    48 x 48 cells in 16 boxes the RAS + deflated composition with 16
    Section 6 vectors per subdomain needs at most a third of one-level RAS's
    FGMRES(30) iterations at delta = 4, and more at delta = 2 (fewer layers,
    as Section 7 reports for its saddle-point runs' overlap trade-off)."""
    from workloads import stokes_cavity_2d
    K, part, b = stokes_cavity_2d(16, 2, 2)
    ev = np.linalg.eigvalsh(K.toarray())
    assert int((ev > 0).sum()) == 2 * 15 * 16 and int((ev < 0).sum()) == 16 * 16
    h = schwarz.setup(K, np.zeros(K.shape[0], dtype=np.int32), 2, 4, spd=False)
    x, it, rr = schwarz.solve(h, b, 1e-8, composition="ras_deflated")
    assert it == 1 and rr <= 1e-10
    K, part, b = stokes_cavity_2d(48, 4, 4)
    its = {}
    for delta, nev in ((4, 16), (4, 0), (2, 16)):
        h = schwarz.setup(K, part, delta, nev, spd=False)
        x, it, rr = schwarz.solve(h, b, 1e-8, composition="ras_deflated")
        assert rr <= 1e-8
        its[delta, nev] = it
    assert 3 * its[4, 16] <= its[4, 0]
    assert its[2, 16] > its[4, 16]


# ----------------------------------------------------------------------------
# RAS (eq. onelevelras) and the deflated coarse correction of Section 7.2
# ----------------------------------------------------------------------------

def _parallel_schwarz_step(A, subs, b, x):
    """One step of the parallel Schwarz method, written from its own
    definition: subdomain i solves its Dirichlet problem on Omega_i with
    the current iterate as data outside Omega_i, and the new iterate takes
    each subdomain's values on its own I_i. Dense numpy solves."""
    Ad = A.toarray()
    n = Ad.shape[0]
    xn = np.full(n, np.nan)
    for s in subs:
        out = np.ones(n, dtype=bool)
        out[s.idx] = False
        u = np.linalg.solve(Ad[np.ix_(s.idx, s.idx)], b[s.idx] - Ad[np.ix_(s.idx, out)] @ x[out])
        xn[s.idx[: s.n_interior]] = u[: s.n_interior]
    return xn


@pytest.mark.parametrize("delta", [1, 2])
def test_ras_step_is_parallel_schwarz_step(delta):
    """x + M_RAS^{-1}(b - A x) equals one parallel Schwarz step from x
    when D_i is the 0/1 partition of unity (Efstathiou and Gander, 2003);
    the additive weighting of eq. onelevelasm does not."""
    rng = np.random.default_rng(8)
    A, part = _small_hc(16)
    h = oracle.setup(A, part, delta, 0)
    b, x = rng.standard_normal((2, A.shape[0]))
    want = _parallel_schwarz_step(A, h.subs, b, x)
    got = x + schwarz.one_level(h, b - A @ x, restricted=True)
    assert np.allclose(got, want, rtol=1e-10, atol=1e-12)
    asm = x + schwarz.one_level(h, b - A @ x)
    assert not np.allclose(asm, want, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("spd", [True, False])
def test_ras_deflated_is_exact_on_the_coarse_space(spd):
    """M^{-1} = Q + M_RAS^{-1}(I - A Q) gives M^{-1} A Z = Z: the coarse
    residual is removed exactly before the one-level part sees it. The
    additive composition does not have this property."""
    rng = np.random.default_rng(9)
    if spd:
        A, part = _small_hc(16)
    else:
        A, _ = convdiff_2d(16, rng)
        part = box_partition_2d(16, 16, 2, 2)
    h = oracle.setup(A, part, 2, 4, spd=spd)
    assert h.n_coarse > 0
    AZ = A @ h.Z
    got = np.column_stack([oracle.apply(h, AZ[:, j], composition="ras_deflated") for j in range(h.n_coarse)])
    assert np.allclose(got, h.Z, rtol=1e-9, atol=1e-10)
    add = np.column_stack([oracle.apply(h, AZ[:, j]) for j in range(h.n_coarse)])
    assert not np.allclose(add, h.Z, rtol=1e-6, atol=1e-6)
    # without coarse vectors the composition is plain RAS
    h0 = oracle.setup(A, part, 2, 0, spd=spd)
    r = rng.standard_normal(A.shape[0])
    assert np.allclose(oracle.apply(h0, r, composition="ras_deflated"),
                       _parallel_schwarz_step(A, h0.subs, r, np.zeros_like(r)), rtol=1e-10, atol=1e-12)


def test_ras_deflated_single_subdomain_and_iterations():
    """N = 1: D_1 = I, no coarse space, M^{-1} = A^{-1} and FGMRES stops
    after one step. On a 32 x 32 convection-diffusion problem with 16 boxes
    (delta = 2, nev = 16) RAS with the deflated correction needs fewer
    FGMRES iterations than the additive composition (Section 7.2 uses it
    for that reason)."""
    rng = np.random.default_rng(4)
    A, _ = convdiff_2d(12, rng)
    part = np.zeros(A.shape[0], dtype=np.int32)
    h = oracle.setup(A, part, 2, 4, spd=False)
    b = rng.standard_normal(A.shape[0])
    assert np.allclose(oracle.apply(h, b, composition="ras_deflated"), spla.spsolve(A.tocsc(), b),
                       rtol=1e-10, atol=1e-12)
    _, it, rr = oracle.solve(h, b, composition="ras_deflated")
    assert it == 1 and rr <= 1e-10
    A, _ = convdiff_2d(32, np.random.default_rng(5))
    part = box_partition_2d(32, 32, 4, 4)
    h = oracle.setup(A, part, 2, 16, spd=False)
    b = np.random.default_rng(6).standard_normal(A.shape[0])
    _, it_add, rr_add = oracle.solve(h, b)
    _, it_ras, rr_ras = oracle.solve(h, b, composition="ras_deflated")
    assert rr_add <= 1e-8 and rr_ras <= 1e-8
    assert it_ras < it_add


def test_relabeling_covariance():
    """A global relabeling P (which changes the ascending order inside every
    layer) gives M'^{-1} = P M^{-1} P^T: the method is independent of the
    within-layer order (Section 2.1 leaves it free)."""
    A, part = _small_hc(14, seed=11)
    n = A.shape[0]
    perm = np.random.default_rng(5).permutation(n)  # new index k holds old perm[k]
    P = sp.csr_matrix((np.ones(n), (np.arange(n), perm)), shape=(n, n))
    A2 = (P @ A @ P.T).tocsr()
    A2.sort_indices()
    part2 = part[perm]
    h1 = oracle.setup(A, part, 2, 3)
    h2 = oracle.setup(A2, part2, 2, 3)
    r = np.random.default_rng(2).standard_normal(n)
    assert np.allclose(P @ oracle.apply(h1, r), oracle.apply(h2, P @ r), rtol=1e-8, atol=1e-10)


# ----------------------------------------------------------------------------
# P13: spectral bounds (Section 4, Theorems upper_bound_1 and upper_bound_2)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("delta", [1, 2])
def test_condition_number_bounds(delta):
    nx = 16
    A = poisson_2d(nx)
    part = box_partition_2d(nx, nx, 2, 2)
    n = A.shape[0]
    nev = 3
    h = oracle.setup(A, part, delta, nev)
    kc = theory.overlap_colors(h.subs, n)
    Minv = schwarz.dense_preconditioner(h)
    lam = theory.preconditioned_spectrum(h, Minv)
    # continuity of the interpolation operator: lambda_max <= k_c + 1
    assert lam[-1] <= kc + 1 + 1e-9
    # Theorem upper_bound_2 with tau^2 = largest discarded GEVP2 eigenvalue
    # and nu = largest GEVP1 eigenvalue (no GEVP1 vector kept)
    tau2, nu = 0.0, 1.0
    for s in h.subs:
        Aii = schwarz.local_matrix(A, s)
        l2, _ = schwarz.gevp2(Aii, s, s.size)
        if l2.size > nev:
            tau2 = max(tau2, l2[nev])
        l1 = sla.eigh(np.diag(s.D()) @ Aii.toarray() @ np.diag(s.D()), Aii.toarray(),
                      eigvals_only=True)
        nu = max(nu, l1[-1])
    lstar = theory.lambda_star(A, h.subs)
    kappa = lam[-1] / lam[0]
    assert kappa <= theory.bound_truncated(kc, nu, np.sqrt(tau2), lstar)


def test_all_kept_bound_and_unit_lower_eigenvalue():
    """Coarse space eq. coarse_space (every harmonic column kept) satisfies
    Theorem upper_bound_1, with nu = the largest GEVP1 eigenvalue when no
    GEVP1 vector is kept."""
    nx = 12
    A = poisson_2d(nx)
    part = box_partition_2d(nx, nx, 2, 2)
    n = A.shape[0]
    subs = [schwarz.overlap(A, part, i, 1) for i in range(4)]
    nu = 1.0
    for s in subs:
        Ad = schwarz.local_matrix(A, s).toarray()
        nu = max(nu, sla.eigh(np.diag(s.D()) @ Ad @ np.diag(s.D()), Ad, eigvals_only=True)[-1])
    Z = theory.coarse_space_v1(A, subs, nu + 1.0)  # no GEVP1 vector above nu + 1
    h = oracle.setup(A, part, 1, 0, Z=Z)
    kc = theory.overlap_colors(h.subs, n)
    lam = theory.preconditioned_spectrum(h, schwarz.dense_preconditioner(h))
    assert lam[-1] / lam[0] <= theory.bound_all_kept(kc, nu)
    assert lam[0] >= 1.0 - 1e-9


# ----------------------------------------------------------------------------
# P14 and the Krylov solvers
# ----------------------------------------------------------------------------

def test_pcg_iterates_minimize_energy_error():
    """k-th PCG iterate minimizes the A-norm error over
    M^{-1}-preconditioned Krylov space K_k(M^{-1}A, M^{-1}b) (x0 = 0)."""
    A, part = _small_hc(10)
    h = oracle.setup(A, part, 1, 2)
    Ad = A.toarray()
    M = schwarz.dense_preconditioner(h)
    b = np.random.default_rng(7).standard_normal(A.shape[0])
    xs = np.linalg.solve(Ad, b)
    for k in (1, 2, 3, 5):
        x, it, _ = krylov.pcg(lambda v: Ad @ v, lambda v: M @ v, b, tol=0.0, maxit=k)
        K = [M @ b]
        for _ in range(k - 1):
            K.append(M @ (Ad @ K[-1]))
        K = np.linalg.qr(np.column_stack(K))[0]
        y = np.linalg.solve(K.T @ Ad @ K, K.T @ b)
        assert np.allclose(x, K @ y, rtol=1e-7, atol=1e-9 * np.abs(xs).max())


def test_fgmres_minimizes_residual_with_fixed_preconditioner():
    rng = np.random.default_rng(8)
    A, _ = convdiff_2d(10, rng)
    Ad = A.toarray()
    part = box_partition_2d(10, 10, 2, 2)
    h = oracle.setup(A, part, 1, 2, spd=False)
    M = schwarz.dense_preconditioner(h)
    b = rng.standard_normal(A.shape[0])
    for k in (1, 3, 6):
        x, it, _ = krylov.fgmres(lambda v: Ad @ v, lambda v: M @ v, b, tol=0.0, restart=30, maxit=k)
        K = [b]
        for _ in range(k - 1):
            K.append(Ad @ (M @ K[-1]))
        K = np.linalg.qr(np.column_stack(K))[0]
        y, *_ = np.linalg.lstsq(Ad @ M @ K, b, rcond=None)
        best = np.linalg.norm(b - Ad @ M @ K @ y)
        assert abs(np.linalg.norm(b - Ad @ x) - best) <= 1e-8 * np.linalg.norm(b)


def test_cg_iteration_bound():
    """eq. cgbound: ||e_k||_A <= 2 ((sqrt(kappa)-1)/(sqrt(kappa)+1))^k ||e_0||_A
    for the preconditioned iteration with kappa(M^{-1}A) from the dense
    spectrum."""
    A, part = _small_hc(14)
    h = oracle.setup(A, part, 2, 4)
    Ad = A.toarray()
    M = schwarz.dense_preconditioner(h)
    lam = theory.preconditioned_spectrum(h, M)
    kap = lam[-1] / lam[0]
    rho = (np.sqrt(kap) - 1) / (np.sqrt(kap) + 1)
    b = np.random.default_rng(9).standard_normal(A.shape[0])
    xs = np.linalg.solve(Ad, b)
    e0 = np.sqrt(xs @ Ad @ xs)
    for k in range(1, 12):
        x, _, _ = krylov.pcg(lambda v: Ad @ v, lambda v: M @ v, b, tol=0.0, maxit=k)
        e = x - xs
        assert np.sqrt(e @ Ad @ e) <= 2 * rho ** k * e0 * (1 + 1e-6) + 1e-12 * e0


def test_config1_iteration_counts():
    """Config-1 instance (64^2 Poisson, 4x4 boxes, delta 1): two-level nev 8
    needs fewer PCG iterations than one-level, which needs fewer than plain
    CG; each count is below the eq. cgbound estimate from its spectrum is not
    computed at this size, so only the ordering and convergence are fixed."""
    from workloads import make_config
    p = make_config(1)
    A = p.A
    _, it_cg, _ = krylov.pcg(lambda v: A @ v, lambda v: v, p.b, 1e-8, 2000)
    h1 = oracle.setup(A, p.part, 1, 0)
    _, it1, rr1 = oracle.solve(h1, p.b)
    h2 = oracle.setup(A, p.part, 1, 8, dense=False)
    _, it2, rr2 = oracle.solve(h2, p.b)
    assert it2 < it1 < it_cg
    assert rr1 <= 1e-8 and rr2 <= 1e-8
    assert h2.n_coarse == 128


def _unpivoted_lu(M):
    """Doolittle LU without pivoting (unit lower L, upper U), textbook loops."""
    n = M.shape[0]
    U = M.astype(np.float64).copy()
    L = np.eye(n)
    for k in range(n - 1):
        L[k + 1:, k] = U[k + 1:, k] / U[k, k]
        U[k + 1:, k:] -= np.outer(L[k + 1:, k], U[k, k:])
        U[k + 1:, k] = 0.0
    return L, U


@pytest.mark.parametrize("general", [False, True])
def test_factor_fill_stays_inside_the_envelope(general):
    """The GPU factorizations, substitutions and explicit inverses skip
    the blocks left of each row's first nonzero of A_ii (and, for LU, above
    each column's first nonzero of its upper part): they rely on Cholesky
    and unpivoted LU creating no fill outside that envelope. Checked on the
    oracle's local matrices (Section 2.3) of a high-contrast diffusion
    problem and of an upwind convection-diffusion problem, whose local
    matrices have a structurally nonsymmetric pattern: every entry outside
    the envelope is exactly zero, and inside it the factors are not all
    zero (the envelope is not trivially the whole triangle)."""
    rng = np.random.default_rng(11)
    if general:
        A = one_way_convection_2d(40, rng)
        part = box_partition_2d(40, 40, 2, 2)
    else:
        A = fv_diffusion_2d(high_contrast_kappa_2d(40, 40, rng))
        part = box_partition_2d(40, 40, 2, 2)
    G = schwarz.sym_pattern(A)
    for i in range(4):
        s = schwarz.overlap(A, part, i, 2, G)
        M = schwarz.local_matrix(A, s).toarray()
        n = M.shape[0]
        nz = M != 0
        row_first = np.array([np.flatnonzero(nz[a, :a + 1])[0] for a in range(n)])
        col_first = np.array([np.flatnonzero(nz[:b + 1, b])[0] for b in range(n)])
        if general:
            L, U = _unpivoted_lu(M)
        else:
            L = np.linalg.cholesky(M)
            U = L.T
        a, b = np.indices((n, n))
        outside_L = (b < row_first[:, None]) & (b <= a)
        outside_U = (a < col_first[None, :]) & (a <= b)
        assert outside_L.any() and outside_U.any()
        assert np.all(L[outside_L] == 0.0)
        assert np.all(U[outside_U] == 0.0)
        # fill does occur inside the envelope
        assert np.count_nonzero(L[~outside_L & (b <= a)]) > np.count_nonzero(np.tril(M))
