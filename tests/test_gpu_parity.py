"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Each test compares the library with the oracle on the same seeded inputs:
integer index sets bit for bit, local solves and the coarse operator to
1e-12 (FP64), eigenvalues to 1e-8 and spans by principal angles where the
spectral gap allows, the apply (with the library's own coarse basis imported
into the oracle) to 1e-10 in FP64 mode, and PCG iteration counts.
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from oracle import schwarz
from tests.gpu_helpers import principal_cosines, say, to_dev, torch_cuda
from workloads import (box_partition_2d, fv_diffusion_2d, high_contrast_kappa_2d, make_config, one_way_convection_2d,
                       poisson_2d, rcb_partition)

pytestmark = pytest.mark.gpu


def _pc(A, part, overlap, nev, **opts):
    import paper_2401_03915_amd as tls
    return tls.Preconditioner(A, part, overlap, nev, **opts)


def _hc_problem(nx, levels, seed):
    rng = np.random.default_rng(seed)
    kappa = high_contrast_kappa_2d(nx, nx, rng)
    A = fv_diffusion_2d(kappa)
    part = rcb_partition((nx, nx), levels, rng, (0.3, 0.7))
    return A, part


# ---------------------------------------------------------------------------
# integer stages: overlap layers (Section 2.1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("delta", [1, 2, 3])
def test_overlap_index_sets_exact(delta):
    A, part = _hc_problem(96, 3, seed=1)
    say("overlap index sets", delta)
    pc = _pc(A, part, delta, 0)
    ex = pc.export()
    N = int(part.max()) + 1
    for i in range(N):
        s = schwarz.overlap(A, part, i, delta)
        a, b = ex["sub_ptr"][i], ex["sub_ptr"][i + 1]
        assert np.array_equal(ex["sub_idx"][a:b], s.idx)
        lp = ex["layer_ptr"][i * (delta + 2):(i + 1) * (delta + 2)]
        sizes = np.diff(lp)
        assert sizes[0] == s.n_interior
        assert list(sizes[1:]) == s.layer_sizes
    pc.close()


def test_worked_example_on_gpu():
    """Index sets of the Section 2.1 example. They depend only on the
    pattern, so an SPD tridiagonal matrix with the example's pattern is used
    (the printed example matrix itself is not SPD)."""
    import scipy.sparse as sp
    from workloads import worked_example_7x7
    A7, part = worked_example_7x7()
    A = sp.diags([-np.ones(6), 4 * np.ones(7), -np.ones(6)], [-1, 0, 1]).tocsr()
    assert np.array_equal(A.toarray() != 0, A7.toarray() != 0)
    for delta, expect in ((1, [[1, 2, 3, 4], [4, 5, 6, 7, 3]]), (2, [[1, 2, 3, 4, 5], [4, 5, 6, 7, 3, 2]])):
        say("worked example", delta)
        pc = _pc(A, part, delta, 0, matrix_kind=0)
        ex = pc.export()
        got = [list(ex["sub_idx"][ex["sub_ptr"][i]:ex["sub_ptr"][i + 1]] + 1) for i in range(2)]
        assert got == expect
        pc.close()


@pytest.mark.parametrize("delta,precision,tol", [(1, 0, 1e-10), (2, 0, 1e-10), (3, 0, 1e-10), (2, 1, 1e-5)])
def test_structurally_nonsymmetric_pattern(delta, precision, tol):
    """graph(A + A^T) (Section 2.1) on a matrix whose pattern is not
    symmetric (one-way upwind coupling in x): the overlap lists and layer
    sizes equal the oracle's exactly, some of them hold unknowns reached only
    through A^T (so the transposed pattern changes Omega_i), and the apply of
    the Section 6 two-level method with the library's basis imported into
    the oracle matches it."""
    torch = torch_cuda()
    m = 48
    A = one_way_convection_2d(m, np.random.default_rng(7))
    part = box_partition_2d(m, m, 3, 3)
    say("nonsymmetric pattern", delta, precision)
    pc = _pc(A, part, delta, 4, matrix_kind=1, precision=precision)
    ex = pc.export(Z=True)
    through_t = False
    for i in range(9):
        s = schwarz.overlap(A, part, i, delta)
        a, b = ex["sub_ptr"][i], ex["sub_ptr"][i + 1]
        assert np.array_equal(ex["sub_idx"][a:b], s.idx)
        sizes = np.diff(ex["layer_ptr"][i * (delta + 2):(i + 1) * (delta + 2)])
        assert sizes[0] == s.n_interior and list(sizes[1:]) == s.layer_sizes
        # layer-1 nodes that no row of I_i references: reached through A^T only
        interior = s.idx[:s.n_interior]
        by_rows = np.unique(A[interior].indices)
        layer1 = s.idx[s.n_interior:s.n_interior + s.layer_sizes[0]]
        only_t = np.setdiff1d(layer1, by_rows)
        if only_t.size:
            # each such node's own row references I_i: an edge of A^T
            assert np.all(A[only_t][:, interior].getnnz(axis=1) > 0)
            through_t = True
    assert through_t
    h = oracle.setup(A, part, delta, 4, spd=False, Z=ex["Z"])
    rng = np.random.default_rng(16)
    worst = 0.0
    for _ in range(5):
        r = rng.standard_normal(A.shape[0])
        z = pc.apply(to_dev(r))
        torch.cuda.synchronize()
        z_ref = oracle.apply(h, r)
        worst = max(worst, np.linalg.norm(z.cpu().numpy() - z_ref) / np.linalg.norm(z_ref))
    say("  worst apply error", worst)
    assert worst <= tol
    pc.close()


# ---------------------------------------------------------------------------
# local factorization and solves (Section 2.3)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision,refine,rows", [(0, 0, 1), (1, 0, 1), (1, 1, 1), (1, 2, 1), (0, 0, 2), (1, 0, 2),
                                                   (1, 1, 2), (1, 0, 3), (1, 0, 4), (1, 1, 4)])
def test_local_solves(precision, refine, rows):
    """Local solves by substitution against the oracle's sparse LU on
    high-contrast subdomains of a few thousand rows (many tiles and a ragged
    tail), with tasks of one to four block rows (solve_rows; a row count
    that the task size does not divide leaves a shorter task at the end). FP64: 1e-11. FP32: the forward error
    of a backward-stable solve,
    bounded by e_32 = 20 cond(A_ii) u_32. With s local_refine steps (FP64
    residual from the sparse A_ii, FP32 correction) the error contracts by
    at most e_32 per step down to the FP64 floor: the bound is
    e_32^(s+1) + 20 cond(A_ii) u_64, and at most the FP32-mode bar 1e-5."""
    A, part = _hc_problem(128, 2, seed=2)
    say("local solves", precision, refine, rows)
    pc = _pc(A, part, 2, 0, precision=precision, local_refine=refine, solve_rows=rows)
    assert pc.info()["local_refine"] == refine and pc.info()["solve_rows"] == rows
    rng = np.random.default_rng(0)
    for i in range(int(part.max()) + 1):
        s = schwarz.overlap(A, part, i, 2)
        Aii = schwarz.local_matrix(A, s).tocsc()
        b = rng.standard_normal(s.size)
        x_ref = spla.spsolve(Aii, b)
        x = pc.local_solve(i, b)
        err = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
        if precision == 0:
            tol = 1e-11
        else:
            lmax = spla.eigsh(Aii, 1, which="LA", return_eigenvectors=False)[0]
            lmin = spla.eigsh(Aii, 1, sigma=0.0, which="LM", return_eigenvectors=False)[0]
            e32 = 20 * (lmax / lmin) * 2.0 ** -24
            tol = e32 if refine == 0 else min(1e-5, e32 ** (refine + 1) + 20 * (lmax / lmin) * 2.0 ** -53)
        say("  subdomain", i, "m", s.size, "err", err, "bound", tol)
        assert err <= tol
    pc.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_local_inverse_solves(precision):
    """Option local_inverse: each local solve is one product with the
    explicit A_ii^{-1} (formed as L^{-T} W, W = L^{-1}, by a block back
    substitution inside the tile profile, as here, or as W^T W when the
    profile is wide). Four subdomains of a few thousand
    rows (block rows of up to 70 tiles, so several chunks per row and a
    ragged last tile), against the oracle's sparse LU. The explicit inverse
    carries a forward error of order cond(A_ii) u, as the substitutions do:
    the bound is 20 cond(A_ii) u, with cond from ARPACK and u the unit
    roundoff of the local precision."""
    A, part = _hc_problem(128, 2, seed=2)
    say("local inverse solves", precision)
    pc = _pc(A, part, 2, 0, precision=precision, local_inverse=1)
    assert pc.info()["local_inverse"] == 1
    u = 2.0 ** -53 if precision == 0 else 2.0 ** -24
    rng = np.random.default_rng(0)
    for i in range(int(part.max()) + 1):
        s = schwarz.overlap(A, part, i, 2)
        Aii = schwarz.local_matrix(A, s).tocsc()
        lmax = spla.eigsh(Aii, 1, which="LA", return_eigenvectors=False)[0]
        lmin = spla.eigsh(Aii, 1, sigma=0.0, which="LM", return_eigenvectors=False)[0]
        cond = lmax / lmin
        b = rng.standard_normal(s.size)
        x_ref = spla.spsolve(Aii, b)
        x = pc.local_solve(i, b)
        err = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
        say("  subdomain", i, "m", s.size, "cond %.1e" % cond, "err", err)
        assert err <= 20 * cond * u
    pc.close()


def _tile_profile_counts(A, part, delta, general):
    """Tiles one forward and one backward substitution read when each local
    factor skips the tiles left of its rows' first nonzero (and, for LU,
    above its columns' first nonzero), from the oracle's Omega_i and A_ii,
    and the lower tiles of all factors."""
    G = schwarz.sym_pattern(A)
    fwd = bwd = lower = 0
    for i in range(int(part.max()) + 1):
        s = schwarz.overlap(A, part, i, delta, G)
        C = schwarz.local_matrix(A, s).tocoo()
        nt = -(-s.size // 64)
        fr, fc = np.arange(nt), np.arange(nt)
        lo, up = C.col <= C.row, C.row <= C.col
        np.minimum.at(fr, C.row[lo] // 64, C.col[lo] // 64)
        np.minimum.at(fc, C.col[up] // 64, C.row[up] // 64)
        r = np.arange(nt)
        fwd += int(np.sum(r - fr + 1))
        bwd += int(np.sum(r - (fc if general else fr) + 1))
        lower += nt * (nt + 1) // 2
    return fwd, bwd, lower


@pytest.mark.parametrize("general", [False, True])
def test_tile_profile_and_local_inverse_choice(general):
    """The tile profiles the factorizations and substitutions skip by
    (fill stays inside the envelope of A_ii, so the tiles left of each tile
    row's first nonzero, and for LU above each tile column's first nonzero,
    stay zero): the tile counts the library reports equal those of the
    oracle's local matrices; with local_inverse = 2 the explicit inverse is
    formed exactly when the two substitutions would read more tiles than the
    product (all lower tiles); both variants give the same apply (FP64, 1e-10 against
    the oracle with the library's basis)."""
    torch = torch_cuda()
    if general:
        A = one_way_convection_2d(96, np.random.default_rng(5))
        part = box_partition_2d(96, 96, 3, 3)
    else:
        A, part = _hc_problem(160, 4, seed=7)
    delta = 2
    fwd, bwd, lower = _tile_profile_counts(A, part, delta, general)
    say("tile profile", "general" if general else "spd", fwd, bwd, lower)
    kind = 1 if general else 0
    pc = _pc(A, part, delta, 4, matrix_kind=kind, local_inverse=0 if general else 2)
    inf = pc.info()
    assert (inf["solve_tiles_fwd"], inf["solve_tiles_bwd"], inf["lower_tiles"]) == (fwd, bwd, lower)
    assert fwd < lower  # the profile skips tiles here
    if general:
        pc.close()
        return
    assert inf["local_inverse"] == int(fwd + bwd > lower)
    other = _pc(A, part, delta, 4, local_inverse=1 - inf["local_inverse"])
    ex = pc.export()
    ref = oracle.schwarz.setup(A, part, delta, 0, spd=True, Z=pc.z_sparse(ex).toarray())
    rng = np.random.default_rng(3)
    for _ in range(2):
        r = rng.standard_normal(A.shape[0])
        want = oracle.schwarz.apply(ref, r)
        for q in (pc, other):
            z = q.apply(to_dev(r))
            torch.cuda.synchronize()
            assert np.linalg.norm(z.cpu().numpy() - want) <= 1e-10 * np.linalg.norm(want)
    pc.close()
    other.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-5)])
def test_local_inverse_apply_and_solve(precision, tol):
    """Option local_inverse on the 64 x 64 Poisson problem: the apply against
    the oracle with the library's own Z imported, PCG iterations equal to
    the oracle's (FP64), graph-captured and eager iterates identical (the
    product's reduction has a fixed order)."""
    torch = torch_cuda()
    p = make_config(1)
    say("local inverse apply", precision)
    pc = _pc(p.A, p.part, 1, 8, precision=precision, local_inverse=1, use_graph=1)
    ex = pc.export(Z=True)
    h = oracle.setup(p.A, p.part, 1, 8, Z=ex["Z"])
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(5):
        r = rng.standard_normal(p.A.shape[0])
        z = pc.apply(to_dev(r))
        torch.cuda.synchronize()
        z_ref = oracle.apply(h, r)
        worst = max(worst, np.linalg.norm(z.cpu().numpy() - z_ref) / np.linalg.norm(z_ref))
    say("  worst apply error", worst)
    assert worst <= tol
    x, it, rr, st = pc.solve(to_dev(p.b), 1e-8)
    x2, it2, _, _ = pc.solve(to_dev(p.b), 1e-8)
    torch.cuda.synchronize()
    pe = _pc(p.A, p.part, 1, 8, precision=precision, local_inverse=1, use_graph=0)
    xe, ite, _, _ = pe.solve(to_dev(p.b), 1e-8)
    torch.cuda.synchronize()
    assert st == 0 and rr <= 1e-8
    assert it == it2 == ite and torch.equal(x, x2) and torch.equal(x, xe)
    if precision == 0:
        _, it_ref, _ = oracle.solve(oracle.setup(p.A, p.part, 1, 8), p.b)
        say("  iterations", it, "oracle", it_ref)
        assert it == it_ref
    pc.close()
    pe.close()


# ---------------------------------------------------------------------------
# coarse space (eq. gevpsvd, eq. coarse_space_2) and A_0
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("delta", [1, 2])
def test_coarse_eigen_parity(delta):
    A = poisson_2d(48)
    part = box_partition_2d(48, 48, 3, 3)
    nev = 6
    say("eigen parity", delta)
    pc = _pc(A, part, delta, nev)
    ex = pc.export(Z=True, A0=True)
    zc = ex["zcol_ptr"]
    for i in range(9):
        s = schwarz.overlap(A, part, i, delta)
        Aii = schwarz.local_matrix(A, s)
        lam_all, W = schwarz.gevp2(Aii, s, s.size)
        k = zc[i + 1] - zc[i]
        assert k == min(nev, lam_all.size)
        lam_gpu = ex["eigvals"][zc[i]:zc[i + 1]]
        assert np.allclose(lam_gpu, lam_all[:k], rtol=1e-8, atol=1e-12)
        # span parity where the cut is not inside a cluster
        if lam_all.size > k and lam_all[k - 1] / lam_all[k] >= 1 + 1e-3:
            Zi, _, _ = schwarz.coarse_block(Aii, s, nev, 0, True)
            Zg = ex["Z"][s.idx[:s.n_interior]][:, zc[i]:zc[i + 1]]
            cos = principal_cosines(Zi, Zg)
            assert np.all(cos >= 1 - 1e-10), cos
    # A_0 = Z^T A Z with the library's own Z
    Zg = ex["Z"]
    A0_ref = Zg.T @ (A @ Zg)
    assert np.allclose(ex["A0"], A0_ref, rtol=1e-12, atol=1e-12 * np.abs(A0_ref).max())
    # orthonormal columns per subdomain
    assert np.allclose(Zg.T @ Zg, np.eye(Zg.shape[1]), atol=1e-12)
    pc.close()


@pytest.mark.parametrize("case", ["poisson_d1", "poisson_d2", "hc64_d2"])
def test_coarse_eigen_parity_fp32(case):
    """eq. gevpsvd in FP32 mode (FP32 factor, FP32 subspace iteration, FP64
    Rayleigh-Ritz) against the oracle's FP64 dense solve of the full pencil:
    relative eigenvalue error <= 1e-4 for every kept pair and largest
    principal angle <= 1e-3 wherever lambda_k / lambda_{k+1} >= 1 + 1e-3."""
    if case.startswith("poisson"):
        A = poisson_2d(48)
        part = box_partition_2d(48, 48, 3, 3)
        delta, nev = (1 if case.endswith("d1") else 2), 6
    else:
        A, part = _hc_problem(64, 3, seed=4)
        delta, nev = 2, 6
    say("eigen parity fp32", case)
    pc = _pc(A, part, delta, nev, precision=1)
    ex = pc.export(Z=True)
    zc = ex["zcol_ptr"]
    worst_l = worst_a = 0.0
    for i in range(int(part.max()) + 1):
        s = schwarz.overlap(A, part, i, delta)
        Aii = schwarz.local_matrix(A, s)
        lam_all, _ = schwarz.gevp2(Aii, s, s.size, dense=True)
        k = zc[i + 1] - zc[i]
        assert k == min(nev, lam_all.size)
        lam_gpu = ex["eigvals"][zc[i]:zc[i + 1]]
        worst_l = max(worst_l, np.max(np.abs(lam_gpu - lam_all[:k]) / lam_all[:k]))
        if lam_all.size > k and lam_all[k - 1] / lam_all[k] >= 1 + 1e-3:
            Zi, _, _ = schwarz.coarse_block(Aii, s, nev, 0, True, dense=True)
            Zg = ex["Z"][s.idx[:s.n_interior]][:, zc[i]:zc[i + 1]]
            cos = np.clip(principal_cosines(Zi, Zg), -1.0, 1.0)
            worst_a = max(worst_a, float(np.arccos(cos.min())))
    say("  worst relative eigenvalue error", worst_l, "worst angle", worst_a)
    assert worst_l <= 1e-4
    assert worst_a <= 1e-3
    pc.close()


def test_gevp1_eigen_parity():
    """eq. uppergevp vectors alone (nev = 0, nev1 > 0, delta = 2): the kept
    eigenvalues lambda > 1 against the oracle's dense solve of the full
    pencil, and the spans of D_i u where the gap allows."""
    A = poisson_2d(48)
    part = box_partition_2d(48, 48, 3, 3)
    nev1, delta = 6, 2
    say("gevp1 parity", delta)
    pc = _pc(A, part, delta, 0, nev1=nev1)
    ex = pc.export(Z=True)
    zc = ex["zcol_ptr"]
    assert np.all(ex["zsrc"] == 1)
    for i in range(9):
        s = schwarz.overlap(A, part, i, delta)
        Aii = schwarz.local_matrix(A, s)
        lam_all, U = schwarz.gevp1(Aii, s, s.size, nu=1.0, dense=True)
        lam_all = lam_all[lam_all > 1 + 1e-10]
        k = zc[i + 1] - zc[i]
        assert k == min(nev1, lam_all.size)
        lam_gpu = ex["eigvals"][zc[i]:zc[i + 1]]
        assert np.allclose(lam_gpu, lam_all[:k], rtol=1e-8, atol=1e-12), (lam_gpu, lam_all[:k])
        if lam_all.size > k and lam_all[k - 1] / lam_all[k] >= 1 + 1e-3:
            Zi, _, _ = schwarz.coarse_block(Aii, s, 0, nev1, True)
            Zg = ex["Z"][s.idx[:s.n_interior]][:, zc[i]:zc[i + 1]]
            cos = principal_cosines(Zi, Zg)
            assert np.all(cos >= 1 - 1e-10), cos
    pc.close()


def test_gevp1_delta1_is_one_plus_gevp2():
    """For delta = 1 the eq. uppergevp pairs above 1 are the eq. gevpsvd pairs
    with lambda_1 = 1 + lambda_2^2 and the same vectors (block algebra of the
    two pencils when Omega' = I_i)."""
    A, part = _hc_problem(64, 3, seed=5)
    N = int(part.max()) + 1
    say("gevp1 vs gevp2 delta 1")
    p2 = _pc(A, part, 1, 5)
    p1 = _pc(A, part, 1, 0, nev1=5)
    e2, e1 = p2.export(Z=True), p1.export(Z=True)
    assert np.array_equal(e2["zcol_ptr"], e1["zcol_ptr"])
    assert np.allclose(e1["eigvals"], 1.0 + e2["eigvals"], rtol=1e-9)
    zc = e2["zcol_ptr"]
    for i in range(N):
        lo, hi = zc[i], zc[i + 1]
        rows = np.flatnonzero(part == i)
        cos = principal_cosines(e2["Z"][rows][:, lo:hi], e1["Z"][rows][:, lo:hi])
        assert np.all(cos >= 1 - 1e-9), cos
    p1.close()
    p2.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-5)])
def test_both_eigenproblems_apply_parity(precision, tol):
    """Z_i = orth([D_i Pi_i W_i, D_i Z_i]) with nev = nev1 = 4 (eq. coarse_space_2):
    per-subdomain span against the oracle (FP64), then the apply with the
    library's basis imported into the oracle."""
    torch = torch_cuda()
    A = poisson_2d(48)
    part = box_partition_2d(48, 48, 3, 3)
    say("gevp1 + gevp2 apply", precision)
    pc = _pc(A, part, 2, 4, nev1=4, precision=precision)
    ex = pc.export(Z=True)
    zc = ex["zcol_ptr"]
    assert set(np.unique(ex["zsrc"])) == {0, 1}
    if precision == 0:
        for i in range(9):
            s = schwarz.overlap(A, part, i, 2)
            Aii = schwarz.local_matrix(A, s)
            lam2, _ = schwarz.gevp2(Aii, s, s.size)
            lam1, _ = schwarz.gevp1(Aii, s, s.size, nu=1.0, dense=True)
            lam1 = lam1[lam1 > 1 + 1e-10]
            gap_ok = (lam2.size <= 4 or lam2[3] / lam2[4] >= 1 + 1e-3) and \
                     (lam1.size <= 4 or lam1[3] / lam1[4] >= 1 + 1e-3)
            if gap_ok:
                Zi, _, _ = schwarz.coarse_block(Aii, s, 4, 4, True)
                Zg = ex["Z"][s.idx[:s.n_interior]][:, zc[i]:zc[i + 1]]
                assert Zg.shape[1] == Zi.shape[1]
                cos = principal_cosines(Zi, Zg)
                assert np.all(cos >= 1 - 1e-9), cos
    h = oracle.setup(A, part, 2, 4, nev1=4, Z=ex["Z"])
    rng = np.random.default_rng(12)
    worst = 0.0
    for _ in range(5):
        r = rng.standard_normal(A.shape[0])
        z = pc.apply(to_dev(r))
        torch.cuda.synchronize()
        z_ref = oracle.apply(h, r)
        worst = max(worst, np.linalg.norm(z.cpu().numpy() - z_ref) / np.linalg.norm(z_ref))
    say("  worst apply error", worst)
    assert worst <= tol
    pc.close()


# ---------------------------------------------------------------------------
# apply (Remark in Section 4.3: the operator M_2^{-1})
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-5)])
def test_apply_with_imported_basis(precision, tol):
    torch = torch_cuda()
    p = make_config(1)
    say("apply parity cfg1", precision)
    pc = _pc(p.A, p.part, 1, 8, precision=precision)
    ex = pc.export(Z=True)
    h = oracle.setup(p.A, p.part, 1, 8, Z=ex["Z"])
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(10):
        r = rng.standard_normal(p.A.shape[0])
        z = pc.apply(to_dev(r))
        torch.cuda.synchronize()
        z_ref = oracle.apply(h, r)
        worst = max(worst, np.linalg.norm(z.cpu().numpy() - z_ref) / np.linalg.norm(z_ref))
    say("  worst apply error", worst)
    assert worst <= tol
    pc.close()


@pytest.mark.parametrize("composition", [0, 1])
@pytest.mark.parametrize("refine,inv,scale", [(0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 0, 1), (2, 0, 0)])
def test_high_contrast_fp32_apply(refine, inv, scale, composition):
    """FP32 mode on high-contrast diffusion (kappa log-uniform in [1, 1e6]
    with 1e6 channels, 16 RCB parts, delta 2): the apply with the library's
    basis imported into the FP64 oracle. The FP32 local solves carry a
    forward error of about cond(A_ii) u_32, which on these subdomains puts
    the apply error at 1.0-1.3e-5 (bound 3e-5 without refinement); one
    local refinement step (FP64 residual from the sparse A_ii) brings it
    under the 1e-5 bound for FP32 mode, two under 1e-8."""
    torch = torch_cuda()
    A, part = _hc_problem(128, 4, seed=6)
    say("high-contrast fp32 apply", refine, inv, scale, composition)
    pc = _pc(A, part, 2, 8, precision=1, local_refine=refine, local_inverse=inv, jacobi_scale=scale,
             composition=composition)
    ex = pc.export(Z=True)
    h = oracle.setup(A, part, 2, 8, Z=ex["Z"])
    rng = np.random.default_rng(17)
    worst = 0.0
    for _ in range(5):
        r = rng.standard_normal(A.shape[0])
        z = pc.apply(to_dev(r))
        torch.cuda.synchronize()
        z_ref = oracle.apply(h, r, composition="ras_deflated" if composition else "additive")
        worst = max(worst, np.linalg.norm(z.cpu().numpy() - z_ref) / np.linalg.norm(z_ref))
    tol = {0: 3e-5, 1: 1e-5, 2: 1e-8}[refine]
    say("  worst apply error", worst, "bound", tol)
    assert worst <= tol
    pc.close()


def test_apply_one_level_and_symmetry():
    torch = torch_cuda()
    A, part = _hc_problem(64, 3, seed=4)
    say("one-level apply")
    pc = _pc(A, part, 2, 0)
    h = oracle.setup(A, part, 2, 0)
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal((2, A.shape[0]))
    zx = pc.apply(to_dev(x))
    zy = pc.apply(to_dev(y))
    torch.cuda.synchronize()
    zx, zy = zx.cpu().numpy(), zy.cpu().numpy()
    assert np.allclose(zx, oracle.apply(h, x), rtol=1e-10, atol=1e-12 * np.abs(zx).max())
    assert abs(y @ zx - x @ zy) <= 1e-12 * abs(y @ zx)
    pc.close()


# ---------------------------------------------------------------------------
# solve (PCG, Section 7.2)
# ---------------------------------------------------------------------------

def test_config1_solve_matches_oracle_iterations():
    torch = torch_cuda()
    p = make_config(1)
    say("cfg1 solve fp64")
    pc = _pc(p.A, p.part, 1, 8)
    x, it, rr, st = pc.solve(to_dev(p.b), 1e-8)
    torch.cuda.synchronize()
    h = oracle.setup(p.A, p.part, 1, 8)
    _, it_ref, _ = oracle.solve(h, p.b)
    say("  iterations", it, "oracle", it_ref, "relres", rr)
    assert st == 0 and rr <= 1e-8
    assert it == it_ref
    xs = spla.spsolve(p.A.tocsc(), p.b)
    assert np.linalg.norm(x.cpu().numpy() - xs) <= 1e-6 * np.linalg.norm(xs)
    pc.close()


def test_single_subdomain_one_iteration():
    torch = torch_cuda()
    A, _ = _hc_problem(40, 1, seed=5)
    part = np.zeros(A.shape[0], dtype=np.int32)
    b = np.random.default_rng(1).standard_normal(A.shape[0])
    say("N=1 solve")
    pc = _pc(A, part, 1, 8)
    assert pc.info()["n_coarse"] == 0
    x, it, rr, st = pc.solve(to_dev(b), 1e-8)
    torch.cuda.synchronize()
    assert it == 1 and rr <= 1e-10
    pc.close()


def test_graph_and_eager_iterates_identical():
    torch = torch_cuda()
    p = make_config(1)
    say("graph vs eager")
    pc1 = _pc(p.A, p.part, 1, 8, use_graph=0)
    pc2 = _pc(p.A, p.part, 1, 8, use_graph=1)
    x1, it1, rr1, _ = pc1.solve(to_dev(p.b), 1e-8)
    x2, it2, rr2, _ = pc2.solve(to_dev(p.b), 1e-8)
    # the graph is replayed: solve twice more with eager work in between
    x3, it3, _, _ = pc2.solve(to_dev(p.b), 1e-8)
    torch.cuda.synchronize()
    assert it1 == it2 == it3
    assert torch.equal(x1, x2) and torch.equal(x2, x3)
    pc1.close()
    pc2.close()


@pytest.mark.parametrize("refine", [0, 1])
def test_fp32_mode_converges(refine):
    """FP32 local factors, solves and eigensolver under the FP64 flexible
    PCG reach the 1e-8 true residual within 5% of the plain FP64 method's
    iterations (high-contrast diffusion, 16 parts, delta 2, nev 8)."""
    torch = torch_cuda()
    A, part = _hc_problem(128, 4, seed=6)
    b = np.random.default_rng(2).standard_normal(A.shape[0])
    say("fp32 solve", refine)
    pc = _pc(A, part, 2, 8, precision=1, local_refine=refine)
    x, it, rr, st = pc.solve(to_dev(b), 1e-8)
    torch.cuda.synchronize()
    pc64 = _pc(A, part, 2, 8, precision=0)
    _, it64, rr64, _ = pc64.solve(to_dev(b), 1e-8)
    say("  fp32 its", it, rr, "fp64 its", it64, rr64)
    assert st == 0 and rr <= 1e-8 and rr64 <= 1e-8
    assert abs(it - it64) <= max(1, int(0.05 * it64))
    pc.close()
    pc64.close()


# ---------------------------------------------------------------------------
# error paths (host-forced, every kernel exits normally)
# ---------------------------------------------------------------------------

def test_error_paths():
    import paper_2401_03915_amd as tls
    A = poisson_2d(16)
    part = box_partition_2d(16, 16, 2, 2)
    say("error paths")
    with pytest.raises(tls.TlsError) as e:
        _pc(A, part, 0, 4)
    assert e.value.status == 1
    bad = part.copy()
    bad[3] = 7  # out of range
    with pytest.raises(tls.TlsError) as e:
        _pc(A, bad, 1, 0)
    assert e.value.status == 1
    neg = -A  # negative definite: Cholesky pivots are negative
    with pytest.raises(tls.TlsError) as e:
        _pc(neg.tocsr(), part, 1, 0)
    assert e.value.status == 2
    with pytest.raises(tls.TlsError) as e:
        _pc(A, part, 1, 4, composition=2)
    assert e.value.status == 1
    with pytest.raises(tls.TlsError) as e:
        _pc(A, part, 1, 4, matrix_kind=1, local_inverse=1)
    assert e.value.status == 1
    import scipy.sparse as sp
    A = A.tocsr()
    # a non-finite value
    nan = A.copy()
    nan.data[5] = np.nan
    with pytest.raises(tls.TlsError) as e:
        _pc(nan, part, 1, 0)
    assert e.value.status == 1 and "non-finite" in str(e.value)
    # columns out of order inside a row (row 17 holds 5 entries), a repeated
    # column, and a column index past n: each is a malformed CSR
    for bad_cols in ("swap", "repeat", "range"):
        ind = A.indices.copy()
        a, b = A.indptr[17], A.indptr[18]
        if bad_cols == "swap":
            ind[a], ind[a + 1] = ind[a + 1], ind[a]
        elif bad_cols == "repeat":
            ind[a + 1] = ind[a]
        else:
            ind[b - 1] = A.shape[0]
        M = A.copy()
        M.indices[:] = ind  # set after construction: no canonicalization or format check
        M.has_sorted_indices = False
        with pytest.raises(tls.TlsError) as e:
            _pc(M, part, 1, 0)
        assert e.value.status == 1 and "malformed CSR" in str(e.value), bad_cols
    # an empty part (parts 0, 1, 3 used, part 2 empty)
    gap = part.copy()
    gap[gap == 2] = 1
    with pytest.raises(tls.TlsError) as e:
        _pc(A, gap, 1, 0)
    assert e.value.status == 1 and "empty" in str(e.value)
    # a zero pivot in the unpivoted local LU (the first row of subdomain 0)
    z = A.tolil()
    z[0, 0] = 0.0
    z = z.tocsr()
    z.eliminate_zeros()
    with pytest.raises(tls.TlsError) as e:
        _pc(z, part, 1, 0, matrix_kind=1)
    assert e.value.status == 3


# ---------------------------------------------------------------------------
# general (nonsymmetric) matrices: LU, Section 6 coarse space, FGMRES
# ---------------------------------------------------------------------------

def _cd_problem(m, p, seed):
    from workloads import convdiff_2d
    rng = np.random.default_rng(seed)
    A, _ = convdiff_2d(m, rng)
    part = box_partition_2d(m, m, p, p)
    return A, part


@pytest.mark.parametrize("precision,refine,rows", [(0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 0, 2), (1, 0, 2), (1, 0, 3),
                                                   (1, 0, 4)])
def test_general_local_solves(precision, refine, rows):
    """LU substitutions (no pivoting) against the oracle's sparse LU on four
    subdomains of about 2.5k rows (delta 2), with tasks of one to four
    block rows. FP64: 1e-11. FP32: forward
    error within e_32 = 20 cond_2(A_ii) u_32 (cond from a dense SVD); with
    one refinement step within min(1e-5, e_32^2 + 20 cond u_64)."""
    A, part = _cd_problem(96, 2, seed=3)
    say("general local solves", precision, refine, rows)
    pc = _pc(A, part, 2, 0, precision=precision, matrix_kind=1, local_refine=refine, solve_rows=rows)
    assert pc.info()["solve_rows"] == rows
    rng = np.random.default_rng(0)
    for i in range(4):
        s = schwarz.overlap(A, part, i, 2)
        Aii = schwarz.local_matrix(A, s).tocsc()
        b = rng.standard_normal(s.size)
        x_ref = spla.spsolve(Aii, b)
        x = pc.local_solve(i, b)
        err = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
        if precision == 0:
            tol = 1e-11
        else:
            sv = np.linalg.svd(Aii.toarray(), compute_uv=False)
            cond = sv[0] / sv[-1]
            e32 = 20 * cond * 2.0 ** -24
            tol = e32 if refine == 0 else min(1e-5, e32 ** 2 + 20 * cond * 2.0 ** -53)
        say("  subdomain", i, "m", s.size, "err", err, "bound", tol)
        assert err <= tol
    pc.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_general_coarse_space_parity(precision):
    """Section 6 coarse vectors against a dense SVD: singular values to 1e-7
    (FP64) or 1e-4 (FP32 mode), spans to 1 - 1e-9 in cosine (FP64) or a
    largest principal angle of 1e-3 (FP32) where the gap allows; A_0 = Z^T A Z
    with the library's own Z to 1e-12."""
    A, part = _cd_problem(64, 3, seed=4)
    nev = 5
    say("general coarse space", precision)
    pc = _pc(A, part, 2, nev, matrix_kind=1, precision=precision)
    ex = pc.export(Z=True, A0=True)
    zc = ex["zcol_ptr"]
    for i in range(9):
        s = schwarz.overlap(A, part, i, 2)
        Aii = schwarz.local_matrix(A, s)
        sig_all, U = schwarz.svd_variant(Aii, s, s.size)
        k = zc[i + 1] - zc[i]
        assert k == min(nev, sig_all.size)
        assert np.allclose(ex["eigvals"][zc[i]:zc[i + 1]], sig_all[:k], rtol=1e-7 if precision == 0 else 1e-4)
        if sig_all.size > k and sig_all[k - 1] / sig_all[k] >= 1 + 1e-3:
            Zg = ex["Z"][s.idx[:s.n_interior]][:, zc[i]:zc[i + 1]]
            cos = principal_cosines(U[:s.n_interior, :k], Zg)
            if precision == 0:
                assert np.all(cos >= 1 - 1e-9), cos
            else:
                assert np.arccos(np.clip(cos.min(), -1.0, 1.0)) <= 1e-3, cos
    Zg = ex["Z"]
    A0_ref = Zg.T @ (A @ Zg)
    assert np.allclose(ex["A0"], A0_ref, rtol=1e-12, atol=1e-12 * np.abs(A0_ref).max())
    pc.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-5)])
def test_general_apply_with_imported_basis(precision, tol):
    torch = torch_cuda()
    A, part = _cd_problem(64, 4, seed=5)
    say("general apply", precision)
    pc = _pc(A, part, 2, 6, precision=precision, matrix_kind=1)
    ex = pc.export(Z=True)
    h = oracle.setup(A, part, 2, 6, spd=False, Z=ex["Z"])
    rng = np.random.default_rng(12)
    worst = 0.0
    for _ in range(5):
        r = rng.standard_normal(A.shape[0])
        z = pc.apply(to_dev(r))
        torch.cuda.synchronize()
        z_ref = oracle.apply(h, r)
        worst = max(worst, np.linalg.norm(z.cpu().numpy() - z_ref) / np.linalg.norm(z_ref))
    say("  worst apply error", worst)
    assert worst <= tol
    pc.close()


def test_general_fgmres_matches_oracle():
    torch = torch_cuda()
    A, part = _cd_problem(64, 4, seed=6)
    b = np.random.default_rng(3).standard_normal(A.shape[0])
    say("general fgmres")
    pc = _pc(A, part, 2, 6, matrix_kind=1, restart=30)
    x, it, rr, st = pc.solve(to_dev(b), 1e-8)
    torch.cuda.synchronize()
    h = oracle.setup(A, part, 2, 6, spd=False)
    _, it_ref, rr_ref = oracle.solve(h, b)
    say("  iterations", it, "oracle", it_ref, "relres", rr)
    assert st == 0 and rr <= 1e-8
    assert abs(it - it_ref) <= max(1, int(0.05 * it_ref))
    xs = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x.cpu().numpy() - xs) <= 1e-6 * np.linalg.norm(xs)
    pc.close()


def test_general_single_subdomain_one_iteration():
    torch = torch_cuda()
    A, _ = _cd_problem(40, 1, seed=7)
    part = np.zeros(A.shape[0], dtype=np.int32)
    b = np.random.default_rng(1).standard_normal(A.shape[0])
    say("general N=1")
    pc = _pc(A, part, 2, 4, matrix_kind=1)
    x, it, rr, st = pc.solve(to_dev(b), 1e-8)
    torch.cuda.synchronize()
    assert it == 1 and rr <= 1e-10
    pc.close()


# ---------------------------------------------------------------------------
# eigenvalue decay against the overlap (Section 7, Fig. 1) and threshold
# selection (lambda^2 > tau^2 in eq. gevpsvd, lambda > nu in eq. uppergevp,
# sigma > tau in Section 6)
# ---------------------------------------------------------------------------

def _diffusion_3d(nx, levels, seed):
    from workloads import fv_diffusion_3d, lognormal_kappa_3d
    rng = np.random.default_rng(seed)
    A = fv_diffusion_3d(lognormal_kappa_3d(nx, rng)).tocsr()
    part = rcb_partition((nx, nx, nx), levels, rng, (0.45, 0.55))
    return A, part


def _gap_threshold(spectra, lo=0.3, hi=0.7):
    """A threshold inside the spread of the given eigenvalues (between the
    lo and hi quantiles of their logarithms) as far as possible, relatively,
    from every one of them; returns it and that distance (log10)."""
    lv = np.log10(np.concatenate([v[v > 0] for v in spectra]))
    xs = np.linspace(np.quantile(lv, lo), np.quantile(lv, hi), 4001)
    dist = np.array([np.min(np.abs(lv - x)) for x in xs])
    b = int(np.argmax(dist))
    return 10.0 ** xs[b], dist[b]


def test_eigenvalue_decay_faster_with_more_layers():
    """3D lognormal diffusion, 8 RCB parts: the 24 largest eq. gevpsvd
    eigenvalues per subdomain for delta = 1, 3, 5 match the oracle's dense
    solve, and their decay lambda_j^2 / lambda_1^2 is faster for larger
    delta (Section 7, Fig. 1). With one threshold tau for all three, fewer
    vectors are kept as delta grows."""
    A, part = _diffusion_3d(16, 3, seed=21)
    N, nev = 8, 24
    med, spectra = {}, {}
    for delta in (1, 3, 5):
        say("decay delta", delta)
        pc = _pc(A, part, delta, nev)
        ex = pc.export()
        zc = ex["zcol_ptr"]
        ratios, spectra[delta] = [], []
        for i in range(N):
            s = schwarz.overlap(A, part, i, delta)
            lam, _ = schwarz.gevp2(schwarz.local_matrix(A, s), s, nev)
            got = ex["eigvals"][zc[i]:zc[i + 1]]
            assert got.size == lam.size == nev
            assert np.allclose(got, lam, rtol=1e-7), (delta, i, np.max(np.abs(got / lam - 1)))
            ratios.append(got / got[0])
            spectra[delta].append(lam)
        med[delta] = np.median(np.array(ratios), axis=0)
        pc.close()
    say("  median decay at j = 8, 16, 23:", {d: med[d][[8, 16, 23]] for d in med})
    for j in (8, 16, 23):
        assert med[1][j] > med[3][j] > med[5][j]
    tau2, margin = _gap_threshold(spectra[3])
    assert margin >= np.log10(1.01)
    kept = {}
    for delta in (1, 3, 5):
        pc = _pc(A, part, delta, nev, tau=float(np.sqrt(tau2)))
        ex = pc.export()
        kept[delta] = int(ex["zcol_ptr"][-1])
        if delta == 3:
            zc = ex["zcol_ptr"]
            for i in range(N):
                want = spectra[3][i][spectra[3][i] > tau2]
                assert zc[i + 1] - zc[i] == want.size
                assert np.allclose(ex["eigvals"][zc[i]:zc[i + 1]], want, rtol=1e-7)
        pc.close()
    say("  kept with tau^2 =", tau2, kept)
    assert kept[1] > kept[3] > kept[5]


def test_threshold_selection_gevp1_and_general():
    """lambda > nu for eq. uppergevp (nev = 0, cap nev1) and sigma > tau for
    the Section 6 variant: per-subdomain counts and values equal the
    oracle's with the threshold placed in a spectral gap."""
    # eq. uppergevp, delta = 2
    A = poisson_2d(48)
    part = box_partition_2d(48, 48, 3, 3)
    spec = []
    for i in range(9):
        s = schwarz.overlap(A, part, i, 2)
        lam, _ = schwarz.gevp1(schwarz.local_matrix(A, s), s, s.size, nu=1.0, dense=True)
        spec.append(lam[lam > 1 + 1e-10][:24])
    nu, margin = _gap_threshold(spec)
    assert margin >= np.log10(1.001)
    say("gevp1 threshold nu =", nu)
    pc = _pc(A, part, 2, 0, nev1=24, nu=float(nu))
    ex = pc.export()
    zc = ex["zcol_ptr"]
    for i in range(9):
        want = spec[i][spec[i] > nu]
        assert zc[i + 1] - zc[i] == want.size
        assert np.allclose(ex["eigvals"][zc[i]:zc[i + 1]], want, rtol=1e-8)
    pc.close()
    # Section 6 singular values, general A
    A, part = _cd_problem(64, 4, seed=5)
    spec = []
    for i in range(16):
        s = schwarz.overlap(A, part, i, 2)
        sig, _ = schwarz.svd_variant(schwarz.local_matrix(A, s), s, 24)
        spec.append(sig)
    tau, margin = _gap_threshold(spec)
    assert margin >= np.log10(1.001)
    say("svd threshold tau =", tau)
    pc = _pc(A, part, 2, 24, matrix_kind=1, tau=float(tau))
    ex = pc.export()
    zc = ex["zcol_ptr"]
    for i in range(16):
        want = spec[i][spec[i] > tau]
        assert zc[i + 1] - zc[i] == want.size
        assert np.allclose(ex["eigvals"][zc[i]:zc[i + 1]], want, rtol=1e-8)
    pc.close()


# ---------------------------------------------------------------------------
# RAS (eq. onelevelras) with the deflated coarse correction (Section 7.2)
# ---------------------------------------------------------------------------

def _ras_case(kind):
    if kind == "spd":
        p = make_config(1)
        return p.A, p.part, 1, 8, True
    if kind == "saddle":
        # symmetric indefinite: MAC Stokes cavity, 48 x 48 cells, 16 boxes
        from workloads import stokes_cavity_2d
        K, part, _ = stokes_cavity_2d(48, 4, 4)
        return K, part, 4, 16, False
    A, part = _cd_problem(64, 4, seed=5)
    return A, part, 2, 6, False


@pytest.mark.parametrize("kind,precision,scale,inv,tol", [("spd", 0, 0, 0, 1e-10), ("spd", 0, 1, 0, 1e-10),
                                                         ("spd", 1, 0, 0, 1e-5), ("spd", 0, 0, 1, 1e-10),
                                                         ("spd", 1, 1, 1, 1e-5), ("general", 0, 0, 0, 1e-10),
                                                         ("general", 1, 0, 0, 1e-5), ("saddle", 0, 0, 0, 1e-10),
                                                         ("saddle", 1, 0, 0, 1e-5)])
def test_ras_deflated_apply_with_imported_basis(kind, precision, scale, inv, tol):
    """z = Q r + M_RAS^{-1}(r - A Q r) with the library's own Z imported
    into the oracle, over several seeded r; for SPD also with the explicit
    local inverses and with Jacobi scaling."""
    torch = torch_cuda()
    A, part, delta, nev, spd = _ras_case(kind)
    say("ras+deflated apply", kind, precision, scale, inv)
    pc = _pc(A, part, delta, nev, precision=precision, matrix_kind=0 if spd else 1, composition=1,
             jacobi_scale=scale, local_inverse=inv)
    ex = pc.export(Z=True)
    h = oracle.setup(A, part, delta, nev, spd=spd, Z=ex["Z"])
    rng = np.random.default_rng(13)
    worst = 0.0
    for _ in range(5):
        r = rng.standard_normal(A.shape[0])
        z = pc.apply(to_dev(r))
        torch.cuda.synchronize()
        z_ref = oracle.apply(h, r, composition="ras_deflated")
        worst = max(worst, np.linalg.norm(z.cpu().numpy() - z_ref) / np.linalg.norm(z_ref))
    say("  worst apply error", worst)
    assert worst <= tol
    # M^{-1} A Z = Z: columns of the library's Z come back through A
    if precision == 0:
        Z = ex["Z"]
        for j in (0, Z.shape[1] // 2, Z.shape[1] - 1):
            z = pc.apply(to_dev(A @ Z[:, j]))
            torch.cuda.synchronize()
            assert np.allclose(z.cpu().numpy(), Z[:, j], rtol=1e-9, atol=1e-9 * np.abs(Z[:, j]).max())
    pc.close()


@pytest.mark.parametrize("kind", ["spd", "general", "saddle"])
def test_ras_one_level_and_single_subdomain(kind):
    """nev = 0 leaves plain RAS; N = 1 gives A^{-1} and one FGMRES step."""
    torch = torch_cuda()
    A, part, delta, _, spd = _ras_case(kind)
    mk = 0 if spd else 1
    say("ras one-level", kind)
    pc = _pc(A, part, delta, 0, matrix_kind=mk, composition=1)
    h = oracle.setup(A, part, delta, 0, spd=spd)
    r = np.random.default_rng(14).standard_normal(A.shape[0])
    z = pc.apply(to_dev(r))
    torch.cuda.synchronize()
    z_ref = oracle.apply(h, r, composition="ras_deflated")
    assert np.allclose(z.cpu().numpy(), z_ref, rtol=1e-10, atol=1e-12 * np.abs(z_ref).max())
    pc.close()
    one = np.zeros(A.shape[0], dtype=np.int32)
    pc = _pc(A, one, delta, 4, matrix_kind=mk, composition=1)
    x, it, rr, st = pc.solve(to_dev(r), 1e-8)
    torch.cuda.synchronize()
    assert st == 0 and it == 1 and rr <= 1e-10
    pc.close()


@pytest.mark.parametrize("kind", ["spd", "general", "saddle"])
def test_ras_deflated_fgmres_matches_oracle(kind):
    """FGMRES(30) with the composition converges like the oracle's (CGS2 on
    the GPU, MGS in the oracle), graph-captured and eager runs give the
    same iterates, and it needs fewer iterations than the additive
    composition on these problems."""
    torch = torch_cuda()
    A, part, delta, nev, spd = _ras_case(kind)
    mk = 0 if spd else 1
    b = np.random.default_rng(15).standard_normal(A.shape[0])
    say("ras+deflated fgmres", kind)
    pc = _pc(A, part, delta, nev, matrix_kind=mk, composition=1, use_graph=1)
    x, it, rr, st = pc.solve(to_dev(b), 1e-8)
    x2, it2, _, _ = pc.solve(to_dev(b), 1e-8)
    torch.cuda.synchronize()
    pc.close()
    pe = _pc(A, part, delta, nev, matrix_kind=mk, composition=1, use_graph=0)
    xe, ite, _, _ = pe.solve(to_dev(b), 1e-8)
    torch.cuda.synchronize()
    pe.close()
    h = oracle.setup(A, part, delta, nev, spd=spd)
    _, it_ref, _ = oracle.solve(h, b, composition="ras_deflated")
    _, it_add, _ = oracle.solve(h, b)
    say("  iterations", it, "oracle", it_ref, "additive (oracle)", it_add, "relres", rr)
    assert st == 0 and rr <= 1e-8
    assert abs(it - it_ref) <= max(1, int(0.05 * it_ref))
    assert it == it2 == ite and torch.equal(x, x2) and torch.equal(x, xe)
    assert it_ref < it_add
    xs = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x.cpu().numpy() - xs) <= 1e-6 * np.linalg.norm(xs)


def test_reused_device_blocks_and_trim():
    """Contexts built on device blocks kept from earlier contexts (not zeroed)
    and after tls_trim solve bit for bit alike."""
    import paper_2401_03915_amd as tls
    torch = torch_cuda()
    A, part = _hc_problem(128, 2, seed=9)
    b = np.random.default_rng(2).standard_normal(A.shape[0])
    xs = []
    for k in range(3):
        if k == 2:
            tls.tls_trim()
        pc = _pc(A, part, 2, 8, local_inverse=1)
        x, it, rr, st = pc.solve(to_dev(b), 1e-8)
        torch.cuda.synchronize()
        assert st == 0 and rr <= 1e-8
        xs.append((x, it))
        pc.close()
    assert xs[0][1] == xs[1][1] == xs[2][1]
    assert torch.equal(xs[0][0], xs[1][0]) and torch.equal(xs[0][0], xs[2][0])


@pytest.mark.parametrize("precision", [0, 1])
def test_grouped_setup_is_bitwise_identical(monkeypatch, precision):
    """With TLS_MEMORY_LIMIT=1 every eigen pass (both eigenproblems) and the
    formation of the explicit inverses run one subdomain at a time; the
    coarse basis, its eigenvalues and the preconditioner are bit for bit
    those of the set-up that does all subdomains at once."""
    torch = torch_cuda()
    A, part = _diffusion_3d(14, 3, seed=21)
    r = to_dev(np.random.default_rng(4).standard_normal(A.shape[0]))
    out = []
    for lim in (None, "1"):
        if lim:
            monkeypatch.setenv("TLS_MEMORY_LIMIT", lim)
        say(f"grouped set-up: precision {precision}, limit {lim}")
        pc = _pc(A, part, 2, 6, nev1=2, precision=precision, local_inverse=1)
        ex = pc.export(Z=True)
        z = pc.apply(r)
        torch.cuda.synchronize()
        out.append((ex, z.cpu().numpy()))
        pc.close()
        monkeypatch.delenv("TLS_MEMORY_LIMIT", raising=False)
    (e0, z0), (e1, z1) = out
    assert e0["zsrc"].tolist().count(1) > 0  # the eq. uppergevp pass kept columns
    for key in ("zcol_ptr", "zsrc", "eigvals", "Z"):
        assert np.array_equal(e0[key], e1[key]), key
    assert np.array_equal(z0, z1)


@pytest.mark.parametrize("precision", [0, 1])
def test_grouped_general_basis_is_bitwise_identical(monkeypatch, precision):
    """With TLS_MEMORY_LIMIT=1 the Section 6 basis (H, its Gram, the
    subspace iteration and V = H v) runs one subdomain at a time; the coarse
    basis, its singular values and the preconditioner are bit for bit those
    of the set-up that does all subdomains at once."""
    torch = torch_cuda()
    A, part = _cd_problem(96, 3, seed=5)
    r = to_dev(np.random.default_rng(6).standard_normal(A.shape[0]))
    out = []
    for lim in (None, "1"):
        if lim:
            monkeypatch.setenv("TLS_MEMORY_LIMIT", lim)
        say(f"grouped general basis: precision {precision}, limit {lim}")
        pc = _pc(A, part, 2, 5, matrix_kind=1, precision=precision)
        ex = pc.export(Z=True)
        z = pc.apply(r)
        torch.cuda.synchronize()
        out.append((ex, z.cpu().numpy()))
        pc.close()
        monkeypatch.delenv("TLS_MEMORY_LIMIT", raising=False)
    (e0, z0), (e1, z1) = out
    assert e0["zcol_ptr"][-1] > 0
    for key in ("zcol_ptr", "zsrc", "eigvals", "Z"):
        assert np.array_equal(e0[key], e1[key]), key
    assert np.array_equal(z0, z1)


@pytest.mark.parametrize("local_inverse", [0, 1])
def test_autotune_cache_reuse(tmp_path, local_inverse):
    """Every autotuned shape (factorization panel width; workgroups and task
    order of the substitutions, or the block side of the product with the
    explicit inverses) is timed by the first setup, written to the cache,
    read back by the second without timing, and the two contexts apply the
    same preconditioner (bitwise, since the picks are equal)."""
    torch = torch_cuda()
    import paper_2401_03915_amd as tls
    A, part = _hc_problem(96, 3, seed=8)
    cache = str(tmp_path / "tune.txt")
    say("autotune cache", local_inverse)
    pc1 = _pc(A, part, 2, 4, autotune=1, tune_cache=cache.encode(), local_inverse=local_inverse)
    i1 = pc1.info()
    lines = open(cache).read().splitlines()
    keys = sorted(line.split(" ")[0] for line in lines)
    assert keys == (["factor:v1", "symv:v1"] if local_inverse else ["factor:v1", "trsv:v7"])
    pc2 = _pc(A, part, 2, 4, autotune=1, tune_cache=cache.encode(), local_inverse=local_inverse)
    i2 = pc2.info()
    assert open(cache).read().splitlines() == lines  # nothing timed or written again
    assert i1["tuned"] == 1 and i2["tuned"] == 2
    assert i1["factor_panel"] == i2["factor_panel"] and i1["factor_panel"] in (4, 8, 16)
    if local_inverse:
        assert i1["symv_block"] == i2["symv_block"] and i1["symv_block"] in (4, 6, 8)
    else:
        assert i1["solve_wgs"] == i2["solve_wgs"] > 0 and i1["solve_order"] == i2["solve_order"]
        assert i1["solve_order_bwd"] == i2["solve_order_bwd"]
    r = to_dev(np.random.default_rng(4).standard_normal(A.shape[0]))
    z1, z2 = pc1.apply(r), pc2.apply(r)
    torch.cuda.synchronize()
    assert torch.equal(z1, z2)
    pc1.close()
    pc2.close()
    del tls


# ---------------------------------------------------------------------------
# learned warm start of the eigensolver (network kernels against the oracle)
# ---------------------------------------------------------------------------

def _gnn_case():
    A, part = _hc_problem(64, 3, seed=6)
    return A, part, 2, 4


def test_gnn_forward_matches_oracle():
    from oracle import gnn
    A, part, delta, nev = _gnn_case()
    N = int(part.max()) + 1
    c_out = 6
    w = 0.3 * np.random.default_rng(21).standard_normal(gnn.n_weights(c_out))
    say("gnn forward")
    pc = _pc(A, part, delta, nev, gnn_train=1)
    X = pc.gnn_forward(w.astype(np.float32), c_out)
    sp_ = pc.export()["sub_ptr"]
    worst = 0.0
    for i in range(N):
        s = schwarz.overlap(A, part, i, delta)
        Aii = schwarz.local_matrix(A, s)
        Xo, _ = gnn.forward(Aii, s.n_interior, s.layer_sizes[-1], w.astype(np.float32).astype(np.float64), c_out)
        Xg = X[sp_[i]:sp_[i + 1]]
        worst = max(worst, np.abs(Xg - Xo).max() / np.abs(Xo).max())
    say("  worst forward error", worst)
    assert worst <= 1e-5
    pc.close()


def test_gnn_loss_and_gradient_match_oracle():
    """Loss and weight gradient of the device backward kernels against the
    oracle's backward pass, with targets from the oracle's dense solve of
    eq. gevpsvd (the spans agree wherever the gap at k allows; the case is
    chosen so that it does for every subdomain)."""
    from oracle import gnn
    A, part, delta, nev = _gnn_case()
    N = int(part.max()) + 1
    c_out = 6
    w = (0.3 * np.random.default_rng(22).standard_normal(gnn.n_weights(c_out))).astype(np.float32)
    say("gnn loss/grad")
    pc = _pc(A, part, delta, nev, gnn_train=1)
    zc = pc.export()["zcol_ptr"]
    loss_g, grad_g = pc.gnn_loss_grad(w, c_out)
    w64 = w.astype(np.float64)
    tot_f, tot_g, nact = 0.0, np.zeros(w.size), 0
    for i in range(N):
        s = schwarz.overlap(A, part, i, delta)
        Aii = schwarz.local_matrix(A, s)
        lam, W = schwarz.gevp2(Aii, s, s.size)
        k = zc[i + 1] - zc[i]
        if k == 0:
            continue
        assert lam.size == k or lam[k - 1] / lam[k] >= 1 + 1e-3, "case must have a spectral gap at k"
        Q = gnn.target_basis(W[:, :k], s.layer_sizes[-1])
        f, g = gnn.loss_grad(Aii, s.n_interior, s.layer_sizes[-1], w64, c_out, Q)
        tot_f += f
        tot_g += g
        nact += 1
    loss_o, grad_o = tot_f / nact, tot_g / nact
    say("  loss", loss_g, loss_o)
    assert abs(loss_g - loss_o) <= 1e-4 * abs(loss_o)
    err = np.linalg.norm(grad_g - grad_o) / np.linalg.norm(grad_o)
    say("  gradient error", err)
    assert err <= 1e-3
    pc.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_gnn_warm_start_keeps_the_result(precision):
    """Any start block (here an untrained network) leads to the same
    eigenvalues within the eigensolver tolerance, the same coarse space and
    the same PCG iterations."""
    torch = torch_cuda()
    from oracle import gnn
    A, part, delta, nev = _gnn_case()
    c_out = 8
    w = (0.3 * np.random.default_rng(23).standard_normal(gnn.n_weights(c_out))).astype(np.float32)
    say("gnn warm start", precision)
    p0 = _pc(A, part, delta, nev, precision=precision)
    p1 = _pc(A, part, delta, nev, precision=precision, gnn_weights=w)
    e0, e1 = p0.export(), p1.export()
    assert np.array_equal(e0["zcol_ptr"], e1["zcol_ptr"])
    tol = 1e-7 if precision == 0 else 1e-3
    assert np.allclose(e0["eigvals"], e1["eigvals"], rtol=tol)
    b = to_dev(np.random.default_rng(24).standard_normal(A.shape[0]))
    _, it0, rr0, _ = p0.solve(b, 1e-8)
    _, it1, rr1, _ = p1.solve(b, 1e-8)
    torch.cuda.synchronize()
    i0, i1 = p0.info(), p1.info()
    say("  iterations", it0, it1, "eig iters", i0["eig_iters_max"], i1["eig_iters_max"], "t_gnn", i1["t_setup"][4])
    assert rr0 <= 1e-8 and rr1 <= 1e-8
    assert abs(it1 - it0) <= max(1, 0.05 * it0)
    assert i1["t_setup"][4] > 0.0
    p0.close()
    p1.close()


def test_gnn_trained_weights_gain_on_layered_elasticity():
    """The committed weights (trained by paper_2401_03915_amd.gnn_train on
    seeds 100-103) on the layered-elasticity workload of seed 0, FP64: the
    training loss is far below that of the initial weights, the warm start
    takes fewer subspace iterations on average than the random start, and
    the final PCG iteration counts and eigen-residuals stay within 5% / the
    tolerance of the method without it."""
    torch = torch_cuda()
    from paper_2401_03915_amd.gnn_train import TRAINED, init_weights, load_weights
    w, c_out = load_weights(TRAINED)
    p = make_config(4)
    say("gnn trained weights: loss")
    pt = _pc(p.A, p.part, p.overlap, p.nev, gnn_train=1)
    loss_trained, _ = pt.gnn_loss_grad(w, c_out)
    loss_init, _ = pt.gnn_loss_grad(init_weights(c_out, 100), c_out)
    pt.close()
    say("  loss trained / initial", loss_trained, loss_init)
    assert loss_trained < 2.0 * loss_init  # losses are negative: at least twice the captured span
    b = to_dev(p.b)
    out = {}
    for name, kw in (("random", {}), ("warm", {"gnn_weights": w})):
        say("gnn trained weights:", name)
        pc = _pc(p.A, p.part, p.overlap, p.nev, use_graph=1, **kw)
        _, it, rr, st = pc.solve(b, 1e-8)
        torch.cuda.synchronize()
        inf = pc.info()
        out[name] = (it, rr, inf["eig_iters_mean"], inf["eig_resid_max"])
        pc.close()
    say("  (PCG iters, relres, mean eig iters, eig resid)", out)
    (it0, rr0, e0, res0), (it1, rr1, e1, res1) = out["random"], out["warm"]
    assert rr0 <= 1e-8 and rr1 <= 1e-8
    assert abs(it1 - it0) <= 0.05 * it0
    assert res1 <= 1e-8 and res0 <= 1e-8  # eig_tol 1e-9; a stalled residual up to 10x is accepted
    assert e1 < e0
