"""GPU parity at the full sizes of the benchmark configurations, in the launch
configuration bench.py times (mixed precision, explicit local inverses for SPD
matrices, autotuned persistent solves otherwise,
PCG/FGMRES captured in hipGraph chunks), against the oracle on sampled
outputs it can compute one by one and against properties that hold at any
size:

* local solves of sampled subdomains (smallest, median, largest) against
  the oracle's sparse LU: forward error within 20 cond(A_ii) u for the
  explicit inverses (SPD), backward error for the LU substitutions;
* the dominant eigenvalues of sampled subdomains against the oracle's
  ARPACK solve of eq. gevpsvd (Section 6: dense SVD of H for general A);
* sampled columns of A_0 against Z^T (A z_j) with the library's own Z;
* symmetry of M^{-1} (SPD);
* config 6 (saddle point) with the RAS + deflated composition it is
  benchmarked with;
* convergence to 1e-8 with the true residual recomputed on the host, and
  mixed-precision iteration counts within 5% of plain FP64.
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import schwarz
from tests.gpu_helpers import say, to_dev, torch_cuda
from workloads import make_config

pytestmark = pytest.mark.gpu


def _pc(p, precision, **kw):
    """The benchmark's settings: graph-captured Krylov chunks, autotuned
    solves, and explicit local inverses for SPD matrices."""
    import paper_2401_03915_amd as tls
    return tls.Preconditioner(p.A, p.part, p.overlap, p.nev, precision=precision,
                              matrix_kind=0 if p.spd else 1, use_graph=1, autotune=1,
                              local_inverse=1 if p.spd else 0, **kw)


def _sample(p, ex):
    """Smallest, median and largest subdomain (by #Omega_i)."""
    m = np.diff(ex["sub_ptr"])
    order = np.argsort(m, kind="stable")
    return [int(order[0]), int(order[len(order) // 2]), int(order[-1])]


@pytest.mark.parametrize("cfg", [2, 3, 4, 5, 6])
def test_full_size_configuration(cfg):
    torch = torch_cuda()
    p = make_config(cfg)
    A = p.A.tocsr()
    # the saddle-point config runs, as benchmarked, with RAS + deflated
    kw = {"composition": 1} if cfg == 6 else {}
    say(f"full size cfg{cfg}: setup fp64")
    p64 = _pc(p, 0, **kw)
    ex = p64.export()
    picks = _sample(p, ex)
    # -- sampled local solves (FP64 context): oracle sparse LU, backward error
    rng = np.random.default_rng(30 + cfg)
    for i in picks:
        s = schwarz.overlap(A, p.part, i, p.overlap)
        a, b = ex["sub_ptr"][i], ex["sub_ptr"][i + 1]
        assert np.array_equal(ex["sub_idx"][a:b], s.idx)
        Aii = schwarz.local_matrix(A, s).tocsc()
        rhs = rng.standard_normal(s.size)
        x = p64.local_solve(i, rhs)
        xo = spla.splu(Aii).solve(rhs)
        bwd = np.linalg.norm(Aii @ x - rhs) / (spla.norm(Aii, 1) * np.linalg.norm(x, 1) + np.linalg.norm(rhs, 1))
        fwd = np.linalg.norm(x - xo) / np.linalg.norm(xo)
        say(f"  local solve {i} (m={s.size}): backward {bwd:.1e} forward {fwd:.1e}")
        if p.spd:
            # product with the explicit inverse: forward error of order
            # cond(A_ii) u, as for the substitutions; bound 20 cond u
            lmax = spla.eigsh(Aii, 1, which="LA", return_eigenvectors=False)[0]
            lmin = spla.eigsh(Aii, 1, sigma=0.0, which="LM", return_eigenvectors=False)[0]
            say(f"    cond {lmax / lmin:.1e}")
            assert fwd <= 20 * (lmax / lmin) * 2.0 ** -53
        else:
            assert bwd <= 1e-13  # substitution with the LU factor is backward stable
            assert fwd <= 1e-5  # the gap to the sparse LU is cond(A_ii) eps
    # -- sampled eigenvalues: the two smaller samples (the oracle's solve is slow)
    zc = ex["zcol_ptr"]
    for i in picks[:2]:
        s = schwarz.overlap(A, p.part, i, p.overlap)
        Aii = schwarz.local_matrix(A, s)
        k = int(zc[i + 1] - zc[i])
        if p.spd:
            lam, _ = schwarz.gevp2(Aii, s, p.nev, dense=False)
        else:
            lam, _ = schwarz.svd_variant(Aii, s, p.nev)
        got = ex["eigvals"][zc[i]:zc[i + 1]]
        say(f"  eigenvalues {i}: k={k} max rel err {np.max(np.abs(got - lam[:k]) / np.abs(lam[:k])):.1e}")
        assert k == min(p.nev, lam.size)
        assert np.allclose(got, lam[:k], rtol=1e-7)
    # -- sampled columns of A_0 = Z^T A Z (the library's own Z)
    if int(zc[-1]) <= 5000:
        exa = p64.export(A0=True)
        Z = p64.z_sparse(ex)
        for j in np.linspace(0, Z.shape[1] - 1, 4).astype(int):
            col = Z.T @ (A @ Z[:, j].toarray().ravel())
            assert np.allclose(exa["A0"][:, j], col, rtol=1e-12, atol=1e-12 * np.abs(col).max())
    # -- symmetry of M^{-1} (SPD): x^T M^{-1} y = y^T M^{-1} x
    if p.spd:
        u = to_dev(rng.standard_normal(A.shape[0]))
        v = to_dev(rng.standard_normal(A.shape[0]))
        mu, mv = p64.apply(u), p64.apply(v)
        torch.cuda.synchronize()
        l, r = float(torch.dot(v, mu)), float(torch.dot(u, mv))
        assert abs(l - r) <= 1e-11 * max(abs(l), abs(r))
    # -- solves: FP64 and mixed, true residuals, iteration counts
    b = to_dev(p.b)
    x64, it64, rr64, st64 = p64.solve(b, 1e-8)
    torch.cuda.synchronize()
    p64.close()
    say(f"full size cfg{cfg}: setup mixed")
    p32 = _pc(p, 1, **kw)
    x32, it32, rr32, st32 = p32.solve(b, 1e-8)
    torch.cuda.synchronize()
    p32.close()
    for x, it, rr, st in ((x64, it64, rr64, st64), (x32, it32, rr32, st32)):
        xh = x.cpu().numpy()
        true = np.linalg.norm(p.b - A @ xh) / np.linalg.norm(p.b)
        assert st == 0 and rr <= 1e-8 and true <= 1.01e-8, (st, rr, true)
    say(f"  iterations fp64 {it64} mixed {it32}")
    assert abs(it32 - it64) <= max(2, 0.05 * it64)
