"""The worker-pool form of the oracle (oracle.pool) against the serial
oracle: the same coarse blocks, the same apply up to the order in which the
one-level contributions are added, the same Krylov iterations (CPU only)."""

import numpy as np
import pytest

import oracle
from oracle import pool
from workloads import box_partition_2d, convdiff_2d, fv_diffusion_2d, high_contrast_kappa_2d, rcb_partition


def _hc(nx=48, levels=3, seed=8):
    rng = np.random.default_rng(seed)
    A = fv_diffusion_2d(high_contrast_kappa_2d(nx, nx, rng, n_channels=4, kmax=1e4))
    return A, rcb_partition((nx, nx), levels, rng, (0.3, 0.7))


@pytest.mark.parametrize("spd", [True, False])
def test_pool_matches_serial_oracle(spd):
    if spd:
        A, part = _hc()
        delta, nev = 2, 5
    else:
        A, _ = convdiff_2d(40, np.random.default_rng(9))
        part = box_partition_2d(40, 40, 3, 3)
        delta, nev = 2, 4
    h = oracle.setup(A, part, delta, nev, spd=spd)
    with pool.Pool(A, part, delta, nev, spd=spd, workers=3) as pl:
        assert pl.n_coarse == h.n_coarse
        Zs = pl.Z.toarray()
        # the same coarse space (workers use one BLAS thread: equal up to rounding)
        assert np.linalg.norm(Zs @ (Zs.T @ h.Z) - h.Z) <= 1e-10 * np.linalg.norm(h.Z)
        rng = np.random.default_rng(1)
        for comp in oracle.schwarz.COMPOSITIONS:
            r = rng.standard_normal(A.shape[0])
            z_ser = oracle.apply(h, r, composition=comp)
            z_par = pl.apply(r, comp)
            assert np.linalg.norm(z_par - z_ser) <= 1e-13 * np.linalg.norm(z_ser)
        b = rng.standard_normal(A.shape[0])
        _, it_s, rr_s = oracle.solve(h, b)
        _, it_p, rr_p = pl.solve(b)
        assert it_s == it_p and rr_p <= 1e-8
        # an imported basis (here a column-scaled copy: same span, same Q)
        Zi = Zs * np.linspace(1.0, 2.0, Zs.shape[1])
        pl.with_basis(Zi)
        r = rng.standard_normal(A.shape[0])
        z1 = pl.apply(r)
        z2 = oracle.apply(oracle.setup(A, part, delta, nev, spd=spd, Z=Zi), r)
        assert np.linalg.norm(z1 - z2) <= 1e-12 * np.linalg.norm(z2)
