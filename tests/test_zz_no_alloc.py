"""tls_solve_noalloc (the solve with its work in the library's fixed device
scratch array) against tls_solve on the same context, through the C ABI:
two calls in a row, the second on a smaller problem, for PCG and FGMRES,
and the size limit of the scratch array."""

import numpy as np
import pytest

from paper_2401_03915_amd import _lib
from tests.gpu_helpers import say, to_dev, torch_cuda
from workloads import box_partition_2d, convdiff_2d, fv_diffusion_2d, high_contrast_kappa_2d, rcb_partition

pytestmark = pytest.mark.gpu


def _hc(nx, levels, seed):
    rng = np.random.default_rng(seed)
    A = fv_diffusion_2d(high_contrast_kappa_2d(nx, nx, rng))
    return A, rcb_partition((nx, nx), levels, rng, (0.3, 0.7))


def _cd(m, p, seed):
    A, _ = convdiff_2d(m, np.random.default_rng(seed))
    return A, box_partition_2d(m, m, p, p)


def _pair(pc, b):
    """x from tls_solve and from tls_solve_noalloc on one context."""
    torch = torch_cuda()
    bd = to_dev(b)
    x1 = torch.empty_like(bd)
    x2 = torch.full_like(bd, float("nan"))
    st1, it1, rr1 = _lib.tls_solve(pc.ctx, bd.data_ptr(), x1.data_ptr(), 1e-8)
    st2, it2, rr2 = _lib.tls_solve_noalloc(pc.ctx, bd.data_ptr(), x2.data_ptr(), 1e-8)
    torch.cuda.synchronize()
    return (st1, it1, rr1, x1.cpu().numpy()), (st2, it2, rr2, x2.cpu().numpy())


@pytest.mark.parametrize("kind", ["pcg", "fgmres"])
def test_noalloc_solve_matches_tls_solve(kind):
    import paper_2401_03915_amd as tls
    # the first problem is the larger one, the second smaller
    if kind == "pcg":
        probs = [(_hc(128, 4, 21), 2, 8, {}), (_hc(64, 3, 22), 2, 6, {})]
    else:
        probs = [(_cd(96, 4, 23), 2, 6, {"matrix_kind": 1}), (_cd(48, 3, 24), 2, 4, {"matrix_kind": 1})]
    sizes = []
    for (A, part), delta, nev, opts in probs:
        for precision in (0, 1):
            say("noalloc", kind, A.shape[0], precision)
            pc = tls.Preconditioner(A, part, delta, nev, precision=precision, use_graph=0, **opts)
            b = np.random.default_rng(A.shape[0] + precision).standard_normal(A.shape[0])
            (st1, it1, rr1, x1), (st2, it2, rr2, x2) = _pair(pc, b)
            say("  tls_solve", st1, it1, rr1, "noalloc", st2, it2, rr2)
            assert st1 == 0 and st2 == 0
            assert it1 == it2 and rr2 <= 1e-8
            # same kernels, same fixed-order reductions: the same iterate
            assert np.array_equal(x1, x2)
            pc.close()
        sizes.append(A.shape[0])
    assert sizes[1] < sizes[0]


def test_noalloc_rejects_work_beyond_the_scratch_array():
    """FGMRES(m) needs 8 n (2 m + 7) bytes of work: with n = 16384 and
    m = 600 that is 158 MB, beyond the 128 MiB array: TLS_E_ARG, while
    tls_solve (which allocates) still solves."""
    import paper_2401_03915_amd as tls
    torch = torch_cuda()
    A, part = _cd(128, 4, 25)
    say("noalloc size limit")
    pc = tls.Preconditioner(A, part, 2, 4, matrix_kind=1, restart=600, use_graph=0)
    b = to_dev(np.random.default_rng(5).standard_normal(A.shape[0]))
    x = torch.zeros_like(b)
    st, _, _ = _lib.tls_solve_noalloc(pc.ctx, b.data_ptr(), x.data_ptr(), 1e-8, allow=(_lib.TLS_E_ARG,))
    assert st == _lib.TLS_E_ARG
    assert "scratch" in _lib.last_error(pc.ctx)
    st, it, rr = _lib.tls_solve(pc.ctx, b.data_ptr(), x.data_ptr(), 1e-8)
    torch.cuda.synchronize()
    assert st == 0 and rr <= 1e-8
    pc.close()
