"""Synthetic PDE matrices, partitions and right-hand sides.

Every generator returns a ``scipy.sparse.csr_matrix`` with int32 indices,
sorted columns and no duplicates, and (where applicable) an int32 ``part``
array with values in [0, N). Unknowns are numbered lexicographically with x
fastest (k = x + nx*y [+ nx*ny*z]).

The benchmark matrices stand in for the finite-element problems of the
paper's numerical section (which are not available here): they have the same
kind of structure (2D/3D diffusion with high-contrast coefficients, 3D
elasticity, nonsymmetric convection-diffusion) and the sizes of the
configurations listed in ``CONFIGS``.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

__all__ = [
    "Problem",
    "CONFIGS",
    "make_config",
    "poisson_2d",
    "fv_diffusion_2d",
    "fv_diffusion_3d",
    "high_contrast_kappa_2d",
    "lognormal_kappa_3d",
    "convdiff_2d",
    "one_way_convection_2d",
    "elasticity_q1_3d",
    "box_partition_2d",
    "box_partition_3d",
    "rcb_partition",
    "rhs",
    "worked_example_7x7",
]


@dataclass
class Problem:
    """A linear system Ax=b with a nonoverlapping partition of its unknowns."""

    name: str
    A: sp.csr_matrix
    part: np.ndarray
    n_parts: int
    overlap: int
    nev: int
    b: np.ndarray
    spd: bool = True
    meta: dict = field(default_factory=dict)


def _finish(rows, cols, vals, n):
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    A.eliminate_zeros()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    return A


# --------------------------------------------------------------------------
# 2D / 3D diffusion
# --------------------------------------------------------------------------

def poisson_2d(nx: int, ny: int | None = None) -> sp.csr_matrix:
    """5-point Laplacian [4; -1 x4] on nx*ny unknowns, Dirichlet boundary
    eliminated (unscaled)."""
    ny = nx if ny is None else ny
    n = nx * ny
    k = np.arange(n)
    x, y = k % nx, k // nx
    rows = [k]
    cols = [k]
    vals = [np.full(n, 4.0)]
    for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        m = (x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny)
        rows.append(k[m])
        cols.append(k[m] + dx + nx * dy)
        vals.append(np.full(int(m.sum()), -1.0))
    return _finish(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n)


def _harmonic(a, b):
    return 2.0 * a * b / (a + b)


def fv_diffusion_2d(kappa: np.ndarray) -> sp.csr_matrix:
    """Cell-centred two-point-flux finite volumes for -div(kappa grad u) on a
    ny x nx grid of unit cells. Interior faces use the harmonic mean
    transmissibility 2 ka kb / (ka + kb); Dirichlet faces use 2 kappa_cell."""
    ny, nx = kappa.shape
    n = nx * ny
    kap = kappa.reshape(-1).astype(np.float64)
    k = np.arange(n)
    x, y = k % nx, k // nx
    diag = np.zeros(n)
    rows, cols, vals = [], [], []
    for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        inside = (x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny)
        nb = k[inside] + dx + nx * dy
        t = _harmonic(kap[k[inside]], kap[nb])
        diag[k[inside]] += t
        rows.append(k[inside])
        cols.append(nb)
        vals.append(-t)
        diag[k[~inside]] += 2.0 * kap[k[~inside]]
    rows.append(k)
    cols.append(k)
    vals.append(diag)
    return _finish(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n)


def fv_diffusion_3d(kappa: np.ndarray) -> sp.csr_matrix:
    """7-point cell-centred finite volumes on an nz x ny x nx grid, same face
    rules as :func:`fv_diffusion_2d`."""
    nz, ny, nx = kappa.shape
    n = nx * ny * nz
    kap = kappa.reshape(-1).astype(np.float64)
    k = np.arange(n)
    x, y, z = k % nx, (k // nx) % ny, k // (nx * ny)
    diag = np.zeros(n)
    rows, cols, vals = [], [], []
    for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        inside = ((x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny)
                  & (z + dz >= 0) & (z + dz < nz))
        nb = k[inside] + dx + nx * dy + nx * ny * dz
        t = _harmonic(kap[k[inside]], kap[nb])
        diag[k[inside]] += t
        rows.append(k[inside])
        cols.append(nb)
        vals.append(-t)
        diag[k[~inside]] += 2.0 * kap[k[~inside]]
    rows.append(k)
    cols.append(k)
    vals.append(diag)
    return _finish(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n)


def high_contrast_kappa_2d(nx: int, ny: int, rng: np.random.Generator,
                           n_channels: int = 20, kmax: float = 1e6) -> np.ndarray:
    """Log-uniform coefficient in [1, kmax] per cell plus ``n_channels``
    axis-aligned full-span stripes (axis x or y with probability 1/2, width
    uniform in {1..4} cells, uniform offset) set to kmax."""
    kappa = 10.0 ** rng.uniform(0.0, np.log10(kmax), size=(ny, nx))
    for _ in range(n_channels):
        axis = rng.integers(0, 2)
        width = int(rng.integers(1, 5))
        if axis == 0:  # stripe along x: a band of rows
            off = int(rng.integers(0, ny - width + 1))
            kappa[off:off + width, :] = kmax
        else:
            off = int(rng.integers(0, nx - width + 1))
            kappa[:, off:off + width] = kmax
    return kappa


def lognormal_kappa_3d(n: int, rng: np.random.Generator, sigma: float = 2.0) -> np.ndarray:
    """kappa = exp(N(0, sigma^2)) independently per cell of an n^3 grid."""
    return np.exp(rng.normal(0.0, sigma, size=(n, n, n)))


# --------------------------------------------------------------------------
# Nonsymmetric convection-diffusion
# --------------------------------------------------------------------------

def convdiff_2d(m: int, rng: np.random.Generator, eps: float = 0.01,
                n_vortex: int = 16) -> tuple[sp.csr_matrix, dict]:
    """-eps Lap u + w . grad u on m x m interior nodes of the unit square
    (h = 1/(m+1)), central differences for diffusion and first-order upwind
    for convection, Dirichlet boundary eliminated. The velocity is
    w = (d psi/dy, -d psi/dx) with psi a sum of ``n_vortex`` Gaussians
    a_k exp(-|x-c_k|^2 / (2 r_k^2)), c_k ~ U[0,1]^2, r_k ~ U(0.05, 0.2),
    a_k = +-1, scaled so that max |w| = 1 over the nodes. The result is a
    nonsingular M-matrix with a symmetric pattern."""
    h = 1.0 / (m + 1)
    c = rng.uniform(0.0, 1.0, size=(n_vortex, 2))
    r = rng.uniform(0.05, 0.2, size=n_vortex)
    a = rng.choice(np.array([-1.0, 1.0]), size=n_vortex)
    k = np.arange(m * m)
    ix, iy = k % m, k // m
    px, py = (ix + 1) * h, (iy + 1) * h
    dpsi_dx = np.zeros(m * m)
    dpsi_dy = np.zeros(m * m)
    for j in range(n_vortex):
        g = a[j] * np.exp(-((px - c[j, 0]) ** 2 + (py - c[j, 1]) ** 2) / (2 * r[j] ** 2))
        dpsi_dx += g * (-(px - c[j, 0]) / r[j] ** 2)
        dpsi_dy += g * (-(py - c[j, 1]) / r[j] ** 2)
    wx, wy = dpsi_dy, -dpsi_dx
    scale = np.max(np.hypot(wx, wy))
    wx, wy = wx / scale, wy / scale
    d = eps / h ** 2
    diag = 4.0 * d + (np.abs(wx) + np.abs(wy)) / h
    rows, cols, vals = [k], [k], [diag]
    # west/east neighbours: upwind picks the west node when wx > 0
    for dx, dy, coef in ((-1, 0, -d - np.maximum(wx, 0.0) / h),
                         (1, 0, -d - np.maximum(-wx, 0.0) / h),
                         (0, -1, -d - np.maximum(wy, 0.0) / h),
                         (0, 1, -d - np.maximum(-wy, 0.0) / h)):
        inside = (ix + dx >= 0) & (ix + dx < m) & (iy + dy >= 0) & (iy + dy < m)
        rows.append(k[inside])
        cols.append(k[inside] + dx + m * dy)
        vals.append(coef[inside])
    A = _finish(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), m * m)
    return A, {"wx": wx, "wy": wy, "eps": eps, "h": h}


def one_way_convection_2d(m: int, rng: np.random.Generator) -> sp.csr_matrix:
    """A structurally nonsymmetric M-matrix on an m x m grid: diffusion in y
    (coupling to (x, y+-1) both ways) and pure upwind convection in x with no
    x-diffusion, so row (x, y) couples to (x-1, y) where the wind blows in +x
    (rows y < m/2) and to (x+1, y) where it blows in -x (rows y >= m/2), and
    never the other way. Wind speeds are U(0.5, 2) per node; the diagonal is
    2 + speed + 0.1, so the matrix is a strictly row diagonally dominant
    Z-matrix: it and every principal submatrix are nonsingular M-matrices,
    and Gaussian elimination without pivoting keeps that property in every
    Schur complement (positive pivots)."""
    k = np.arange(m * m)
    ix, iy = k % m, k // m
    c = rng.uniform(0.5, 2.0, size=m * m)
    east = iy < m // 2
    rows, cols, vals = [k], [k], [2.0 + c + 0.1]
    for dx, dy, coef, sel in ((-1, 0, -c, east), (1, 0, -c, ~east),
                              (0, -1, -np.ones(m * m), np.ones(m * m, dtype=bool)),
                              (0, 1, -np.ones(m * m), np.ones(m * m, dtype=bool))):
        inside = sel & (ix + dx >= 0) & (ix + dx < m) & (iy + dy >= 0) & (iy + dy < m)
        rows.append(k[inside])
        cols.append(k[inside] + dx + m * dy)
        vals.append(coef[inside])
    return _finish(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), m * m)


# --------------------------------------------------------------------------
# 2D Stokes, lid-driven cavity (saddle point)
# --------------------------------------------------------------------------

def stokes_cavity_2d(m: int, px: int, py: int, eps: float = 1e-2) -> tuple[sp.csr_matrix, np.ndarray, np.ndarray]:
    """Lid-driven cavity on the unit square with the staggered (MAC) finite
    differences of -Lap u + grad p = 0, div u = 0 on m x m cells, h = 1/m,
    in the symmetric saddle-point form

        K = [[A, G], [G^T, -eps I]],

    A the 5-point velocity Laplacians (1/h^2; the wall values enter through
    ghost values, the walls normal to a component eliminate it), G the
    pressure gradient (1/h) and G^T = -div; the small pressure block -eps I
    (pressure stabilization) fixes the constant pressure mode and makes K
    quasi-definite. Unknowns: u on the (m-1) x m interior vertical faces,
    then v on the m x (m-1) interior horizontal faces, then p on the m^2
    cells (velocities numbered first). b carries the moving lid (u = 1 on
    y = 1). The partition is px x py boxes of cells; a face belongs to the
    box of the cell to its left (u) or below (v).
    Returns (K, part, b)."""
    h = 1.0 / m
    nu, nv, npr = (m - 1) * m, m * (m - 1), m * m
    iu = lambda i, j: j * (m - 1) + i          # u face (i+1/2, j), i in [0, m-1)
    iv = lambda i, j: nu + j * m + i           # v face (i, j+1/2), j in [0, m-1)
    ip = lambda i, j: nu + nv + j * m + i      # cell (i, j)
    rows, cols, vals = [], [], []
    b = np.zeros(nu + nv + npr)
    d = 1.0 / (h * h)
    # u: neighbours along x are faces (the walls x = 0, 1 hold u = 0, no
    # ghost); along y the walls y = 0, 1 use ghost values u_g = 2 u_w - u
    I, J = np.meshgrid(np.arange(m - 1), np.arange(m), indexing="ij")
    I, J = I.ravel(), J.ravel()
    k = iu(I, J)
    diag = np.full(k.size, 4.0 * d)
    diag += np.where((J == 0) | (J == m - 1), d, 0.0)
    rows.append(k); cols.append(k); vals.append(diag)
    for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        ok = (I + di >= 0) & (I + di < m - 1) & (J + dj >= 0) & (J + dj < m)
        rows.append(k[ok]); cols.append(iu(I[ok] + di, J[ok] + dj)); vals.append(np.full(ok.sum(), -d))
    b[iu(I[J == m - 1], J[J == m - 1])] += 2.0 * d * 1.0  # lid u_w = 1
    # v: symmetric roles; all walls at rest
    I, J = np.meshgrid(np.arange(m), np.arange(m - 1), indexing="ij")
    I, J = I.ravel(), J.ravel()
    k = iv(I, J)
    diag = np.full(k.size, 4.0 * d)
    diag += np.where((I == 0) | (I == m - 1), d, 0.0)
    rows.append(k); cols.append(k); vals.append(diag)
    for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        ok = (I + di >= 0) & (I + di < m) & (J + dj >= 0) & (J + dj < m - 1)
        rows.append(k[ok]); cols.append(iv(I[ok] + di, J[ok] + dj)); vals.append(np.full(ok.sum(), -d))
    # gradient: (grad p)_u(i+1/2, j) = (p(i+1, j) - p(i, j)) / h, and v alike
    I, J = np.meshgrid(np.arange(m - 1), np.arange(m), indexing="ij")
    I, J = I.ravel(), J.ravel()
    for src, sign in ((ip(I + 1, J), 1.0), (ip(I, J), -1.0)):
        rows += [iu(I, J), src]; cols += [src, iu(I, J)]; vals += [np.full(I.size, sign / h)] * 2
    I, J = np.meshgrid(np.arange(m), np.arange(m - 1), indexing="ij")
    I, J = I.ravel(), J.ravel()
    for src, sign in ((ip(I, J + 1), 1.0), (ip(I, J), -1.0)):
        rows += [iv(I, J), src]; cols += [src, iv(I, J)]; vals += [np.full(I.size, sign / h)] * 2
    kp = np.arange(npr) + nu + nv
    rows.append(kp); cols.append(kp); vals.append(np.full(npr, -eps))
    K = _finish(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), nu + nv + npr)
    box = lambda i, j: (j * py // m) * px + (i * px // m)
    I, J = np.meshgrid(np.arange(m - 1), np.arange(m), indexing="ij")
    pu = np.empty(nu, dtype=np.int32); pu[iu(I.ravel(), J.ravel())] = box(I.ravel(), J.ravel())
    I, J = np.meshgrid(np.arange(m), np.arange(m - 1), indexing="ij")
    pv = np.empty(nv, dtype=np.int32); pv[iv(I.ravel(), J.ravel()) - nu] = box(I.ravel(), J.ravel())
    I, J = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    pp = np.empty(npr, dtype=np.int32); pp[ip(I.ravel(), J.ravel()) - nu - nv] = box(I.ravel(), J.ravel())
    return K, np.concatenate([pu, pv, pp]).astype(np.int32), b


# --------------------------------------------------------------------------
# 3D linear elasticity, trilinear hexahedra
# --------------------------------------------------------------------------

def _q1_stiffness(h: float, nu: float) -> np.ndarray:
    """24x24 stiffness of a cube element of side h, Young's modulus 1, with
    2x2x2 Gauss quadrature. Local node a = (ax, ay, az) in {0,1}^3 numbered
    ax + 2 ay + 4 az; dof 3a + component."""
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1.0 / (2 * (1 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2 * mu
    D[3:, 3:] = np.eye(3) * mu
    corners = np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], dtype=float)
    gp = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    K = np.zeros((24, 24))
    for qx in gp:
        for qy in gp:
            for qz in gp:
                q = np.array([qx, qy, qz])
                # d N_a / d xi_d on the reference cube [0,1]^3
                dN = np.zeros((8, 3))
                for a in range(8):
                    f = np.where(corners[a] == 1, q, 1 - q)
                    s = np.where(corners[a] == 1, 1.0, -1.0)
                    dN[a, 0] = s[0] * f[1] * f[2]
                    dN[a, 1] = f[0] * s[1] * f[2]
                    dN[a, 2] = f[0] * f[1] * s[2]
                dN /= h
                B = np.zeros((6, 24))
                for a in range(8):
                    gx, gy, gz = dN[a]
                    B[0, 3 * a + 0] = gx
                    B[1, 3 * a + 1] = gy
                    B[2, 3 * a + 2] = gz
                    B[3, 3 * a + 0] = gy
                    B[3, 3 * a + 1] = gx
                    B[4, 3 * a + 1] = gz
                    B[4, 3 * a + 2] = gy
                    B[5, 3 * a + 0] = gz
                    B[5, 3 * a + 2] = gx
                K += B.T @ D @ B * (h ** 3) / 8.0
    return K


def elasticity_q1_3d(nn: int, E_elem: np.ndarray, nu: float = 0.3) -> tuple[sp.csr_matrix, np.ndarray]:
    """Q1 linear elasticity on an nn^3-node unit-cube grid ((nn-1)^3
    elements, h = 1/(nn-1)), 3 dofs per node, nodes on the face x=0 clamped
    (their dofs removed). ``E_elem`` holds Young's modulus per element,
    shape (ne, ne, ne) indexed [z, y, x]. Returns (A, node_of_dof) where
    node_of_dof maps each kept dof to its grid node (x fastest)."""
    ne = nn - 1
    h = 1.0 / ne
    Ke = _q1_stiffness(h, nu)
    ez, ey, ex = np.meshgrid(np.arange(ne), np.arange(ne), np.arange(ne), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    Ee = E_elem.reshape(-1)
    nodes = np.stack([(ex + (a & 1)) + nn * (ey + ((a >> 1) & 1)) + nn * nn * (ez + ((a >> 2) & 1))
                      for a in range(8)], axis=1)  # (n_el, 8)
    dofs = (3 * nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 24)
    # keep only dofs of nodes with x > 0
    n_all = 3 * nn ** 3
    node_all = np.arange(nn ** 3)
    keep_node = (node_all % nn) > 0
    keep_dof = np.repeat(keep_node, 3)
    newid = -np.ones(n_all, dtype=np.int64)
    newid[keep_dof] = np.arange(int(keep_dof.sum()))
    ld = newid[dofs]  # (n_el, 24)
    rows = np.repeat(ld, 24, axis=1).ravel()
    cols = np.tile(ld, (1, 24)).ravel()
    vals = (Ee[:, None, None] * Ke[None, :, :]).reshape(-1)
    m = (rows >= 0) & (cols >= 0)
    n = int(keep_dof.sum())
    A = _finish(rows[m], cols[m], vals[m], n)
    node_of_dof = np.repeat(node_all[keep_node], 3)
    return A, node_of_dof


# --------------------------------------------------------------------------
# Partitions
# --------------------------------------------------------------------------

def box_partition_2d(nx: int, ny: int, px: int, py: int) -> np.ndarray:
    """Regular px x py boxes: part = (y // (ny/py)) * px + x // (nx/px)."""
    k = np.arange(nx * ny)
    x, y = k % nx, k // nx
    return ((y * py // ny) * px + (x * px // nx)).astype(np.int32)


def box_partition_3d(nx: int, ny: int, nz: int, px: int, py: int, pz: int,
                     x: np.ndarray, y: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Regular boxes on grid coordinates x, y, z (arrays over unknowns)."""
    return ((z * pz // nz) * (px * py) + (y * py // ny) * px + (x * px // nx)).astype(np.int32)


def rcb_partition(shape: tuple[int, ...], levels: int, rng: np.random.Generator,
                  ratio: tuple[float, float] = (0.3, 0.7)) -> np.ndarray:
    """Randomised recursive coordinate bisection of a grid of cells.

    ``shape`` is (nx, ny) or (nx, ny, nz) (x fastest in the numbering).
    Boxes are cut breadth-first, level by level; each box is cut across its
    longest side (ties broken towards x, then y) at
    lo + clamp(round(r * len), 1, len - 1) with r ~ U(ratio). The leaves of
    the last level, in breadth-first order, are the parts 0 .. 2^levels - 1.
    """
    dim = len(shape)
    boxes = [tuple((0, s) for s in shape)]
    for _ in range(levels):
        nxt = []
        for box in boxes:
            lens = [hi - lo for lo, hi in box]
            ax = int(np.argmax(lens))  # first maximum: x before y before z
            lo, hi = box[ax]
            ln = hi - lo
            r = rng.uniform(*ratio)
            cut = lo + int(min(max(round(r * ln), 1), ln - 1))
            left = list(box)
            right = list(box)
            left[ax] = (lo, cut)
            right[ax] = (cut, hi)
            nxt.append(tuple(left))
            nxt.append(tuple(right))
        boxes = nxt
    part = np.empty(shape[::-1], dtype=np.int32)  # indexed [z][y][x]
    for pid, box in enumerate(boxes):
        sl = tuple(slice(lo, hi) for lo, hi in box[::-1])
        part[sl] = pid
    if dim == 2:
        return part.reshape(-1)
    return part.reshape(-1)


def rhs(n: int, seed: int) -> np.ndarray:
    """b ~ N(0, 1) from PCG64(seed)."""
    return np.random.default_rng(seed).standard_normal(n)


# --------------------------------------------------------------------------
# The 7x7 example of the paper's notation section
# --------------------------------------------------------------------------

def worked_example_7x7() -> tuple[sp.csr_matrix, np.ndarray]:
    """The tridiagonal 7x7 matrix with entries 1..20 row by row and the two
    interior sets {1,2,3}, {4,5,6,7} (1-based) used in the paper's notation
    section (Section 2.1). Returned with 0-based numbering."""
    dense = np.zeros((7, 7))
    # the printed matrix skips the value 6: its third row reads 7, 8, 9
    entries = [(0, 0, 1), (0, 1, 2), (1, 0, 3), (1, 1, 4), (1, 2, 5), (2, 1, 7), (2, 2, 8),
               (2, 3, 9), (3, 2, 10), (3, 3, 11), (3, 4, 12), (4, 3, 13), (4, 4, 14),
               (4, 5, 15), (5, 4, 16), (5, 5, 17), (5, 6, 18), (6, 5, 19), (6, 6, 20)]
    for i, j, val in entries:
        dense[i, j] = val
    A = sp.csr_matrix(dense)
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    part = np.array([0, 0, 0, 1, 1, 1, 1], dtype=np.int32)
    return A, part


def layered_elasticity(nn: int, thick: int, phase: int) -> tuple[sp.csr_matrix, np.ndarray, int]:
    """Q1 elasticity on nn^3 nodes with Young's modulus in z-slabs of
    ``thick`` elements alternating 1 / 1e4 (shifted by ``phase``), nu = 0.3,
    face x = 0 clamped; partition into boxes of 6^3 nodes. Returns
    (A, part, n_parts)."""
    ne = nn - 1
    zc = np.arange(ne)
    layer = ((zc + phase) // thick) % 2
    E1d = np.where(layer == 0, 1.0, 1e4)
    E = np.broadcast_to(E1d[:, None, None], (ne, ne, ne)).copy()
    A, node_of_dof = elasticity_q1_3d(nn, E)
    x = node_of_dof % nn
    y = (node_of_dof // nn) % nn
    z = node_of_dof // (nn * nn)
    pb = max(1, nn // 6)
    part = box_partition_3d(nn, nn, nn, pb, pb, pb, x, y, z)
    return A, part, pb ** 3


def elasticity_training_instances(count: int, seed0: int = 100, nn: int = 48):
    """Seeded training instances for the warm-start network: the layered
    elasticity family with slab thickness uniform in {2..8} and a uniform
    phase. Yields (seed, thick, phase, A, part, n_parts)."""
    for j in range(count):
        rng = np.random.default_rng(seed0 + j)
        thick = int(rng.integers(2, 9))
        phase = int(rng.integers(0, thick))
        A, part, nparts = layered_elasticity(nn, thick, phase)
        yield seed0 + j, thick, phase, A, part, nparts


# --------------------------------------------------------------------------
# Benchmark configurations
# --------------------------------------------------------------------------

CONFIGS = {
    1: "2D 5-point Poisson 64x64, 4x4 boxes, overlap 1, nev 8 (SPD, PCG)",
    2: "2D high-contrast FV diffusion 1024x1024, 256 RCB parts, overlap 2, nev 16 (SPD, PCG)",
    3: "3D lognormal FV diffusion 128^3, 1024 RCB parts, overlap 1, nev 12 (SPD, PCG)",
    4: "3D Q1 elasticity 48^3 nodes, 512 boxes, overlap 1, nev 20 (SPD, PCG)",
    5: "2D upwind convection-diffusion 1024x1024, 256 boxes, overlap 2, nev 16 (general, FGMRES(30))",
    6: "2D Stokes lid-driven cavity, MAC 694x694 cells (1,443,520 unknowns), 256 boxes, overlap 6, nev 16 "
       "(symmetric indefinite saddle point, general path, RAS + deflated, FGMRES(30))",
}


def weak_scaling_poisson_3d(n_parts: int, seed: int = 0, per_part: float = 29791 / 2, overlap: int = 1,
                            nev: int = 12) -> Problem:
    """Weak-scaling instance: the constant-coefficient 3D Poisson problem (the
    7-point finite-volume Laplacian of kappa = 1 with Dirichlet faces) on a
    cube of side round((per_part * N)^(1/3)) cells, cut by exact recursive
    bisection into N = 2^L boxes of about per_part unknowns (the default
    gives the 31^3 grid with 2 parts and the 191^3 grid with 512). b is
    seeded as in make_config."""
    levels = int(round(np.log2(n_parts)))
    if 2 ** levels != n_parts:
        raise ValueError("n_parts must be a power of two")
    side = int(round((per_part * n_parts) ** (1.0 / 3.0)))
    A = fv_diffusion_3d(np.ones((side, side, side)))
    part = rcb_partition((side, side, side), levels, np.random.default_rng(seed), (0.5, 0.5))
    return Problem(f"weak{n_parts}", A, part, n_parts, overlap, nev, rhs(A.shape[0], seed + 1000), True,
                   {"grid": (side, side, side), "levels": levels})


def make_config(cfg: int, seed: int = 0, scale: int | None = None) -> Problem:
    """Build benchmark configuration ``cfg`` (1..6).

    ``scale`` shrinks the grid side (and the partition accordingly) for tests
    while keeping the structure: e.g. ``make_config(2, scale=128)`` is a
    128x128 instance with 2^(levels) parts scaled down.
    """
    rng = np.random.default_rng(seed)
    if cfg == 1:
        nx = scale or 64
        A = poisson_2d(nx)
        part = box_partition_2d(nx, nx, 4, 4)
        return Problem("cfg1", A, part, 16, 1, 8, rhs(A.shape[0], seed + 1000), True,
                       {"grid": (nx, nx)})
    if cfg == 2:
        nx = scale or 1024
        levels = 8 if scale is None else max(2, int(round(8 + 2 * np.log2(nx / 1024))))
        kappa = high_contrast_kappa_2d(nx, nx, rng)
        A = fv_diffusion_2d(kappa)
        part = rcb_partition((nx, nx), levels, rng, (0.3, 0.7))
        return Problem("cfg2", A, part, 2 ** levels, 2, 16, rhs(A.shape[0], seed + 1000), True,
                       {"grid": (nx, nx), "levels": levels})
    if cfg == 3:
        nx = scale or 128
        levels = 10 if scale is None else max(2, int(round(10 + 3 * np.log2(nx / 128))))
        kappa = lognormal_kappa_3d(nx, rng)
        A = fv_diffusion_3d(kappa)
        part = rcb_partition((nx, nx, nx), levels, rng, (0.45, 0.55))
        return Problem("cfg3", A, part, 2 ** levels, 1, 12, rhs(A.shape[0], seed + 1000), True,
                       {"grid": (nx, nx, nx), "levels": levels})
    if cfg == 4:
        nn = scale or 48
        A, part, nparts = layered_elasticity(nn, 4, 0)
        return Problem("cfg4", A, part, nparts, 1, 20, rhs(A.shape[0], seed + 1000), True,
                       {"nodes": nn, "E_layers": (4, 0)})
    if cfg == 5:
        m = scale or 1024
        A, meta = convdiff_2d(m, rng)
        p = 16 if scale is None else max(2, m // 64)
        part = box_partition_2d(m, m, p, p)
        return Problem("cfg5", A, part, p * p, 2, 16, rhs(A.shape[0], seed + 1000), False,
                       {"grid": (m, m)})
    if cfg == 6:
        # the paper's 2D lid-driven cavity has 1,444,003 Taylor-Hood unknowns;
        # 694^2 MAC cells give 1,443,520. b is the lid (deterministic).
        m = scale or 694
        p = 16 if scale is None else max(2, m // 43)
        K, part, b = stokes_cavity_2d(m, p, p)
        return Problem("cfg6", K, part, p * p, 6, 16, b, False, {"grid": (m, m), "saddle_point": True})
    raise ValueError(f"unknown configuration {cfg}")
