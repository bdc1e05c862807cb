// Galerkin coarse operator A_00 = R_0 A R_0^T = Z^T A Z (Section 4.1), its
// FP64 factorization, and the coarse correction R_0^T A_00^{-1} R_0 r of the
// apply.
//
// Z is block-diagonal over the nonoverlapping partition (D_i is zero outside
// I_i), so block (p, q) of Z^T A Z is nonzero only for subdomains p, q that
// are adjacent in graph(A). For each p the rows I_p of A Z restricted to the
// columns of p's neighbours are formed by a row-owned SpMM (deterministic),
// then the block row Z_p^T (A Z)_{I_p, .} is one MFMA GEMM.
#include <algorithm>

#include "batched.hpp"
#include "kernels.hpp"

namespace tls {

namespace {

__global__ void k_adjacency(int n, const int* __restrict__ rp, const int* __restrict__ ci, const int* __restrict__ part,
                            int N, uint8_t* adj) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  int p = part[g];
  for (int j = rp[g]; j < rp[g + 1]; j++) adj[(size_t)p * N + part[ci[j]]] = 1;
}

// W_p[ipos(g) + (slotoff + b) * nI_p] = sum_{c in row g, part c = q} A_gc Z_q[ipos(c), b]
__global__ void k_az(int n, const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ val,
                     const int* __restrict__ part, const int* __restrict__ ipos, const int* __restrict__ nI,
                     const int* __restrict__ adj_ptr, const int* __restrict__ adj_q, const int* __restrict__ adj_col,
                     const int64_t* __restrict__ woff, const int* __restrict__ kz, const int64_t* __restrict__ zoff,
                     const double* __restrict__ Z, double* W) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int p = part[g];
  const int j = ipos[g];
  const int nIp = nI[p];
  double* Wp = W + woff[p];
  for (int e = rp[g]; e < rp[g + 1]; e++) {
    const int c = ci[e];
    const int q = part[c];
    const int kq = kz[q];
    if (kq == 0) continue;
    int lo = adj_ptr[p], hi = adj_ptr[p + 1] - 1;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (adj_q[mid] < q)
        lo = mid + 1;
      else
        hi = mid;
    }
    const int co = adj_col[lo];
    const double a = val[e];
    const double* Zq = Z + zoff[q] + ipos[c];
    const int nIq = nI[q];
    for (int b = 0; b < kq; b++) Wp[j + (int64_t)(co + b) * nIp] += a * Zq[(int64_t)b * nIq];
  }
}

// scatter block row p (k_p x ncols) into the lower tile storage of A_0
__global__ void k_scatter_a0(int N, const int* __restrict__ kz, const int* __restrict__ zcol,
                             const int* __restrict__ adj_ptr, const int* __restrict__ adj_q,
                             const int* __restrict__ adj_col, const int64_t* __restrict__ boff, const double* __restrict__ B,
                             int nt0, int kind, double* A0) {
  const int p = blockIdx.x;
  const int kp = kz[p];
  if (kp == 0) return;
  for (int s = adj_ptr[p]; s < adj_ptr[p + 1]; s++) {
    const int q = adj_q[s];
    const int kq = kz[q];
    const int co = adj_col[s];
    for (int e = threadIdx.x; e < kp * kq; e += blockDim.x) {
      int a = e % kp, b = e / kp;
      int R = zcol[p] + a, Cc = zcol[q] + b;
      if (kind == 1 || R >= Cc) *elem_ptr(A0, kind, nt0, R, Cc) = B[boff[p] + a + (int64_t)(co + b) * kp];
    }
  }
}

__global__ void k_pad_identity0(int nC, int M0, int nt0, int kind, double* A0) {
  for (int a = nC + blockIdx.x * blockDim.x + threadIdx.x; a < M0; a += gridDim.x * blockDim.x)
    *elem_ptr(A0, kind, nt0, a, a) = 1.0;
}

// y0[zcol_p + a] = sum_{j < nI_p} Z_p[j, a] r[I_p[j]]
__global__ void __launch_bounds__(256) k_restrict(const int* __restrict__ kz, const int* __restrict__ zcol,
                                                  const int* __restrict__ nI, const int* __restrict__ sub_ptr,
                                                  const int* __restrict__ sub_idx, const int64_t* __restrict__ zoff,
                                                  const double* __restrict__ Z, const double* __restrict__ r,
                                                  double* y0, const int* __restrict__ done) {
  if (*done) return;
  const int p = blockIdx.y, a = blockIdx.x;
  if (a >= kz[p]) return;
  const int n = nI[p];
  const double* z = Z + zoff[p] + (int64_t)a * n;
  const int* idx = sub_idx + sub_ptr[p];
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) s += z[j] * r[idx[j]];
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) y0[zcol[p] + a] = red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------------------
// LU with partial pivoting of A_0 for general A. The coarse operator of an
// indefinite or nonsymmetric A (for instance a saddle-point matrix) can
// have arbitrarily small leading minors, so its rows are pivoted: P A_0 =
// L U by right-looking panels of 64 columns on a dense column-major copy D
// (leading dimension M0), then L and U go back into the tile storage with
// the inverses of their diagonal tiles, and every coarse solve permutes its
// right-hand side first.
// ---------------------------------------------------------------------------
// Copy between the full tile storage (tile (r, c) at r nt + c) and the
// dense column-major matrix: to_dense = 1 tiles -> D, 0 D -> tiles.
__global__ void k_tiles_dense(int nt, int64_t M0, double* tiles, double* D, int to_dense) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < M0 * M0; x += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(x % M0), b = (int)(x / M0);
    const int64_t t = ((int64_t)(a / TS) * nt + b / TS) * TS2 + (b % TS) * TS + a % TS;
    if (to_dense)
      D[x] = tiles[t];
    else
      tiles[t] = D[x];
  }
}

// Columns [j0, j1) of D, rows [j0, n), one workgroup: in groups of 8
// columns, each column's pivot search, the row interchange across the whole
// panel, the multipliers and the update of the rest of its group; then the
// group's rows of the later panel columns (unit-lower solve) and the rank-8
// update of the rows below.
constexpr int LU_PANEL_THREADS = 1024;
constexpr int LU_GROUP = 8;

__global__ void __launch_bounds__(LU_PANEL_THREADS) k_lu_panel(int n, int64_t ld, int j0, int j1, double* D, int* piv,
                                                               int* err) {
  constexpr int NW = LU_PANEL_THREADS / 64;
  __shared__ double s_v[NW];
  __shared__ int s_i[NW];
  __shared__ int s_p;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int c0 = j0; c0 < j1; c0 += LU_GROUP) {
    const int c1 = min(c0 + LU_GROUP, j1);
    for (int j = c0; j < c1; j++) {
      double best = -1.0;
      int bi = j;
      for (int i = j + tid; i < n; i += LU_PANEL_THREADS) {
        const double v = fabs(D[i + j * ld]);
        if (v > best) {
          best = v;
          bi = i;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ov > best || (ov == best && oi < bi)) {
          best = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        s_v[wave] = best;
        s_i[wave] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        double bv = s_v[0];
        int p = s_i[0];
        for (int w = 1; w < NW; w++)
          if (s_v[w] > bv || (s_v[w] == bv && s_i[w] < p)) {
            bv = s_v[w];
            p = s_i[w];
          }
        s_p = p;
        piv[j] = p;
      }
      __syncthreads();
      const int p = s_p;
      if (p != j && tid < j1 - j0) {
        const int64_t c = (int64_t)(j0 + tid) * ld;
        const double t = D[j + c];
        D[j + c] = D[p + c];
        D[p + c] = t;
      }
      __syncthreads();
      double d = D[j + j * ld];
      if (!(fabs(d) > 0.0) || !isfinite(d)) {
        if (tid == 0) atomicOr(err, ERR_PIVOT);
        d = 1.0;
      }
      const double inv = 1.0 / d;
      for (int i = j + 1 + tid; i < n; i += LU_PANEL_THREADS) {
        const double l = D[i + j * ld] * inv;
        D[i + j * ld] = l;
        for (int c = j + 1; c < c1; c++) D[i + c * ld] -= l * D[j + c * ld];
      }
      __syncthreads();
    }
    if (c1 >= j1) break;
    // rows [c0, c1) of the columns [c1, j1): unit-lower solve with the group's L
    if (tid < j1 - c1) {
      double* Dc = D + (int64_t)(c1 + tid) * ld;
      for (int r = c0 + 1; r < c1; r++) {
        double acc = Dc[r];
        for (int k = c0; k < r; k++) acc -= D[r + (int64_t)k * ld] * Dc[k];
        Dc[r] = acc;
      }
    }
    __syncthreads();
    // rows [c1, n) of the columns [c1, j1): minus L_(rows, group) U_(group, cols)
    for (int i = c1 + tid; i < n; i += LU_PANEL_THREADS) {
      double l[LU_GROUP];
#pragma unroll
      for (int k = 0; k < LU_GROUP; k++) l[k] = c0 + k < c1 ? D[i + (int64_t)(c0 + k) * ld] : 0.0;
      for (int c = c1; c < j1; c++) {
        double acc = D[i + (int64_t)c * ld];
#pragma unroll
        for (int k = 0; k < LU_GROUP; k++)
          if (c0 + k < c1) acc -= l[k] * D[c0 + k + (int64_t)c * ld];
        D[i + (int64_t)c * ld] = acc;
      }
    }
    __syncthreads();
  }
}

// The same panel factorization with the group's columns held in registers
// (rows c0 + t + 1024 q, q < R, by thread t) for n - j0 <= 1024 R, R <= 4 (no
// spills at 1024 threads per workgroup): the pivot
// search, the row interchange and the updates inside the group then cost no
// global-memory round trips. Same operations in the same order as
// k_lu_panel.
template <int R>
__global__ void __launch_bounds__(LU_PANEL_THREADS) k_lu_panel_reg(int n, int64_t ld, int j0, int j1, double* D,
                                                                   int* piv, int* err) {
  constexpr int NT = LU_PANEL_THREADS, NW = NT / 64, G = LU_GROUP;
  __shared__ double s_v[NW];
  __shared__ int s_i[NW];
  __shared__ int s_p;
  __shared__ double s_rj[G], s_rp[G];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int c0 = j0; c0 < j1; c0 += G) {
    const int c1 = min(c0 + G, j1), g = c1 - c0;
    double x[R][G];
#pragma unroll
    for (int q = 0; q < R; q++) {
      const int r = c0 + tid + NT * q;
#pragma unroll
      for (int k = 0; k < G; k++) x[q][k] = (r < n && k < g) ? D[r + (int64_t)(c0 + k) * ld] : 0.0;
    }
#pragma unroll
    for (int jj = 0; jj < G; jj++) {
      if (jj >= g) break;
      const int j = c0 + jj;
      double best = -1.0;
      int bi = j;
#pragma unroll
      for (int q = 0; q < R; q++) {
        const int r = c0 + tid + NT * q;
        const double v = fabs(x[q][jj]);
        if (r >= j && r < n && v > best) {
          best = v;
          bi = r;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ov > best || (ov == best && oi < bi)) {
          best = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        s_v[wave] = best;
        s_i[wave] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        double bv = s_v[0];
        int p = s_i[0];
        for (int w = 1; w < NW; w++)
          if (s_v[w] > bv || (s_v[w] == bv && s_i[w] < p)) {
            bv = s_v[w];
            p = s_i[w];
          }
        s_p = p;
        piv[j] = p;
      }
      __syncthreads();
      const int p = s_p;
      // the owners of rows j and p publish their group rows
#pragma unroll
      for (int q = 0; q < R; q++) {
        const int r = c0 + tid + NT * q;
        if (r == j)
#pragma unroll
          for (int k = 0; k < G; k++) s_rj[k] = x[q][k];
        if (r == p)
#pragma unroll
          for (int k = 0; k < G; k++) s_rp[k] = x[q][k];
      }
      // the interchange in the panel columns outside the group (global)
      if (p != j && tid < j1 - j0 && (j0 + tid < c0 || j0 + tid >= c1)) {
        const int64_t c = (int64_t)(j0 + tid) * ld;
        const double t = D[j + c];
        D[j + c] = D[p + c];
        D[p + c] = t;
      }
      __syncthreads();
      // new row j = old row p, new row p = old row j
#pragma unroll
      for (int q = 0; q < R; q++) {
        const int r = c0 + tid + NT * q;
        if (r == j)
#pragma unroll
          for (int k = 0; k < G; k++) x[q][k] = s_rp[k];
        if (r == p && p != j)
#pragma unroll
          for (int k = 0; k < G; k++) x[q][k] = s_rj[k];
      }
      double d = s_rp[jj];
      if (!(fabs(d) > 0.0) || !isfinite(d)) {
        if (tid == 0) atomicOr(err, ERR_PIVOT);
        d = 1.0;
      }
      const double inv = 1.0 / d;
#pragma unroll
      for (int q = 0; q < R; q++) {
        const int r = c0 + tid + NT * q;
        if (r > j && r < n) {
          const double l = x[q][jj] * inv;
          x[q][jj] = l;
#pragma unroll
          for (int k = jj + 1; k < G; k++)
            if (k < g) x[q][k] -= l * s_rp[k];
        }
      }
      __syncthreads();  // s_rj / s_rp are reused by the next column
    }
#pragma unroll
    for (int q = 0; q < R; q++) {
      const int r = c0 + tid + NT * q;
      if (r < n)
#pragma unroll
        for (int k = 0; k < G; k++)
          if (k < g) D[r + (int64_t)(c0 + k) * ld] = x[q][k];
    }
    __syncthreads();
    if (c1 >= j1) break;
    // rows [c0, c1) of the columns [c1, j1): unit-lower solve with the group's L
    if (tid < j1 - c1) {
      double* Dc = D + (int64_t)(c1 + tid) * ld;
      for (int r = c0 + 1; r < c1; r++) {
        double acc = Dc[r];
        for (int k = c0; k < r; k++) acc -= D[r + (int64_t)k * ld] * Dc[k];
        Dc[r] = acc;
      }
    }
    __syncthreads();
    // rows [c1, n) of the columns [c1, j1): minus L_(rows, group) U_(group, cols)
#pragma unroll
    for (int q = 0; q < R; q++) {
      const int i = c0 + tid + NT * q;
      if (i >= c1 && i < n)
        for (int c = c1; c < j1; c++) {
          double acc = D[i + (int64_t)c * ld];
#pragma unroll
          for (int k = 0; k < G; k++)
            if (c0 + k < c1) acc -= x[q][k] * D[c0 + k + (int64_t)c * ld];
          D[i + (int64_t)c * ld] = acc;
        }
    }
    __syncthreads();
  }
}

// The panel's interchanges applied, in order, to every column outside it.
__global__ void k_lu_swap_rest(int n, int64_t ld, int j0, int j1, const int* __restrict__ piv, double* D) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= n || (col >= j0 && col < j1)) return;
  double* Dc = D + (int64_t)col * ld;
  for (int j = j0; j < j1; j++) {
    const int p = piv[j];
    if (p != j) {
      const double t = Dc[j];
      Dc[j] = Dc[p];
      Dc[p] = t;
    }
  }
}

// U_12 = L_11^{-1} A_12 for the columns [j1, n) (L_11 unit lower, rows and
// columns [j0, j1), j1 - j0 <= 64): one workgroup of 64 per 64 columns, the
// blocks staged in LDS, thread t solving column t.
__global__ void __launch_bounds__(64) k_lu_trsm_row(int n, int64_t ld, int j0, int j1, double* D) {
  constexpr int P = TS + 1;
  __shared__ double Ls[TS * P];
  __shared__ double Xs[TS * P];
  const int w = j1 - j0, t = threadIdx.x;
  const int cb = j1 + blockIdx.x * TS;
  const int nc = min(TS, n - cb);
  for (int c = 0; c < w; c++) Ls[t + c * P] = t < w ? D[j0 + t + (int64_t)(j0 + c) * ld] : 0.0;
  for (int c = 0; c < nc; c++) Xs[t + c * P] = t < w ? D[j0 + t + (int64_t)(cb + c) * ld] : 0.0;
  __syncthreads();
  if (t < nc) {
    for (int r = 1; r < w; r++) {
      double acc = Xs[r + t * P];
      for (int k = 0; k < r; k++) acc -= Ls[r + k * P] * Xs[k + t * P];
      Xs[r + t * P] = acc;
    }
  }
  __syncthreads();
  for (int c = 0; c < nc; c++)
    if (t < w) D[j0 + t + (int64_t)(cb + c) * ld] = Xs[t + c * P];
}

// Inverses of the diagonal tiles of the LU factor in the layout the
// substitutions read: strictly below the diagonal the unit-lower L_kk^{-1},
// on and above it U_kk^{-1}. One workgroup of 64 per tile.
__global__ void __launch_bounds__(64) k_lu_tile_inverses(int nt, const double* __restrict__ tiles, double* dinv) {
  constexpr int L1 = TS + 1;
  __shared__ double Ls[TS * L1];
  __shared__ double Xs[TS * L1];
  const int k = blockIdx.x, j = threadIdx.x;
  const double* t = tiles + ((int64_t)k * nt + k) * TS2;
  for (int b = 0; b < TS; b++) Ls[j + b * L1] = t[b * TS + j];
  __syncthreads();
  double* out = dinv + (int64_t)k * TS2 + (int64_t)j * TS;
  for (int r = 0; r < TS; r++) {
    double v = (r == j) ? 1.0 : 0.0;
    for (int l = 0; l < r; l++) v -= Ls[r + l * L1] * Xs[l * L1 + j];
    Xs[r * L1 + j] = r < j ? 0.0 : v;
    if (r > j) out[r] = v;
  }
  for (int r = TS - 1; r >= 0; r--) {
    double v = (r == j) ? 1.0 : 0.0;
    for (int l = r + 1; l < TS; l++) v -= Ls[r + l * L1] * Xs[l * L1 + j];
    v = r > j ? 0.0 : v / Ls[r + r * L1];
    Xs[r * L1 + j] = v;
    if (r <= j) out[r] = v;
  }
}

// dst[i] = src[perm[i]] (skipped once the Krylov loop has converged)
__global__ void k_permute(int n, const int* __restrict__ perm, const double* __restrict__ src, double* dst,
                          const int* __restrict__ done) {
  if (done && *done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

__global__ void k_copy_vec(int n, const double* __restrict__ src, double* dst, const int* __restrict__ done) {
  if (done && *done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace

// P A_0 = L U (see the kernels above); A_0's tiles are overwritten by L and
// U, dinv0 receives the inverses of the diagonal tiles, perm0 the row order.
static void factor_coarse_lu_pivoted(tls_ctx* c) {
  hipStream_t s = c->stream;
  const int n = c->M0, nt = c->nt0;
  const int64_t ld = n;
  DBuf<double> D;
  DBuf<int> piv;
  D.alloc((size_t)n * n);
  piv.alloc(n);
  // the trailing-update descriptors of every panel, on the device before
  // the loop, so that the panels run back to back without host waits
  const int npan = div_up(n, TS);
  std::vector<GemmPlan> plans(npan);
  for (int k = 0; k + 1 < npan; k++) {
    const int j0 = k * TS, j1 = j0 + TS;
    gemm_plan(plans[k], {GemmDesc{n - j1, n - j1, j1 - j0, n, n, j1 + (int64_t)j0 * ld, j0 + (int64_t)j1 * ld,
                                  j1 + (int64_t)j1 * ld, ld}},
              s);
  }
  hipLaunchKernelGGL(k_tiles_dense, dim3(2048), dim3(256), 0, s, nt, (int64_t)n, c->A0.p, D.p, 1);
  TLS_LAUNCH_CHECK();
  for (int k = 0; k < npan; k++) {
    const int j0 = k * TS, j1 = std::min(j0 + TS, n);
    const int rows = n - j0;
    if (rows <= 2 * LU_PANEL_THREADS)
      hipLaunchKernelGGL(k_lu_panel_reg<2>, dim3(1), dim3(LU_PANEL_THREADS), 0, s, n, ld, j0, j1, D.p, piv.p,
                         c->errflag.p);
    else if (rows <= 4 * LU_PANEL_THREADS)
      hipLaunchKernelGGL(k_lu_panel_reg<4>, dim3(1), dim3(LU_PANEL_THREADS), 0, s, n, ld, j0, j1, D.p, piv.p,
                         c->errflag.p);
    else  // more rows than 4 per thread would not fit the registers of a 1024-thread workgroup
      hipLaunchKernelGGL(k_lu_panel, dim3(1), dim3(LU_PANEL_THREADS), 0, s, n, ld, j0, j1, D.p, piv.p, c->errflag.p);
    hipLaunchKernelGGL(k_lu_swap_rest, dim3(div_up(n, 256)), dim3(256), 0, s, n, ld, j0, j1, piv.p, D.p);
    TLS_LAUNCH_CHECK();
    if (j1 < n) {
      hipLaunchKernelGGL(k_lu_trsm_row, dim3(div_up(n - j1, TS)), dim3(64), 0, s, n, ld, j0, j1, D.p);
      TLS_LAUNCH_CHECK();
      gemm_run<double>(s, plans[k], false, false, D.p, D.p, D.p, -1.0, 1.0);
    }
  }
  hipLaunchKernelGGL(k_tiles_dense, dim3(2048), dim3(256), 0, s, nt, (int64_t)n, c->A0.p, D.p, 0);
  hipLaunchKernelGGL(k_lu_tile_inverses, dim3(nt), dim3(64), 0, s, nt, c->A0.p, c->dinv0.p);
  TLS_LAUNCH_CHECK();
  // the interchanges in order give the row order of P
  const std::vector<int> hp = download(piv.p, n, s);
  std::vector<int> perm(n);
  for (int i = 0; i < n; i++) perm[i] = i;
  for (int j = 0; j < n; j++) std::swap(perm[j], perm[hp[j]]);
  c->perm0.upload(perm, s);
  c->y0t.alloc(n);
  TLS_HIP(hipStreamSynchronize(s));
}

void build_coarse_operator(tls_ctx* c) {
  hipStream_t s = c->stream;
  const int N = c->N;
  if (c->nC == 0) {
    c->nnz0 = 0;
    return;
  }
  std::vector<int> kz(N);
  for (int i = 0; i < N; i++) kz[i] = c->h_zcol[i + 1] - c->h_zcol[i];
  // subdomain adjacency
  DBuf<uint8_t> adj;
  adj.alloc((size_t)N * N);
  TLS_HIP(hipMemsetAsync(adj.p, 0, (size_t)N * N, s));
  hipLaunchKernelGGL(k_adjacency, dim3(div_up(c->n, 256)), dim3(256), 0, s, c->n, c->row_ptr.p, c->col_idx.p,
                     c->part.p, N, adj.p);
  TLS_LAUNCH_CHECK();
  auto h_adj = download(adj.p, (size_t)N * N, s);
  std::vector<int> adj_ptr(N + 1, 0), adj_q, adj_col;
  std::vector<int64_t> woff(N + 1, 0), boff(N + 1, 0);
  int64_t nnz0 = 0;
  for (int p = 0; p < N; p++) {
    int col = 0;
    for (int q = 0; q < N; q++)
      if (h_adj[(size_t)p * N + q] && kz[q] > 0) {
        adj_q.push_back(q);
        adj_col.push_back(col);
        col += kz[q];
      }
    adj_ptr[p + 1] = (int)adj_q.size();
    woff[p + 1] = woff[p] + (int64_t)c->h_nI[p] * col;
    boff[p + 1] = boff[p] + (int64_t)kz[p] * col;
    nnz0 += (int64_t)kz[p] * col;
  }
  c->nnz0 = nnz0;
  DBuf<int> d_adj_ptr, d_adj_q, d_adj_col, d_kz;
  DBuf<int64_t> d_woff, d_boff;
  d_adj_ptr.upload(adj_ptr, s);
  d_adj_q.upload(adj_q, s);
  d_adj_col.upload(adj_col, s);
  d_kz.upload(kz, s);
  d_woff.upload(woff, s);
  d_boff.upload(boff, s);
  DBuf<double> W, B;
  W.alloc(woff[N]);
  B.alloc(boff[N]);
  TLS_HIP(hipMemsetAsync(W.p, 0, sizeof(double) * woff[N], s));
  hipLaunchKernelGGL(k_az, dim3(div_up(c->n, 256)), dim3(256), 0, s, c->n, c->row_ptr.p, c->col_idx.p, c->val.p,
                     c->part.p, c->ipos.p, c->d_nI.p, d_adj_ptr.p, d_adj_q.p, d_adj_col.p, d_woff.p, d_kz.p,
                     c->zoff.p, c->Z.p, W.p);
  TLS_LAUNCH_CHECK();
  // block rows Z_p^T W_p (MFMA fp64)
  std::vector<GemmDesc> gd;
  for (int p = 0; p < N; p++) {
    int ncols = 0;
    for (int sidx = adj_ptr[p]; sidx < adj_ptr[p + 1]; sidx++) ncols += kz[adj_q[sidx]];
    if (kz[p] == 0 || ncols == 0) continue;
    gd.push_back(GemmDesc{kz[p], ncols, c->h_nI[p], c->h_nI[p], c->h_nI[p], c->h_zoff[p], woff[p], boff[p],
                          (int64_t)kz[p]});
  }
  batched_gemm<double>(s, gd, true, false, c->Z.p, W.p, B.p, 1.0, 0.0);
  W.release();
  // tile storage of A_0
  c->M0 = div_up(c->nC, TS) * TS;
  c->nt0 = c->M0 / TS;
  const int64_t a0_elems = tiles_of(c->kind, c->nt0) * TS2;
  c->A0.alloc(a0_elems);
  TLS_HIP(hipMemsetAsync(c->A0.p, 0, sizeof(double) * a0_elems, s));
  hipLaunchKernelGGL(k_scatter_a0, dim3(N), dim3(256), 0, s, N, d_kz.p, c->zcol.p, d_adj_ptr.p, d_adj_q.p,
                     d_adj_col.p, d_boff.p, B.p, c->nt0, c->kind, c->A0.p);
  hipLaunchKernelGGL(k_pad_identity0, dim3(1), dim3(64), 0, s, c->nC, c->M0, c->nt0, c->kind, c->A0.p);
  TLS_LAUNCH_CHECK();
  TLS_HIP(hipStreamSynchronize(s));
  c->kz_dev.upload(kz, s);
  // single-matrix layout for the coarse factor and solves
  std::vector<int> one_m{c->nC}, one_nt{c->nt0};
  std::vector<int64_t> zero64{0, a0_elems}, voff{0, c->M0}, toff{0, c->nt0};
  c->one_m.upload(one_m, s);
  c->one_nI.upload(one_m, s);
  c->one_nP.upload(one_m, s);
  c->one_nt.upload(one_nt, s);
  c->one_foff.upload(zero64, s);
  c->one_voff.upload(voff, s);
  c->one_toff.upload(toff, s);
  c->A0_orig.alloc(a0_elems);
  TLS_HIP(hipMemcpyAsync(c->A0_orig.p, c->A0.p, sizeof(double) * a0_elems, hipMemcpyDeviceToDevice, s));
  TLS_HIP(hipMemsetAsync(c->errflag.p, 0, sizeof(int), s));
  c->dinv0.alloc((size_t)c->nt0 * TS2);
  if (c->kind == 0)
    factor_tiles_f64(s, 1, one_nt, c->layout0(), c->A0.p, c->dinv0.p, c->errflag.p);
  else
    factor_coarse_lu_pivoted(c);
  if (download(c->errflag.p, 1, s)[0] & ERR_PIVOT) {
    if (c->kind == 0) fail(TLS_E_NOT_SPD, "coarse operator Z^T A Z is not positive definite");
    fail(TLS_E_SINGULAR, "zero pivot in the LU factorization of the coarse operator Z^T A Z");
  }
  if (c->kind == 0 && c->opt.local_inverse) {
    // explicit A_0^{-1}: the coarse solve becomes one streaming product
    // instead of two chains of nt0 dependent block rows
    form_inverse_f64(s, 1, one_nt, c->layout0(), c->A0.p, c->dinv0.p);
    // blocks of 4 x 4 tiles: a single matrix needs more workgroups to
    // stream at full rate next to the local products
    build_symv_work(c->inv0_work, s, 1, one_nt, std::vector<int64_t>{0}, std::vector<int64_t>{0}, false, 4);
    c->inv0_formed = true;
  }
  build_plan(c->plan0_fwd, false, one_nt, toff, 1, s);
  build_plan(c->plan0_bwd, true, one_nt, toff, 1, s);
  c->counters0.alloc(4);
  c->y0.alloc(c->M0);
  TLS_HIP(hipMemsetAsync(c->counters0.p, 0, sizeof(int) * 4, s));
  TLS_HIP(hipMemsetAsync(c->y0.p, 0, sizeof(double) * c->M0, s));
  TLS_HIP(hipStreamSynchronize(s));
}

void coarse_restrict(tls_ctx* c, const double* r, const int* done) {
  if (c->nC == 0) return;
  int kmax = 0;
  for (int i = 0; i < c->N; i++) kmax = std::max(kmax, c->h_zcol[i + 1] - c->h_zcol[i]);
  hipLaunchKernelGGL(k_restrict, dim3(kmax, c->N), dim3(256), 0, c->stream, c->kz_dev.p, c->zcol.p, c->d_nI.p,
                     c->sub_ptr.p, c->sub_idx.p, c->zoff.p, c->Z.p, r, c->y0.p, done);
  TLS_LAUNCH_CHECK();
}

void coarse_solve(tls_ctx* c, const int* done) {
  if (c->nC == 0) return;
  hipStream_t s = c->stream;
  if (c->inv0_formed) {
    symv_solve_f64(s, c->inv0_work, c->A0.p, c->y0.p, done);
    return;
  }
  if (c->kind == 1) {
    // y0 <- P y0 before L U y = P r
    hipLaunchKernelGGL(k_permute, dim3(div_up(c->M0, 256)), dim3(256), 0, s, c->M0, c->perm0.p, c->y0.p, c->y0t.p,
                       done);
    hipLaunchKernelGGL(k_copy_vec, dim3(div_up(c->M0, 256)), dim3(256), 0, s, c->M0, c->y0t.p, c->y0.p, done);
    TLS_LAUNCH_CHECK();
  }
  solve_begin(s, c->counters0.p, done);
  const int grid = std::min(c->plan0_fwd.ntasks, 512);
  trsv_f64(s, c->kind == 0 ? 0 : 2, c->plan0_fwd, c->counters0.p + 0, c->counters0.p + 2, c->layout0(), c->A0.p,
           c->dinv0.p, c->y0.p, c->errflag.p, done, grid);
  trsv_f64(s, c->kind == 0 ? 1 : 3, c->plan0_bwd, c->counters0.p + 1, c->counters0.p + 2, c->layout0(), c->A0.p,
           c->dinv0.p, c->y0.p, c->errflag.p, done, grid);
}

}  // namespace tls
