// Local matrices A_ii = R_i A R_i^T (Section 2.3), their batched dense
// factorization, and the batched triangular solves that apply A_ii^{-1}
// (eq. onelevelasm) - the HBM-bound hot loop of every preconditioner apply.
//
// Factorization: right-looking tiled Cholesky over all subdomains at once.
// Step k factors the diagonal tile (k,k) of every subdomain with nt_i > k
// (one workgroup each, in LDS), solves the tiles below it (one wave per
// tile), then updates every trailing lower tile with a 64x64x64 MFMA
// product (one workgroup per tile). Subdomains are sorted by size, so the
// active set at step k is a prefix and tile indices are decoded from
// per-step prefix tables.
//
// Triangular solves: one persistent kernel per direction. A task is one
// 64-row block of one subdomain; tasks are handed out in dependency order by
// an atomic counter, a task waits (bounded spin) on per-block ready flags of
// the blocks it reads, streams its tiles through a 256-thread GEMV and
// finishes with a one-wave substitution on the diagonal tile.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "kernels.hpp"
#include "mfma.hpp"

namespace tls {

namespace {

// ---------------------------------------------------------------------------
// Gather
// ---------------------------------------------------------------------------

template <class T>
__global__ void k_pad_identity(int N, LocalLayout lay, int kind, T* fac) {
  int i = blockIdx.x;
  int m = lay.m[i], nt = lay.nt[i];
  T* base = fac + lay.foff[i];
  for (int a = m + threadIdx.x; a < nt * TS; a += blockDim.x) *elem_ptr_l(base, lay, i, kind, nt, a, a) = T(1);
}

// scale[voff_i + a] = 1 / sqrt(A[g][g]) for the Jacobi-scaled variant
__global__ void k_jacobi_scale(int total, const int* __restrict__ sub_idx, const int* __restrict__ sub_of_pos,
                               const int* __restrict__ sub_ptr, const int64_t* __restrict__ voff,
                               const int* __restrict__ rp, const int* __restrict__ ci,
                               const double* __restrict__ val, double* scale, int* err) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  int g = sub_idx[p];
  int i = sub_of_pos[p];
  double d = 0.0;
  for (int j = rp[g]; j < rp[g + 1]; j++)
    if (ci[j] == g) d = val[j];
  if (!(d > 0.0)) {
    atomicOr(err, ERR_PIVOT);
    d = 1.0;
  }
  scale[voff[i] + (p - sub_ptr[i])] = 1.0 / sqrt(d);
}

// prof[toff_i + r] = r: the diagonal tile (padding rows hold the identity);
// for LU also the column profile at prof[sum_nt + toff_i + c] = c
__global__ void k_prof_init(int N, LocalLayout lay, int64_t colp, int* prof) {
  const int i = blockIdx.x;
  for (int r = threadIdx.x; r < lay.nt[i]; r += blockDim.x) {
    prof[lay.toff[i] + r] = r;
    if (colp) prof[colp + lay.toff[i] + r] = r;
  }
}

template <class T>
__global__ void k_gather(int total, const int* __restrict__ sub_idx, const int* __restrict__ sub_of_pos,
                         const int* __restrict__ sub_ptr, const int* __restrict__ layer_ptr, int stride,
                         const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ val,
                         const double* __restrict__ scale, LocalLayout lay, int kind, T* fac, int* prof,
                         int64_t colp) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  int i = sub_of_pos[p];
  int a = p - sub_ptr[i];
  int g = sub_idx[p];
  int nt = lay.nt[i];
  const int* lp = layer_ptr + (size_t)i * stride;
  double sa = scale && fac ? scale[lay.voff[i] + a] : 1.0;
  for (int j = rp[g]; j < rp[g + 1]; j++) {
    // position of column c in Omega_i (every layer is ascending), or -1
    int q = find_local_pos(ci[j], sub_idx, lp, stride - 1);
    if (q < 0) continue;
    int b = q - sub_ptr[i];
    if (kind == 0 && b > a) continue;  // Cholesky stores the lower triangle
    if (!fac) {
      // first pass, the tile profiles: rows of the lower part, and (LU)
      // columns of the upper part
      if (b <= a) atomicMin(&prof[lay.toff[i] + a / TS], b / TS);
      if (colp && a <= b) atomicMin(&prof[colp + lay.toff[i] + b / TS], a / TS);
      continue;
    }
    double v = val[j];
    if (scale) v *= sa * scale[lay.voff[i] + b];
    *elem_ptr_l(fac + lay.foff[i], lay, i, kind, nt, a, b) = (T)v;
  }
}

// ---------------------------------------------------------------------------
// Batched tiled Cholesky
// ---------------------------------------------------------------------------

__device__ inline int find_slot(const int64_t* pref, int count, int64_t bid) {
  // largest j in [0, count) with pref[j] <= bid
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (pref[mid] <= bid)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// value of lane b of v, for every lane
__device__ inline float bcast(float v, int b) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), b));
}
__device__ inline double bcast(double v, int b) {
  long long u = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), b);
  int hi = __builtin_amdgcn_readlane((int)(u >> 32), b);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Cholesky of the diagonal tile (k, k) of every active subdomain by one
// wavefront: lane a holds row a in registers, and entry (a, j) is formed
// from the dot product of rows a and j (row j broadcast by readlane), so
// no barrier is needed. Then the inverse L_kk^{-1} (FP64, lane j computes
// column j) goes to dinv[(toff_i + k) * 64^2]: it serves the tile
// triangular solves of column k and the apply's triangular solves.
template <class T>
__global__ void __launch_bounds__(64) k_potrf(int k, const int* __restrict__ order, LocalLayout lay, T* fac,
                                              T* dinv, int* err) {
  constexpr int L1 = TS + 1;
  __shared__ double Ls[TS * L1];
  const int i = order[blockIdx.x];
  const int nt = lay.nt[i];
  T* tile = fac + lay.foff[i] + tile_off(lay, i, 0, nt, k, k);
  const int a = threadIdx.x;
  T row[TS];
#pragma unroll
  for (int b = 0; b < TS; b++) row[b] = tile[b * TS + a];
  bool bad = false;
#pragma unroll
  for (int j = 0; j < TS; j++) {
    // four partial sums, so that the products of a row do not wait on each other
    T v0 = row[j], v1 = T(0), v2 = T(0), v3 = T(0);
#pragma unroll
    for (int l = 0; l < j; l += 4) {
      v0 -= row[l] * bcast(row[l], j);
      if (l + 1 < j) v1 -= row[l + 1] * bcast(row[l + 1], j);
      if (l + 2 < j) v2 -= row[l + 2] * bcast(row[l + 2], j);
      if (l + 3 < j) v3 -= row[l + 3] * bcast(row[l + 3], j);
    }
    const T v = (v0 + v1) + (v2 + v3);
    T d = bcast(v, j);
    if (!(d > T(0))) {
      bad = true;
      d = T(1);
    }
    d = sqrt(d);
    row[j] = a == j ? d : (a > j ? v / d : T(0));
  }
  if (bad && a == 0) atomicOr(err, ERR_PIVOT);
#pragma unroll
  for (int b = 0; b < TS; b++) {
    tile[b * TS + a] = row[b];
    Ls[a + b * L1] = (double)row[b];
  }
  __shared__ double rdiag[TS];
  __syncthreads();
  rdiag[a] = 1.0 / Ls[a + a * L1];  // reciprocals of the diagonal, one per lane
  __syncthreads();
  const int j = a;
  T* out = dinv + (lay.toff[i] + k) * TS2 + (int64_t)j * TS;
  double x[TS];
#pragma unroll
  for (int r = 0; r < TS; r++) {
    double v0 = (r == j) ? 1.0 : 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
#pragma unroll
    for (int l = 0; l < r; l += 4) {
      v0 -= Ls[r + l * L1] * x[l];
      if (l + 1 < r) v1 -= Ls[r + (l + 1) * L1] * x[l + 1];
      if (l + 2 < r) v2 -= Ls[r + (l + 2) * L1] * x[l + 2];
      if (l + 3 < r) v3 -= Ls[r + (l + 3) * L1] * x[l + 3];
    }
    x[r] = r < j ? 0.0 : ((v0 + v1) + (v2 + v3)) * rdiag[r];
  }
#pragma unroll
  for (int r = 0; r < TS; r++) out[r] = (T)x[r];
}

template <class T>
struct LdsLd;
template <>
struct LdsLd<float> {
  static constexpr int v = TS + 16;
};
template <>
struct LdsLd<double> {
  static constexpr int v = TS;
};

// Pitch of a tile staged "k fastest" in LDS (operand (i, kk) at [i * P + kk]),
// read by the MFMA loops with lanes li (16 rows or columns) and lk (4 k).
// LDS has 32 four-byte banks; 32-bit reads are served per half wave (lk in
// {0, 1} or {2, 3}), 64-bit reads per 16 lanes. P = 66 (= 2 mod 32) puts a
// half wave's FP32 reads on 32 distinct banks, an odd P = 65 gives 16
// distinct bank pairs for FP64. (A pitch of 68 put lanes li and li + 8 on one
// bank: 1-2 conflict cycles per FP32 read, 6-12 per FP64 read, measured.)
template <class T>
struct KfPitch;
template <>
struct KfPitch<float> {
  static constexpr int v = TS + 2;
};
template <>
struct KfPitch<double> {
  static constexpr int v = TS + 1;
};

// X = A_rk L_kk^{-T} for the tiles (r, k), r > k (MFMA with the inverse
// formed by k_potrf): X(a, b) = sum_l A(a, l) Linv(b, l), written over A_rk.
template <class T>
__global__ void __launch_bounds__(256) k_trsm(int k, const int64_t* __restrict__ pref, int nact,
                                              const int* __restrict__ order, LocalLayout lay, T* fac,
                                              const T* __restrict__ dinv, const int4* __restrict__ tasks) {
  constexpr int LD = LdsLd<T>::v;
  __shared__ T As[TS * LD];
  __shared__ T Bs[TS * LD];
  const int64_t bid = blockIdx.x;
  int i, r;
  if (tasks) {  // explicit list (tiles inside the profile): x = i, y = r
    i = tasks[bid].x;
    r = tasks[bid].y;
  } else {
    const int j = find_slot(pref, nact, bid);
    i = order[j];
    r = k + 1 + (int)(bid - pref[j]);
  }
  const int nt = lay.nt[i];
  T* A = fac + lay.foff[i] + tile_off(lay, i, 0, nt, r, k);
  const T* Li = dinv + (lay.toff[i] + k) * TS2;
  const int tid = threadIdx.x;
  for (int e = tid; e < TS2; e += 256) {
    const int a = e % TS, b = e / TS;
    As[b * LD + a] = A[e];
    Bs[b * LD + a] = Li[e];
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) acc[x][y] = Mfma<T>::zero();
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll 4
  for (int kk = 0; kk < TS; kk += 4) {
    T a0 = As[(kk + lk) * LD + wr + li];
    T a1 = As[(kk + lk) * LD + wr + 16 + li];
    T b0 = Bs[(kk + lk) * LD + wc + li];
    T b1 = Bs[(kk + lk) * LD + wc + 16 + li];
    acc[0][0] = Mfma<T>::mac(a0, b0, acc[0][0]);
    acc[0][1] = Mfma<T>::mac(a0, b1, acc[0][1]);
    acc[1][0] = Mfma<T>::mac(a1, b0, acc[1][0]);
    acc[1][1] = Mfma<T>::mac(a1, b1, acc[1][1]);
  }
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int col = wc + 16 * y + li;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int row = wr + 16 * x + Mfma<T>::row(lane, q);
        A[col * TS + row] = acc[x][y][q];
      }
    }
}

// Blocked trailing update: C_rc -= sum_{k in [kb, kb+kn)} L_rk L_ck^T with
// K = 64 kn (MFMA). mode 0: tiles (r, c) with kf <= c <= r < nt (trailing
// lower triangle from tile column kf); mode 1: tiles (r, c) with
// kf <= c < kl (a few panel columns), c <= r < nt. The next k-tile pair is
// prefetched into registers while the current one is multiplied.
template <class T>
__global__ void __launch_bounds__(256) k_update_blk(int mode, int kb, int kn, int kf, int kl,
                                                    const int64_t* __restrict__ pref, int nact,
                                                    const int* __restrict__ order, LocalLayout lay, T* fac,
                                                    const int4* __restrict__ tasks) {
  constexpr int LD = LdsLd<T>::v;
  __shared__ T As[TS * LD];
  __shared__ T Bs[TS * LD];
  const int64_t bid = blockIdx.x;
  int i, r, c;
  if (tasks) {  // explicit list: tile (y, z) of subdomain x, K tiles [w & 0xFFFFFF, + w >> 24)
    const int4 q = tasks[bid];
    i = q.x;
    r = q.y;
    c = q.z;
    kb = q.w & 0xFFFFFF;
    kn = q.w >> 24;
  } else {
    const int j = find_slot(pref, nact, bid);
    i = order[j];
    int64_t t = bid - pref[j];
    if (mode == 0) {
      int rr = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
      while ((int64_t)(rr + 1) * (rr + 2) / 2 <= t) rr++;
      while ((int64_t)rr * (rr + 1) / 2 > t) rr--;
      int cc = (int)(t - (int64_t)rr * (rr + 1) / 2);
      r = kf + rr;
      c = kf + cc;
    } else {
      const int nt_ = lay.nt[i];
      c = kf;
      while (t >= nt_ - c) {
        t -= nt_ - c;
        c++;
      }
      r = c + (int)t;
    }
  }
  const int nt = lay.nt[i];
  T* base = fac + lay.foff[i];
  T* C = base + tile_off(lay, i, 0, nt, r, c);
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) acc[x][y] = Mfma<T>::zero();
  constexpr int PER = TS2 / 256;
  T pa[PER], pb[PER];
  {
    const T* Lr = base + tile_off(lay, i, 0, nt, r, kb);
    const T* Lc = base + tile_off(lay, i, 0, nt, c, kb);
#pragma unroll
    for (int u = 0; u < PER; u++) {
      pa[u] = Lr[tid + 256 * u];
      pb[u] = Lc[tid + 256 * u];
    }
  }
  for (int k = 0; k < kn; k++) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; u++) {
      const int e = tid + 256 * u;
      const int a = e % TS, b = e / TS;
      As[b * LD + a] = pa[u];
      Bs[b * LD + a] = pb[u];
    }
    __syncthreads();
    if (k + 1 < kn) {
      const T* Lr = base + tile_off(lay, i, 0, nt, r, kb + k + 1);
      const T* Lc = base + tile_off(lay, i, 0, nt, c, kb + k + 1);
#pragma unroll
      for (int u = 0; u < PER; u++) {
        pa[u] = Lr[tid + 256 * u];
        pb[u] = Lc[tid + 256 * u];
      }
    }
#pragma unroll 4
    for (int kk = 0; kk < TS; kk += 4) {
      T a0 = As[(kk + lk) * LD + wr + li];
      T a1 = As[(kk + lk) * LD + wr + 16 + li];
      T b0 = Bs[(kk + lk) * LD + wc + li];
      T b1 = Bs[(kk + lk) * LD + wc + 16 + li];
      acc[0][0] = Mfma<T>::mac(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<T>::mac(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<T>::mac(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<T>::mac(a1, b1, acc[1][1]);
    }
  }
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      int col = wc + 16 * y + li;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        int row = wr + 16 * x + Mfma<T>::row(lane, q);
        C[col * TS + row] -= acc[x][y][q];
      }
    }
}

// ---------------------------------------------------------------------------
// Batched tiled LU without pivoting (general A; full tile storage)
// ---------------------------------------------------------------------------

// A_kk = L_kk U_kk (L unit lower, U upper, stored together) by one
// wavefront: lane a holds row a in registers; at step j the multipliers of
// column j are formed and row j (broadcast by readlane) is eliminated from
// the rows below, with no barrier. Then the inverses (FP64, lane j computes
// column j) go to dinv[(toff_i + k) * 64^2], packed like the tile: the unit
// lower inverse strictly below the diagonal, the upper inverse on and above.
template <class T>
__global__ void __launch_bounds__(64) k_getrf(int k, const int* __restrict__ order, LocalLayout lay, T* fac,
                                              T* dinv, int* err) {
  constexpr int L1 = TS + 1;
  __shared__ double Ls[TS * L1];
  __shared__ double Xs[TS * L1];
  const int i = order[blockIdx.x];
  const int nt = lay.nt[i];
  T* tile = fac + lay.foff[i] + tile_off(lay, i, 1, nt, k, k);
  const int a = threadIdx.x;
  T row[TS];
#pragma unroll
  for (int b = 0; b < TS; b++) row[b] = tile[b * TS + a];
  bool bad = false;
#pragma unroll
  for (int j = 0; j < TS; j++) {
    T d = bcast(row[j], j);
    if (!(fabs(d) > T(0)) || !isfinite(d)) {
      bad = true;
      d = T(1);
    }
    const T l = row[j] / d;
#pragma unroll
    for (int c = j + 1; c < TS; c++) {
      const T u = bcast(row[c], j);
      if (a > j) row[c] -= l * u;
    }
    if (a > j) row[j] = l;
  }
  if (bad && a == 0) atomicOr(err, ERR_PIVOT);
#pragma unroll
  for (int b = 0; b < TS; b++) {
    tile[b * TS + a] = row[b];
    Ls[a + b * L1] = (double)row[b];
  }
  __syncthreads();
  // thread j forms column j of both inverses; the column lives in LDS (Xs,
  // column j owned by thread j), since two 64-entry FP64 columns in
  // registers spill
  const int j = a;
  T* out = dinv + (lay.toff[i] + k) * TS2 + (int64_t)j * TS;
  // unit lower part: L x = e_j, entries below the diagonal
  for (int r = 0; r < TS; r++) {
    double v = (r == j) ? 1.0 : 0.0;
#pragma unroll 8
    for (int l = 0; l < r; l++) v -= Ls[r + l * L1] * Xs[l * L1 + j];
    Xs[r * L1 + j] = r < j ? 0.0 : v;
    if (r > j) out[r] = (T)v;
  }
  // upper part: U y = e_j, entries on and above the diagonal; rows below r
  // of Xs already hold y when row r is formed
  for (int r = TS - 1; r >= 0; r--) {
    double v = (r == j) ? 1.0 : 0.0;
#pragma unroll 8
    for (int l = r + 1; l < TS; l++) v -= Ls[r + l * L1] * Xs[l * L1 + j];
    v = r > j ? 0.0 : v / Ls[r + r * L1];
    Xs[r * L1 + j] = v;
    if (r <= j) out[r] = (T)v;
  }
}

// Panels of step k with the inverses from k_getrf (MFMA): the first half of
// the grid forms U_kc = L_kk^{-1} A_kc (c > k), the second half
// L_rk = A_rk U_kk^{-1} (r > k); the result overwrites the tile.
template <class T>
__global__ void __launch_bounds__(256) k_trsm_lu(int k, const int64_t* __restrict__ pref, int nact, int64_t half,
                                                 const int* __restrict__ order, LocalLayout lay, T* fac,
                                                 const T* __restrict__ dinv, const int4* __restrict__ tasks) {
  constexpr int LD = LdsLd<T>::v;
  constexpr int LDB = KfPitch<T>::v;  // conflict-free store and MFMA read of Bs
  __shared__ T As[TS * LD];     // As[kk * LD + row] = left operand (row, kk)
  __shared__ T Bs[TS * LDB];    // Bs[col * LDB + kk] = right operand (kk, col)
  int64_t bid = blockIdx.x;
  bool colpanel;
  int i, o;
  if (tasks) {  // explicit list (tiles inside the profiles): x = i, y = o, z = 1 for the L tile (o, k)
    i = tasks[bid].x;
    o = tasks[bid].y;
    colpanel = tasks[bid].z != 0;
  } else {
    colpanel = bid >= half;
    if (colpanel) bid -= half;
    const int j = find_slot(pref, nact, bid);
    i = order[j];
    o = k + 1 + (int)(bid - pref[j]);
  }
  const int nt = lay.nt[i];
  T* base = fac + lay.foff[i];
  const T* Di = dinv + (lay.toff[i] + k) * TS2;
  T* X = base + (colpanel ? tile_off(lay, i, 1, nt, o, k) : tile_off(lay, i, 1, nt, k, o));
  const int tid = threadIdx.x;
  for (int e = tid; e < TS2; e += 256) {
    const int a = e % TS, b = e / TS;  // element (a, b) of a column-major tile
    const T d = Di[e];
    if (!colpanel) {
      // left: unit lower inverse (a > b; 1 on the diagonal); right: A_ko
      As[b * LD + a] = a > b ? d : (a == b ? T(1) : T(0));
      Bs[b * LDB + a] = X[e];
    } else {
      // left: A_ok; right: upper inverse (a <= b)
      As[b * LD + a] = X[e];
      Bs[b * LDB + a] = a <= b ? d : T(0);
    }
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) acc[x][y] = Mfma<T>::zero();
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll 4
  for (int kk = 0; kk < TS; kk += 4) {
    T a0 = As[(kk + lk) * LD + wr + li];
    T a1 = As[(kk + lk) * LD + wr + 16 + li];
    T b0 = Bs[(wc + li) * LDB + kk + lk];
    T b1 = Bs[(wc + 16 + li) * LDB + kk + lk];
    acc[0][0] = Mfma<T>::mac(a0, b0, acc[0][0]);
    acc[0][1] = Mfma<T>::mac(a0, b1, acc[0][1]);
    acc[1][0] = Mfma<T>::mac(a1, b0, acc[1][0]);
    acc[1][1] = Mfma<T>::mac(a1, b1, acc[1][1]);
  }
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int col = wc + 16 * y + li;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int row = wr + 16 * x + Mfma<T>::row(lane, q);
        X[col * TS + row] = acc[x][y][q];
      }
    }
}

// Blocked LU update: C_rc -= sum_{k in [kb, kb+kn)} L_rk U_kc (MFMA, the
// next k-tile pair prefetched into registers). mode 0: the trailing square
// r, c >= kl (kl clipped to nt); mode 1 (kn = 1, k = kb): the rest of the
// panel, rows k < r < kl with every column c > k, and rows r >= kl with
// panel columns k < c < kl.
template <class T>
__global__ void __launch_bounds__(256) k_update_lu(int mode, int kb, int kn, int kl, const int64_t* __restrict__ pref,
                                                   int nact, const int* __restrict__ order, LocalLayout lay, T* fac,
                                                   const int4* __restrict__ tasks) {
  constexpr int LD = LdsLd<T>::v;
  // U_kc is kept as stored (k fastest), with the conflict-free pitch for
  // both the store and the MFMA read
  constexpr int LDB = KfPitch<T>::v;
  __shared__ T As[TS * LD];
  __shared__ T Bs[TS * LDB];
  const int64_t bid = blockIdx.x;
  int i, r, c;
  if (tasks) {  // explicit list: tile (y, z) of subdomain x, K tiles [w & 0xFFFFFF, + w >> 24)
    const int4 q = tasks[bid];
    i = q.x;
    r = q.y;
    c = q.z;
    kb = q.w & 0xFFFFFF;
    kn = q.w >> 24;
  } else {
    const int j = find_slot(pref, nact, bid);
    i = order[j];
    const int nt_ = lay.nt[i];
    const int kli = min(kl, nt_);
    int64_t t = bid - pref[j];
    if (mode == 0) {
      const int w = nt_ - kli;
      r = kli + (int)(t / w);
      c = kli + (int)(t % w);
    } else {
      const int k = kb;
      const int64_t ra = kli - k - 1, ca = nt_ - k - 1;
      if (t < ra * ca) {
        r = k + 1 + (int)(t / ca);
        c = k + 1 + (int)(t % ca);
      } else {
        t -= ra * ca;
        const int cb = kli - k - 1;
        r = kli + (int)(t / cb);
        c = k + 1 + (int)(t % cb);
      }
    }
  }
  const int nt = lay.nt[i];
  T* base = fac + lay.foff[i];
  T* C = base + tile_off(lay, i, 1, nt, r, c);
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) acc[x][y] = Mfma<T>::zero();
  constexpr int PER = TS2 / 256;
  T pa[PER], pb[PER];
  {
    const T* Lr = base + tile_off(lay, i, 1, nt, r, kb);
    const T* Uc = base + tile_off(lay, i, 1, nt, kb, c);
#pragma unroll
    for (int u = 0; u < PER; u++) {
      pa[u] = Lr[tid + 256 * u];
      pb[u] = Uc[tid + 256 * u];
    }
  }
  for (int k = 0; k < kn; k++) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; u++) {
      const int e = tid + 256 * u;
      const int a = e % TS, b = e / TS;
      As[b * LD + a] = pa[u];   // As[kk][row] = L(row, kk)
      Bs[b * LDB + a] = pb[u];  // Bs[col][kk] = U(kk, col)
    }
    __syncthreads();
    if (k + 1 < kn) {
      const T* Lr = base + tile_off(lay, i, 1, nt, r, kb + k + 1);
      const T* Uc = base + tile_off(lay, i, 1, nt, kb + k + 1, c);
#pragma unroll
      for (int u = 0; u < PER; u++) {
        pa[u] = Lr[tid + 256 * u];
        pb[u] = Uc[tid + 256 * u];
      }
    }
#pragma unroll 4
    for (int kk = 0; kk < TS; kk += 4) {
      T a0 = As[(kk + lk) * LD + wr + li];
      T a1 = As[(kk + lk) * LD + wr + 16 + li];
      T b0 = Bs[(wc + li) * LDB + kk + lk];
      T b1 = Bs[(wc + 16 + li) * LDB + kk + lk];
      acc[0][0] = Mfma<T>::mac(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<T>::mac(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<T>::mac(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<T>::mac(a1, b1, acc[1][1]);
    }
  }
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int col = wc + 16 * y + li;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int row = wr + 16 * x + Mfma<T>::row(lane, q);
        C[col * TS + row] -= acc[x][y][q];
      }
    }
}

// Right-looking LU blocked by panels of PW tile columns (as the Cholesky
// path): for each k of the panel, the diagonal tile (k_getrf), the row and
// column strips (k_trsm_lu) and the rest of the panel (k_update_lu mode 1);
// then the trailing square once with K = 64 PW (mode 0).
// With tile profiles (profile pr of the rows of the lower part, the first
// tile column of row r holding a nonzero left of or on the diagonal; pc of
// the columns of the upper part, the first tile row of column c holding one
// above or on the diagonal), L has no fill left of pr(r) and U none above
// pc(c), so only the terms L_rk U_kc with k >= max(pr(r), pc(c)) are formed,
// from explicit task lists. Returns the arithmetic of the tasks (2 per
// multiply-add; triangular products counted at half).
template <class T>
double factor_tiles_lu(hipStream_t s, int N, const std::vector<int>& nt, const LocalLayout& lay, T* fac, T* dinv,
                       int* err, int PW = 8, const int* pr = nullptr, const int* pc = nullptr,
                       const std::vector<int64_t>* toff = nullptr) {
  std::vector<int> order(N);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nt[a] > nt[b]; });
  const int maxnt = N ? nt[order[0]] : 0;
  struct Launch {
    int kind, k, kb, kn, kl, nact;
    int64_t off, total, half;
  };
  std::vector<Launch> launches;
  std::vector<int64_t> pref;
  std::vector<int4> tasks;
  const bool prof = pr != nullptr;
  const double t3 = (double)TS * TS * TS;
  double flops = 0.0;
  auto active = [&](int k) {
    int a = 0;
    while (a < N && nt[order[a]] > k) a++;
    return a;
  };
  std::vector<int> R, C;
  for (int k0 = 0; k0 < maxnt; k0 += PW) {
    const int kl = k0 + PW;
    for (int k = k0; k < std::min(kl, maxnt); k++) {
      const int act = active(k);
      launches.push_back(Launch{0, k, 0, 0, 0, act, 0, 0, 0});
      flops += act * 2.0 * t3 / 3.0;
      if (prof) {
        // L tiles (o, k) with pr(o) <= k and U tiles (k, o) with pc(o) <= k,
        // then the panel's part of their products
        const int64_t off1 = (int64_t)tasks.size();
        for (int a = 0; a < act; a++) {
          const int i = order[a];
          const int *fr = pr + (*toff)[i], *fc = pc + (*toff)[i];
          for (int o = k + 1; o < nt[i]; o++) {
            if (fr[o] <= k) tasks.push_back(int4{i, o, 1, 0});
            if (fc[o] <= k) tasks.push_back(int4{i, o, 0, 0});
          }
        }
        const int64_t n1 = (int64_t)tasks.size() - off1;
        flops += (double)n1 * t3;
        if (n1 > 0) launches.push_back(Launch{1, k, 0, 0, 0, act, off1, n1, 0});
        const int64_t off2 = (int64_t)tasks.size();
        for (int a = 0; a < act; a++) {
          const int i = order[a];
          const int *fr = pr + (*toff)[i], *fc = pc + (*toff)[i];
          R.clear();
          C.clear();
          for (int o = k + 1; o < nt[i]; o++) {
            if (fr[o] <= k) R.push_back(o);
            if (fc[o] <= k) C.push_back(o);
          }
          // the panel: rows k < r < kl with every column, rows r >= kl with the panel's columns
          for (int r : R)
            for (int c : C)
              if (r < kl || c < kl) tasks.push_back(int4{i, r, c, k | (1 << 24)});
        }
        const int64_t n2 = (int64_t)tasks.size() - off2;
        flops += 2.0 * (double)n2 * t3;
        if (n2 > 0) launches.push_back(Launch{2, k, k, 1, kl, act, off2, n2, 0});
        continue;
      }
      {
        int64_t off = (int64_t)pref.size(), tot = 0;
        for (int a = 0; a < act; a++) {
          pref.push_back(tot);
          tot += nt[order[a]] - k - 1;
        }
        pref.push_back(tot);
        flops += 2.0 * (double)tot * t3;
        if (tot > 0) launches.push_back(Launch{1, k, 0, 0, 0, act, off, 2 * tot, tot});
      }
      {
        int64_t off = (int64_t)pref.size(), tot = 0;
        for (int a = 0; a < act; a++) {
          pref.push_back(tot);
          const int64_t n_ = nt[order[a]], kli = std::min<int64_t>(kl, n_);
          tot += (kli - k - 1) * (n_ - k - 1) + (n_ - kli) * (kli - k - 1);
        }
        pref.push_back(tot);
        flops += 2.0 * (double)tot * t3;
        if (tot > 0) launches.push_back(Launch{2, k, k, 1, kl, act, off, tot, 0});
      }
    }
    const int act = active(kl);
    if (act <= 0) continue;
    if (prof) {
      const int64_t off = (int64_t)tasks.size();
      for (int a = 0; a < act; a++) {
        const int i = order[a];
        const int *fr = pr + (*toff)[i], *fc = pc + (*toff)[i];
        R.clear();
        C.clear();
        for (int o = kl; o < nt[i]; o++) {
          if (fr[o] < kl) R.push_back(o);
          if (fc[o] < kl) C.push_back(o);
        }
        for (int r : R)
          for (int c : C) {
            const int kb = std::max(k0, std::max(fr[r], fc[c]));
            tasks.push_back(int4{i, r, c, kb | ((kl - kb) << 24)});
            flops += 2.0 * t3 * (kl - kb);
          }
      }
      const int64_t n3 = (int64_t)tasks.size() - off;
      if (n3 > 0) launches.push_back(Launch{3, kl, k0, PW, kl, act, off, n3, 0});
      continue;
    }
    int64_t off = (int64_t)pref.size(), tot = 0;
    for (int a = 0; a < act; a++) {
      pref.push_back(tot);
      const int64_t w = nt[order[a]] - kl;
      tot += w * w;
    }
    pref.push_back(tot);
    flops += 2.0 * (double)tot * t3 * PW;
    if (tot > 0) launches.push_back(Launch{3, kl, k0, PW, kl, act, off, tot, 0});
  }
  DBuf<int> d_order;
  DBuf<int64_t> d_pref;
  DBuf<int4> d_tasks;
  d_order.upload(order, s);
  d_pref.upload(pref, s);
  d_tasks.upload(tasks, s);
  for (const Launch& L : launches) {
    const int4* tk = prof && L.kind > 0 ? d_tasks.p + L.off : nullptr;
    const int64_t* pf = prof ? nullptr : d_pref.p + L.off;
    switch (L.kind) {
      case 0:
        hipLaunchKernelGGL(k_getrf<T>, dim3(L.nact), dim3(64), 0, s, L.k, d_order.p, lay, fac, dinv, err);
        break;
      case 1:
        hipLaunchKernelGGL(k_trsm_lu<T>, dim3((unsigned)L.total), dim3(256), 0, s, L.k, pf, L.nact, L.half,
                           d_order.p, lay, fac, dinv, tk);
        break;
      case 2:
        hipLaunchKernelGGL(k_update_lu<T>, dim3((unsigned)L.total), dim3(256), 0, s, 1, L.kb, L.kn, L.kl, pf, L.nact,
                           d_order.p, lay, fac, tk);
        break;
      default:
        hipLaunchKernelGGL(k_update_lu<T>, dim3((unsigned)L.total), dim3(256), 0, s, 0, L.kb, L.kn, L.kl, pf, L.nact,
                           d_order.p, lay, fac, tk);
        break;
    }
    TLS_LAUNCH_CHECK();
  }
  TLS_HIP(hipStreamSynchronize(s));
  return flops;
}

// Right-looking Cholesky blocked by panels of PW tile columns: inside a
// panel every step updates only the panel's remaining columns; the rest of
// the trailing matrix is updated once per panel with K = 64 * PW, which cuts
// its read-modify-write traffic by PW.
//
// With a tile profile (prof[toff_i + r] = f_i(r), the first tile column of
// row r that holds a nonzero of A_ii), the factor has no fill left of f_i(r)
// (fill stays inside the envelope), so only the terms L_rk L_ck^T with
// k >= max(f(r), f(c)) are formed: the kernels take explicit task lists,
// built here, instead of enumerating every tile. Returns the arithmetic of
// the tasks (2 per multiply-add; triangular products counted at half).
template <class T>
double factor_tiles(hipStream_t s, int N, const std::vector<int>& nt, const LocalLayout& lay, T* fac, T* dinv,
                    int* err, int PW = 8, const int* prof = nullptr, const std::vector<int64_t>* toff = nullptr) {
  std::vector<int> order(N);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nt[a] > nt[b]; });
  const int maxnt = N ? nt[order[0]] : 0;
  struct Launch {
    int kind;  // 0 potrf, 1 trsm, 2 panel update, 3 trailing update
    int k, kb, kn, kf, kl, nact;
    int64_t off, total;
  };
  std::vector<Launch> launches;
  std::vector<int64_t> pref;
  std::vector<int4> tasks;
  const double t3 = (double)TS * TS * TS;
  double flops = 0.0;
  auto active = [&](int k) {
    int a = 0;
    while (a < N && nt[order[a]] > k) a++;
    return a;
  };
  auto fp = [&](int i) { return prof + (*toff)[i]; };
  std::vector<int> rows;
  for (int k0 = 0; k0 < maxnt; k0 += PW) {
    const int kl = k0 + PW;
    for (int k = k0; k < std::min(kl, maxnt); k++) {
      const int act = active(k);
      launches.push_back(Launch{0, k, 0, 0, 0, 0, act, 0, act});
      flops += act * t3 / 3.0;
      if (prof) {
        // rows below k with a nonzero tile in column k: the trsm tiles, and
        // the panel columns c < kl among them get the term of column k
        const int64_t off1 = (int64_t)tasks.size();
        for (int a = 0; a < act; a++) {
          const int i = order[a];
          const int* f = fp(i);
          for (int r = k + 1; r < nt[i]; r++)
            if (f[r] <= k) tasks.push_back(int4{i, r, k, 0});
        }
        const int64_t n1 = (int64_t)tasks.size() - off1;
        if (n1 > 0) launches.push_back(Launch{1, k, 0, 0, 0, 0, act, off1, n1});
        flops += (double)n1 * t3;
        const int64_t off2 = (int64_t)tasks.size();
        for (int a = 0; a < act; a++) {
          const int i = order[a];
          const int* f = fp(i);
          rows.clear();
          for (int r = k + 1; r < nt[i]; r++)
            if (f[r] <= k) rows.push_back(r);
          for (size_t x = 0; x < rows.size() && rows[x] < kl; x++)
            for (size_t y = x; y < rows.size(); y++) {
              tasks.push_back(int4{i, rows[y], rows[x], k | (1 << 24)});
              flops += (y == x ? 1.0 : 2.0) * t3;
            }
        }
        const int64_t n2 = (int64_t)tasks.size() - off2;
        if (n2 > 0) launches.push_back(Launch{2, k, k, 1, k + 1, kl, act, off2, n2});
        continue;
      }
      // trsm: tiles (r, k), r > k
      {
        int64_t off = (int64_t)pref.size(), tot = 0;
        for (int a = 0; a < act; a++) {
          pref.push_back(tot);
          tot += nt[order[a]] - k - 1;
        }
        pref.push_back(tot);
        flops += (double)tot * t3;
        if (tot > 0) launches.push_back(Launch{1, k, 0, 0, 0, 0, act, off, tot});
      }
      // panel columns c in (k, k0 + PW): tiles (r, c), c <= r
      {
        const int kf = k + 1;
        int64_t off = (int64_t)pref.size(), tot = 0;
        for (int a = 0; a < act; a++) {
          pref.push_back(tot);
          const int n_ = nt[order[a]];
          for (int cc = kf; cc < std::min(kl, n_); cc++) {
            tot += n_ - cc;
            flops += (2.0 * (n_ - cc) - 1.0) * t3;
          }
        }
        pref.push_back(tot);
        if (tot > 0) launches.push_back(Launch{2, k, k, 1, kf, kl, act, off, tot});
      }
    }
    // trailing update from column k0 + PW with the whole panel
    const int act = active(kl);
    if (act <= 0) continue;
    if (prof) {
      const int64_t off = (int64_t)tasks.size();
      for (int a = 0; a < act; a++) {
        const int i = order[a];
        const int* f = fp(i);
        rows.clear();
        for (int r = kl; r < nt[i]; r++)
          if (f[r] < kl) rows.push_back(r);
        for (size_t x = 0; x < rows.size(); x++)
          for (size_t y = x; y < rows.size(); y++) {
            const int kb = std::max(k0, std::max(f[rows[x]], f[rows[y]]));
            tasks.push_back(int4{i, rows[y], rows[x], kb | ((kl - kb) << 24)});
            flops += (y == x ? 1.0 : 2.0) * t3 * (kl - kb);
          }
      }
      const int64_t n3 = (int64_t)tasks.size() - off;
      if (n3 > 0) launches.push_back(Launch{3, kl, k0, PW, kl, 0, act, off, n3});
      continue;
    }
    int64_t off = (int64_t)pref.size(), tot = 0;
    for (int a = 0; a < act; a++) {
      pref.push_back(tot);
      const int64_t T_ = nt[order[a]] - kl;
      tot += T_ * (T_ + 1) / 2;
      flops += (double)T_ * T_ * t3 * PW;
    }
    pref.push_back(tot);
    if (tot > 0) launches.push_back(Launch{3, kl, k0, PW, kl, 0, act, off, tot});
  }
  DBuf<int> d_order;
  DBuf<int64_t> d_pref;
  DBuf<int4> d_tasks;
  d_order.upload(order, s);
  d_pref.upload(pref, s);
  d_tasks.upload(tasks, s);
  for (const Launch& L : launches) {
    const int4* tk = prof && L.kind > 0 ? d_tasks.p + L.off : nullptr;
    const int64_t* pf = prof ? nullptr : d_pref.p + L.off;
    switch (L.kind) {
      case 0:
        hipLaunchKernelGGL(k_potrf<T>, dim3(L.nact), dim3(64), 0, s, L.k, d_order.p, lay, fac, dinv, err);
        break;
      case 1:
        hipLaunchKernelGGL(k_trsm<T>, dim3((unsigned)L.total), dim3(256), 0, s, L.k, pf, L.nact, d_order.p, lay,
                           fac, dinv, tk);
        break;
      case 2:
        hipLaunchKernelGGL(k_update_blk<T>, dim3((unsigned)L.total), dim3(256), 0, s, 1, L.kb, L.kn, L.kf, L.kl, pf,
                           L.nact, d_order.p, lay, fac, tk);
        break;
      default:
        hipLaunchKernelGGL(k_update_blk<T>, dim3((unsigned)L.total), dim3(256), 0, s, 0, L.kb, L.kn, L.kf, 0, pf,
                           L.nact, d_order.p, lay, fac, tk);
        break;
    }
    TLS_LAUNCH_CHECK();
  }
  TLS_HIP(hipStreamSynchronize(s));
  return flops;
}

// ---------------------------------------------------------------------------
// Persistent triangular solves
// ---------------------------------------------------------------------------

template <class T>
struct Vec4;
template <>
struct Vec4<float> {
  typedef f32x4 type;
};
template <>
struct Vec4<double> {
  typedef f64x4 type;
};

// Unroll depth of the tile loop: tiles whose loads are issued together.
template <class T>
struct TrsvUnroll;
template <>
struct TrsvUnroll<float> {
  static constexpr int v = 4;
};
template <>
struct TrsvUnroll<double> {
  static constexpr int v = 2;
};

__device__ inline int load_flag(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Values that other workgroups of the same launch produce are exchanged
// with device-coherent accesses (relaxed agent-scope atomics: they bypass
// the per-XCD caches), so publishing a block needs no cache write-back and
// reading one no invalidation: the producer waits for its coherent stores to
// complete (s_waitcnt) before it stores the ready flag, and the consumer only
// issues its coherent loads after it has seen the flag.
template <class T>
__device__ inline T load_shared(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ inline void store_shared(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class V>
__device__ inline V stream_load(const V* p) {
  return __builtin_nontemporal_load(p);
}

constexpr long long SPIN_LIMIT = 1ll << 26;

// Run by the 64 lanes of wave 0 of a solve task: from block row c, stepping
// towards `stop` (exclusive), the first row that is neither ready (its flag
// holds this epoch) nor skippable (backward with a profile g: g(cc) >
// need_row, so the task reads nothing of row cc). 64 rows are checked per
// round, one per lane, so a task whose dependencies are long solved (or
// skipped) passes them in a few rounds instead of one memory round trip per
// row. Waits, within SPIN_LIMIT polls, until at least one row is
// available. CAP: at most 64 rows are passed (one round), so the caller can
// keep what the lanes read about those rows in a 64-entry table.
// With CAP each lane also returns, for its row c + step * lane, the
// profile entry (g_out; 0 without g) and the entry of the per-row table cb
// (cb_out; 0 without cb), read in the same polls as the flags, so that
// nothing more is loaded once the rows are ready.
template <bool BWD, bool CAP = false>
__device__ inline int wait_rows(int c, int stop, const int* fl, int epoch, const int* __restrict__ g, int need_row,
                                int* err, const int64_t* __restrict__ cb = nullptr, int* g_out = nullptr,
                                int64_t* cb_out = nullptr) {
  const int lane = threadIdx.x & 63;
  constexpr int step = BWD ? -1 : 1;
  int lim = c;
  long long spins = 0;
  for (;;) {
    for (;;) {
      const int cc = lim + step * lane;
      const bool inr = BWD ? (cc > stop) : (cc < stop);
      // the profile entry, the table entry and the flag are loaded together (one round trip)
      const int gv = (inr && g) ? g[cc] : 0;
      const int64_t bv = (CAP && inr && cb) ? cb[cc] : 0;
      const int fv = inr ? load_flag(&fl[cc]) : 0;
      const bool ok = inr && ((g && gv > need_row) || fv == epoch);
      if (CAP) {
        if (g_out) *g_out = gv;
        if (cb_out) *cb_out = bv;
      }
      const uint64_t m = __ballot(ok);
      const int run = ~m == 0ull ? 64 : __builtin_ctzll(~m);
      lim += step * run;
      if (CAP || run < 64) break;
    }
    if (lim != c) break;
    if (++spins > SPIN_LIMIT) {
      if (lane == 0) atomicOr(err, ERR_WAIT);
      lim += step;
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return lim;
}

// Solve modes of the persistent triangular-solve kernel.
//   FWD_L : L y = b, L lower with its diagonal (Cholesky), block rows ascending
//   BWD_LT: L^T x = y (Cholesky), block rows descending, tiles read transposed
//   FWD_UL: L y = b, L unit lower (LU), ascending
//   BWD_U : U x = y, U upper with its diagonal (LU), descending
enum TrsvMode { FWD_L = 0, BWD_LT = 1, FWD_UL = 2, BWD_U = 3 };

// The diagonal block is applied through its precomputed inverse (dinv, one
// 64 x 64 tile per block row, at (toff_i + r) * TS2, formed by k_potrf or k_getrf): the
// right-hand side is reduced into LDS and multiplied by that tile with all
// 256 threads, instead of a 64-step substitution on one wave.
template <class T, int MODE>
__global__ void __launch_bounds__(256) k_trsv(const int4* __restrict__ tasks, int ntasks, int* counter,
                                              int* flags, const int* __restrict__ epoch_ptr, LocalLayout lay,
                                              const T* __restrict__ fac, const T* __restrict__ dinv, T* x,
                                              int* err, const int* __restrict__ done, const int* __restrict__ prof) {
  if (*done) return;
  constexpr bool BWD = (MODE == BWD_LT || MODE == BWD_U);
  constexpr bool TRANS = (MODE == BWD_LT);
  constexpr int KIND = (MODE == FWD_UL || MODE == BWD_U) ? 1 : 0;
  constexpr int U = TrsvUnroll<T>::v;
  typedef typename Vec4<T>::type V4;
  // partial sums: 16 rows of RP; the transposed modes store down a column
  // (16 lanes, one per row), so their rows are padded to spread the banks
  constexpr int RP = (MODE == BWD_LT) ? TS + 4 : TS;
  __shared__ T s_red[16 * RP];
  __shared__ T s_rhs[TS];
  __shared__ int s_task, s_lim;
  __shared__ int s_g[BWD ? 64 : 1];
  __shared__ int64_t s_cb[BWD ? 64 : 1];
  const int tid = threadIdx.x;
  const int rg = tid & 15, cg = tid >> 4;
  const int epoch = *epoch_ptr;
  for (;;) {
    if (tid == 0) s_task = atomicAdd(counter, 1);
    __syncthreads();
    const int t = s_task;
    if (t >= ntasks) break;
    const int i = tasks[t].x, r = tasks[t].y;
    const int nt = lay.nt[i];
    const T* base = fac + lay.foff[i];
    T* xi = x + lay.voff[i];
    int* fl = flags + lay.toff[i];
    // inverse of the diagonal tile -> registers (rows 4rg..4rg+3 of columns
    // cg + 16j), loaded while the task waits; the LU tile packs the unit
    // lower inverse below the diagonal and the upper inverse on and above it
    V4 dv[4];
    {
      const T* dt = dinv + (lay.toff[i] + r) * TS2;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        dv[j] = stream_load(reinterpret_cast<const V4*>(dt + (cg + 16 * j) * TS + 4 * rg));
        if (MODE == FWD_UL || MODE == BWD_U) {
          const int col = cg + 16 * j, r0 = 4 * rg;
          const bool lower = MODE == FWD_UL;
          if (lower ? !(r0 + 0 > col) : !(r0 + 0 <= col)) dv[j].x = T(0);
          if (lower ? !(r0 + 1 > col) : !(r0 + 1 <= col)) dv[j].y = T(0);
          if (lower ? !(r0 + 2 > col) : !(r0 + 2 <= col)) dv[j].z = T(0);
          if (lower ? !(r0 + 3 > col) : !(r0 + 3 <= col)) dv[j].w = T(0);
        }
      }
    }
    T acc[4] = {T(0), T(0), T(0), T(0)};
    // blocks this task reads: forward c = 0 .. r-1, backward c = nt-1 .. r+1;
    // with tile profiles, forward starts at the row profile f(r), and
    // backward skips the blocks whose profile entry g(c) exceeds r (they
    // hold only zeros): for Cholesky g = f (the tile (c, r) of L), for LU g
    // is the column profile of U (the tile (r, c))
    const int* fp = prof ? prof + lay.toff[i] : nullptr;
    int c = BWD ? nt - 1 : (fp ? fp[r] : 0);
    // block this row takes from block row cc: forward (r, cc) = row base + cc;
    // backward (cc, r) of L (Cholesky) or (r, cc) of U (LU, by columns)
    // (the subdomain's row and column bases, read without re-reading toff)
    const int64_t* trw = lay.trow ? lay.trow + lay.toff[i] : nullptr;
    const int64_t* tcl = lay.tcol ? lay.tcol + lay.toff[i] : nullptr;
    auto rowb = [&](int q) -> int64_t { return trw ? trw[q] : tile_index(KIND, nt, q, 0); };
    const int64_t rb0 = BWD ? 0 : rowb(r);
    auto tile_at = [&](int cc) -> const T* {
      int64_t t;
      if (!BWD)
        t = rb0 + cc;
      else if (TRANS)
        t = rowb(cc) + r;
      else
        t = tcl ? tcl[cc] + r : (int64_t)r * nt + cc;
      return base + t * TS2;
    };
    const int step = BWD ? -1 : 1;
    // the block next to the diagonal is almost always the last dependency:
    // load it, and this row's right-hand side, while the task waits
    const int c_last = BWD ? r + 1 : r - 1;
    const bool has_last = BWD ? (r + 1 < nt) : (r > 0);
    V4 vlast[4];
    // (only if that block is stored: inside the profile, when there is one)
    if (has_last && (!fp || (BWD ? fp[c_last] <= r : fp[r] <= c_last))) {
      const T* tile = tile_at(c_last);
#pragma unroll
      for (int j = 0; j < 4; j++) vlast[j] = stream_load(reinterpret_cast<const V4*>(tile + (cg + 16 * j) * TS + 4 * rg));
    }
    const T brow = tid < 64 ? xi[r * TS + tid] : T(0);
    while (BWD ? (c > r) : (c < r)) {
      if (tid < 64) {
        int gq = 0;
        int64_t bq = 0;
        const int lim =
            wait_rows<BWD, BWD>(c, r, fl, epoch, BWD ? fp : nullptr, r, err, BWD ? (TRANS ? trw : tcl) : nullptr,
                                &gq, &bq);
        if (BWD && tid < c - lim) {
          // each column's profile entry and block base, for all threads
          const int cc = c - tid;
          s_g[tid] = gq;
          s_cb[tid] = TRANS ? (trw ? bq : tile_index(KIND, nt, cc, 0)) + r : (tcl ? bq + r : (int64_t)r * nt + cc);
        }
        if (tid == 0) s_lim = lim;
      }
      __syncthreads();
      const int lim = s_lim;
      const int cnt = BWD ? c - lim : lim - c;
      int done_tiles = 0;
      // groups of U tiles: all loads first, then the arithmetic
      for (; done_tiles + U <= cnt; done_tiles += U) {
        V4 v[U][4];
        T xs[U][4];
#pragma unroll
        for (int u = 0; u < U; u++) {
          const int cc = c + step * (done_tiles + u);
          if (BWD && s_g[done_tiles + u] > r) {
#pragma unroll
            for (int j = 0; j < 4; j++) {
              v[u][j] = V4{T(0), T(0), T(0), T(0)};
              xs[u][j] = T(0);
            }
            continue;
          }
          const T* tile = BWD ? base + s_cb[done_tiles + u] * TS2 : tile_at(cc);
          if (cc == c_last) {
#pragma unroll
            for (int j = 0; j < 4; j++) v[u][j] = vlast[j];
          } else {
#pragma unroll
            for (int j = 0; j < 4; j++)
              v[u][j] = stream_load(reinterpret_cast<const V4*>(tile + (cg + 16 * j) * TS + 4 * rg));
          }
          const T* xc = xi + cc * TS;
          if (!TRANS) {
#pragma unroll
            for (int j = 0; j < 4; j++) xs[u][j] = load_shared(xc + cg + 16 * j);
          } else {
#pragma unroll
            for (int j = 0; j < 4; j++) xs[u][j] = load_shared(xc + 4 * rg + j);
          }
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
          if (!TRANS) {
#pragma unroll
            for (int j = 0; j < 4; j++) {
              acc[0] += v[u][j].x * xs[u][j];
              acc[1] += v[u][j].y * xs[u][j];
              acc[2] += v[u][j].z * xs[u][j];
              acc[3] += v[u][j].w * xs[u][j];
            }
          } else {
#pragma unroll
            for (int j = 0; j < 4; j++)
              acc[j] += v[u][j].x * xs[u][0] + v[u][j].y * xs[u][1] + v[u][j].z * xs[u][2] + v[u][j].w * xs[u][3];
          }
        }
      }
      for (; done_tiles < cnt; done_tiles++) {
        const int cc = c + step * done_tiles;
        if (BWD && s_g[done_tiles] > r) continue;
        const T* tile = BWD ? base + s_cb[done_tiles] * TS2 : tile_at(cc);
        const T* xc = xi + cc * TS;
        const bool pre = cc == c_last;
        if (!TRANS) {
#pragma unroll
          for (int j = 0; j < 4; j++) {
            int col = cg + 16 * j;
            V4 v = pre ? vlast[j] : stream_load(reinterpret_cast<const V4*>(tile + col * TS + 4 * rg));
            T xv = load_shared(xc + col);
            acc[0] += v.x * xv;
            acc[1] += v.y * xv;
            acc[2] += v.z * xv;
            acc[3] += v.w * xv;
          }
        } else {
          T xv[4];
#pragma unroll
          for (int q = 0; q < 4; q++) xv[q] = load_shared(xc + 4 * rg + q);
#pragma unroll
          for (int j = 0; j < 4; j++) {
            int col = cg + 16 * j;
            V4 v = pre ? vlast[j] : stream_load(reinterpret_cast<const V4*>(tile + col * TS + 4 * rg));
            acc[j] += v.x * xv[0] + v.y * xv[1] + v.z * xv[2] + v.w * xv[3];
          }
        }
      }
      c = lim;
      __syncthreads();
    }
    // reduce the partial sums into the right-hand side of the diagonal block
    if (!TRANS) {
#pragma unroll
      for (int q = 0; q < 4; q++) s_red[cg * RP + 4 * rg + q] = acc[q];
    } else {
#pragma unroll
      for (int j = 0; j < 4; j++) s_red[rg * RP + cg + 16 * j] = acc[j];
    }
    __syncthreads();
    if (tid < 64) {
      T sum = T(0);
#pragma unroll
      for (int g = 0; g < 16; g++) sum += s_red[g * RP + tid];
      s_rhs[tid] = brow - sum;
    }
    __syncthreads();
    // x_r = (diagonal tile)^{-1} rhs, or its transpose for BWD_LT
    T a2[4] = {T(0), T(0), T(0), T(0)};
    if (!TRANS) {
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const T rv = s_rhs[cg + 16 * j];
        a2[0] += dv[j].x * rv;
        a2[1] += dv[j].y * rv;
        a2[2] += dv[j].z * rv;
        a2[3] += dv[j].w * rv;
      }
#pragma unroll
      for (int q = 0; q < 4; q++) s_red[cg * RP + 4 * rg + q] = a2[q];
    } else {
      const T r0 = s_rhs[4 * rg], r1 = s_rhs[4 * rg + 1], r2 = s_rhs[4 * rg + 2], r3 = s_rhs[4 * rg + 3];
#pragma unroll
      for (int j = 0; j < 4; j++) a2[j] = dv[j].x * r0 + dv[j].y * r1 + dv[j].z * r2 + dv[j].w * r3;
#pragma unroll
      for (int j = 0; j < 4; j++) s_red[rg * RP + cg + 16 * j] = a2[j];
    }
    __syncthreads();
    if (tid < 64) {
      const int lane = tid;
      T val = T(0);
#pragma unroll
      for (int g = 0; g < 16; g++) val += s_red[g * RP + lane];
      if (MODE == FWD_UL) val += s_rhs[lane];  // unit diagonal of L
      store_shared(xi + r * TS + lane, val);
      __builtin_amdgcn_s_waitcnt(0);  // the coherent stores above have completed
      if (lane == 0) __hip_atomic_store(&fl[r], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }
}

// Backward solve with many right-hand sides on the tile storage, with the
// upper block U_II of an LU factor or, LT = true, with L_II^T of a Cholesky
// factor (U_jk = L_kj^T, read from the lower tile (k, j)). X_i is
// column-major with leading dimension ldx (M_i = 64 nt_i when ldx = 0), its
// 64 q-th columns one "column block". Subdomain i has nb_i = ceil(#I_i / 64)
// tile rows; a global step s stands for its tile row k = nb_i - 1 - s, so
// all subdomains start from their own last row. Rows of the last tile that
// lie outside I have zero right-hand sides and stay zero, so solving with
// the whole diagonal tile is exact.

// X_k <- U_kk^{-1} X_k (packed inverse from the factorization: the upper
// part for LU, the transpose of the lower part for Cholesky), one
// workgroup per (subdomain, column block); MFMA.
template <class T, bool LT>
__global__ void __launch_bounds__(256) k_bsolve_diag(int s, const int64_t* __restrict__ pref, int nact,
                                                     const int* __restrict__ order, LocalLayout lay,
                                                     const int* __restrict__ nb, const int64_t* __restrict__ xoff,
                                                     int64_t ldx, const T* __restrict__ dinv, T* X) {
  constexpr int LD = LdsLd<T>::v;
  constexpr int LDK = KfPitch<T>::v;
  __shared__ T As[TS * (LD > LDK ? LD : LDK)];  // A = U_kk^{-1}: LT As[row * LDK + kk], else As[kk * LD + row]
  __shared__ T Bs[TS * LDK];                    // Bs[col * LDK + kk] = X_k(kk, col)
  const int64_t bid = blockIdx.x;
  const int j = find_slot(pref, nact, bid);
  const int i = order[j];
  const int q = (int)(bid - pref[j]);
  const int k = nb[i] - 1 - s;
  const int64_t M = ldx > 0 ? ldx : (int64_t)lay.nt[i] * TS;
  T* Xk = X + xoff[i] + (int64_t)q * TS * M + (int64_t)k * TS;
  const T* Di = dinv + (lay.toff[i] + k) * TS2;
  const int tid = threadIdx.x;
  for (int e = tid; e < TS2; e += 256) {
    const int a = e % TS, b = e / TS;
    if (LT)
      As[b * LDK + a] = a >= b ? Di[e] : T(0);  // A(b, a) = L_kk^{-1}(a, b)
    else
      As[b * LD + a] = a <= b ? Di[e] : T(0);
    Bs[b * LDK + a] = Xk[(int64_t)b * M + a];
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) acc[x][y] = Mfma<T>::zero();
#pragma unroll 4
  for (int kk = 0; kk < TS; kk += 4) {
    T a0 = LT ? As[(wr + li) * LDK + kk + lk] : As[(kk + lk) * LD + wr + li];
    T a1 = LT ? As[(wr + 16 + li) * LDK + kk + lk] : As[(kk + lk) * LD + wr + 16 + li];
    T b0 = Bs[(wc + li) * LDK + kk + lk];
    T b1 = Bs[(wc + 16 + li) * LDK + kk + lk];
    acc[0][0] = Mfma<T>::mac(a0, b0, acc[0][0]);
    acc[0][1] = Mfma<T>::mac(a0, b1, acc[0][1]);
    acc[1][0] = Mfma<T>::mac(a1, b0, acc[1][0]);
    acc[1][1] = Mfma<T>::mac(a1, b1, acc[1][1]);
  }
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int col = wc + 16 * y + li;
#pragma unroll
      for (int qq = 0; qq < 4; qq++) {
        const int row = wr + 16 * x + Mfma<T>::row(lane, qq);
        Xk[(int64_t)col * M + row] = acc[x][y][qq];
      }
    }
}

// Row ranges of one update launch for subdomain i, in its tile rows:
// mode 0 (step s inside the panel starting at s0): rows [lo, k) with
// k = nb - 1 - s, the panel's rows not yet solved, from the single solved
// block X_k; mode 1 (after the panel): rows [0, k0) from the panel's
// blocks X_{k0..k1-1}, k1 = nb - s0, k0 = max(0, k1 - pw).
struct BsolveRange {
  int jlo, jhi, klo, khi;
};
__host__ __device__ inline BsolveRange bsolve_range(int mode, int s, int s0, int pw, int nb) {
  BsolveRange r;
  const int k1 = nb - s0;
  const int k0 = k1 - pw > 0 ? k1 - pw : 0;
  if (mode == 0) {
    const int k = nb - 1 - s;
    r.jlo = k0;
    r.jhi = k;
    r.klo = k;
    r.khi = k + 1;
  } else {
    r.jlo = 0;
    r.jhi = k0;
    r.klo = k0;
    r.khi = k1;
  }
  return r;
}

// X_j -= sum_{k in [klo, khi)} U_jk X_k for the rows j of bsolve_range, one
// workgroup per (subdomain, row, column block); MFMA, the next tile pair
// prefetched into registers.
template <class T, bool LT>
__global__ void __launch_bounds__(256) k_bsolve_update(int mode, int s, int s0, int pw,
                                                       const int64_t* __restrict__ pref, int nact,
                                                       const int* __restrict__ order, LocalLayout lay,
                                                       const int* __restrict__ nb, const int* __restrict__ nq,
                                                       const int64_t* __restrict__ xoff, int64_t ldx,
                                                       const T* __restrict__ fac, T* X,
                                                       const int4* __restrict__ tasks, const int* __restrict__ prof) {
  constexpr int LD = LdsLd<T>::v;
  constexpr int LDB = KfPitch<T>::v;
  __shared__ T As[TS * (LD > LDB ? LD : LDB)];  // A = U_jk: LT As[row * LDB + kk], else As[kk * LD + row]
  __shared__ T Bs[TS * LDB];                    // Bs[col * LDB + kk] = X_k(kk, col)
  const int64_t bid = blockIdx.x;
  int i, j, q;
  BsolveRange rg;
  if (tasks) {  // explicit list: subdomain x, row y, column block z, K tiles [w & 0xFFFFFF, + w >> 24)
    const int4 tk = tasks[bid];
    i = tk.x;
    j = tk.y;
    q = tk.z;
    rg.klo = tk.w & 0xFFFFFF;
    rg.khi = rg.klo + (tk.w >> 24);
  } else {
    const int slot = find_slot(pref, nact, bid);
    i = order[slot];
    const int64_t t = bid - pref[slot];
    rg = bsolve_range(mode, s, s0, pw, nb[i]);
    q = (int)(t % nq[i]);
    j = rg.jlo + (int)(t / nq[i]);
  }
  const int nt = lay.nt[i];
  // with a profile g (LT: the rows of L, tile (k, j) is zero when g(k) > j;
  // LU: the columns of U, tile (j, k) is zero when g(k) > j) zero tiles are skipped
  const int* g = prof ? prof + lay.toff[i] : nullptr;
  int k0 = rg.klo;
  while (k0 < rg.khi && g && g[k0] > j) k0++;
  if (k0 >= rg.khi) return;
  const int64_t M = ldx > 0 ? ldx : (int64_t)nt * TS;
  const T* base = fac + lay.foff[i];
  T* Xq = X + xoff[i] + (int64_t)q * TS * M;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) acc[x][y] = Mfma<T>::zero();
  constexpr int PER = TS2 / 256;
  T pa[PER], pb[PER];
  {
    const T* U = base + (LT ? tile_off(lay, i, 0, nt, k0, j) : tile_off(lay, i, 1, nt, j, k0));
    const T* Xk = Xq + (int64_t)k0 * TS;
#pragma unroll
    for (int u = 0; u < PER; u++) {
      const int e = tid + 256 * u;
      pa[u] = U[e];
      pb[u] = Xk[(int64_t)(e / TS) * M + e % TS];
    }
  }
  for (int k = k0; k < rg.khi;) {
    int kn = k + 1;
    while (kn < rg.khi && g && g[kn] > j) kn++;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; u++) {
      const int e = tid + 256 * u;
      const int a = e % TS, b = e / TS;
      if (LT)
        As[b * LDB + a] = pa[u];  // L_kj(a, b) = U_jk(b, a)
      else
        As[b * LD + a] = pa[u];
      Bs[b * LDB + a] = pb[u];
    }
    __syncthreads();
    if (kn < rg.khi) {
      const T* U = base + (LT ? tile_off(lay, i, 0, nt, kn, j) : tile_off(lay, i, 1, nt, j, kn));
      const T* Xk = Xq + (int64_t)kn * TS;
#pragma unroll
      for (int u = 0; u < PER; u++) {
        const int e = tid + 256 * u;
        pa[u] = U[e];
        pb[u] = Xk[(int64_t)(e / TS) * M + e % TS];
      }
    }
#pragma unroll 4
    for (int kk = 0; kk < TS; kk += 4) {
      T a0 = LT ? As[(wr + li) * LDB + kk + lk] : As[(kk + lk) * LD + wr + li];
      T a1 = LT ? As[(wr + 16 + li) * LDB + kk + lk] : As[(kk + lk) * LD + wr + 16 + li];
      T b0 = Bs[(wc + li) * LDB + kk + lk];
      T b1 = Bs[(wc + 16 + li) * LDB + kk + lk];
      acc[0][0] = Mfma<T>::mac(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<T>::mac(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<T>::mac(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<T>::mac(a1, b1, acc[1][1]);
    }
    k = kn;
  }
  T* Xj = Xq + (int64_t)j * TS;
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int col = wc + 16 * y + li;
#pragma unroll
      for (int qq = 0; qq < 4; qq++) {
        const int row = wr + 16 * x + Mfma<T>::row(lane, qq);
        Xj[(int64_t)col * M + row] -= acc[x][y][qq];
      }
    }
}

// ---------------------------------------------------------------------------
// Explicit inverse of the SPD local matrices (option local_inverse): from the
// Cholesky factor, W = L^{-1} (block lower triangular, same packed tile
// layout), then S = A_ii^{-1} = W^T W over the lower tiles with full
// symmetric diagonal tiles, written over the factor. Each local solve is
// then one product with S, which reads the lower tiles once, instead of a
// forward and a backward substitution that read them twice.
//
// W is formed right-looking by panels of PW block rows. Row j of W, for
// k < j: W_jk = -L_jj^{-1} sum_{l=k}^{j-1} L_jl W_lk. The W buffer starts at
// zero; after each panel the rows below it accumulate the panel's terms
// (k_tinv_update), and the panel's own terms are added when the row is
// finished (k_tinv_row). W_jj = L_jj^{-1} comes from the factorization.

// Finish row j (panel starting at j0) for the tiles k <= j of one
// subdomain: one workgroup per (subdomain, k).
template <class T>
__global__ void __launch_bounds__(256) k_tinv_row(int j, int j0, const int64_t* __restrict__ pref, int nact,
                                                  const int* __restrict__ order, LocalLayout lay,
                                                  const int64_t* __restrict__ woff, const T* __restrict__ fac,
                                                  const T* __restrict__ dinv, T* W, const int* __restrict__ prof) {
  constexpr int LD = LdsLd<T>::v;  // A operand (row, kk) at [kk * LD + row]
  constexpr int LDB = KfPitch<T>::v;  // B operand (kk, col) at [col * LDB + kk]
  __shared__ T As[TS * LD];
  __shared__ T Bs[TS * LDB];
  const int64_t bid = blockIdx.x;
  const int slot = find_slot(pref, nact, bid);
  const int i = order[slot];
  const int k = (int)(bid - pref[slot]);
  const int nt = lay.nt[i];
  const T* Lb = fac + lay.foff[i];
  T* Wb = W + woff[i];
  T* Wjk = Wb + tile_index(0, nt, j, k) * TS2;
  const T* Dj = dinv + (lay.toff[i] + j) * TS2;
  const int tid = threadIdx.x;
  if (k == j) {
    for (int e = tid; e < TS2; e += 256) Wjk[e] = Dj[e];
    return;
  }
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc[2][2];
  // start from the accumulated terms of earlier panels (none with a
  // profile: every term of the row is added here)
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int col = wc + 16 * y + li;
#pragma unroll
      for (int q = 0; q < 4; q++)
        acc[x][y][q] = prof ? T(0) : Wjk[col * TS + wr + 16 * x + Mfma<T>::row(lane, q)];
    }
  // L_jl = 0 left of the profile of row j
  const int l0 = max(max(k, j0), prof ? prof[lay.toff[i] + j] : 0);
  for (int l = l0; l < j; l++) {
    const T* Ljl = Lb + tile_off(lay, i, 0, nt, j, l);
    const T* Wlk = Wb + tile_index(0, nt, l, k) * TS2;
    __syncthreads();
    for (int e = tid; e < TS2; e += 256) {
      const int a = e % TS, b = e / TS;
      As[b * LD + a] = Ljl[e];
      Bs[b * LDB + a] = Wlk[e];
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < TS; kk += 4) {
      T a0 = As[(kk + lk) * LD + wr + li];
      T a1 = As[(kk + lk) * LD + wr + 16 + li];
      T b0 = Bs[(wc + li) * LDB + kk + lk];
      T b1 = Bs[(wc + 16 + li) * LDB + kk + lk];
      acc[0][0] = Mfma<T>::mac(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<T>::mac(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<T>::mac(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<T>::mac(a1, b1, acc[1][1]);
    }
  }
  // W_jk = -L_jj^{-1} acc
  __syncthreads();
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int col = wc + 16 * y + li;
#pragma unroll
      for (int q = 0; q < 4; q++) Bs[col * LDB + wr + 16 * x + Mfma<T>::row(lane, q)] = acc[x][y][q];
    }
  for (int e = tid; e < TS2; e += 256) As[(e / TS) * LD + e % TS] = Dj[e];
  __syncthreads();
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) acc[x][y] = Mfma<T>::zero();
#pragma unroll 4
  for (int kk = 0; kk < TS; kk += 4) {
    T a0 = As[(kk + lk) * LD + wr + li];
    T a1 = As[(kk + lk) * LD + wr + 16 + li];
    T b0 = Bs[(wc + li) * LDB + kk + lk];
    T b1 = Bs[(wc + 16 + li) * LDB + kk + lk];
    acc[0][0] = Mfma<T>::mac(a0, b0, acc[0][0]);
    acc[0][1] = Mfma<T>::mac(a0, b1, acc[0][1]);
    acc[1][0] = Mfma<T>::mac(a1, b0, acc[1][0]);
    acc[1][1] = Mfma<T>::mac(a1, b1, acc[1][1]);
  }
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int col = wc + 16 * y + li;
#pragma unroll
      for (int q = 0; q < 4; q++) Wjk[col * TS + wr + 16 * x + Mfma<T>::row(lane, q)] = -acc[x][y][q];
    }
}

// After the panel [j0, j1): W_rk += sum_{l in [max(k, j0), j1)} L_rl W_lk
// for the rows r >= j1 and columns k < j1 of every active subdomain
// (t -> r = j1 + t / j1, k = t % j1); MFMA, the next pair prefetched.
template <class T>
__global__ void __launch_bounds__(256) k_tinv_update(int j0, int j1, const int64_t* __restrict__ pref, int nact,
                                                     const int* __restrict__ order, LocalLayout lay,
                                                     const int64_t* __restrict__ woff, const T* __restrict__ fac,
                                                     T* W) {
  constexpr int LD = LdsLd<T>::v;
  constexpr int LDB = KfPitch<T>::v;
  __shared__ T As[TS * LD];
  __shared__ T Bs[TS * LDB];
  const int64_t bid = blockIdx.x;
  const int slot = find_slot(pref, nact, bid);
  const int i = order[slot];
  const int64_t t = bid - pref[slot];
  const int r = j1 + (int)(t / j1);
  const int k = (int)(t % j1);
  const int nt = lay.nt[i];
  const T* Lb = fac + lay.foff[i];
  T* Wb = W + woff[i];
  const int l0 = k > j0 ? k : j0;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) acc[x][y] = Mfma<T>::zero();
  constexpr int PER = TS2 / 256;
  T pa[PER], pb[PER];
  {
    const T* Lrl = Lb + tile_off(lay, i, 0, nt, r, l0);
    const T* Wlk = Wb + tile_index(0, nt, l0, k) * TS2;
#pragma unroll
    for (int u = 0; u < PER; u++) {
      pa[u] = Lrl[tid + 256 * u];
      pb[u] = Wlk[tid + 256 * u];
    }
  }
  for (int l = l0; l < j1; l++) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; u++) {
      const int e = tid + 256 * u;
      As[(e / TS) * LD + e % TS] = pa[u];
      Bs[(e / TS) * LDB + e % TS] = pb[u];
    }
    __syncthreads();
    if (l + 1 < j1) {
      const T* Lrl = Lb + tile_off(lay, i, 0, nt, r, l + 1);
      const T* Wlk = Wb + tile_index(0, nt, l + 1, k) * TS2;
#pragma unroll
      for (int u = 0; u < PER; u++) {
        pa[u] = Lrl[tid + 256 * u];
        pb[u] = Wlk[tid + 256 * u];
      }
    }
#pragma unroll 4
    for (int kk = 0; kk < TS; kk += 4) {
      T a0 = As[(kk + lk) * LD + wr + li];
      T a1 = As[(kk + lk) * LD + wr + 16 + li];
      T b0 = Bs[(wc + li) * LDB + kk + lk];
      T b1 = Bs[(wc + 16 + li) * LDB + kk + lk];
      acc[0][0] = Mfma<T>::mac(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<T>::mac(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<T>::mac(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<T>::mac(a1, b1, acc[1][1]);
    }
  }
  T* Wrk = Wb + tile_index(0, nt, r, k) * TS2;
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int col = wc + 16 * y + li;
#pragma unroll
      for (int q = 0; q < 4; q++) Wrk[col * TS + wr + 16 * x + Mfma<T>::row(lane, q)] += acc[x][y][q];
    }
}

// S_rc = sum_{k=r}^{nt-1} W_kr^T W_kc for every lower tile (r >= c), written
// over the factor; one workgroup per tile, the longest sums (small r) of
// the largest subdomains first. Both operands are kept as stored (kk
// fastest).
template <class T>
__global__ void __launch_bounds__(256) k_tinv_lauum(const int64_t* __restrict__ pref, int nact,
                                                    const int* __restrict__ order, LocalLayout lay,
                                                    const int64_t* __restrict__ woff, const T* __restrict__ W,
                                                    T* S) {
  constexpr int LDA = KfPitch<T>::v;  // A operand (row, kk) at [row * LDA + kk]
  constexpr int LDB = KfPitch<T>::v;  // B operand (kk, col) at [col * LDB + kk]
  __shared__ T As[TS * LDA];
  __shared__ T Bs[TS * LDB];
  const int64_t bid = blockIdx.x;
  const int slot = find_slot(pref, nact, bid);
  const int i = order[slot];
  const int64_t t = bid - pref[slot];
  int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((int64_t)(r + 1) * (r + 2) / 2 <= t) r++;
  while ((int64_t)r * (r + 1) / 2 > t) r--;
  const int c = (int)(t - (int64_t)r * (r + 1) / 2);
  const int nt = lay.nt[i];
  const T* Wb = W + woff[i];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) acc[x][y] = Mfma<T>::zero();
  constexpr int PER = TS2 / 256;
  T pa[PER], pb[PER];
  {
    const T* Wkr = Wb + tile_index(0, nt, r, r) * TS2;
    const T* Wkc = Wb + tile_index(0, nt, r, c) * TS2;
#pragma unroll
    for (int u = 0; u < PER; u++) {
      pa[u] = Wkr[tid + 256 * u];
      pb[u] = Wkc[tid + 256 * u];
    }
  }
  for (int k = r; k < nt; k++) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; u++) {
      const int e = tid + 256 * u;
      As[(e / TS) * LDA + e % TS] = pa[u];  // A(row = e / TS, kk = e % TS) = W_kr(kk, row)
      Bs[(e / TS) * LDB + e % TS] = pb[u];  // B(kk = e % TS, col = e / TS) = W_kc(kk, col)
    }
    __syncthreads();
    if (k + 1 < nt) {
      const T* Wkr = Wb + tile_index(0, nt, k + 1, r) * TS2;
      const T* Wkc = Wb + tile_index(0, nt, k + 1, c) * TS2;
#pragma unroll
      for (int u = 0; u < PER; u++) {
        pa[u] = Wkr[tid + 256 * u];
        pb[u] = Wkc[tid + 256 * u];
      }
    }
#pragma unroll 4
    for (int kk = 0; kk < TS; kk += 4) {
      T a0 = As[(wr + li) * LDA + kk + lk];
      T a1 = As[(wr + 16 + li) * LDA + kk + lk];
      T b0 = Bs[(wc + li) * LDB + kk + lk];
      T b1 = Bs[(wc + 16 + li) * LDB + kk + lk];
      acc[0][0] = Mfma<T>::mac(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<T>::mac(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<T>::mac(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<T>::mac(a1, b1, acc[1][1]);
    }
  }
  T* Src = S + lay.foff[i] + tile_index(0, nt, r, c) * TS2;
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int col = wc + 16 * y + li;
#pragma unroll
      for (int q = 0; q < 4; q++) Src[col * TS + wr + 16 * x + Mfma<T>::row(lane, q)] = acc[x][y][q];
    }
}

// With a narrow profile, S = A_ii^{-1} = L^{-T} W is formed by a block back
// substitution rather than by W^T W: L^T S = W gives, for the lower tiles,
//   S_rk = L_rr^{-T} (W_rk - sum_{c > r, f(c) <= r} L_cr^T S_ck),   k <= r,
// where only the rows c whose profile reaches column r contribute. Rows are
// done in descending order (one launch per r, one workgroup per tile
// (r, k)); S_rk replaces W_rk, which nothing reads afterwards (the terms of
// later rows read S_ck with c > r). The diagonal tile comes out full
// (symmetric), as the symmetric product wants it.
template <class T>
__global__ void __launch_bounds__(256) k_sinv_row(int r, const int64_t* __restrict__ pref, int nact,
                                                  const int* __restrict__ order, LocalLayout lay,
                                                  const int64_t* __restrict__ woff, const int* __restrict__ prof,
                                                  const T* __restrict__ fac, const T* __restrict__ dinv, T* W) {
  constexpr int LDA = KfPitch<T>::v;  // A operand (row, kk) at [row * LDA + kk]
  constexpr int LDB = KfPitch<T>::v;  // B operand (kk, col) at [col * LDB + kk]
  __shared__ T As[TS * LDA];
  __shared__ T Bs[TS * LDB];
  const int64_t bid = blockIdx.x;
  const int slot = find_slot(pref, nact, bid);
  const int i = order[slot];
  const int k = (int)(bid - pref[slot]);
  const int nt = lay.nt[i];
  const T* Lb = fac + lay.foff[i];
  T* Wb = W + woff[i];
  const int* f = prof + lay.toff[i];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) acc[x][y] = Mfma<T>::zero();
  constexpr int PER = TS2 / 256;
  T pa[PER], pb[PER];
  // the rows c > r with f(c) <= r, in ascending order; operands of the next
  // one are loaded while the current one is multiplied
  int c = r + 1;
  while (c < nt && f[c] > r) c++;
  if (c < nt) {
    const T* Lcr = Lb + tile_off(lay, i, 0, nt, c, r);
    const T* Sck = Wb + tile_index(0, nt, c, k) * TS2;
#pragma unroll
    for (int u = 0; u < PER; u++) {
      pa[u] = Lcr[tid + 256 * u];
      pb[u] = Sck[tid + 256 * u];
    }
  }
  while (c < nt) {
    int cn = c + 1;
    while (cn < nt && f[cn] > r) cn++;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; u++) {
      const int e = tid + 256 * u;
      As[(e / TS) * LDA + e % TS] = pa[u];  // A(row = e / TS, kk = e % TS) = L_cr(kk, row)
      Bs[(e / TS) * LDB + e % TS] = pb[u];  // B(kk = e % TS, col = e / TS) = S_ck(kk, col)
    }
    __syncthreads();
    if (cn < nt) {
      const T* Lcr = Lb + tile_off(lay, i, 0, nt, cn, r);
      const T* Sck = Wb + tile_index(0, nt, cn, k) * TS2;
#pragma unroll
      for (int u = 0; u < PER; u++) {
        pa[u] = Lcr[tid + 256 * u];
        pb[u] = Sck[tid + 256 * u];
      }
    }
#pragma unroll 4
    for (int kk = 0; kk < TS; kk += 4) {
      T a0 = As[(wr + li) * LDA + kk + lk];
      T a1 = As[(wr + 16 + li) * LDA + kk + lk];
      T b0 = Bs[(wc + li) * LDB + kk + lk];
      T b1 = Bs[(wc + 16 + li) * LDB + kk + lk];
      acc[0][0] = Mfma<T>::mac(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<T>::mac(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<T>::mac(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<T>::mac(a1, b1, acc[1][1]);
    }
    c = cn;
  }
  // right-hand side W_rk - acc into Bs (B operand layout), L_rr^{-1} into As
  // read transposed: A(row, kk) = L_rr^{-1}(kk, row)
  T* Wrk = Wb + tile_index(0, nt, r, k) * TS2;
  const T* Dr = dinv + (lay.toff[i] + r) * TS2;
  __syncthreads();
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int col = wc + 16 * y + li;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int row = wr + 16 * x + Mfma<T>::row(lane, q);
        Bs[col * LDB + row] = Wrk[col * TS + row] - acc[x][y][q];
      }
    }
  for (int e = tid; e < TS2; e += 256) As[(e / TS) * LDA + e % TS] = Dr[e];
  __syncthreads();
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) acc[x][y] = Mfma<T>::zero();
#pragma unroll 4
  for (int kk = 0; kk < TS; kk += 4) {
    T a0 = As[(wr + li) * LDA + kk + lk];
    T a1 = As[(wr + 16 + li) * LDA + kk + lk];
    T b0 = Bs[(wc + li) * LDB + kk + lk];
    T b1 = Bs[(wc + 16 + li) * LDB + kk + lk];
    acc[0][0] = Mfma<T>::mac(a0, b0, acc[0][0]);
    acc[0][1] = Mfma<T>::mac(a0, b1, acc[0][1]);
    acc[1][0] = Mfma<T>::mac(a1, b0, acc[1][0]);
    acc[1][1] = Mfma<T>::mac(a1, b1, acc[1][1]);
  }
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int col = wc + 16 * y + li;
#pragma unroll
      for (int q = 0; q < 4; q++) Wrk[col * TS + wr + 16 * x + Mfma<T>::row(lane, q)] = acc[x][y][q];
    }
}

// y_i = S_i x_i for every subdomain. The lower tiles are cut into blocks of
// B x B tiles (block row R, block column C <= R; B = 8 by default, or 4 for
// a single matrix, which then has enough blocks to fill the GPU; the
// autotuner may pick 4, 6 or 8 for the local inverses); one workgroup
// streams one block row by row (the tiles of a row are consecutive in
// storage). Thread t holds rows 4 (t % 16) + w and columns t / 16 + 16 u
// (w, u = 0..3) of each tile (four 16-byte non-temporal loads). For each
// tile row r of the block it writes the block's part of y_r; for each tile
// column c it writes the sum of S_rc^T x_r over the block's tiles below the
// diagonal (the terms of y_c that the upper triangle would hold). Partial
// sums per block rather than per tile keep the writes to about 2 / B of
// a 64-value vector per tile: interleaved with the read stream, writes cost
// far more than their size. k_symv_reduce adds the partial sums of each row
// in a fixed order.
// One block: subdomain factor at foff, x at voff; tile rows [r0, r1), tile
// columns [c0, c1) (only c <= r is stored); its partial sums at
// out * B * TS in the row and column arrays.
struct alignas(16) SymvBlock {
  int64_t foff, voff;
  int32_t r0, r1, c0, c1;
  int32_t out, pad_;
};

typedef float f32x4_nt __attribute__((ext_vector_type(4)));
typedef double f64x2_nt __attribute__((ext_vector_type(2)));

// four consecutive elements with non-temporal 16-byte loads
__device__ inline void load4(const float* p, float (&v)[4]) {
  const f32x4_nt q = stream_load(reinterpret_cast<const f32x4_nt*>(p));
  v[0] = q[0];
  v[1] = q[1];
  v[2] = q[2];
  v[3] = q[3];
}
__device__ inline void load4(const double* p, double (&v)[4]) {
  const f64x2_nt q0 = stream_load(reinterpret_cast<const f64x2_nt*>(p));
  const f64x2_nt q1 = stream_load(reinterpret_cast<const f64x2_nt*>(p) + 1);
  v[0] = q0[0];
  v[1] = q0[1];
  v[2] = q1[0];
  v[3] = q1[1];
}

// Lane moves within rows of 16 lanes (DPP): mirror l -> 15 - l, half mirror
// l -> 7 - l within each half row, and the quad swaps l ^ 1, l ^ 2.
template <int CTRL>
__device__ inline float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int DPP_ROW_MIRROR = 0x140, DPP_ROW_HALF_MIRROR = 0x141, DPP_QUAD_XOR1 = 0xB1, DPP_QUAD_XOR2 = 0x4E;

// Sum z[0..3] over the 16 lanes of a row (reduce-scatter, 5 lane moves):
// on return lane l of the row holds the total of z[(l & 15) >> 2].
template <class T>
__device__ inline T reduce_scatter4_16(const T (&z)[4], int lane) {
  const bool hi8 = (lane & 8) != 0, hi4 = (lane & 4) != 0;
  // partner l ^ 15 (mirror) has bit 3 flipped: keep z[0], z[1] (bit 3 clear) or z[2], z[3]
  const T k0 = (hi8 ? z[2] : z[0]) + dpp_move<DPP_ROW_MIRROR>(hi8 ? z[0] : z[2]);
  const T k1 = (hi8 ? z[3] : z[1]) + dpp_move<DPP_ROW_MIRROR>(hi8 ? z[1] : z[3]);
  // partner within the half row has bit 2 flipped (bit 3 kept)
  T v = (hi4 ? k1 : k0) + dpp_move<DPP_ROW_HALF_MIRROR>(hi4 ? k0 : k1);
  v += dpp_move<DPP_QUAD_XOR1>(v);
  v += dpp_move<DPP_QUAD_XOR2>(v);
  return v;
}

template <class T, int B>
__global__ void __launch_bounds__(256) k_symv(const SymvBlock* __restrict__ blocks, const T* __restrict__ S,
                                              const T* __restrict__ x, T* RP, T* CP,
                                              const int* __restrict__ done) {
  if (*done) return;
  __shared__ T red[4][TS];
  __shared__ T rbuf[B * TS];  // row partial sums of the block
  __shared__ T cbuf[B * TS];  // column partial sums of the block
  const SymvBlock bk = blocks[blockIdx.x];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int a0 = 4 * (tid & 15), b0 = tid >> 4;
  const T* Sb = S + bk.foff + 4 * tid;
  const T* xi = x + bk.voff;
  T cacc[B][4];
#pragma unroll
  for (int k = 0; k < B; k++)
#pragma unroll
    for (int u = 0; u < 4; u++) cacc[k][u] = T(0);
  for (int r = bk.r0; r < bk.r1; r++) {
    const int ce = r + 1 < bk.c1 ? r + 1 : bk.c1;  // tiles c0 .. ce - 1 of row r
    const T* rowp = Sb + ((int64_t)r * (r + 1) / 2 + bk.c0) * TS2;
    T xr[4];
#pragma unroll
    for (int w = 0; w < 4; w++) xr[w] = xi[r * TS + a0 + w];
    T yrow[4] = {T(0), T(0), T(0), T(0)};
    T vn[4][4], xn[4];
#pragma unroll
    for (int u = 0; u < 4; u++) load4(rowp + 1024 * u, vn[u]);
#pragma unroll
    for (int u = 0; u < 4; u++) xn[u] = xi[bk.c0 * TS + b0 + 16 * u];
#pragma unroll
    for (int k = 0; k < B; k++) {
      const int c = bk.c0 + k;
      if (c < ce) {
        T v[4][4], xc[4];  // v[u][w] = S(a0 + w, b0 + 16 u) of tile (r, c)
#pragma unroll
        for (int u = 0; u < 4; u++) {
          xc[u] = xn[u];
#pragma unroll
          for (int w = 0; w < 4; w++) v[u][w] = vn[u][w];
        }
        if (c + 1 < ce) {
#pragma unroll
          for (int u = 0; u < 4; u++) load4(rowp + (int64_t)(k + 1) * TS2 + 1024 * u, vn[u]);
#pragma unroll
          for (int u = 0; u < 4; u++) xn[u] = xi[(c + 1) * TS + b0 + 16 * u];
        }
#pragma unroll
        for (int w = 0; w < 4; w++)
#pragma unroll
          for (int u = 0; u < 4; u++) yrow[w] += v[u][w] * xc[u];
        if (c < r) {
#pragma unroll
          for (int u = 0; u < 4; u++)
#pragma unroll
            for (int w = 0; w < 4; w++) cacc[k][u] += v[u][w] * xr[w];
        }
      }
    }
    // rows a0 + w of y_r: add over the 16 threads with this tid % 16 (4 per
    // wave, lanes 16 apart, then the 4 waves)
#pragma unroll
    for (int w = 0; w < 4; w++) {
      T sum = yrow[w];
      sum += __shfl_xor(sum, 16);
      sum += __shfl_xor(sum, 32);
      yrow[w] = sum;
    }
    if (lane < 16)
#pragma unroll
      for (int w = 0; w < 4; w++) red[wave][a0 + w] = yrow[w];
    __syncthreads();
    if (tid < TS) rbuf[(r - bk.r0) * TS + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
    __syncthreads();
  }
  // column sums: the 16 lanes holding column b0 + 16 u of a tile form one
  // DPP row
#pragma unroll
  for (int k = 0; k < B; k++) {
    const T zs = reduce_scatter4_16(cacc[k], tid);
    if ((tid & 3) == 0) cbuf[k * TS + b0 + 16 * ((tid & 15) >> 2)] = zs;
  }
  __syncthreads();
  const int nr = bk.r1 - bk.r0, nc = bk.c1 - bk.c0;
  T* rp = RP + (int64_t)bk.out * B * TS;
  T* cp = CP + (int64_t)bk.out * B * TS;
  for (int e = tid; e < nr * TS; e += 256) rp[e] = rbuf[e];
  for (int e = tid; e < nc * TS; e += 256) cp[e] = cbuf[e];
}

// y_r = sum over the blocks of block row R = r / B of their row partial
// sum for r, plus sum over the blocks of block column R (block rows R' >= R)
// of their column partial sum for r; fixed order, x overwritten. One
// 64-thread workgroup per tile row; blk0 = first block of the subdomain.
struct alignas(16) SymvRow {
  int64_t voff;
  int32_t r, nbr, blk0, pad_;
};

template <class T, int B>
__global__ void __launch_bounds__(64) k_symv_reduce(const SymvRow* __restrict__ rows, const T* __restrict__ RP,
                                                    const T* __restrict__ CP, T* x, const int* __restrict__ done) {
  if (*done) return;
  const SymvRow rw = rows[blockIdx.x];
  const int a = threadIdx.x;
  const int R = rw.r / B, rho = rw.r % B;
  T s0 = T(0), s1 = T(0);
  for (int C = 0; C <= R; C++)
    s0 += RP[((int64_t)(rw.blk0 + R * (R + 1) / 2 + C) * B + rho) * TS + a];
  for (int Rp = R; Rp < rw.nbr; Rp++)
    s1 += CP[((int64_t)(rw.blk0 + Rp * (Rp + 1) / 2 + R) * B + rho) * TS + a];
  x[rw.voff + (int64_t)rw.r * TS + a] = s0 + s1;
}


// The same substitution by tasks of up to S consecutive block rows of one
// subdomain (S = 2; FP32 also 3 and 4). A task first accumulates, for all its rows, the blocks
// of the rows solved by earlier tasks (waiting on their flags as k_trsv
// does), then solves its rows one after the other with the blocks between
// them, taking the solved values from LDS, and publishes all its rows with
// one store completion and one flag each. On a long dependency chain this
// halves the number of round trips through memory (flag, values, store
// completion) on the chain. Task (x, y, z) = (subdomain, first row, number
// of rows); rows go up from y forward and down from y backward.
template <class T, int MODE, int S>
__global__ void __launch_bounds__(256) k_trsv_sr(const int4* __restrict__ tasks, int ntasks, int* counter,
                                                 int* flags, const int* __restrict__ epoch_ptr, LocalLayout lay,
                                                 const T* __restrict__ fac, const T* __restrict__ dinv, T* x,
                                                 int* err, const int* __restrict__ done,
                                                 const int* __restrict__ prof) {
  if (*done) return;
  constexpr bool BWD = (MODE == BWD_LT || MODE == BWD_U);
  constexpr bool TRANS = (MODE == BWD_LT);
  constexpr int KIND = (MODE == FWD_UL || MODE == BWD_U) ? 1 : 0;
  // columns whose tiles load together: with three FP32 rows a task takes
  // the previous task's three rows (its last dependencies) in one group, so
  // that their tiles and values arrive in one round trip
  constexpr int G = (sizeof(T) == 4 && S == 3) ? 3 : (TrsvUnroll<T>::v / S > 0 ? TrsvUnroll<T>::v / S : 1);
  constexpr int NIN = S * (S - 1) / 2;
  // the last dependency's tiles preloaded in registers (FP32, 2 rows; with
  // 3 rows that dependency loads in one group with the two before it), the
  // blocks between the task's rows in registers (2 rows) or in LDS (each
  // thread keeps its own pieces there)
  constexpr bool PRE = sizeof(T) == 4 && S <= 2;
  constexpr bool VIN_LDS = S > 2;
  static_assert(S <= 2 || sizeof(T) == 4, "tasks of more than two rows are built for FP32 only");
  typedef typename Vec4<T>::type V4;
  // partial sums: 16 rows of RP; the transposed modes store down a column
  // (16 lanes, one per row), so their rows are padded to spread the banks
  constexpr int RP = (MODE == BWD_LT) ? TS + 4 : TS;
  __shared__ T s_red[16 * RP];
  __shared__ T s_rhs[TS];
  __shared__ T s_x[S][TS];
  __shared__ T s_in[VIN_LDS ? NIN * TS2 : 1];
  __shared__ int s_task, s_lim;
  // backward: per column of the current wait round, its profile entry and
  // block base, read once by wave 0 instead of once per tile load
  __shared__ int s_g[BWD ? 64 : 1];
  __shared__ int64_t s_cb[BWD ? 64 : 1];
  const int tid = threadIdx.x;
  const int rg = tid & 15, cg = tid >> 4;
  const int epoch = *epoch_ptr;
  constexpr int step = BWD ? -1 : 1;
  const V4 zero4 = V4{T(0), T(0), T(0), T(0)};
  for (;;) {
    if (tid == 0) s_task = atomicAdd(counter, 1);
    __syncthreads();
    const int t = s_task;
    if (t >= ntasks) break;
    const int4 tk = tasks[t];
    const int i = tk.x, r0 = tk.y, cnt = tk.z;
    const int nt = lay.nt[i];
    const T* base = fac + lay.foff[i];
    T* xi = x + lay.voff[i];
    int* fl = flags + lay.toff[i];
    const int* fp = prof ? prof + lay.toff[i] : nullptr;
    // is the block that row rs takes from block row cc inside the profile?
    auto live = [&](int rs, int cc) { return !fp || (BWD ? fp[cc] <= rs : fp[rs] <= cc); };
    // block row rs takes from block row cc: forward (rs, cc) = row base of
    // rs + cc (row bases of the task's rows kept in registers); backward
    // (cc, rs) of L or (rs, cc) of U, from the base of cc
    const int64_t* trw = lay.trow ? lay.trow + lay.toff[i] : nullptr;
    const int64_t* tcl = lay.tcol ? lay.tcol + lay.toff[i] : nullptr;
    auto rowb = [&](int q) -> int64_t { return trw ? trw[q] : tile_index(KIND, nt, q, 0); };
    int64_t rb[S];
#pragma unroll
    for (int q = 0; q < S; q++) rb[q] = (!BWD && q < cnt) ? rowb(r0 + step * q) : 0;
    // base of block row cc for the backward blocks: (cc, rs) of L at
    // rowb(cc) + rs, (rs, cc) of U at tcol(cc) + rs
    auto colb = [&](int cc) -> int64_t { return TRANS ? rowb(cc) : (tcl ? tcl[cc] : (int64_t)cc); };
    const int64_t cstride = TRANS || tcl ? 1 : nt;
    // q: the row's place in the task (rs = r0 + step q); cb = colb(cc) for backward
    auto tile_of = [&](int q, int cc, int64_t cb) {
      const int rs = r0 + step * q;
      const int64_t t = BWD ? cb + (int64_t)rs * cstride : rb[q] + cc;
      return base + t * TS2;
    };
    // diagonal-tile inverses and the blocks between the task's rows -> registers
    V4 dv[S][4];
#pragma unroll
    for (int q = 0; q < S; q++) {
      const int rs = r0 + step * q;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        dv[q][j] = zero4;
        if (q < cnt) {
          dv[q][j] = stream_load(reinterpret_cast<const V4*>(dinv + (lay.toff[i] + rs) * TS2 + (cg + 16 * j) * TS +
                                                             4 * rg));
          if (MODE == FWD_UL || MODE == BWD_U) {
            const int col = cg + 16 * j, a0 = 4 * rg;
            const bool lower = MODE == FWD_UL;
            if (lower ? !(a0 + 0 > col) : !(a0 + 0 <= col)) dv[q][j].x = T(0);
            if (lower ? !(a0 + 1 > col) : !(a0 + 1 <= col)) dv[q][j].y = T(0);
            if (lower ? !(a0 + 2 > col) : !(a0 + 2 <= col)) dv[q][j].z = T(0);
            if (lower ? !(a0 + 3 > col) : !(a0 + 3 <= col)) dv[q][j].w = T(0);
          }
        }
      }
    }
    V4 vin[VIN_LDS || NIN == 0 ? 1 : NIN][4];
    auto vin_slot = [&](int idx, int j) -> V4* {
      return reinterpret_cast<V4*>(&s_in[(VIN_LDS ? idx * TS2 : 0) + (cg + 16 * j) * TS + 4 * rg]);
    };
#pragma unroll
    for (int s = 1; s < S; s++)
#pragma unroll
      for (int q = 0; q < s; q++) {
        const int rs = r0 + step * s, rq = r0 + step * q;
        const bool on = s < cnt && live(rs, rq);
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const V4 v = on ? stream_load(reinterpret_cast<const V4*>(tile_of(s, rq, BWD ? colb(rq) : 0) + (cg + 16 * j) * TS + 4 * rg))
                          : zero4;
          if (VIN_LDS)
            *vin_slot(s * (s - 1) / 2 + q, j) = v;
          else
            vin[VIN_LDS ? 0 : s * (s - 1) / 2 + q][j] = v;
        }
      }
    T brow[S];
#pragma unroll
    for (int q = 0; q < S; q++) brow[q] = (tid < 64 && q < cnt) ? xi[(r0 + step * q) * TS + tid] : T(0);
    T acc[S][4];
#pragma unroll
    for (int q = 0; q < S; q++)
#pragma unroll
      for (int j = 0; j < 4; j++) acc[q][j] = T(0);
    // rows solved by earlier tasks: forward c in [min f(rs), r0), backward c in (r0, nt)
    int c = BWD ? nt - 1 : 0;
    if (!BWD && fp) {
      c = r0;
#pragma unroll
      for (int q = 0; q < S; q++)
        if (q < cnt) c = min(c, fp[r0 + q]);
    }
    int fr[S];  // forward: the profile entries of the task's rows
#pragma unroll
    for (int q = 0; q < S; q++) fr[q] = (!BWD && fp && q < cnt) ? fp[r0 + q] : 0;
    const int c_last = r0 - step;  // the previous task's last row: almost always the last dependency
    V4 vlast[PRE ? S : 1][4];
    if (PRE) {
      const bool has = BWD ? (c_last < nt) : (c_last >= 0);
#pragma unroll
      for (int q = 0; q < (PRE ? S : 1); q++) {
        const int rs = r0 + step * q;
        const bool on = has && q < cnt && live(rs, c_last);
#pragma unroll
        for (int j = 0; j < 4; j++)
          vlast[q][j] =
              on ? stream_load(reinterpret_cast<const V4*>(tile_of(q, c_last, BWD ? colb(c_last) : 0) + (cg + 16 * j) * TS + 4 * rg)) : zero4;
      }
    }
    while (BWD ? (c > r0) : (c < r0)) {
      if (tid < 64) {
        // backward: the task's rows are r0 and below, so row cc is read only if g(cc) <= r0
        int gq = 0;
        int64_t bq = 0;
        const int lim =
            wait_rows<BWD, BWD>(c, r0, fl, epoch, BWD ? fp : nullptr, r0, err, BWD ? (TRANS ? trw : tcl) : nullptr,
                                &gq, &bq);
        if (BWD && tid < c - lim) {
          const int cc = c - tid;
          s_g[tid] = gq;
          s_cb[tid] = TRANS ? (trw ? bq : tile_index(KIND, nt, cc, 0)) : (tcl ? bq : (int64_t)cc);
        }
        if (tid == 0) s_lim = lim;
      }
      __syncthreads();
      const int lim = s_lim;
      const int ncol = BWD ? c - lim : lim - c;
      for (int d = 0; d < ncol; d += G) {
        V4 v[G][S][4];
        T xs[G][4];
#pragma unroll
        for (int g = 0; g < G; g++) {
          const int cc = c + step * (d + g);
          const bool col_on = d + g < ncol;
          const int64_t cb = BWD && col_on ? s_cb[d + g] : 0;
          const int gc = BWD && col_on ? s_g[d + g] : 0;
#pragma unroll
          for (int q = 0; q < S; q++) {
            const int rs = r0 + step * q;
            const bool on = col_on && q < cnt && (BWD ? gc <= rs : fr[q] <= cc);
            const bool pre = PRE && cc == c_last;
#pragma unroll
            for (int j = 0; j < 4; j++)
              v[g][q][j] = !on ? zero4
                               : (pre ? vlast[PRE ? q : 0][j]
                                      : stream_load(reinterpret_cast<const V4*>(tile_of(q, cc, cb) + (cg + 16 * j) * TS +
                                                                                4 * rg)));
          }
          const T* xc = xi + cc * TS;
#pragma unroll
          for (int j = 0; j < 4; j++)
            xs[g][j] = col_on ? load_shared(TRANS ? xc + 4 * rg + j : xc + cg + 16 * j) : T(0);
        }
#pragma unroll
        for (int g = 0; g < G; g++)
#pragma unroll
          for (int q = 0; q < S; q++) {
            if (!TRANS) {
#pragma unroll
              for (int j = 0; j < 4; j++) {
                acc[q][0] += v[g][q][j].x * xs[g][j];
                acc[q][1] += v[g][q][j].y * xs[g][j];
                acc[q][2] += v[g][q][j].z * xs[g][j];
                acc[q][3] += v[g][q][j].w * xs[g][j];
              }
            } else {
#pragma unroll
              for (int j = 0; j < 4; j++)
                acc[q][j] += v[g][q][j].x * xs[g][0] + v[g][q][j].y * xs[g][1] + v[g][q][j].z * xs[g][2] +
                             v[g][q][j].w * xs[g][3];
            }
          }
      }
      c = lim;
      __syncthreads();
    }
    // the task's rows in order, each with the blocks of the rows solved before it here
#pragma unroll
    for (int s = 0; s < S; s++) {
      if (s >= cnt) break;
#pragma unroll
      for (int q = 0; q < s; q++) {
        const int idx = s * (s - 1) / 2 + q;
        V4 w[4];
#pragma unroll
        for (int j = 0; j < 4; j++) w[j] = VIN_LDS ? *vin_slot(idx, j) : vin[VIN_LDS ? 0 : idx][j];
        if (!TRANS) {
#pragma unroll
          for (int j = 0; j < 4; j++) {
            const T xv = s_x[q][cg + 16 * j];
            acc[s][0] += w[j].x * xv;
            acc[s][1] += w[j].y * xv;
            acc[s][2] += w[j].z * xv;
            acc[s][3] += w[j].w * xv;
          }
        } else {
          const T x0 = s_x[q][4 * rg], x1 = s_x[q][4 * rg + 1], x2 = s_x[q][4 * rg + 2], x3 = s_x[q][4 * rg + 3];
#pragma unroll
          for (int j = 0; j < 4; j++) acc[s][j] += w[j].x * x0 + w[j].y * x1 + w[j].z * x2 + w[j].w * x3;
        }
      }
      if (!TRANS) {
#pragma unroll
        for (int q = 0; q < 4; q++) s_red[cg * RP + 4 * rg + q] = acc[s][q];
      } else {
#pragma unroll
        for (int j = 0; j < 4; j++) s_red[rg * RP + cg + 16 * j] = acc[s][j];
      }
      __syncthreads();
      if (tid < 64) {
        T sum = T(0);
#pragma unroll
        for (int g = 0; g < 16; g++) sum += s_red[g * RP + tid];
        s_rhs[tid] = brow[s] - sum;
      }
      __syncthreads();
      T a2[4] = {T(0), T(0), T(0), T(0)};
      if (!TRANS) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const T rv = s_rhs[cg + 16 * j];
          a2[0] += dv[s][j].x * rv;
          a2[1] += dv[s][j].y * rv;
          a2[2] += dv[s][j].z * rv;
          a2[3] += dv[s][j].w * rv;
        }
#pragma unroll
        for (int q = 0; q < 4; q++) s_red[cg * RP + 4 * rg + q] = a2[q];
      } else {
        const T q0 = s_rhs[4 * rg], q1 = s_rhs[4 * rg + 1], q2 = s_rhs[4 * rg + 2], q3 = s_rhs[4 * rg + 3];
#pragma unroll
        for (int j = 0; j < 4; j++) a2[j] = dv[s][j].x * q0 + dv[s][j].y * q1 + dv[s][j].z * q2 + dv[s][j].w * q3;
#pragma unroll
        for (int j = 0; j < 4; j++) s_red[rg * RP + cg + 16 * j] = a2[j];
      }
      __syncthreads();
      if (tid < 64) {
        T val = T(0);
#pragma unroll
        for (int g = 0; g < 16; g++) val += s_red[g * RP + tid];
        if (MODE == FWD_UL) val += s_rhs[tid];  // unit diagonal of L
        s_x[s][tid] = val;
        store_shared(xi + (r0 + step * s) * TS + tid, val);
      }
      __syncthreads();
    }
    if (tid < 64) {
      __builtin_amdgcn_s_waitcnt(0);  // the coherent stores of every row have completed
      if (tid == 0)
        for (int s = 0; s < cnt; s++)
          __hip_atomic_store(&fl[r0 + step * s], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }
}

__global__ void k_solve_begin(int* counters, const int* done) {
  if (*done) return;
  counters[0] = 0;
  counters[1] = 0;
  counters[2] += 1;
}

template <class T, int S>
void trsv_rows_s(hipStream_t s, int mode, SolvePlan& p, int grid, int* counter, const int* epoch,
                 const LocalLayout& lay, const T* fac, const T* dinv, T* x, int* err, const int* done,
                 const int* prof) {
  const int ntasks = p.ntasks;
  switch (mode) {
    case FWD_L:
      hipLaunchKernelGGL((k_trsv_sr<T, FWD_L, S>), dim3(grid), dim3(256), 0, s, p.tasks.p, ntasks, counter, p.flags.p,
                         epoch, lay, fac, dinv, x, err, done, prof);
      break;
    case BWD_LT:
      hipLaunchKernelGGL((k_trsv_sr<T, BWD_LT, S>), dim3(grid), dim3(256), 0, s, p.tasks.p, ntasks, counter, p.flags.p,
                         epoch, lay, fac, dinv, x, err, done, prof);
      break;
    case FWD_UL:
      hipLaunchKernelGGL((k_trsv_sr<T, FWD_UL, S>), dim3(grid), dim3(256), 0, s, p.tasks.p, ntasks, counter, p.flags.p,
                         epoch, lay, fac, dinv, x, err, done, prof);
      break;
    default:
      hipLaunchKernelGGL((k_trsv_sr<T, BWD_U, S>), dim3(grid), dim3(256), 0, s, p.tasks.p, ntasks, counter, p.flags.p,
                         epoch, lay, fac, dinv, x, err, done, prof);
      break;
  }
  TLS_LAUNCH_CHECK();
}

template <class T>
void trsv_rows(hipStream_t s, int mode, SolvePlan& p, int grid, int* counter, const int* epoch,
               const LocalLayout& lay, const T* fac, const T* dinv, T* x, int* err, const int* done,
               const int* prof);
template <>
void trsv_rows<float>(hipStream_t s, int mode, SolvePlan& p, int grid, int* counter, const int* epoch,
                      const LocalLayout& lay, const float* fac, const float* dinv, float* x, int* err,
                      const int* done, const int* prof) {
  switch (p.rows) {
    case 2:
      trsv_rows_s<float, 2>(s, mode, p, grid, counter, epoch, lay, fac, dinv, x, err, done, prof);
      break;
    case 3:
      trsv_rows_s<float, 3>(s, mode, p, grid, counter, epoch, lay, fac, dinv, x, err, done, prof);
      break;
    case 4:
      trsv_rows_s<float, 4>(s, mode, p, grid, counter, epoch, lay, fac, dinv, x, err, done, prof);
      break;
    default:
      fail(TLS_E_ARG, "triangular-solve tasks of 1 to 4 block rows");
  }
}
template <>
void trsv_rows<double>(hipStream_t s, int mode, SolvePlan& p, int grid, int* counter, const int* epoch,
                       const LocalLayout& lay, const double* fac, const double* dinv, double* x, int* err,
                       const int* done, const int* prof) {
  if (p.rows != 2) fail(TLS_E_ARG, "FP64 triangular-solve tasks of 1 or 2 block rows");
  trsv_rows_s<double, 2>(s, mode, p, grid, counter, epoch, lay, fac, dinv, x, err, done, prof);
}

template <class T>
void trsv(hipStream_t s, int mode, SolvePlan& p, int* counter, const int* epoch, const LocalLayout& lay,
          const T* fac, const T* dinv, T* x, int* err, const int* done, int grid, const int* prof = nullptr) {
  const int ntasks = p.ntasks;
  if (ntasks == 0) return;
  // more workgroups than tasks handed out ahead of their dependencies
  grid = std::max(p.early + 1, std::min(grid, ntasks));
  if (p.rows > 1) {
    trsv_rows<T>(s, mode, p, grid, counter, epoch, lay, fac, dinv, x, err, done, prof);
    return;
  }
  switch (mode) {
    case FWD_L:
      hipLaunchKernelGGL((k_trsv<T, FWD_L>), dim3(grid), dim3(256), 0, s, p.tasks.p, ntasks, counter, p.flags.p, epoch,
                         lay, fac, dinv, x, err, done, prof);
      break;
    case BWD_LT:
      hipLaunchKernelGGL((k_trsv<T, BWD_LT>), dim3(grid), dim3(256), 0, s, p.tasks.p, ntasks, counter, p.flags.p,
                         epoch, lay, fac, dinv, x, err, done, prof);
      break;
    case FWD_UL:
      hipLaunchKernelGGL((k_trsv<T, FWD_UL>), dim3(grid), dim3(256), 0, s, p.tasks.p, ntasks, counter, p.flags.p,
                         epoch, lay, fac, dinv, x, err, done, prof);
      break;
    default:
      hipLaunchKernelGGL((k_trsv<T, BWD_U>), dim3(grid), dim3(256), 0, s, p.tasks.p, ntasks, counter, p.flags.p, epoch,
                         lay, fac, dinv, x, err, done, prof);
      break;
  }
  TLS_LAUNCH_CHECK();
}

}  // namespace

void factor_tiles_f64(hipStream_t s, int N, const std::vector<int>& nt, const LocalLayout& lay, double* fac,
                      double* dinv, int* err) {
  factor_tiles<double>(s, N, nt, lay, fac, dinv, err);
}

void trsv_f64(hipStream_t s, int mode, SolvePlan& p, int* counter, const int* epoch, const LocalLayout& lay,
              const double* fac, const double* dinv, double* x, int* err, const int* done, int grid) {
  trsv<double>(s, mode, p, counter, epoch, lay, fac, dinv, x, err, done, grid);
}


void solve_begin(hipStream_t s, int* counters, const int* done) {
  hipLaunchKernelGGL(k_solve_begin, dim3(1), dim3(1), 0, s, counters, done);
  TLS_LAUNCH_CHECK();
}

// The tile profiles of every A_ii (a pass of the gather loop that only
// records, per tile row, the first tile column holding a nonzero of the
// lower part, and for LU per tile column the first tile row of the upper
// part), then the storage of the factors: the tiles inside the profiles,
// row by row (for LU the strictly upper tiles column by column after the
// rows). The full packed offsets are kept for the explicit inverses.
static void profile_storage(tls_ctx* c, int stride) {
  hipStream_t s = c->stream;
  const int total = c->h_sub_ptr[c->N];
  const LocalLayout lay = c->layout();
  const int64_t colp = c->kind == 1 ? c->sum_nt : 0;
  c->prof.alloc(c->sum_nt + colp);
  hipLaunchKernelGGL(k_prof_init, dim3(c->N), dim3(256), 0, s, c->N, lay, colp, c->prof.p);
  TLS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gather<float>, dim3(div_up(total, 256)), dim3(256), 0, s, total, c->sub_idx.p,
                     c->sub_of_pos.p, c->sub_ptr.p, c->layer_ptr.p, stride, c->row_ptr.p, c->col_idx.p, c->val.p,
                     nullptr, lay, c->kind, (float*)nullptr, c->prof.p, colp);
  TLS_LAUNCH_CHECK();
  c->h_prof = download(c->prof.p, c->sum_nt + colp, s);
  const int N = c->N;
  c->h_soff = c->h_foff;
  c->h_trow.assign(c->sum_nt, 0);
  if (c->kind == 1) c->h_tcol.assign(c->sum_nt, 0);
  for (int i = 0; i < N; i++) {
    const int64_t t0 = c->h_toff[i];
    int64_t cnt = 0;
    // tile (r, c) at trow[r] + c (row storage), (r, c) above the diagonal
    // at tcol[c] + r (LU, column storage)
    for (int r = 0; r < c->h_nt[i]; r++) {
      c->h_trow[t0 + r] = cnt - c->h_prof[t0 + r];
      cnt += r - c->h_prof[t0 + r] + 1;
    }
    if (c->kind == 1)
      for (int cc = 0; cc < c->h_nt[i]; cc++) {
        c->h_tcol[t0 + cc] = cnt - c->h_prof[c->sum_nt + t0 + cc];
        cnt += cc - c->h_prof[c->sum_nt + t0 + cc];
      }
    c->h_foff[i + 1] = c->h_foff[i] + cnt * TS2;
  }
  c->fac_elems = c->h_foff[N];
  c->d_foff.upload(c->h_foff, s);
  c->d_trow.upload(c->h_trow, s);
  if (c->kind == 1) c->d_tcol.upload(c->h_tcol, s);
  c->prof_store = true;
  TLS_HIP(hipStreamSynchronize(s));
}

void gather_local(tls_ctx* c) {
  hipStream_t s = c->stream;
  const int total = c->h_sub_ptr[c->N];
  LocalLayout lay = c->layout();
  const int stride = c->delta + 2;
  const double* scale = nullptr;
  if (c->opt.jacobi_scale) {
    c->scale.alloc(c->sum_M);
    TLS_HIP(hipMemsetAsync(c->scale.p, 0, sizeof(double) * c->sum_M, s));
    TLS_HIP(hipMemsetAsync(c->errflag.p, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_jacobi_scale, dim3(div_up(total, 256)), dim3(256), 0, s, total, c->sub_idx.p,
                       c->sub_of_pos.p, c->sub_ptr.p, c->d_voff.p, c->row_ptr.p, c->col_idx.p, c->val.p,
                       c->scale.p, c->errflag.p);
    TLS_LAUNCH_CHECK();
    if (download(c->errflag.p, 1, s)[0]) fail(TLS_E_NOT_SPD, "non-positive diagonal entry (Jacobi scaling)");
    scale = c->scale.p;
  }
  if (!c->prof_store) profile_storage(c, stride);
  lay = c->layout();
  const int64_t colp = c->kind == 1 ? c->sum_nt : 0;
  if (c->fp32) {
    c->fac32.alloc(c->fac_elems);
    TLS_HIP(hipMemsetAsync(c->fac32.p, 0, sizeof(float) * c->fac_elems, s));
    hipLaunchKernelGGL(k_pad_identity<float>, dim3(c->N), dim3(64), 0, s, c->N, lay, c->kind, c->fac32.p);
    TLS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gather<float>, dim3(div_up(total, 256)), dim3(256), 0, s, total, c->sub_idx.p,
                       c->sub_of_pos.p, c->sub_ptr.p, c->layer_ptr.p, stride, c->row_ptr.p, c->col_idx.p,
                       c->val.p, scale, lay, c->kind, c->fac32.p, c->prof.p, colp);
  } else {
    c->fac64.alloc(c->fac_elems);
    TLS_HIP(hipMemsetAsync(c->fac64.p, 0, sizeof(double) * c->fac_elems, s));
    hipLaunchKernelGGL(k_pad_identity<double>, dim3(c->N), dim3(64), 0, s, c->N, lay, c->kind, c->fac64.p);
    TLS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gather<double>, dim3(div_up(total, 256)), dim3(256), 0, s, total, c->sub_idx.p,
                       c->sub_of_pos.p, c->sub_ptr.p, c->layer_ptr.p, stride, c->row_ptr.p, c->col_idx.p,
                       c->val.p, scale, lay, c->kind, c->fac64.p, c->prof.p, colp);
  }
  TLS_LAUNCH_CHECK();
  TLS_HIP(hipStreamSynchronize(s));
}

void factor_local(tls_ctx* c) {
  TLS_HIP(hipMemsetAsync(c->errflag.p, 0, sizeof(int), c->stream));
  // both factorizations form the inverses of the diagonal tiles as they go
  if (c->fp32)
    c->dinv32.alloc((size_t)c->sum_nt * TS2);
  else
    c->dinv64.alloc((size_t)c->sum_nt * TS2);
  if (c->kind == 0) {
    const int* prof = c->h_prof.empty() ? nullptr : c->h_prof.data();
    if (c->fp32)
      c->flops_factor = factor_tiles<float>(c->stream, c->N, c->h_nt, c->layout(), c->fac32.p, c->dinv32.p,
                                            c->errflag.p, c->factor_panel, prof, &c->h_toff);
    else
      c->flops_factor = factor_tiles<double>(c->stream, c->N, c->h_nt, c->layout(), c->fac64.p, c->dinv64.p,
                                             c->errflag.p, c->factor_panel, prof, &c->h_toff);
  } else {
    const int* pr = c->h_prof.empty() ? nullptr : c->h_prof.data();
    const int* pc = pr ? pr + c->sum_nt : nullptr;
    if (c->fp32)
      c->flops_factor = factor_tiles_lu<float>(c->stream, c->N, c->h_nt, c->layout(), c->fac32.p, c->dinv32.p,
                                               c->errflag.p, c->factor_panel, pr, pc, &c->h_toff);
    else
      c->flops_factor = factor_tiles_lu<double>(c->stream, c->N, c->h_nt, c->layout(), c->fac64.p, c->dinv64.p,
                                                c->errflag.p, c->factor_panel, pr, pc, &c->h_toff);
  }
  int err = download(c->errflag.p, 1, c->stream)[0];
  if (err & ERR_PIVOT) {
    if (c->kind == 0) fail(TLS_E_NOT_SPD, "non-positive pivot in a local Cholesky factorization");
    fail(TLS_E_SINGULAR, "zero or non-finite pivot in a local LU factorization (no pivoting)");
  }
  TLS_HIP(hipStreamSynchronize(c->stream));
}

void build_plan(SolvePlan& p, bool bwd, const std::vector<int>& nt, const std::vector<int64_t>& toff, int order,
                hipStream_t s, int S, const std::vector<int>* width) {
  // A task is S consecutive block rows (the last task of a subdomain may
  // hold fewer); task q of subdomain i covers rows qS .. (forward) or
  // nt_i - 1 - qS down (backward) and has "position" q in its dependency
  // chain of n_i = ceil(nt_i / S) tasks. Every ordering below sorts a
  // subdomain's tasks by position, so a task only ever waits on tasks
  // handed out before it (nt below counts tasks):
  //   1 level order         key = position
  //   2 normalized progress key = position / nt_i
  //   3 longest chain first key = position + (max nt - nt_i)
  //   4, 5 progress with a lead for large subdomains:
  //         key = position / nt_i * (1 - lead * nt_i / max nt), lead 0.3 / 0.6,
  //         so that the long rows of the largest chains are handed out
  //         before the end and stream most of their tiles early
  // With the tiles each row reads (width, at toff_i + r), the widest tasks
  // (at most EARLY of them, each reading at least 64 tiles) are handed out
  // ahead of their place, by one position per LEAD_TILES tiles, so that they
  // stream their blocks while the chain catches up instead of after it.
  // Such a task may wait on tasks handed out after it; with fewer early
  // tasks than resident workgroups some workgroup is always free to take
  // those, so every wait still ends.
  constexpr int EARLY = 64, LEAD_TILES = 24;
  const int N = (int)nt.size();
  std::vector<int> nq(N);
  for (int i = 0; i < N; i++) nq[i] = (nt[i] + S - 1) / S;
  int maxnt = 0;
  for (int v : nq) maxnt = std::max(maxnt, v);
  std::vector<std::vector<int>> lead(N);
  if (width) {
    struct Wide {
      int64_t w;
      int i, pos;
    };
    std::vector<Wide> wide;
    for (int i = 0; i < N; i++) {
      lead[i].assign(nq[i], 0);
      for (int pos = 0; pos < nq[i]; pos++) {
        int64_t w = 0;
        for (int q = 0; q < S && pos * S + q < nt[i]; q++) {
          const int r = bwd ? nt[i] - 1 - (pos * S + q) : pos * S + q;
          w += (*width)[toff[i] + r];
        }
        if (w >= 64) wide.push_back(Wide{w, i, pos});
      }
    }
    std::stable_sort(wide.begin(), wide.end(), [](const Wide& a, const Wide& b) { return a.w > b.w; });
    for (size_t k = 0; k < wide.size() && k < (size_t)EARLY; k++)
      lead[wide[k].i][wide[k].pos] = (int)std::min<int64_t>(wide[k].pos, wide[k].w / LEAD_TILES);
  }
  p.early = 0;
  for (const auto& l : lead)
    for (int v : l) p.early += v > 0;
  struct Item {
    double key;
    int i, pos;
  };
  std::vector<Item> items;
  for (int i = 0; i < N; i++)
    for (int pos0 = 0; pos0 < nq[i]; pos0++) {
      const int pos = width ? pos0 - lead[i][pos0] : pos0;  // position the key is computed from
      double key;
      if (order == 2)
        key = (pos + 0.5) / nq[i];
      else if (order == 3)
        key = (double)(pos + maxnt - nq[i]);
      else if (order >= 4)
        key = (pos + 0.5) / nq[i] * (1.0 - (order == 4 ? 0.3 : 0.6) * nq[i] / std::max(maxnt, 1));
      else
        key = (double)pos;
      items.push_back(Item{key, i, pos0});
    }
  std::stable_sort(items.begin(), items.end(), [&](const Item& a, const Item& b) {
    if (a.key != b.key) return a.key < b.key;
    if (nq[a.i] != nq[b.i]) return nq[a.i] > nq[b.i];
    if (a.i != b.i) return a.i < b.i;
    return a.pos < b.pos;
  });
  std::vector<int4> tasks;
  tasks.reserve(items.size());
  for (const Item& it : items) {
    const int first = it.pos * S, rows = std::min(S, nt[it.i] - first);
    tasks.push_back(make_int4(it.i, bwd ? nt[it.i] - 1 - first : first, rows, 0));
  }
  p.rows = S;
  const int64_t rows = N ? toff[N] : 0;
  p.tasks.upload(tasks, s);
  p.ntasks = (int)tasks.size();
  p.flags.alloc(std::max<int64_t>(rows, 1));
  p.order = order;
  TLS_HIP(hipMemsetAsync(p.flags.p, 0, sizeof(int) * std::max<int64_t>(rows, 1), s));
  TLS_HIP(hipStreamSynchronize(s));
}

void build_local_plans(tls_ctx* c, int order, int rows, int order_b) {
  if (order_b <= 0) order_b = order;
  // tiles each row reads inside the profiles: forward r - f(r), backward
  // the rows c > r whose profile g reaches r (g = f for Cholesky, the
  // column profile of U for LU)
  std::vector<int> wf, wb;
  if (!c->h_prof.empty()) {
    wf.assign(c->sum_nt, 0);
    wb.assign(c->sum_nt, 0);
    const int* g = c->h_prof.data() + (c->kind == 1 ? c->sum_nt : 0);
    for (int i = 0; i < c->N; i++) {
      const int64_t t0 = c->h_toff[i];
      const int nt = c->h_nt[i];
      for (int r = 0; r < nt; r++) {
        wf[t0 + r] = r - c->h_prof[t0 + r];
        for (int cc = r + 1; cc < nt; cc++) wb[t0 + r] += g[t0 + cc] <= r;
      }
    }
  }
  build_plan(c->plan_fwd, false, c->h_nt, c->h_toff, order, c->stream, rows, wf.empty() ? nullptr : &wf);
  build_plan(c->plan_bwd, true, c->h_nt, c->h_toff, order_b, c->stream, rows, wb.empty() ? nullptr : &wb);
  c->solve_order = order;
  c->solve_order_b = order_b;
  c->solve_rows = rows;
}

void build_solve_tasks(tls_ctx* c) {
  c->counters.alloc(4);
  TLS_HIP(hipMemsetAsync(c->counters.p, 0, sizeof(int) * 4, c->stream));
  build_local_plans(c, 4, 1);
  // padding entries must stay zero: the padded identity rows then solve to 0
  if (c->fp32) {
    c->xloc32.alloc(c->sum_M);
    TLS_HIP(hipMemsetAsync(c->xloc32.p, 0, sizeof(float) * c->sum_M, c->stream));
  } else {
    c->xloc64.alloc(c->sum_M);
    TLS_HIP(hipMemsetAsync(c->xloc64.p, 0, sizeof(double) * c->sum_M, c->stream));
  }
  TLS_HIP(hipStreamSynchronize(c->stream));
}

template <class T>
void bsolve_interior_impl(tls_ctx* c, const T* dinv, T* X, const std::vector<int>& nq,
                          const std::vector<int64_t>& xoff, int64_t ldx) {
  constexpr int PW = 8;
  hipStream_t s = c->stream;
  const int N = c->N;
  std::vector<int> nb(N), order;
  for (int i = 0; i < N; i++) {
    nb[i] = nq[i] > 0 ? (c->h_nI[i] + TS - 1) / TS : 0;
    if (nb[i] > 0) order.push_back(i);
  }
  if (order.empty()) return;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nb[a] > nb[b]; });
  const int maxnb = nb[order[0]];
  struct Launch {
    int kind, s, s0, nact;
    int64_t off, total;
    bool listed;  // explicit task list (tiles inside the profiles)
  };
  std::vector<Launch> launches;
  std::vector<int64_t> pref;
  std::vector<int4> tasks;
  // profile of the blocks read: the rows of L (Cholesky, tile (k, j) is
  // zero when f(k) > j) or the columns of U (LU, tile (j, k) zero when
  // g(k) > j)
  const bool use_prof = !c->h_prof.empty();
  const int* gh = use_prof ? c->h_prof.data() + (c->kind == 1 ? c->sum_nt : 0) : nullptr;
  auto active = [&](int step) {
    int a = 0;
    while (a < (int)order.size() && nb[order[a]] > step) a++;
    return a;
  };
  auto add_update = [&](int mode, int step, int s0) {
    const int act = active(mode == 0 ? step : s0);
    if (use_prof) {
      const int64_t off = (int64_t)tasks.size();
      for (int a = 0; a < act; a++) {
        const int i = order[a];
        const int* g = gh + c->h_toff[i];
        const BsolveRange rg = bsolve_range(mode, step, s0, PW, nb[i]);
        for (int j = rg.jlo; j < rg.jhi; j++) {
          bool any = false;
          for (int k = rg.klo; k < rg.khi && !any; k++) any = g[k] <= j;
          if (!any) continue;
          for (int q = 0; q < nq[i]; q++) tasks.push_back(int4{i, j, q, rg.klo | ((rg.khi - rg.klo) << 24)});
        }
      }
      const int64_t n = (int64_t)tasks.size() - off;
      if (n > 0) launches.push_back(Launch{1 + mode, step, s0, act, off, n, true});
      return;
    }
    const int64_t off = (int64_t)pref.size();
    int64_t tot = 0;
    for (int a = 0; a < act; a++) {
      const int i = order[a];
      pref.push_back(tot);
      const BsolveRange rg = bsolve_range(mode, step, s0, PW, nb[i]);
      if (rg.jhi > rg.jlo) tot += (int64_t)(rg.jhi - rg.jlo) * nq[i];
    }
    pref.push_back(tot);
    if (tot > 0) launches.push_back(Launch{1 + mode, step, s0, act, off, tot, false});
  };
  for (int s0 = 0; s0 < maxnb; s0 += PW) {
    for (int st = s0; st < std::min(s0 + PW, maxnb); st++) {
      const int act = active(st);
      const int64_t off = (int64_t)pref.size();
      int64_t tot = 0;
      for (int a = 0; a < act; a++) {
        pref.push_back(tot);
        tot += nq[order[a]];
      }
      pref.push_back(tot);
      launches.push_back(Launch{0, st, s0, act, off, tot, false});
      add_update(0, st, s0);
    }
    add_update(1, 0, s0);
  }
  DBuf<int> d_order, d_nb, d_nq;
  DBuf<int64_t> d_pref, d_xoff;
  DBuf<int4> d_tasks;
  d_order.upload(order, s);
  d_nb.upload(nb, s);
  d_nq.upload(nq, s);
  d_pref.upload(pref, s);
  d_xoff.upload(xoff, s);
  d_tasks.upload(tasks, s);
  const int* gd = use_prof ? c->prof.p + (c->kind == 1 ? c->sum_nt : 0) : nullptr;
  LocalLayout lay = c->layout();
  const T* fac = c->fp32 ? reinterpret_cast<const T*>(c->fac32.p) : reinterpret_cast<const T*>(c->fac64.p);
  const bool lt = c->kind == 0;
  auto diag = lt ? k_bsolve_diag<T, true> : k_bsolve_diag<T, false>;
  auto update = lt ? k_bsolve_update<T, true> : k_bsolve_update<T, false>;
  for (const Launch& L : launches) {
    if (L.kind == 0)
      hipLaunchKernelGGL(diag, dim3((unsigned)L.total), dim3(256), 0, s, L.s, d_pref.p + L.off, L.nact, d_order.p,
                         lay, d_nb.p, d_xoff.p, ldx, dinv, X);
    else
      hipLaunchKernelGGL(update, dim3((unsigned)L.total), dim3(256), 0, s, L.kind - 1, L.s, L.s0, PW,
                         L.listed ? nullptr : d_pref.p + L.off, L.nact, d_order.p, lay, d_nb.p, d_nq.p, d_xoff.p,
                         ldx, fac, X, L.listed ? d_tasks.p + L.off : nullptr, gd);
    TLS_LAUNCH_CHECK();
  }
  TLS_HIP(hipStreamSynchronize(s));
}

void local_bsolve_interior(tls_ctx* c, float* X, const std::vector<int>& nq, const std::vector<int64_t>& xoff,
                           int64_t ldx) {
  bsolve_interior_impl<float>(c, c->dinv32.p, X, nq, xoff, ldx);
}
void local_bsolve_interior(tls_ctx* c, double* X, const std::vector<int>& nq, const std::vector<int64_t>& xoff,
                           int64_t ldx) {
  bsolve_interior_impl<double>(c, c->dinv64.p, X, nq, xoff, ldx);
}

// S = A^{-1} over the lower tiles of N Cholesky factors (tile counts nt,
// layout lay, elems elements in all), from their factors and diagonal-tile
// inverses; a scratch buffer of the factors' size holds W = L^{-1}.
// One group of subdomains (ids in `order`, largest first) whose W blocks
// sit at woff[i] of W.
template <class T>
static void inverse_group(hipStream_t s, const std::vector<int>& order, const std::vector<int>& nt,
                          const LocalLayout& lay, const int64_t* woff, T* fac, const T* dinv, T* W) {
  constexpr int PW = 8;
  const int N = (int)order.size();
  const int maxnt = N ? nt[order[0]] : 0;
  auto active = [&](int j) {
    int a = 0;
    while (a < N && nt[order[a]] > j) a++;
    return a;
  };
  struct Launch {
    int kind, j, j0, j1, nact;
    int64_t off, total;
  };
  std::vector<Launch> launches;
  std::vector<int64_t> pref;
  for (int j0 = 0; j0 < maxnt; j0 += PW) {
    const int j1 = j0 + PW;
    for (int j = j0; j < std::min(j1, maxnt); j++) {
      const int act = active(j);
      const int64_t off = (int64_t)pref.size();
      for (int a = 0; a <= act; a++) pref.push_back((int64_t)a * (j + 1));
      launches.push_back(Launch{0, j, j0, j1, act, off, (int64_t)act * (j + 1)});
    }
    const int act = active(j1);
    if (act > 0) {
      const int64_t off = (int64_t)pref.size();
      int64_t tot = 0;
      for (int a = 0; a < act; a++) {
        pref.push_back(tot);
        tot += (int64_t)(nt[order[a]] - j1) * j1;
      }
      pref.push_back(tot);
      launches.push_back(Launch{1, 0, j0, j1, act, off, tot});
    }
  }
  {
    const int act = active(0);
    const int64_t off = (int64_t)pref.size();
    int64_t tot = 0;
    for (int a = 0; a < act; a++) {
      pref.push_back(tot);
      const int64_t n = nt[order[a]];
      tot += n * (n + 1) / 2;
    }
    pref.push_back(tot);
    if (tot > 0) launches.push_back(Launch{2, 0, 0, 0, act, off, tot});
  }
  DBuf<int> d_order;
  DBuf<int64_t> d_pref;
  d_order.upload(order, s);
  d_pref.upload(pref, s);
  for (const Launch& L : launches) {
    if (L.total <= 0) continue;
    switch (L.kind) {
      case 0:
        hipLaunchKernelGGL(k_tinv_row<T>, dim3((unsigned)L.total), dim3(256), 0, s, L.j, L.j0, d_pref.p + L.off,
                           L.nact, d_order.p, lay, woff, fac, dinv, W, nullptr);
        break;
      case 1:
        hipLaunchKernelGGL(k_tinv_update<T>, dim3((unsigned)L.total), dim3(256), 0, s, L.j0, L.j1, d_pref.p + L.off,
                           L.nact, d_order.p, lay, woff, fac, W);
        break;
      default:
        hipLaunchKernelGGL(k_tinv_lauum<T>, dim3((unsigned)L.total), dim3(256), 0, s, d_pref.p + L.off, L.nact,
                           d_order.p, lay, woff, W, fac);
        break;
    }
    TLS_LAUNCH_CHECK();
  }
  TLS_HIP(hipStreamSynchronize(s));
}

// The profile variant for one group: W = L^{-1} row by row (each row j
// needs only the rows l >= f(j) of its profile; one launch per j), then
// S = L^{-T} W by descending rows (k_sinv_row), then S copied over the
// factor. prof is the device copy of the profile.
template <class T>
static void inverse_group_profile(hipStream_t s, const std::vector<int>& order, const std::vector<int>& nt,
                                  const LocalLayout& lay, const int64_t* woff_d, const std::vector<int64_t>& woff,
                                  const std::vector<int64_t>& foff, T* fac, const T* dinv, T* W, const int* prof,
                                  bool copy_back) {
  const int N = (int)order.size();
  const int maxnt = N ? nt[order[0]] : 0;
  auto active = [&](int j) {
    int a = 0;
    while (a < N && nt[order[a]] > j) a++;
    return a;
  };
  std::vector<int64_t> pref;
  std::vector<std::pair<int64_t, int>> rows;  // prefix offset, active count per row j
  for (int j = 0; j < maxnt; j++) {
    const int act = active(j);
    rows.push_back({(int64_t)pref.size(), act});
    for (int a = 0; a <= act; a++) pref.push_back((int64_t)a * (j + 1));
  }
  DBuf<int> d_order;
  DBuf<int64_t> d_pref;
  d_order.upload(order, s);
  d_pref.upload(pref, s);
  for (int j = 0; j < maxnt; j++) {
    const int act = rows[j].second;
    hipLaunchKernelGGL(k_tinv_row<T>, dim3((unsigned)((int64_t)act * (j + 1))), dim3(256), 0, s, j, 0,
                       d_pref.p + rows[j].first, act, d_order.p, lay, woff_d, fac, dinv, W, prof);
    TLS_LAUNCH_CHECK();
  }
  for (int r = maxnt - 1; r >= 0; r--) {
    const int act = rows[r].second;
    hipLaunchKernelGGL(k_sinv_row<T>, dim3((unsigned)((int64_t)act * (r + 1))), dim3(256), 0, s, r,
                       d_pref.p + rows[r].first, act, d_order.p, lay, woff_d, prof, fac, dinv, W);
    TLS_LAUNCH_CHECK();
  }
  if (copy_back)
    for (int i : order)
      TLS_HIP(hipMemcpyAsync(fac + foff[i], W + woff[i], sizeof(T) * tiles_of(0, nt[i]) * TS2,
                             hipMemcpyDeviceToDevice, s));
  TLS_HIP(hipStreamSynchronize(s));
}

// Arithmetic of the two ways of forming S from L (2 per multiply-add,
// triangular products at half): with the profile (W row by row, S by the
// back substitution) and dense (W by panels, S = W^T W).
struct InverseFlops {
  double profile = 0.0, dense = 0.0;
};
inline InverseFlops inverse_flops(const std::vector<int>& nt, const int* prof, const std::vector<int64_t>& toff) {
  InverseFlops fl;
  const double t3 = (double)TS * TS * TS;
  for (size_t i = 0; i < nt.size(); i++) {
    const int n = nt[i];
    fl.dense += 2.0 / 3.0 * std::pow((double)TS * n, 3);
    if (!prof) continue;
    const int* f = prof + toff[i];
    for (int j = 0; j < n; j++)
      for (int k = 0; k < j; k++) {
        const int l0 = std::max(k, f[j]);
        if (j > l0) fl.profile += (2.0 * (j - l0) + 1.0) * t3;
      }
    for (int r = 0; r < n; r++) {
      int cnt = 0;
      for (int c = r + 1; c < n; c++) cnt += f[c] <= r;
      fl.profile += (r + 1) * (2.0 * cnt + 1.0) * t3;
    }
  }
  return fl;
}

// W holds the blocks of one group of subdomains at a time. The groups
// (largest subdomains first) are cut so that W fits in the memory budget
// (devmem::budget, 90% of what is still available); when everything fits
// there is one group.
// With a profile (prof, device) and fac_buf, the buffer that holds the
// factors with offsets foff: when W fits beside the factors it takes their
// layout, the result is formed there and the two buffers are swapped (no
// clearing, no copy: the profile variant writes every lower tile of W).
template <class T>
void form_inverse_tiles(hipStream_t s, int N, const std::vector<int>& nt, const LocalLayout& lay, T* fac,
                        const T* dinv, const int* prof = nullptr, const std::vector<int64_t>* foff = nullptr,
                        DBuf<T>* fac_buf = nullptr, bool must_swap = false) {
  std::vector<int> order(N);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nt[a] > nt[b]; });
  const int64_t budget = (int64_t)(devmem::budget() / sizeof(T));
  if (prof && fac_buf && N > 0 && must_swap) {
    // profile storage: the factors cannot hold the full inverses, which are
    // formed in a buffer of their own with the full packed offsets (the
    // result's layout) and then take the factors' place; the subdomains go
    // in groups that fit the memory budget, each straight into its place
    const int64_t need = (*foff)[N - 1] + tiles_of(0, nt[N - 1]) * TS2;
    DBuf<int64_t> d_woff;
    d_woff.upload(*foff, s);
    DBuf<T> W;
    W.alloc(need);
    const int64_t room = std::max<int64_t>((int64_t)(devmem::budget() / sizeof(T)), 1);
    std::vector<int> g;
    int64_t tot = 0;
    for (int a = 0; a <= N; a++) {
      const int64_t e = a < N ? tiles_of(0, nt[order[a]]) * TS2 : 0;
      if (a == N || (!g.empty() && tot + e > room)) {
        inverse_group_profile<T>(s, g, nt, lay, d_woff.p, *foff, *foff, fac, dinv, W.p, prof, false);
        g.clear();
        tot = 0;
      }
      if (a < N) {
        g.push_back(order[a]);
        tot += e;
      }
    }
    fac_buf->swap(W);
    return;
  }
  if (prof && fac_buf && N > 0) {
    const int64_t need = (*foff)[N - 1] + tiles_of(0, nt[N - 1]) * TS2;
    if (need <= budget) {
      DBuf<int64_t> d_woff;
      d_woff.upload(*foff, s);
      DBuf<T> W;
      W.alloc(need);
      inverse_group_profile<T>(s, order, nt, lay, d_woff.p, *foff, *foff, fac, dinv, W.p, prof, false);
      fac_buf->swap(W);
      return;
    }
  }
  std::vector<std::vector<int>> groups;
  std::vector<int64_t> woff(N, 0);
  int64_t wmax = 1, tot = 0;
  for (int a = 0; a < N; a++) {
    const int i = order[a];
    const int64_t e = tiles_of(0, nt[i]) * TS2;
    if (groups.empty() || tot + e > budget) {
      groups.emplace_back();
      tot = 0;
    }
    groups.back().push_back(i);
    woff[i] = tot;
    tot += e;
    wmax = std::max(wmax, tot);
  }
  DBuf<int64_t> d_woff;
  d_woff.upload(woff, s);
  DBuf<T> W;
  W.alloc(wmax);
  for (const auto& g : groups) {
    TLS_HIP(hipMemsetAsync(W.p, 0, sizeof(T) * wmax, s));
    if (prof)
      inverse_group_profile<T>(s, g, nt, lay, d_woff.p, woff, *foff, fac, dinv, W.p, prof, true);
    else
      inverse_group<T>(s, g, nt, lay, d_woff.p, fac, dinv, W.p);
  }
}

// Work list of the symmetric product over N matrices (tile counts nt,
// factor offsets foff, vector offsets voff): blocks of block x block
// tiles, the largest matrices first, one reduction row per tile row.
void build_symv_work(SymvWork& w, hipStream_t s, int N, const std::vector<int>& nt,
                     const std::vector<int64_t>& foff, const std::vector<int64_t>& voff, bool fp32, int block) {
  if (block != 4 && block != 6 && block != 8) fail(TLS_E_ARG, "symmetric-product blocks of 4, 6 or 8 tiles");
  const int SB = block;
  w.block = block;
  std::vector<int> order(N);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nt[a] > nt[b]; });
  std::vector<int> blk0(N, 0);
  int64_t nblk = 0;
  for (int i = 0; i < N; i++) {
    const int64_t nbr = (nt[i] + SB - 1) / SB;
    blk0[i] = (int)nblk;
    nblk += nbr * (nbr + 1) / 2;
  }
  if (nblk > (int64_t)INT32_MAX / SB) fail(TLS_E_ARG, "too many tiles for the symmetric-product work list");
  std::vector<SymvBlock> blocks;
  std::vector<SymvRow> rows;
  blocks.reserve(nblk);
  for (int i : order) {
    const int nbr = (nt[i] + SB - 1) / SB;
    for (int R = 0; R < nbr; R++)
      for (int C = 0; C <= R; C++) {
        SymvBlock bk;
        bk.foff = foff[i];
        bk.voff = voff[i];
        bk.r0 = R * SB;
        bk.r1 = std::min(nt[i], (R + 1) * SB);
        bk.c0 = C * SB;
        bk.c1 = std::min(nt[i], (C + 1) * SB);
        bk.out = blk0[i] + R * (R + 1) / 2 + C;
        bk.pad_ = 0;
        blocks.push_back(bk);
      }
  }
  for (int i = 0; i < N; i++)
    for (int r = 0; r < nt[i]; r++) {
      SymvRow rw;
      rw.voff = voff[i];
      rw.r = r;
      rw.nbr = (nt[i] + SB - 1) / SB;
      rw.blk0 = blk0[i];
      rw.pad_ = 0;
      rows.push_back(rw);
    }
  static_assert(sizeof(SymvBlock) == 48 && sizeof(SymvRow) == 32, "descriptor layout");
  w.nblocks = (int64_t)blocks.size();
  w.nrows = (int64_t)rows.size();
  w.blocks.alloc(blocks.size() * 3);
  TLS_HIP(hipMemcpyAsync(w.blocks.p, blocks.data(), sizeof(SymvBlock) * blocks.size(), hipMemcpyHostToDevice, s));
  w.rows.alloc(rows.size() * 2);
  TLS_HIP(hipMemcpyAsync(w.rows.p, rows.data(), sizeof(SymvRow) * rows.size(), hipMemcpyHostToDevice, s));
  const int64_t npart = std::max<int64_t>(nblk * SB * TS, 1);
  if (fp32) {
    w.RP32.alloc(npart);
    w.CP32.alloc(npart);
  } else {
    w.RP64.alloc(npart);
    w.CP64.alloc(npart);
  }
  TLS_HIP(hipStreamSynchronize(s));
}

void solve_tile_counts(const tls_ctx* c, int64_t* fwd, int64_t* bwd, int64_t* lower) {
  int64_t f = 0, b = 0, d = 0;
  const bool prof = !c->h_prof.empty();
  for (int i = 0; i < c->N; i++) {
    const int nt = c->h_nt[i];
    const int64_t t0 = c->h_toff[i];
    d += (int64_t)nt * (nt + 1) / 2;
    for (int r = 0; r < nt; r++) {
      f += prof ? r - c->h_prof[t0 + r] + 1 : r + 1;
      b += prof ? r - c->h_prof[(c->kind == 1 ? c->sum_nt : 0) + t0 + r] + 1 : r + 1;
    }
  }
  *fwd = f;
  *bwd = b;
  *lower = d;
}

bool inverse_pays(const tls_ctx* c) {
  if (c->kind != 0) return false;
  int64_t f, b, d;
  solve_tile_counts(c, &f, &b, &d);
  // the inverses need a full packed buffer beside the profile-stored factors
  const double need = (double)d * TS2 * (c->fp32 ? 4 : 8);
  return f + b > d && need <= 0.9 * (double)devmem::available();
}

void form_local_inverse(tls_ctx* c) {
  if (c->kind != 0) fail(TLS_E_ARG, "local_inverse applies to SPD matrices only");
  hipStream_t s = c->stream;
  // the profile variant when the factors are stored by profile, or when it
  // saves at least half of the arithmetic
  const bool ps = c->prof_store;
  const InverseFlops fl = inverse_flops(c->h_nt, c->h_prof.empty() ? nullptr : c->h_prof.data(), c->h_toff);
  const bool use_prof = ps || (!c->h_prof.empty() && fl.profile < 0.5 * fl.dense);
  c->flops_inverse = use_prof ? fl.profile : fl.dense;
  const int* prof = use_prof ? c->prof.p : nullptr;
  // the inverses fill the full packed triangles (offsets h_soff with profile storage)
  const std::vector<int64_t>* so = ps ? &c->h_soff : &c->h_foff;
  if (c->fp32)
    form_inverse_tiles<float>(s, c->N, c->h_nt, c->layout(), c->fac32.p, c->dinv32.p, prof, so, &c->fac32, ps);
  else
    form_inverse_tiles<double>(s, c->N, c->h_nt, c->layout(), c->fac64.p, c->dinv64.p, prof, so, &c->fac64, ps);
  if (ps) {
    // the storage now holds the inverses, in the full packed layout
    c->prof_store = false;
    c->h_foff = c->h_soff;
    c->fac_elems = c->h_foff[c->N];
    c->d_foff.upload(c->h_foff, s);
  }
  build_symv_work(c->inv_work, s, c->N, c->h_nt, c->h_foff, c->h_voff, c->fp32, c->symv_block);
  c->inv_formed = true;
}

void form_inverse_f64(hipStream_t s, int N, const std::vector<int>& nt, const LocalLayout& lay, double* fac,
                      const double* dinv) {
  form_inverse_tiles<double>(s, N, nt, lay, fac, dinv);
}

template <class T>
void symv_solve_t(hipStream_t s, const SymvWork& w, const T* S, T* x, T* RP, T* CP, const int* done,
                  hipEvent_t ev_begin, hipEvent_t ev_mid, hipEvent_t ev_end) {
  if (ev_begin) TLS_HIP(hipEventRecord(ev_begin, s));
  auto prod = w.block == 4 ? k_symv<T, 4> : w.block == 6 ? k_symv<T, 6> : k_symv<T, 8>;
  auto reduce = w.block == 4 ? k_symv_reduce<T, 4> : w.block == 6 ? k_symv_reduce<T, 6> : k_symv_reduce<T, 8>;
  if (w.nblocks > 0)
    hipLaunchKernelGGL(prod, dim3((unsigned)w.nblocks), dim3(256), 0, s,
                       reinterpret_cast<const SymvBlock*>(w.blocks.p), S, x, RP, CP, done);
  TLS_LAUNCH_CHECK();
  if (ev_mid) TLS_HIP(hipEventRecord(ev_mid, s));
  if (w.nrows > 0)
    hipLaunchKernelGGL(reduce, dim3((unsigned)w.nrows), dim3(64), 0, s,
                       reinterpret_cast<const SymvRow*>(w.rows.p), RP, CP, x, done);
  TLS_LAUNCH_CHECK();
  if (ev_end) TLS_HIP(hipEventRecord(ev_end, s));
}

void symv_solve_f64(hipStream_t s, SymvWork& w, const double* S, double* x, const int* done) {
  symv_solve_t<double>(s, w, S, x, w.RP64.p, w.CP64.p, done, nullptr, nullptr, nullptr);
}

void local_solve(tls_ctx* c, const int* done, hipEvent_t ev_begin, hipEvent_t ev_mid, hipEvent_t ev_end) {
  hipStream_t s = c->stream;
  LocalLayout lay = c->layout();
  if (c->inv_formed) {
    SymvWork& w = c->inv_work;
    if (c->fp32)
      symv_solve_t<float>(s, w, c->fac32.p, c->xloc32.p, w.RP32.p, w.CP32.p, done, ev_begin, ev_mid, ev_end);
    else
      symv_solve_t<double>(s, w, c->fac64.p, c->xloc64.p, w.RP64.p, w.CP64.p, done, ev_begin, ev_mid, ev_end);
    return;
  }
  solve_begin(s, c->counters.p, done);
  if (ev_begin) TLS_HIP(hipEventRecord(ev_begin, s));
  const int fm = c->kind == 0 ? FWD_L : FWD_UL, bm = c->kind == 0 ? BWD_LT : BWD_U;
  // forward: row profile; backward: the row profile again (Cholesky, read
  // by columns) or the column profile of U (LU)
  const int* prof = c->h_prof.empty() ? nullptr : c->prof.p;
  const int* profb = prof && c->kind == 1 ? prof + c->sum_nt : prof;
  if (c->fp32) {
    trsv<float>(s, fm, c->plan_fwd, c->counters.p + 0, c->counters.p + 2, lay, c->fac32.p, c->dinv32.p, c->xloc32.p,
                c->errflag.p, done, c->solve_grid, prof);
    if (ev_mid) TLS_HIP(hipEventRecord(ev_mid, s));
    trsv<float>(s, bm, c->plan_bwd, c->counters.p + 1, c->counters.p + 2, lay, c->fac32.p, c->dinv32.p, c->xloc32.p,
                c->errflag.p, done, c->solve_grid, profb);
  } else {
    trsv<double>(s, fm, c->plan_fwd, c->counters.p + 0, c->counters.p + 2, lay, c->fac64.p, c->dinv64.p, c->xloc64.p,
                 c->errflag.p, done, c->solve_grid, prof);
    if (ev_mid) TLS_HIP(hipEventRecord(ev_mid, s));
    trsv<double>(s, bm, c->plan_bwd, c->counters.p + 1, c->counters.p + 2, lay, c->fac64.p, c->dinv64.p, c->xloc64.p,
                 c->errflag.p, done, c->solve_grid, profb);
  }
  if (ev_end) TLS_HIP(hipEventRecord(ev_end, s));
}

}  // namespace tls
