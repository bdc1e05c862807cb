// Coarse basis of eq. coarse_space_2 (SPD A): the dominant eigenvectors of
// Pi_i^T D_i A_ii D_i Pi_i w = lambda^2 A_ii w (eq. gevpsvd), mapped to
// D_i Pi_i w.
//
// Reduction used here (exact, derived from the block form of Pi_i that the
// paper writes before Proposition gevpsvd). Order Omega_i as
// [I, G = Gamma_{1:delta-1}, T = Gamma_delta] and let L be the Cholesky
// factor of A_ii with blocks L_II, L_GI, L_GG, L_TI, L_TG, L_TT. Then
//   E = -A_{Omega',Omega'}^{-1} A_{Omega',T} (eq. HOp), H = rows I of E,
//   F := L_II^T H = -L_TI^T + L_GI^T L_GG^{-T} L_TG^T,
//   Pi_i^T D_i A_ii D_i Pi_i is zero outside its (T,T) block K = F^T F,
//   and the Schur complement of A_ii onto T is S_T = L_TT L_TT^T.
// A nonzero eigenpair (lambda^2, w) therefore satisfies K w_T = lambda^2 S_T w_T,
// i.e. C z = lambda^2 z with C = L_TT^{-1} K L_TT^{-T}, w_T = L_TT^{-T} z, and
// the coarse vector is D_i Pi_i w = [H w_T; 0] = [L_II^{-T} F w_T; 0].
// C is #T x #T; its top eigenpairs come from subspace iteration with
// Rayleigh-Ritz.
#include <algorithm>
#include <chrono>
#include <climits>
#include <type_traits>
#include <cmath>

#include "batched.hpp"
#include "kernels.hpp"

namespace tls {

namespace {

constexpr int PMAX = 48;      // largest subspace block
constexpr int OVER_MIN = 8;   // the block keeps at least this many extra vectors: k <= PMAX - OVER_MIN
constexpr int KMAX = 2 * PMAX;  // most coarse columns of one subdomain (both eigenproblems)

struct EigLayout {
  const int* nI;
  const int* nG;
  const int* nT;
  const int* m;
  const int* nt;
  const int64_t* foff;
  const int64_t* o_F;    // nI*nT
  const int64_t* o_GI;   // nG*nI
  const int64_t* o_TG;   // nG*nT
  const int64_t* o_GG;   // nG*nG
  const int64_t* o_TT;   // nT*nT
  const int64_t* o_X;    // M_i x 64 nq_i right-hand-side blocks (general: H)
  const int* kreq;
  LocalLayout fl;        // the factors' storage (tile profiles)
};

// Blocks of the local factor copied to dense column-major buffers.
// SPD (Cholesky, lower tiles):
//   mode 0: F = -L_TI^T (nI x nT)    mode 1: Tm = L_TG^T (nG x nT)
//   mode 2: L_GG^T (upper, nG x nG) mode 3: L_GI (nG x nI)
//   mode 4: L_TT (lower, nT x nT)   mode 5: L_TT^T (upper, nT x nT)
// General (LU, full tiles; U upper with its diagonal):
//   mode 6: U_GT (nG x nT)          mode 7: U_GG (upper, nG x nG)
//   mode 8: U_IG (nI x nG)          mode 9: -U_IT into rows < nI of X (leading dim M_i)
template <class S, class D>
__global__ void k_extract(int mode, EigLayout e, const S* __restrict__ fac, D* out) {
  const int i = blockIdx.y;
  const int nI = e.nI[i], nG = e.nG[i], nT = e.nT[i], nt = e.nt[i];
  const int nP = nI + nG;
  const S* base = fac + e.foff[i];
  const int kind = mode >= 6 ? 1 : 0;
  int rows, cols;
  int64_t off, ld;
  switch (mode) {
    case 0: rows = nI; cols = nT; off = e.o_F[i]; break;
    case 1: rows = nG; cols = nT; off = e.o_TG[i]; break;
    case 2: rows = nG; cols = nG; off = e.o_GG[i]; break;
    case 3: rows = nG; cols = nI; off = e.o_GI[i]; break;
    case 6: rows = nG; cols = nT; off = e.o_TG[i]; break;
    case 7: rows = nG; cols = nG; off = e.o_GG[i]; break;
    case 8: rows = nI; cols = nG; off = e.o_GI[i]; break;
    case 9: rows = nI; cols = nT; off = e.o_X[i]; break;
    default: rows = nT; cols = nT; off = e.o_TT[i]; break;
  }
  ld = mode == 9 ? (int64_t)nt * TS : rows;
  if (e.kreq[i] <= 0) return;
  const int64_t total = (int64_t)rows * cols;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    int a = (int)(x % rows), b = (int)(x / rows);
    // element (r, q) of the factor, zero where its tile is not stored
    auto el = [&](int r, int q) -> S {
      return tile_in(e.fl, i, kind, r / TS, q / TS) ? *elem_ptr_l(base, e.fl, i, kind, nt, r, q) : S(0);
    };
    S v = S(0);
    switch (mode) {
      case 0: v = -el(nP + b, a); break;
      case 1: v = el(nP + b, nI + a); break;
      case 2: v = b >= a ? el(nI + b, nI + a) : S(0); break;
      case 3: v = el(nI + a, b); break;
      case 4: v = a >= b ? el(nP + a, nP + b) : S(0); break;
      case 5: v = b >= a ? el(nP + b, nP + a) : S(0); break;
      case 6: v = el(nI + a, nP + b); break;
      case 7: v = b >= a ? el(nI + a, nI + b) : S(0); break;
      case 8: v = el(a, nI + b); break;
      default: v = -el(a, nP + b); break;
    }
    out[off + a + (int64_t)b * ld] = (D)v;
  }
}

// F = -L_TI^T (nI x nT, column-major; SPD tile storage) as k_extract mode 0
// does, through 64 x 64 chunks staged in LDS: the factor is read down its
// columns (contiguous inside a tile) and F written down its columns.
template <class T>
__global__ void __launch_bounds__(256) k_extract_f(EigLayout e, const T* __restrict__ fac, T* out) {
  const int i = blockIdx.y;
  if (e.kreq[i] <= 0) return;
  const int nI = e.nI[i], nT = e.nT[i], nt = e.nt[i];
  const int nP = nI + e.nG[i];
  const T* base = fac + e.foff[i];
  T* F = out + e.o_F[i];
  const int na = (nI + TS - 1) / TS, nbk = (nT + TS - 1) / TS;
  __shared__ T t[TS][TS + 1];
  for (int chunk = blockIdx.x; chunk < na * nbk; chunk += gridDim.x) {
    const int A0 = (chunk % na) * TS, B0 = (chunk / na) * TS;
    __syncthreads();
    for (int x = threadIdx.x; x < TS2; x += 256) {
      const int bb = x % TS, aa = x / TS;  // factor element (nP + B0 + bb, A0 + aa)
      const int a = A0 + aa, b = B0 + bb;
      t[aa][bb] = (a < nI && b < nT && tile_in(e.fl, i, 0, (nP + b) / TS, a / TS))
                      ? -*elem_ptr_l(base, e.fl, i, 0, nt, nP + b, a)
                      : T(0);
    }
    __syncthreads();
    for (int x = threadIdx.x; x < TS2; x += 256) {
      const int aa = x % TS, bb = x / TS;
      const int a = A0 + aa, b = B0 + bb;
      if (a < nI && b < nT) F[a + (int64_t)b * nI] = t[aa][bb];
    }
  }
}

template <class S, class D>
__global__ void k_convert(int64_t count, const S* __restrict__ in, D* out) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < count; x += (int64_t)gridDim.x * blockDim.x)
    out[x] = (D)in[x];
}

// out = in^T (symmetrize = 0) or out = (in + in^T) / 2 (symmetrize = 1) for
// each subdomain's nT x nT column-major block; 64 x 64 tiles staged through
// LDS so that both the reads and the writes are contiguous.
template <class U>
__global__ void __launch_bounds__(256) k_transpose_blocks(const int* __restrict__ nT_, const int64_t* __restrict__ off,
                                                          const int* __restrict__ kreq, const U* in, U* out,
                                                          int symmetrize) {
  const int i = blockIdx.y;
  if (kreq[i] <= 0) return;
  const int n = nT_[i];
  const int nb = (n + TS - 1) / TS;
  const U* a = in + off[i];
  U* b = out + off[i];
  __shared__ U t[TS][TS + 1];
  for (int tile = blockIdx.x; tile < nb * nb; tile += gridDim.x) {
    const int tr = tile % nb, tc = tile / nb;  // output tile: rows tr, columns tc
    __syncthreads();
    for (int e = threadIdx.x; e < TS2; e += 256) {
      const int x = e % TS, y = e / TS;
      const int r = tc * TS + x, c = tr * TS + y;  // t[y][x] = in(tc 64 + x, tr 64 + y)
      t[y][x] = (r < n && c < n) ? a[r + (int64_t)c * n] : U(0);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < TS2; e += 256) {
      const int x = e % TS, y = e / TS;
      const int r = tr * TS + x, c = tc * TS + y;
      if (r < n && c < n) {
        const U tv = t[x][y];  // in(c, r)
        b[r + (int64_t)c * n] = symmetrize ? U(0.5) * (a[r + (int64_t)c * n] + tv) : tv;
      }
    }
  }
}

// out (precision D) = the symmetric nT x nT block whose tiles on and below the
// block diagonal are in `in` (precision S, column-major, as a syrk GEMM
// leaves them): those tiles are converted, the ones above are the
// transposes of their mirror tiles (64 x 64 LDS staging, contiguous reads
// and writes).
template <class S, class D>
__global__ void __launch_bounds__(256) k_sym_from_lower(const int* __restrict__ nT_, const int64_t* __restrict__ off,
                                                        const int* __restrict__ kreq, const S* __restrict__ in,
                                                        D* out) {
  const int i = blockIdx.y;
  if (kreq[i] <= 0) return;
  const int n = nT_[i];
  const int nb = (n + TS - 1) / TS;
  const S* a = in + off[i];
  D* b = out + off[i];
  __shared__ D t[TS][TS + 1];
  for (int tile = blockIdx.x; tile < nb * nb; tile += gridDim.x) {
    const int tr = tile % nb, tc = tile / nb;  // output tile: rows tr, columns tc
    if (tr >= tc) {
      for (int e = threadIdx.x; e < TS2; e += 256) {
        const int r = tr * TS + e % TS, c = tc * TS + e / TS;
        if (r < n && c < n) b[r + (int64_t)c * n] = (D)a[r + (int64_t)c * n];
      }
      continue;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < TS2; e += 256) {
      const int x = e % TS, y = e / TS;
      const int r = tc * TS + x, c = tr * TS + y;  // t[y][x] = in(tc 64 + x, tr 64 + y), a lower tile
      t[y][x] = (r < n && c < n) ? (D)a[r + (int64_t)c * n] : D(0);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < TS2; e += 256) {
      const int x = e % TS, y = e / TS;
      const int r = tr * TS + x, c = tc * TS + y;
      if (r < n && c < n) b[r + (int64_t)c * n] = t[x][y];  // in(c, r)
    }
  }
}

__device__ inline double hash_uniform(uint64_t seed, uint64_t i, uint64_t r, uint64_t c) {
  // splitmix64 finalizer over a counter built from (seed, i, r, c)
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * ((i << 42) ^ (c << 32) ^ r ^ 0x5851F42D4C957F2Dull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return ((double)(z >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
}

__device__ inline double block_sum(double v, double* red) {
  // 256 threads: wave shuffle then 4 partials
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return s;
}

// Eight sums at once over the 256 threads of the block (red: 32 values);
// every thread gets the totals.
__device__ inline void block_sum8(double (&v)[8], double* red) {
#pragma unroll
  for (int m = 0; m < 8; m++)
    for (int o = 32; o > 0; o >>= 1) v[m] += __shfl_xor(v[m], o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int m = 0; m < 8; m++) red[w * 8 + m] = v[m];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 8; m++) v[m] = red[m] + red[8 + m] + red[16 + m] + red[24 + m];
  __syncthreads();
}

// Cyclic Jacobi on the symmetric p x p matrix H (LDS, leading dim PMAX) with
// round-robin parallel ordering; S accumulates the rotations.
__device__ void jacobi_eig(double* H, double* S, int p, double* cs, double* red) {
  const int tid = threadIdx.x;
  const int pe = p + (p & 1);  // even number of players; index p is a dummy if p is odd
  for (int e = tid; e < PMAX * PMAX; e += 256) S[e] = ((e / PMAX) == (e % PMAX)) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 40; sweep++) {
    // off-diagonal norm vs total
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < p * p; e += 256) {
      int a = e % p, b = e / p;
      double h = H[b * PMAX + a];
      tot += h * h;
      if (a != b) off += h * h;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    if (off <= 1e-30 * tot || tot == 0.0) break;
    for (int rnd = 0; rnd < pe - 1; rnd++) {
      const int npairs = pe / 2;
      if (tid < npairs) {
        int a, b;
        if (tid == 0) {
          a = 0;
          b = (rnd % (pe - 1)) + 1;
        } else {
          a = ((rnd + tid) % (pe - 1)) + 1;
          b = ((rnd - tid + (pe - 1)) % (pe - 1)) + 1;
        }
        if (a > b) {
          int t = a;
          a = b;
          b = t;
        }
        double c = 1.0, s = 0.0;
        if (b < p) {
          double hab = H[b * PMAX + a];
          if (hab != 0.0) {
            double tau = (H[b * PMAX + b] - H[a * PMAX + a]) / (2.0 * hab);
            double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        cs[4 * tid + 0] = c;
        cs[4 * tid + 1] = s;
        cs[4 * tid + 2] = a;
        cs[4 * tid + 3] = b;
      }
      __syncthreads();
      // columns: H <- H J, S <- S J
      for (int e = tid; e < npairs * p; e += 256) {
        int j = e / p, x = e % p;
        int a = (int)cs[4 * j + 2], b = (int)cs[4 * j + 3];
        if (b >= p) continue;
        double c = cs[4 * j], s = cs[4 * j + 1];
        double ha = H[a * PMAX + x], hb = H[b * PMAX + x];
        H[a * PMAX + x] = c * ha - s * hb;
        H[b * PMAX + x] = s * ha + c * hb;
        double sa = S[a * PMAX + x], sb = S[b * PMAX + x];
        S[a * PMAX + x] = c * sa - s * sb;
        S[b * PMAX + x] = s * sa + c * sb;
      }
      __syncthreads();
      // rows: H <- J^T H
      for (int e = tid; e < npairs * p; e += 256) {
        int j = e / p, x = e % p;
        int a = (int)cs[4 * j + 2], b = (int)cs[4 * j + 3];
        if (b >= p) continue;
        double c = cs[4 * j], s = cs[4 * j + 1];
        double ha = H[x * PMAX + a], hb = H[x * PMAX + b];
        H[x * PMAX + a] = c * ha - s * hb;
        H[x * PMAX + b] = s * ha + c * hb;
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Batched subspace iteration with Rayleigh-Ritz for the top-k eigenpairs of
// the symmetric PSD blocks C_i (n_i x n_i). The products with C_i and the
// n x p by p x p products are variable-size MFMA GEMMs over all active
// subdomains (precision T: FP32 in mixed mode, FP64 otherwise); the p x p
// pieces (Jacobi eigensolver, Cholesky) run one workgroup per subdomain in
// FP64. Iteration: W = (C + sigma I) Y, H = Y^T W = S Theta S^T, V = W S,
// U = Y S (Ritz vectors), residuals ||V_j - theta_j U_j||, then
// Y <- orth(V) (CholQR2 with column equilibration). sigma = 1e-7 trace(C)
// keeps the block full rank when C has a null space.
// ---------------------------------------------------------------------------

// C_w = C + sigma I in precision T, and the start block: columns >= cw
// random, the first cw = min(c0, p) from Ywarm (normalized, with a 1e-3
// random component so that the block keeps full rank).
template <class T>
__global__ void __launch_bounds__(256) k_ss_init(const int* __restrict__ ids, const int* __restrict__ n_,
                                                 const int* __restrict__ p_, const int64_t* __restrict__ oC,
                                                 const int64_t* __restrict__ oY, const double* __restrict__ C64,
                                                 T* Cw, T* Y, const double* __restrict__ Ywarm, int c0,
                                                 uint64_t seed, double* sigma_out) {
  __shared__ double red[16];
  const int i = ids[blockIdx.x];
  const int n = n_[i], p = p_[i], tid = threadIdx.x;
  const double* C = C64 + oC[i];
  double tr = 0.0;
  for (int r = tid; r < n; r += 256) tr += C[r + (int64_t)r * n];
  tr = block_sum(tr, red);
  const double sigma = 1e-7 * tr;
  T* Ci = Cw + oC[i];
  for (int64_t e = tid; e < (int64_t)n * n; e += 256) {
    const int r = (int)(e % n), c = (int)(e / n);
    Ci[e] = (T)(C[e] + (r == c ? sigma : 0.0));
  }
  T* Yi = Y + oY[i];
  const int cw = min(c0, p);
  for (int64_t e = tid; e < (int64_t)n * p; e += 256) {
    const int r = (int)(e % n), c = (int)(e / n);
    if (c >= cw) Yi[e] = (T)hash_uniform(seed, i, r, c);
  }
  const double rs = 1e-3 * sqrt(3.0 / n);
  for (int c = 0; c < cw; c++) {
    const double* y = Ywarm + oY[i] + (int64_t)c * n;
    double s2 = 0.0;
    for (int r = tid; r < n; r += 256) s2 += y[r] * y[r];
    s2 = block_sum(s2, red);
    const double inv = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
    for (int r = tid; r < n; r += 256) Yi[r + (int64_t)c * n] = (T)(y[r] * inv + rs * hash_uniform(seed, i, r, c));
  }
  if (tid == 0) sigma_out[i] = sigma;
}

// R_i = D R'^{-1} where D = diag(G)^{-1/2} and R'^T R' = D G D (Cholesky of
// the equilibrated Gram matrix, FP64), so that Y R_i has orthonormal columns.
// Right-looking Cholesky with the row of R and the trailing update spread
// over the 64 threads; then thread c solves column c of R'^{-1}.
template <class T>
__global__ void __launch_bounds__(64) k_ss_chol(const int* __restrict__ ids, const int* __restrict__ p_,
                                                const T* __restrict__ G, T* R, int* err) {
  __shared__ double A[PMAX * PMAX];
  __shared__ double X[PMAX * PMAX];
  __shared__ double d[PMAX];
  __shared__ int s_bad;
  const int i = ids[blockIdx.x];
  const int p = p_[i], tid = threadIdx.x;
  const T* Gi = G + (int64_t)i * PMAX * PMAX;
  if (tid == 0) s_bad = 0;
  for (int e = tid; e < p * p; e += 64) A[(e % p) + (e / p) * PMAX] = (double)Gi[e];
  __syncthreads();
  if (tid < p) {
    const double g = A[tid + tid * PMAX];
    d[tid] = g > 0.0 ? 1.0 / sqrt(g) : 1.0;
  }
  __syncthreads();
  for (int e = tid; e < p * p; e += 64) {
    const int a = e % p, b = e / p;
    A[a + b * PMAX] *= d[a] * d[b];
  }
  __syncthreads();
  // upper Cholesky A = R^T R in place (R in the upper triangle)
  for (int j = 0; j < p; j++) {
    if (tid == 0) {
      double v = A[j + j * PMAX];
      if (!(v > 1e-28)) {
        s_bad = 1;
        v = 1e-28;
      }
      A[j + j * PMAX] = sqrt(v);
    }
    __syncthreads();
    const double rjj = A[j + j * PMAX];
    if (tid > j && tid < p) A[j + tid * PMAX] /= rjj;
    __syncthreads();
    const int w = p - j - 1;
    for (int e = tid; e < w * w; e += 64) {
      const int a = j + 1 + e % w, c = j + 1 + e / w;
      if (c >= a) A[a + c * PMAX] -= A[j + a * PMAX] * A[j + c * PMAX];
    }
    __syncthreads();
  }
  // X = R^{-1} (upper): column c by thread c, rows c down to 0
  if (tid < p) {
    const int c = tid;
    for (int a = p - 1; a > c; a--) X[a + c * PMAX] = 0.0;
    X[c + c * PMAX] = 1.0 / A[c + c * PMAX];
    for (int a = c - 1; a >= 0; a--) {
      double t = 0.0;
      for (int b = a + 1; b <= c; b++) t += A[a + b * PMAX] * X[b + c * PMAX];
      X[a + c * PMAX] = -t / A[a + a * PMAX];
    }
  }
  __syncthreads();
  if (tid == 0 && s_bad) atomicOr(err, ERR_EIG);
  T* Ri = R + (int64_t)i * PMAX * PMAX;
  for (int e = tid; e < p * p; e += 64) {
    const int a = e % p, b = e / p;
    Ri[e] = (T)(a <= b ? d[a] * X[a + b * PMAX] : 0.0);
  }
}

// Rayleigh-Ritz on H = Y^T W (p x p): S (eigenvectors, columns sorted by
// descending eigenvalue) and theta.
template <class T>
__global__ void __launch_bounds__(256) k_ss_rr(const int* __restrict__ ids, const int* __restrict__ p_,
                                               const T* __restrict__ Hm, T* Sout, double* th) {
  __shared__ double H[PMAX * PMAX];
  __shared__ double S[PMAX * PMAX];
  __shared__ double cs[4 * (PMAX / 2 + 1)];
  __shared__ double red[16];
  __shared__ int perm[PMAX];
  const int i = ids[blockIdx.x];
  const int p = p_[i], tid = threadIdx.x;
  const T* Hi = Hm + (int64_t)i * PMAX * PMAX;
  for (int e = tid; e < PMAX * PMAX; e += 256) H[e] = 0.0;
  __syncthreads();
  for (int e = tid; e < p * p; e += 256) {
    const int a = e % p, b = e / p;
    H[b * PMAX + a] = 0.5 * ((double)Hi[a + b * p] + (double)Hi[b + a * p]);
  }
  __syncthreads();
  jacobi_eig(H, S, p, cs, red);
  if (tid == 0) {
    for (int a = 0; a < p; a++) perm[a] = a;
    for (int a = 0; a < p; a++) {
      int best = a;
      for (int b = a + 1; b < p; b++)
        if (H[perm[b] * PMAX + perm[b]] > H[perm[best] * PMAX + perm[best]]) best = b;
      const int t = perm[a];
      perm[a] = perm[best];
      perm[best] = t;
    }
  }
  __syncthreads();
  T* Si = Sout + (int64_t)i * PMAX * PMAX;
  for (int e = tid; e < p * p; e += 256) {
    const int l = e % p, j = e / p;
    Si[e] = (T)S[perm[j] * PMAX + l];
  }
  if (tid < p) th[(int64_t)i * PMAX + tid] = H[perm[tid] * PMAX + perm[tid]];
}

// Largest relative residual ||V_j - theta_j U_j|| / theta_0 over the first
// min(k, p) Ritz pairs; converged when it is <= tol (or when p == n). With a
// selection threshold (thresh > 0) only the pairs that may be kept count:
// those whose shifted Ritz value is above 0.9 thresh (Ritz values grow
// towards the eigenvalues as the iteration proceeds), and always the first.
template <class T>
__global__ void __launch_bounds__(256) k_ss_resid(const int* __restrict__ ids, const int* __restrict__ n_,
                                                  const int* __restrict__ p_, const int* __restrict__ k_,
                                                  const int64_t* __restrict__ oY, const T* __restrict__ V,
                                                  const T* __restrict__ U, const double* __restrict__ th,
                                                  const double* __restrict__ sigma, double thresh, double tol,
                                                  double* res, int* conv) {
  __shared__ double red[16];
  const int i = ids[blockIdx.x];
  const int n = n_[i], p = p_[i], tid = threadIdx.x;
  const double* t = th + (int64_t)i * PMAX;
  int kp = min(k_[i], p);
  if (thresh > 0.0)
    for (int j = 1; j < kp; j++)
      if (t[j] - sigma[i] <= 0.9 * thresh) {
        kp = j;
        break;
      }
  const double th0 = fmax(t[0], 1e-300);
  const T* Vi = V + oY[i];
  const T* Ui = U + oY[i];
  double mx = 0.0;
  for (int j = 0; j < kp; j++) {
    double r2 = 0.0;
    for (int r = tid; r < n; r += 256) {
      const double dv = (double)Vi[r + (int64_t)j * n] - t[j] * (double)Ui[r + (int64_t)j * n];
      r2 += dv * dv;
    }
    r2 = block_sum(r2, red);
    mx = fmax(mx, sqrt(r2) / th0);
  }
  if (tid == 0) {
    res[i] = mx;
    conv[i] = (mx <= tol || p == n) ? 1 : 0;
  }
}

__global__ void k_flag_eig(int* err) { atomicOr(err, ERR_EIG); }

// Selection (descending, minus the shift, above floor_rel * top and thresh)
// and output of the kept eigenvectors (FP64, n x kf at oZ[i]).
template <class T>
__global__ void __launch_bounds__(256) k_ss_final(const int* __restrict__ ids, const int* __restrict__ n_,
                                                  const int* __restrict__ p_, const int* __restrict__ k_,
                                                  const int64_t* __restrict__ oY, const T* __restrict__ U,
                                                  const double* __restrict__ th, const double* __restrict__ sigma,
                                                  double thresh, double floor_rel, const int64_t* __restrict__ oZ,
                                                  double* zv, const int* __restrict__ o_th, double* theta,
                                                  int* kfound) {
  __shared__ int s_kf;
  const int i = ids[blockIdx.x];
  const int n = n_[i], p = p_[i], kp = min(k_[i], p), tid = threadIdx.x;
  const double* t = th + (int64_t)i * PMAX;
  if (tid == 0) {
    const double top = t[0] - sigma[i];
    int kf = 0;
    for (int j = 0; j < kp; j++) {
      const double v = t[j] - sigma[i];
      if (v > floor_rel * top && v > thresh && top > 0.0)
        kf++;
      else
        break;
    }
    for (int j = 0; j < kf; j++) theta[o_th[i] + j] = t[j] - sigma[i];
    kfound[i] = kf;
    s_kf = kf;
  }
  __syncthreads();
  const int kf = s_kf;
  const T* Ui = U + oY[i];
  for (int64_t e = tid; e < (int64_t)n * kf; e += 256) zv[oZ[i] + e] = (double)Ui[e];
}

// Orthonormalize the coarse columns of subdomain i (rows I_i), dropping
// columns that are numerically dependent, and store them as Z_i (fp64).
template <class T>
__global__ void __launch_bounds__(256) k_orth(const int* __restrict__ nI_, const int* __restrict__ kf_,
                                              const int64_t* __restrict__ voff, const int64_t* __restrict__ xoff,
                                              const int* __restrict__ nt_, int64_t colstride, const T* __restrict__ xr,
                                              const double* __restrict__ scale,
                                              const int64_t* __restrict__ zoff, double* Z, int* kfinal,
                                              int* keep_idx) {
  __shared__ double red[32];
  __shared__ double dsh[KMAX];
  const int i = blockIdx.x;
  const int nI = nI_[i], k = kf_[i];
  double* Zi = Z + zoff[i];
  const int tid = threadIdx.x;
  int kept = 0;
  // every thread reads and writes only its own rows r = tid + 256 m of the
  // columns, so only the reductions need barriers
  for (int a = 0; a < k; a++) {
    double* v = Zi + (int64_t)kept * nI;
    double n0 = 0.0;
    for (int r = tid; r < nI; r += 256) {
      double x = (double)xr[xoff[i] + (int64_t)a * (colstride > 0 ? colstride : (int64_t)nt_[i] * TS) + r];
      if (scale) x *= scale[voff[i] + r];
      v[r] = x;
      n0 += x * x;
    }
    n0 = sqrt(block_sum(n0, red));
    // classical Gram-Schmidt, twice: all projections of a pass from one set
    // of dot products (eight per sweep and reduction), then one update sweep
    for (int pass = 0; pass < 2 && kept > 0; pass++) {
      for (int b0 = 0; b0 < kept; b0 += 8) {
        double pd[8];
#pragma unroll
        for (int m = 0; m < 8; m++) pd[m] = 0.0;
        for (int r = tid; r < nI; r += 256) {
          const double vr = v[r];
#pragma unroll
          for (int m = 0; m < 8; m++)
            if (b0 + m < kept) pd[m] += Zi[(int64_t)(b0 + m) * nI + r] * vr;
        }
        block_sum8(pd, red);
        if (tid == 0)
#pragma unroll
          for (int m = 0; m < 8; m++)
            if (b0 + m < kept) dsh[b0 + m] = pd[m];
      }
      __syncthreads();
      for (int r = tid; r < nI; r += 256) {
        double acc = v[r];
#pragma unroll 4
        for (int b = 0; b < kept; b++) acc -= dsh[b] * Zi[(int64_t)b * nI + r];
        v[r] = acc;
      }
      __syncthreads();
    }
    double nr = 0.0;
    for (int r = tid; r < nI; r += 256) nr += v[r] * v[r];
    nr = sqrt(block_sum(nr, red));
    if (nr > 1e-10 * n0 && nr > 0.0) {
      for (int r = tid; r < nI; r += 256) v[r] /= nr;
      if (tid == 0) keep_idx[i * KMAX + kept] = a;
      kept++;
    }
    __syncthreads();
  }
  if (tid == 0) kfinal[i] = kept;
}

}  // namespace

// Per-subdomain sizes of one symmetric eigen pass over the blocks
// [I, G, T] of the local factors, with the offsets of its dense buffers.
struct PassDims {
  std::vector<int> nI, nG, nT, kreq;
  std::vector<int64_t> oF, oGI, oTG, oGG, oTT, oY, oZv;
  std::vector<int> oth;
  int kmax = 0;
  int over = 0;  // subspace block p = k + over (default over = k of the pass)
  bool general = false;
};

// Buffer offsets from the sizes and kreq (subdomains with kreq = 0 take no room).
static void pass_offsets(PassDims& d) {
  const int N = (int)d.nI.size();
  for (auto* v : {&d.oF, &d.oGI, &d.oTG, &d.oGG, &d.oTT, &d.oY, &d.oZv}) v->assign(N + 1, 0);
  d.oth.assign(N + 1, 0);
  d.kmax = 0;
  for (int i = 0; i < N; i++) {
    d.kmax = std::max(d.kmax, d.kreq[i]);
    const int p = std::min(d.nT[i], std::min(PMAX, d.kreq[i] + d.over));
    const bool act = d.kreq[i] > 0;
    const int64_t nG = d.nG[i];
    d.oF[i + 1] = d.oF[i] + (act && !d.general ? (int64_t)d.nI[i] * d.nT[i] : 0);
    d.oGI[i + 1] = d.oGI[i] + (act ? nG * d.nI[i] : 0);
    d.oTG[i + 1] = d.oTG[i] + (act ? nG * d.nT[i] : 0);
    d.oGG[i + 1] = d.oGG[i] + (act ? nG * nG : 0);
    d.oTT[i + 1] = d.oTT[i] + (act ? (int64_t)d.nT[i] * d.nT[i] : 0);
    d.oY[i + 1] = d.oY[i] + (act ? (int64_t)d.nT[i] * std::max(p, 1) : 0);
    d.oZv[i + 1] = d.oZv[i] + (int64_t)d.nT[i] * d.kreq[i];
    d.oth[i + 1] = d.oth[i] + d.kreq[i];
  }
}

static PassDims pass_dims(const tls_ctx* c, const std::vector<int>& nG, int nev, bool general) {
  const int N = c->N;
  PassDims d;
  d.nI.resize(N);
  d.nG = nG;
  d.nT.resize(N);
  d.kreq.resize(N);
  d.general = general;
  d.over = c->opt.eig_oversample >= 0 ? c->opt.eig_oversample : nev;
  for (int i = 0; i < N; i++) {
    d.nI[i] = c->h_nI[i];
    d.nT[i] = c->h_m[i] - d.nI[i] - nG[i];
    int k = std::min(std::min(nev, d.nT[i]), PMAX - OVER_MIN);
    if (general) k = std::min(k, d.nI[i]);
    d.kreq[i] = std::max(k, 0);
  }
  pass_offsets(d);
  return d;
}

// The same pass restricted to the subdomains [i0, i1).
static PassDims pass_restrict(const PassDims& d, int i0, int i1) {
  PassDims r = d;
  for (int i = 0; i < (int)d.kreq.size(); i++)
    if (i < i0 || i >= i1) r.kreq[i] = 0;
  pass_offsets(r);
  return r;
}

// Device copies of the per-subdomain tables of a pass.
struct PassDev {
  DBuf<int> nI, nG, nT, kreq, oth;
  DBuf<int64_t> oF, oGI, oTG, oGG, oTT, oY, oZv, oXH;
  void upload(const PassDims& d, const std::vector<int64_t>& oXH_h, hipStream_t s) {
    nI.upload(d.nI, s);
    nG.upload(d.nG, s);
    nT.upload(d.nT, s);
    kreq.upload(d.kreq, s);
    oth.upload(d.oth, s);
    oF.upload(d.oF, s);
    oGI.upload(d.oGI, s);
    oTG.upload(d.oTG, s);
    oGG.upload(d.oGG, s);
    oTT.upload(d.oTT, s);
    oY.upload(d.oY, s);
    oZv.upload(d.oZv, s);
    oXH.upload(oXH_h, s);
  }
  EigLayout layout(const tls_ctx* c) const {
    return EigLayout{nI.p, nG.p, nT.p, c->d_m.p, c->d_nt.p, c->d_foff.p, oF.p, oGI.p, oTG.p, oGG.p, oTT.p, oXH.p,
                     kreq.p, c->layout()};
  }
};

// Result of the subspace iteration of one pass (host copies).
struct PassEig {
  std::vector<int> kf;         // pairs kept per subdomain
  std::vector<double> theta;   // their eigenvalues of C, at oth[i] + j
  double resid_max = 0.0;
  int iters_max = 0;
  double iters_sum = 0.0;
  int n_solved = 0;
};

// Top eigenpairs of C (nT x nT per subdomain, fp64, in C64) by subspace
// iteration; the eigenvectors land in zv (nT x kf, offsets oZv).
// Batched subspace iteration driver (kernels above) in precision T.
template <class T>
static PassEig subspace_batched(tls_ctx* c, const PassDims& d, PassDev& dv, const DBuf<double>& C64,
                                DBuf<double>& zv, double thresh, const double* Ywarm, int c0) {
  hipStream_t s = c->stream;
  const int N = c->N;
  std::vector<int> p(N, 0), all;
  for (int i = 0; i < N; i++) {
    if (d.kreq[i] <= 0 || d.nT[i] <= 0) continue;
    p[i] = std::min(d.nT[i], std::min(PMAX, d.kreq[i] + d.over));
    all.push_back(i);
  }
  PassEig e;
  e.kf.assign(N, 0);
  e.theta.assign(std::max(d.oth[N], 1), 0.0);
  zv.alloc(std::max<int64_t>(d.oZv[N], 1));
  if (all.empty()) return e;
  DBuf<int> d_p, ids, conv, kfound;
  d_p.upload(p, s);
  DBuf<T> Cw, Y, W, V, U, Hb, Sb;
  DBuf<double> th, sig, res, theta;
  Cw.alloc(std::max<int64_t>(d.oTT[N], 1));
  for (auto* b : {&Y, &W, &V, &U}) b->alloc(std::max<int64_t>(d.oY[N], 1));
  Hb.alloc((size_t)N * PMAX * PMAX);
  Sb.alloc((size_t)N * PMAX * PMAX);
  th.alloc((size_t)N * PMAX);
  sig.alloc(N);
  res.alloc(N);
  conv.alloc(N);
  kfound.alloc(N);
  theta.alloc(std::max(d.oth[N], 1));
  ids.upload(all, s);
  DBuf<double> nowarm;
  if (!Ywarm) nowarm.alloc(1);
  hipLaunchKernelGGL(k_ss_init<T>, dim3((unsigned)all.size()), dim3(256), 0, s, ids.p, dv.nT.p, d_p.p, dv.oTT.p,
                     dv.oY.p, C64.p, Cw.p, Y.p, Ywarm ? Ywarm : nowarm.p, Ywarm ? c0 : 0, (uint64_t)c->opt.seed,
                     sig.p);
  TLS_LAUNCH_CHECK();
  GemmPlan pCY, pTN, pNP;  // n x p = C Y;  p x p = X^T Y;  n x p = X (p x p)
  std::vector<int> act = all;
  auto plans = [&](const std::vector<int>& a) {
    std::vector<GemmDesc> g1, g2, g3;
    for (int i : a) {
      const int n = d.nT[i], pi = p[i];
      const int64_t oS = (int64_t)i * PMAX * PMAX;
      g1.push_back(GemmDesc{n, pi, n, n, n, d.oTT[i], d.oY[i], d.oY[i], (int64_t)n});
      g2.push_back(GemmDesc{pi, pi, n, n, n, d.oY[i], d.oY[i], oS, (int64_t)pi});
      g3.push_back(GemmDesc{n, pi, pi, n, pi, d.oY[i], oS, d.oY[i], (int64_t)n});
    }
    gemm_plan(pCY, g1, s);
    gemm_plan(pTN, g2, s);
    gemm_plan(pNP, g3, s);
    ids.upload(a, s);
    TLS_HIP(hipStreamSynchronize(s));
  };
  // Y <- orth(X) by CholQR with equilibration, twice; X is overwritten
  auto orth = [&](T* X) {
    for (int pass = 0; pass < 2; pass++) {
      T* src = pass == 0 ? X : Y.p;
      T* dst = pass == 0 ? Y.p : X;
      gemm_run<T>(s, pTN, true, false, src, src, Hb.p, T(1), T(0));
      hipLaunchKernelGGL(k_ss_chol<T>, dim3((unsigned)act.size()), dim3(64), 0, s, ids.p, d_p.p, Hb.p, Sb.p,
                         c->errflag.p);
      TLS_LAUNCH_CHECK();
      gemm_run<T>(s, pNP, false, false, src, Sb.p, dst, T(1), T(0));
    }
    // the result of the second pass is in X: copy it back into Y
    TLS_HIP(hipMemcpyAsync(Y.p, X, sizeof(T) * std::max<int64_t>(d.oY[N], 1), hipMemcpyDeviceToDevice, s));
  };
  plans(act);
  TLS_HIP(hipMemcpyAsync(V.p, Y.p, sizeof(T) * std::max<int64_t>(d.oY[N], 1), hipMemcpyDeviceToDevice, s));
  orth(V.p);
  const double tol = c->opt.eig_tol > 0 ? c->opt.eig_tol : (c->fp32 ? 1e-5 : 1e-9);
  const int maxit = c->opt.eig_maxit;
  std::vector<int> iters(N, 0);
  std::vector<double> hres(N, 0.0);
  std::vector<std::vector<double>> res_hist(N);
  for (int it = 1; it <= maxit && !act.empty(); it++) {
    gemm_run<T>(s, pCY, false, false, Cw.p, Y.p, W.p, T(1), T(0));      // W = C Y
    gemm_run<T>(s, pTN, true, false, Y.p, W.p, Hb.p, T(1), T(0));       // H = Y^T W
    hipLaunchKernelGGL(k_ss_rr<T>, dim3((unsigned)act.size()), dim3(256), 0, s, ids.p, d_p.p, Hb.p, Sb.p, th.p);
    TLS_LAUNCH_CHECK();
    gemm_run<T>(s, pNP, false, false, W.p, Sb.p, V.p, T(1), T(0));      // V = W S
    gemm_run<T>(s, pNP, false, false, Y.p, Sb.p, U.p, T(1), T(0));      // U = Y S
    hipLaunchKernelGGL(k_ss_resid<T>, dim3((unsigned)act.size()), dim3(256), 0, s, ids.p, dv.nT.p, d_p.p,
                       dv.kreq.p, dv.oY.p, V.p, U.p, th.p, sig.p, thresh, tol, res.p, conv.p);
    TLS_LAUNCH_CHECK();
    auto h_conv = download(conv.p, N, s);
    auto h_res = download(res.p, N, s);
    std::vector<int> next;
    for (int i : act) {
      iters[i] = it;
      hres[i] = h_res[i];
      if (std::isnan(h_res[i])) fail(TLS_E_NOCONV, "local eigensolver: NaN residual in subdomain " + std::to_string(i));
      // stagnation at the rounding floor of the working precision: accept a
      // residual below 10 tol that has not dropped 5% in four iterations
      auto& hist = res_hist[i];
      hist.push_back(h_res[i]);
      if (!h_conv[i] && hist.size() > 4 && h_res[i] <= 10.0 * tol && h_res[i] > 0.95 * hist[hist.size() - 5])
        h_conv[i] = 1;
      if (!h_conv[i] && it < maxit) next.push_back(i);
      if (!h_conv[i] && it == maxit) {
        hipLaunchKernelGGL(k_flag_eig, dim3(1), dim3(1), 0, s, c->errflag.p);
        TLS_LAUNCH_CHECK();
      }
    }
    if (next.empty()) break;
    if (next.size() != act.size()) {
      act = next;
      plans(act);
    }
    orth(V.p);  // Y <- orth(V)
  }
  ids.upload(all, s);
  hipLaunchKernelGGL(k_ss_final<T>, dim3((unsigned)all.size()), dim3(256), 0, s, ids.p, dv.nT.p, d_p.p, dv.kreq.p,
                     dv.oY.p, U.p, th.p, sig.p, thresh, 1e-12, dv.oZv.p, zv.p, dv.oth.p, theta.p, kfound.p);
  TLS_LAUNCH_CHECK();
  auto kf = download(kfound.p, N, s);
  auto tt = download(theta.p, std::max(d.oth[N], 1), s);
  for (int i : all) {
    e.kf[i] = kf[i];
    e.resid_max = std::max(e.resid_max, hres[i]);
    e.iters_max = std::max(e.iters_max, iters[i]);
    e.iters_sum += iters[i];
  }
  e.n_solved = (int)all.size();
  e.theta = tt;
  return e;
}

// Ypre (optional): FP64 start block holding c0 warm columns per subdomain.
static PassEig run_subspace(tls_ctx* c, const PassDims& d, PassDev& dv, const DBuf<double>& C64, DBuf<double>& zv,
                            double thresh, DBuf<double>* Ypre = nullptr, int c0 = 0) {
  const double* yw = Ypre ? Ypre->p : nullptr;
  if (c->fp32) return subspace_batched<float>(c, d, dv, C64, zv, thresh, yw, c0);
  return subspace_batched<double>(c, d, dv, C64, zv, thresh, yw, c0);
}

// One SPD pass (see the file header): F = -L_TI^T + L_GI^T L_GG^{-T} L_TG^T,
// C = L_TT^{-1} F^T F L_TT^{-T}, top pairs of C, then the vectors
// F L_TT^{-T} z written as column colbase[i] + j of the per-column padded
// buffer XV (column j of every subdomain is padded local vector j, stride
// sum_M); a backward solve with the whole factor then turns [V; 0] into
// [L_II^{-T} V; 0].
// gevp2: the eq. gevpsvd pass (the learned warm start and the training
// targets belong to it).
template <class T>
static PassEig spd_pass(tls_ctx* c, const T* fac, const PassDims& d, double thresh, const std::vector<int>& colbase,
                        T* XV, bool gevp2) {
  hipStream_t s = c->stream;
  const int N = c->N;
  PassDev dv;
  dv.upload(d, std::vector<int64_t>(N + 1, 0), s);
  const EigLayout el = dv.layout(c);
  const dim3 eg(64, N);
  DBuf<T> F, GI, TG, GGt, K;
  DBuf<double> LTT, LTTt, C64, C64b;
  // buffers are taken as late and given back as early as the steps allow:
  // the nT x nT blocks dominate the memory of a pass
  K.alloc(std::max<int64_t>(d.oTT[N], 1));
  F.alloc(std::max<int64_t>(d.oF[N], 1));
  hipLaunchKernelGGL(k_extract_f<T>, eg, dim3(256), 0, s, el, fac, F.p);
  TLS_LAUNCH_CHECK();
  if (d.oGG[N] > 0) {
    GI.alloc(d.oGI[N]);
    TG.alloc(d.oTG[N]);
    GGt.alloc(d.oGG[N]);
    hipLaunchKernelGGL((k_extract<T, T>), eg, dim3(256), 0, s, 1, el, fac, TG.p);
    hipLaunchKernelGGL((k_extract<T, T>), eg, dim3(256), 0, s, 2, el, fac, GGt.p);
    hipLaunchKernelGGL((k_extract<T, T>), eg, dim3(256), 0, s, 3, el, fac, GI.p);
    TLS_LAUNCH_CHECK();
    // Tm = L_GG^{-T} L_TG^T ; F += L_GI^T Tm
    std::vector<TriDesc> td;
    for (int i = 0; i < N; i++)
      if (d.kreq[i] > 0 && d.nG[i] > 0) td.push_back(TriDesc{d.nG[i], d.nT[i], d.oGG[i], d.oTG[i], (int64_t)d.nG[i]});
    batched_trsm<T>(s, td, UPPER_BWD, GGt.p, TG.p, c->errflag.p);
    std::vector<GemmDesc> gd;
    for (int i = 0; i < N; i++)
      if (d.kreq[i] > 0 && d.nG[i] > 0)
        gd.push_back(GemmDesc{d.nI[i], d.nT[i], d.nG[i], d.nG[i], d.nG[i], d.oGI[i], d.oTG[i], d.oF[i],
                              (int64_t)d.nI[i]});
    batched_gemm<T>(s, gd, true, false, GI.p, TG.p, F.p, T(1), T(1));
    GI.release();
    TG.release();
    GGt.release();
  }
  // K = F^T F: only the tiles on and below the block diagonal (K is
  // symmetric). Without G layers (delta = 1) F = -L_TI^T, and column t of F
  // is zero above the tile profile of row t of L: each 64-column block of F
  // starts at the first interior row its profile reaches, and the K loop of
  // each tile of K starts at the later of its two blocks' starts.
  DBuf<int> kst;
  {
    std::vector<int> hk;
    std::vector<int64_t> kofs(N, -1);
    if (!c->h_prof.empty())
      for (int i = 0; i < N; i++) {
        if (d.kreq[i] <= 0 || d.nG[i] > 0) continue;
        kofs[i] = (int64_t)hk.size();
        const int t0 = d.nI[i];  // first T row in Omega_i (no G rows)
        for (int b = 0; b * TS < d.nT[i]; b++) {
          const int r0 = t0 + b * TS, r1 = std::min(t0 + d.nT[i], r0 + TS) - 1;
          int f = INT32_MAX;
          for (int tile = r0 / TS; tile <= r1 / TS; tile++) f = std::min(f, c->h_prof[c->h_toff[i] + tile]);
          hk.push_back(std::min(f * TS, d.nI[i]));
        }
      }
    kst.upload(hk, s);
    std::vector<GemmDesc> gd;
    for (int i = 0; i < N; i++)
      if (d.kreq[i] > 0) {
        GemmDesc g{d.nT[i], d.nT[i], d.nI[i], d.nI[i], d.nI[i], d.oF[i], d.oF[i], d.oTT[i], (int64_t)d.nT[i]};
        g.syrk = 1;
        g.kstart = kofs[i] >= 0 ? kst.p + kofs[i] : nullptr;
        gd.push_back(g);
      }
    batched_gemm<T>(s, gd, true, false, F.p, F.p, K.p, T(1), T(0));
  }
  // C = L_TT^{-1} K L_TT^{-T}: X = L^{-1} K; C = L^{-1} X^T, in the local
  // precision (FP32 in mixed mode, where the factor itself is FP32); the
  // subspace iteration takes C in FP64
  std::vector<TriDesc> td;
  for (int i = 0; i < N; i++)
    if (d.kreq[i] > 0) td.push_back(TriDesc{d.nT[i], d.nT[i], d.oTT[i], d.oTT[i], (int64_t)d.nT[i]});
  C64.alloc(std::max<int64_t>(d.oTT[N], 1));
  if (std::is_same<T, float>::value) {
    DBuf<T> Cc, Ccb;
    Cc.alloc(std::max<int64_t>(d.oTT[N], 1));
    hipLaunchKernelGGL((k_sym_from_lower<T, T>), eg, dim3(256), 0, s, dv.nT.p, dv.oTT.p, dv.kreq.p, K.p, Cc.p);
    TLS_LAUNCH_CHECK();
    K.release();
    DBuf<T> LTTc;
    LTTc.alloc(std::max<int64_t>(d.oTT[N], 1));
    hipLaunchKernelGGL((k_extract<T, T>), eg, dim3(256), 0, s, 4, el, fac, LTTc.p);
    TLS_LAUNCH_CHECK();
    Ccb.alloc(std::max<int64_t>(d.oTT[N], 1));
    batched_trsm<T>(s, td, LOWER_FWD, LTTc.p, Cc.p, c->errflag.p);
    hipLaunchKernelGGL(k_transpose_blocks<T>, eg, dim3(256), 0, s, dv.nT.p, dv.oTT.p, dv.kreq.p, Cc.p, Ccb.p, 0);
    TLS_LAUNCH_CHECK();
    batched_trsm<T>(s, td, LOWER_FWD, LTTc.p, Ccb.p, c->errflag.p);
    hipLaunchKernelGGL(k_transpose_blocks<T>, eg, dim3(256), 0, s, dv.nT.p, dv.oTT.p, dv.kreq.p, Ccb.p, Cc.p, 1);
    TLS_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_convert<T, double>), dim3(1024), dim3(256), 0, s, (int64_t)d.oTT[N], Cc.p, C64.p);
    TLS_LAUNCH_CHECK();
    TLS_HIP(hipStreamSynchronize(s));  // Cc, Ccb, LTTc are freed on return from this block
  } else {
    hipLaunchKernelGGL((k_sym_from_lower<T, double>), eg, dim3(256), 0, s, dv.nT.p, dv.oTT.p, dv.kreq.p, K.p, C64.p);
    TLS_LAUNCH_CHECK();
    K.release();
    LTT.alloc(std::max<int64_t>(d.oTT[N], 1));
    hipLaunchKernelGGL((k_extract<T, double>), eg, dim3(256), 0, s, 4, el, fac, LTT.p);
    TLS_LAUNCH_CHECK();
    C64b.alloc(std::max<int64_t>(d.oTT[N], 1));
    batched_trsm<double>(s, td, LOWER_FWD, LTT.p, C64.p, c->errflag.p);
    hipLaunchKernelGGL(k_transpose_blocks<double>, eg, dim3(256), 0, s, dv.nT.p, dv.oTT.p, dv.kreq.p, C64.p, C64b.p,
                       0);
    TLS_LAUNCH_CHECK();
    batched_trsm<double>(s, td, LOWER_FWD, LTT.p, C64b.p, c->errflag.p);
    hipLaunchKernelGGL(k_transpose_blocks<double>, eg, dim3(256), 0, s, dv.nT.p, dv.oTT.p, dv.kreq.p, C64b.p, C64.p,
                       1);
    TLS_LAUNCH_CHECK();
  }
  if (download(c->errflag.p, 1, s)[0] & ERR_PIVOT) fail(TLS_E_NOT_SPD, "zero pivot in a Schur-complement block");
  LTT.release();
  C64b.release();
  LTTt.alloc(std::max<int64_t>(d.oTT[N], 1));
  hipLaunchKernelGGL((k_extract<T, double>), eg, dim3(256), 0, s, 5, el, fac, LTTt.p);
  TLS_LAUNCH_CHECK();
  DBuf<double> zv;
  DBuf<double> Ywarm;
  int c0 = 0;
  if (gevp2 && c->opt.gnn_weights) {
    // start block = L_TT^T X_T: the network guesses the rows T of the
    // eigenvectors w, and z = L_TT^T w_T are the eigenvectors of C
    const auto t0 = std::chrono::steady_clock::now();
    gnn_forward(c, c->opt.gnn_weights, c->opt.gnn_c_out, false);
    c0 = std::min(c->opt.gnn_c_out, PMAX);
    std::vector<int64_t> oX(N + 1, 0);
    for (int i = 0; i < N; i++) oX[i + 1] = oX[i] + (d.kreq[i] > 0 ? (int64_t)d.nT[i] * c0 : 0);
    DBuf<double> Xg;
    Xg.alloc(std::max<int64_t>(oX[N], 1));
    gnn_take_rows(c, d.nT, d.kreq, oX, c0, Xg.p);
    Ywarm.alloc(std::max<int64_t>(d.oY[N], 1));
    std::vector<GemmDesc> gw;
    for (int i = 0; i < N; i++) {
      if (d.kreq[i] <= 0) continue;
      const int p = std::min(d.nT[i], std::min(PMAX, d.kreq[i] + d.over));
      const int cw = std::min(c0, p);
      gw.push_back(GemmDesc{d.nT[i], cw, d.nT[i], d.nT[i], d.nT[i], d.oTT[i], oX[i], d.oY[i], (int64_t)d.nT[i]});
    }
    batched_gemm<double>(s, gw, false, false, LTTt.p, Xg.p, Ywarm.p, 1.0, 0.0);
    TLS_HIP(hipStreamSynchronize(s));
    c->t_setup[4] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  PassEig e = run_subspace(c, d, dv, C64, zv, thresh, c0 > 0 ? &Ywarm : nullptr, c0);
  C64.release();
  // w_T = L_TT^{-T} z ; V = F w_T into columns colbase[i] + j of XV
  std::vector<TriDesc> tw;
  for (int i = 0; i < N; i++)
    if (e.kf[i] > 0) tw.push_back(TriDesc{d.nT[i], e.kf[i], d.oTT[i], d.oZv[i], (int64_t)d.nT[i]});
  batched_trsm<double>(s, tw, UPPER_BWD, LTTt.p, zv.p, c->errflag.p);
  if (gevp2 && c->opt.gnn_train) gnn_keep_targets(c, d.nT, e.kf, zv.p, d.oZv);
  DBuf<T> wT;
  wT.alloc(std::max<int64_t>(d.oZv[N], 1));
  hipLaunchKernelGGL((k_convert<double, T>), dim3(1024), dim3(256), 0, s, (int64_t)d.oZv[N], zv.p, wT.p);
  TLS_LAUNCH_CHECK();
  std::vector<GemmDesc> gd;
  for (int i = 0; i < N; i++)
    if (e.kf[i] > 0)
      gd.push_back(GemmDesc{d.nI[i], e.kf[i], d.nT[i], d.nI[i], d.nT[i], d.oF[i], d.oZv[i],
                            c->h_voff[i] + (int64_t)colbase[i] * c->sum_M, c->sum_M});
  batched_gemm<T>(s, gd, false, false, F.p, wT.p, XV, T(1), T(0));
  TLS_HIP(hipStreamSynchronize(s));
  return e;
}

// Peak device bytes of subdomain i in an SPD pass: the nT x nT blocks (K,
// two FP64 copies of C, L_TT and the working copy Cw), F, the G blocks, the
// subspace blocks and the eigenvectors.
static int64_t spd_pass_bytes(const PassDims& d, int i, int64_t tsz) {
  if (d.kreq[i] <= 0) return 0;
  const int64_t tt = (int64_t)d.nT[i] * d.nT[i], nG = d.nG[i];
  return tt * (24 + 2 * tsz) + ((int64_t)d.nI[i] * d.nT[i] + nG * (nG + d.nI[i] + d.nT[i])) * tsz +
         (d.oY[i + 1] - d.oY[i]) * 4 * tsz + (d.oZv[i + 1] - d.oZv[i]) * (8 + tsz);
}

// spd_pass over groups of consecutive subdomains whose buffers fit in the
// memory budget (devmem::budget; one group when all fit). The
// learned warm start and its training targets work on all subdomains at
// once, so a pass that uses them is not split.
template <class T>
static PassEig spd_pass_grouped(tls_ctx* c, const T* fac, const PassDims& d, double thresh,
                                const std::vector<int>& colbase, T* XV, bool gevp2) {
  const int N = c->N;
  const bool whole = gevp2 && (c->opt.gnn_weights || c->opt.gnn_train);
  const int64_t budget = (int64_t)devmem::budget();
  std::vector<std::pair<int, int>> groups;
  int64_t acc = 0;
  for (int i = 0; i < N; i++) {
    const int64_t b = spd_pass_bytes(d, i, sizeof(T));
    if (groups.empty() || (!whole && acc + b > budget)) {
      groups.push_back({i, i});
      acc = 0;
    }
    groups.back().second = i + 1;
    acc += b;
  }
  if (groups.size() <= 1) return spd_pass<T>(c, fac, d, thresh, colbase, XV, gevp2);
  PassEig e;
  e.kf.assign(N, 0);
  e.theta.assign(std::max(d.oth[N], 1), 0.0);
  for (const auto& g : groups) {
    const PassDims dg = pass_restrict(d, g.first, g.second);
    if (dg.kmax == 0) continue;
    const PassEig eg = spd_pass<T>(c, fac, dg, thresh, colbase, XV, gevp2);
    for (int i = g.first; i < g.second; i++) {
      e.kf[i] = eg.kf[i];
      for (int j = 0; j < eg.kf[i]; j++) e.theta[d.oth[i] + j] = eg.theta[dg.oth[i] + j];
    }
    e.resid_max = std::max(e.resid_max, eg.resid_max);
    e.iters_max = std::max(e.iters_max, eg.iters_max);
    e.iters_sum += eg.iters_sum;
    e.n_solved += eg.n_solved;
  }
  return e;
}

// Orthonormalize the columns of every subdomain into Z (fp64) and record
// the kept columns, their eigenvalues and which eigenproblem each came from.
template <class T>
static void finish_basis(tls_ctx* c, const std::vector<int>& ncols, const std::vector<double>& colval,
                         const std::vector<int>& colsrc, const std::vector<int64_t>& colval_off,
                         const DBuf<int64_t>& d_xoff, int64_t colstride, const T* XV) {
  hipStream_t s = c->stream;
  const int N = c->N;
  std::vector<int64_t> oZ(N + 1, 0);
  for (int i = 0; i < N; i++) oZ[i + 1] = oZ[i] + (int64_t)c->h_nI[i] * ncols[i];
  DBuf<int64_t> d_oZ;
  DBuf<int> d_nI, kf, kfin, keep;
  d_oZ.upload(oZ, s);
  d_nI.upload(std::vector<int>(c->h_nI.begin(), c->h_nI.end()), s);
  kf.upload(ncols, s);
  DBuf<double> Zt;
  Zt.alloc(std::max<int64_t>(oZ[N], 1));
  kfin.alloc(N);
  keep.alloc((size_t)N * KMAX);
  hipLaunchKernelGGL(k_orth<T>, dim3(N), dim3(256), 0, s, d_nI.p, kf.p, c->d_voff.p, d_xoff.p, c->d_nt.p, colstride,
                     XV, c->opt.jacobi_scale ? c->scale.p : nullptr, d_oZ.p, Zt.p, kfin.p, keep.p);
  TLS_LAUNCH_CHECK();
  auto h_kfin = download(kfin.p, N, s);
  auto h_keep = download(keep.p, (size_t)N * KMAX, s);
  c->h_zcol.assign(N + 1, 0);
  c->h_zoff = oZ;
  c->h_eig.clear();
  c->h_zsrc.clear();
  for (int i = 0; i < N; i++) {
    c->h_zcol[i + 1] = c->h_zcol[i] + h_kfin[i];
    for (int a = 0; a < h_kfin[i]; a++) {
      const int src = h_keep[(size_t)i * KMAX + a];
      c->h_eig.push_back(colval[colval_off[i] + src]);
      c->h_zsrc.push_back(colsrc[colval_off[i] + src]);
    }
  }
  c->nC = c->h_zcol[N];
  c->Z.alloc(std::max<int64_t>(oZ[N], 1));
  TLS_HIP(hipMemcpyAsync(c->Z.p, Zt.p, sizeof(double) * std::max<int64_t>(oZ[N], 1), hipMemcpyDeviceToDevice, s));
  c->zcol.upload(c->h_zcol, s);
  c->zoff.upload(c->h_zoff, s);
  TLS_HIP(hipStreamSynchronize(s));
}

static void empty_basis(tls_ctx* c) {
  c->nC = 0;
  c->h_zcol.assign(c->N + 1, 0);
  c->h_zoff.assign(c->N + 1, 0);
  c->h_eig.clear();
  c->h_zsrc.clear();
  c->zcol.upload(c->h_zcol, c->stream);
  c->zoff.upload(c->h_zoff, c->stream);
  c->Z.alloc(1);
}

// SPD: eq. gevpsvd (blocks [I, G, T] with G = Gamma_{1:delta-1},
// T = Gamma_delta) and, when nev1 > 0, eq. uppergevp. For the latter, with
// Omega_i = [I, O] and L = [[L_II, 0], [L_OI, L_OO]], the nonzero part of
// D_i A_ii D_i u = lambda A_ii u is, after u = L^{-T} v, the matrix V V^T
// with V = [I; -L_OO^{-1} L_OI]: lambda = 1 + kappa where kappa are the
// eigenvalues of C1 = L_OO^{-1} L_OI L_OI^T L_OO^{-T}, and rows I of the
// eigenvector are proportional to L_II^{-T} L_OI^T L_OO^{-T} y. That is
// the same pass with G empty and T = O (F = -L_OI^T); lambda > nu keeps
// kappa > nu - 1.
template <class T>
static void basis_spd(tls_ctx* c, T* fac) {
  hipStream_t s = c->stream;
  const int N = c->N;
  std::vector<int> nG2(N), nG1(N, 0);
  for (int i = 0; i < N; i++) nG2[i] = c->h_nP[i] - c->h_nI[i];
  const PassDims d2 = pass_dims(c, nG2, c->nev, false);
  const int nev1 = c->opt.nev1;
  const PassDims d1 = pass_dims(c, nG1, nev1, false);
  if (d2.kmax == 0 && d1.kmax == 0) {
    empty_basis(c);
    return;
  }
  int kcols = 0;
  for (int i = 0; i < N; i++) kcols = std::max(kcols, d2.kreq[i] + d1.kreq[i]);
  kcols = (std::max(kcols, 1) + TS - 1) / TS * TS;  // whole column blocks for the backward solve
  DBuf<T> XV;
  XV.alloc((size_t)kcols * c->sum_M);
  TLS_HIP(hipMemsetAsync(XV.p, 0, sizeof(T) * kcols * c->sum_M, s));
  TLS_HIP(hipMemsetAsync(c->errflag.p, 0, sizeof(int), s));
  const double tau2 = c->opt.tau > 0 ? c->opt.tau * c->opt.tau : -1.0;  // lambda^2 > tau^2
  PassEig e2, e1;
  e2.kf.assign(N, 0);
  e1.kf.assign(N, 0);
  if (d2.kmax > 0) e2 = spd_pass_grouped<T>(c, fac, d2, tau2, std::vector<int>(N, 0), XV.p, true);
  if (d1.kmax > 0) {
    const double nu = c->opt.nu > 0 ? c->opt.nu : 1.0;
    e1 = spd_pass_grouped<T>(c, fac, d1, nu - 1.0, e2.kf, XV.p, false);  // lambda = 1 + kappa > nu
  }
  c->eig_resid_max = std::max(e2.resid_max, e1.resid_max);
  c->eig_iters_max = std::max(e2.iters_max, e1.iters_max);
  c->eig_iters_mean = (e2.iters_sum + e1.iters_sum) / std::max(1, e2.n_solved + e1.n_solved);
  // x = L^{-T} [V; 0]: rows I are L_II^{-T} V (the rows outside I stay
  // zero), all columns of a subdomain at once by the blocked MFMA solve
  std::vector<int> ncols(N), nq(N);
  for (int i = 0; i < N; i++) {
    ncols[i] = e2.kf[i] + e1.kf[i];
    nq[i] = (ncols[i] + TS - 1) / TS;
  }
  local_bsolve_interior(c, XV.p, nq, c->h_voff, c->sum_M);
  // eigenvalue and source of every column: lambda^2 (eq. gevpsvd) or lambda (eq. uppergevp)
  std::vector<double> colval;
  std::vector<int> colsrc;
  std::vector<int64_t> coff(N + 1, 0);
  for (int i = 0; i < N; i++) {
    for (int j = 0; j < e2.kf[i]; j++) {
      colval.push_back(e2.theta[d2.oth[i] + j]);
      colsrc.push_back(0);
    }
    for (int j = 0; j < e1.kf[i]; j++) {
      colval.push_back(1.0 + e1.theta[d1.oth[i] + j]);
      colsrc.push_back(1);
    }
    coff[i + 1] = colval.size();
  }
  finish_basis<T>(c, ncols, colval, colsrc, coff, c->d_voff, c->sum_M, XV.p);
}

// One pass of the general basis over the subdomains with kreq > 0: H, its
// Gram, the subspace iteration, and V = H v into XV at oXV[i].
template <class T>
static PassEig general_pass(tls_ctx* c, T* fac, const PassDims& d, double tau2, const std::vector<int64_t>& oXV,
                            T* XV) {
  hipStream_t s = c->stream;
  const int N = c->N;
  const std::vector<int>& nI = d.nI;
  const std::vector<int>& nG = d.nG;
  const std::vector<int>& nT = d.nT;
  const std::vector<int>& kreq = d.kreq;
  const std::vector<int64_t>& oGI = d.oGI;
  const std::vector<int64_t>& oTG = d.oTG;
  const std::vector<int64_t>& oGG = d.oGG;
  const std::vector<int64_t>& oTT = d.oTT;
  const std::vector<int64_t>& oZv = d.oZv;
  std::vector<int> nqH(N, 0);
  std::vector<int64_t> oXH(N + 1, 0);
  for (int i = 0; i < N; i++) {
    const int64_t M = (int64_t)c->h_nt[i] * TS;
    nqH[i] = kreq[i] > 0 ? (nT[i] + TS - 1) / TS : 0;
    oXH[i + 1] = oXH[i] + M * TS * nqH[i];
  }
  PassDev dv;
  dv.upload(d, oXH, s);
  const EigLayout el = dv.layout(c);
  const dim3 eg(64, N);
  TLS_HIP(hipMemsetAsync(c->errflag.p, 0, sizeof(int), s));
  DBuf<T> GI, TG, GGt, K, XH;
  DBuf<double> C64;
  K.alloc(std::max<int64_t>(oTT[N], 1));
  C64.alloc(std::max<int64_t>(oTT[N], 1));
  if (oGG[N] > 0) {
    GI.alloc(oGI[N]);
    TG.alloc(oTG[N]);
    GGt.alloc(oGG[N]);
  }
  // with A_ii = L U ordered [I, G, T]: H = U_II^{-1} (-U_IT + U_IG U_GG^{-1} U_GT)
  XH.alloc(std::max<int64_t>(oXH[N], 1));
  TLS_HIP(hipMemsetAsync(XH.p, 0, sizeof(T) * std::max<int64_t>(oXH[N], 1), s));
  hipLaunchKernelGGL((k_extract<T, T>), eg, dim3(256), 0, s, 9, el, fac, XH.p);
  TLS_LAUNCH_CHECK();
  if (oGG[N] > 0) {
    hipLaunchKernelGGL((k_extract<T, T>), eg, dim3(256), 0, s, 6, el, fac, TG.p);
    hipLaunchKernelGGL((k_extract<T, T>), eg, dim3(256), 0, s, 7, el, fac, GGt.p);
    hipLaunchKernelGGL((k_extract<T, T>), eg, dim3(256), 0, s, 8, el, fac, GI.p);
    TLS_LAUNCH_CHECK();
    std::vector<TriDesc> td;
    for (int i = 0; i < N; i++)
      if (kreq[i] > 0) td.push_back(TriDesc{nG[i], nT[i], oGG[i], oTG[i], (int64_t)nG[i]});
    batched_trsm<T>(s, td, UPPER_BWD, GGt.p, TG.p, c->errflag.p);
    std::vector<GemmDesc> gd;
    for (int i = 0; i < N; i++)
      if (kreq[i] > 0 && nG[i] > 0)
        gd.push_back(GemmDesc{nI[i], nT[i], nG[i], nI[i], nG[i], oGI[i], oTG[i], oXH[i],
                              (int64_t)c->h_nt[i] * TS});
    batched_gemm<T>(s, gd, false, false, GI.p, TG.p, XH.p, T(1), T(1));
  }
  if (download(c->errflag.p, 1, s)[0] & ERR_PIVOT) fail(TLS_E_SINGULAR, "zero pivot in a local U_GG block");
  // H = U_II^{-1} X (rows I); rows G, T of XH stay zero
  local_bsolve_interior(c, XH.p, nqH, oXH, 0);
  // K = H^T H
  std::vector<GemmDesc> gd;
  for (int i = 0; i < N; i++) {
    const int M = c->h_nt[i] * TS;
    if (kreq[i] > 0) gd.push_back(GemmDesc{nT[i], nT[i], nI[i], M, M, oXH[i], oXH[i], oTT[i], (int64_t)nT[i]});
  }
  batched_gemm<T>(s, gd, true, false, XH.p, XH.p, K.p, T(1), T(0));
  hipLaunchKernelGGL((k_convert<T, double>), dim3(1024), dim3(256), 0, s, (int64_t)oTT[N], K.p, C64.p);
  TLS_LAUNCH_CHECK();
  K.release();
  GI.release();
  TG.release();
  GGt.release();
  DBuf<double> zv;
  PassEig e = run_subspace(c, d, dv, C64, zv, tau2);
  C64.release();
  // left singular directions: V = H v
  DBuf<T> wT;
  wT.alloc(std::max<int64_t>(oZv[N], 1));
  hipLaunchKernelGGL((k_convert<double, T>), dim3(1024), dim3(256), 0, s, (int64_t)oZv[N], zv.p, wT.p);
  TLS_LAUNCH_CHECK();
  std::vector<GemmDesc> gv;
  for (int i = 0; i < N; i++) {
    const int M = c->h_nt[i] * TS;
    if (e.kf[i] > 0) gv.push_back(GemmDesc{nI[i], e.kf[i], nT[i], M, nT[i], oXH[i], oZv[i], oXV[i], (int64_t)M});
  }
  batched_gemm<T>(s, gv, false, false, XH.p, wT.p, XV, T(1), T(0));
  TLS_HIP(hipStreamSynchronize(s));
  return e;
}

// Peak device bytes of subdomain i in a general pass: H (M x nT rounded up
// to whole tiles), the nT x nT Gram in T and FP64 with the subspace
// iteration's working copy, the G blocks, the subspace blocks and the
// singular vectors.
static int64_t general_pass_bytes(const PassDims& d, int i, int64_t M, int64_t tsz) {
  if (d.kreq[i] <= 0) return 0;
  const int64_t tt = (int64_t)d.nT[i] * d.nT[i], nG = d.nG[i];
  const int64_t nqH = (d.nT[i] + TS - 1) / TS;
  return M * TS * nqH * tsz + tt * (24 + tsz) + nG * (nG + d.nI[i] + d.nT[i]) * tsz +
         (d.oY[i + 1] - d.oY[i]) * 4 * 8 + (d.oZv[i + 1] - d.oZv[i]) * (8 + tsz);
}

// General A (Section 6): H = rows I of -A_{O'O'}^{-1} A_{O'T}; the dominant
// right singular vectors v of H from the Gram H^T H, coarse vectors H v.
// The passes run on groups of consecutive subdomains whose buffers fit in
// the memory budget (devmem::budget; one group when all fit).
template <class T>
static void basis_general(tls_ctx* c, T* fac) {
  hipStream_t s = c->stream;
  const int N = c->N;
  std::vector<int> nGv(N);
  for (int i = 0; i < N; i++) nGv[i] = c->h_nP[i] - c->h_nI[i];
  const PassDims d = pass_dims(c, nGv, c->nev, true);
  if (d.kmax == 0) {
    empty_basis(c);
    return;
  }
  std::vector<int64_t> oXV(N + 1, 0);
  for (int i = 0; i < N; i++) oXV[i + 1] = oXV[i] + (int64_t)c->h_nt[i] * TS * TS * (d.kreq[i] > 0 ? 1 : 0);
  DBuf<int64_t> d_oXV;
  d_oXV.upload(oXV, s);
  DBuf<T> XV;
  XV.alloc(std::max<int64_t>(oXV[N], 1));
  TLS_HIP(hipMemsetAsync(XV.p, 0, sizeof(T) * std::max<int64_t>(oXV[N], 1), s));
  // sigma^2 > tau^2 when a threshold is given
  const double tau2 = c->opt.tau > 0 ? c->opt.tau * c->opt.tau : -1.0;
  const int64_t budget = (int64_t)devmem::budget();
  std::vector<std::pair<int, int>> groups;
  int64_t acc = 0;
  for (int i = 0; i < N; i++) {
    const int64_t b = general_pass_bytes(d, i, (int64_t)c->h_nt[i] * TS, sizeof(T));
    if (groups.empty() || acc + b > budget) {
      groups.push_back({i, i});
      acc = 0;
    }
    groups.back().second = i + 1;
    acc += b;
  }
  PassEig e;
  e.kf.assign(N, 0);
  e.theta.assign(std::max(d.oth[N], 1), 0.0);
  for (const auto& g : groups) {
    const PassDims dg = groups.size() == 1 ? d : pass_restrict(d, g.first, g.second);
    if (dg.kmax == 0) continue;
    const PassEig eg = general_pass<T>(c, fac, dg, tau2, oXV, XV.p);
    for (int i = g.first; i < g.second; i++) {
      e.kf[i] = eg.kf[i];
      for (int j = 0; j < eg.kf[i]; j++) e.theta[d.oth[i] + j] = eg.theta[dg.oth[i] + j];
    }
    e.resid_max = std::max(e.resid_max, eg.resid_max);
    e.iters_max = std::max(e.iters_max, eg.iters_max);
    e.iters_sum += eg.iters_sum;
    e.n_solved += eg.n_solved;
  }
  c->eig_resid_max = e.resid_max;
  c->eig_iters_max = e.iters_max;
  c->eig_iters_mean = e.iters_sum / std::max(1, e.n_solved);
  // the reported value of a column is sigma = sqrt(eigenvalue of H^T H)
  std::vector<double> colval;
  std::vector<int> colsrc;
  std::vector<int64_t> coff(N + 1, 0);
  for (int i = 0; i < N; i++) {
    for (int j = 0; j < e.kf[i]; j++) {
      colval.push_back(std::sqrt(std::max(e.theta[d.oth[i] + j], 0.0)));
      colsrc.push_back(2);
    }
    coff[i + 1] = colval.size();
  }
  finish_basis<T>(c, e.kf, colval, colsrc, coff, d_oXV, 0, XV.p);
}

void build_coarse_basis(tls_ctx* c) {
  if ((c->nev == 0 && c->opt.nev1 == 0) || c->delta == 0) {
    empty_basis(c);
    return;
  }
  if (c->kind == 1) {
    if (c->fp32)
      basis_general<float>(c, c->fac32.p);
    else
      basis_general<double>(c, c->fac64.p);
  } else {
    if (c->fp32)
      basis_spd<float>(c, c->fac32.p);
    else
      basis_spd<double>(c, c->fac64.p);
  }
}

}  // namespace tls
