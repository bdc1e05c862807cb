// Batched variable-size MFMA GEMM and many-RHS triangular solves.
#include <algorithm>

#include "batched.hpp"
#include "mfma.hpp"

namespace tls {

namespace {

__device__ inline int find_desc(const int64_t* pref, int count, int64_t bid) {
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

template <class T>
struct GemmPadK;
// k-fastest pitch KC + pad: LDS has 32 four-byte banks, 32-bit reads are
// served per half wave and 64-bit reads per 16 lanes; 34 (= 2 mod 32) and
// the odd 33 keep those on distinct banks
template <>
struct GemmPadK<float> {
  static constexpr int v = 2;
};
template <>
struct GemmPadK<double> {
  static constexpr int v = 1;
};

// One 64x64 tile of C per 256-thread workgroup; K in chunks of KC = 32, the
// next chunk loaded into registers while the current one is used. An
// operand whose consecutive elements in memory run along m (or n) is staged
// m-fastest ([k][m], pitch PM); one whose elements run along k is staged
// k-fastest ([m][k], pitch PK). Either way the LDS stores and the MFMA reads
// fall on distinct banks. C may be B's storage when
// M <= 64: each workgroup reads all of K before it writes its tile.
template <class T, bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm(const GemmDesc* __restrict__ desc, const int64_t* __restrict__ pref,
                                              int nd, const T* __restrict__ A, const T* __restrict__ B, T* C,
                                              T alpha, T beta) {
  constexpr int KC = 32;
  constexpr int PM = 64 + 16;
  constexpr int PK = KC + GemmPadK<T>::v;
  constexpr int PER = 64 * KC / 256;  // elements of each operand per thread and chunk
  __shared__ T As[TA ? 64 * PK : KC * PM];
  __shared__ T Bs[TB ? KC * PM : 64 * PK];
  const int64_t bid = blockIdx.x;
  const int di = find_desc(pref, nd, bid);
  const GemmDesc g = desc[di];
  const int64_t t = bid - pref[di];
  const int tm = (g.M + 63) / 64;
  const int bm = (int)(t % tm) * 64, bn = (int)(t / tm) * 64;
  if (g.syrk && bn > bm) return;  // above the block diagonal of a symmetric C
  const int kbeg = g.kstart ? max(g.kstart[bm / 64], g.kstart[bn / 64]) / KC * KC : 0;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) acc[x][y] = Mfma<T>::zero();
  T ra[PER], rb[PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PER; q++) {
      const int e = tid + 256 * q;
      int m, k;
      if (!TA) {
        m = e & 63;
        k = e >> 6;
      } else {
        k = e & (KC - 1);
        m = e / KC;
      }
      const int gm = bm + m, gk = k0 + k;
      T v = T(0);
      if (gm < g.M && gk < g.K)
        v = TA ? A[g.a_off + gk + (int64_t)gm * g.lda] : A[g.a_off + gm + (int64_t)gk * g.lda];
      ra[q] = v;
      int n2, k2;
      if (!TB) {
        k2 = e & (KC - 1);
        n2 = e / KC;
      } else {
        n2 = e & 63;
        k2 = e >> 6;
      }
      const int gn = bn + n2, gk2 = k0 + k2;
      T w = T(0);
      if (gn < g.N && gk2 < g.K)
        w = TB ? B[g.b_off + gn + (int64_t)gk2 * g.ldb] : B[g.b_off + gk2 + (int64_t)gn * g.ldb];
      rb[q] = w;
    }
  };
  load(kbeg);
  for (int k0 = kbeg; k0 < g.K; k0 += KC) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; q++) {
      const int e = tid + 256 * q;
      if (!TA)
        As[(e >> 6) * PM + (e & 63)] = ra[q];
      else
        As[(e / KC) * PK + (e & (KC - 1))] = ra[q];
      if (!TB)
        Bs[(e / KC) * PK + (e & (KC - 1))] = rb[q];
      else
        Bs[(e >> 6) * PM + (e & 63)] = rb[q];
    }
    __syncthreads();
    if (k0 + KC < g.K) load(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      T a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; x++)
        a[x] = TA ? As[(wr + 16 * x + li) * PK + kk + lk] : As[(kk + lk) * PM + wr + 16 * x + li];
#pragma unroll
      for (int y = 0; y < 2; y++)
        b[y] = TB ? Bs[(kk + lk) * PM + wc + 16 * y + li] : Bs[(wc + 16 * y + li) * PK + kk + lk];
      acc[0][0] = Mfma<T>::mac(a[0], b[0], acc[0][0]);
      acc[0][1] = Mfma<T>::mac(a[0], b[1], acc[0][1]);
      acc[1][0] = Mfma<T>::mac(a[1], b[0], acc[1][0]);
      acc[1][1] = Mfma<T>::mac(a[1], b[1], acc[1][1]);
    }
  }
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      int col = bn + wc + 16 * y + li;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        int row = bm + wr + 16 * x + Mfma<T>::row(lane, q);
        if (row < g.M && col < g.N) {
          T* p = C + g.c_off + row + (int64_t)col * g.ldc;
          T v = alpha * acc[x][y][q];
          if (beta != T(0)) v += beta * (*p);
          *p = v;
        }
      }
    }
}

// Inverse of one diagonal block (w x w, w <= 64) of a column-major
// triangular matrix per 64-thread workgroup, in FP64; thread j computes
// column j. Output: 64 x 64 column-major (rows/columns >= w unused).
template <class T>
__global__ void __launch_bounds__(64) k_tri_inv(const TriDesc* __restrict__ desc, const int2* __restrict__ blk,
                                                const int64_t* __restrict__ ioff, int mode, const T* __restrict__ Mat,
                                                T* inv, int* err) {
  constexpr int L1 = 65;
  __shared__ double Ls[64 * L1];
  const int2 bb = blk[blockIdx.x];
  const TriDesc d = desc[bb.x];
  const int k0 = 64 * bb.y;
  const int w = min(64, d.n - k0);
  const T* M = Mat + d.m_off + k0 + (int64_t)k0 * d.n;
  const int j = threadIdx.x;
  for (int e = j; e < w * w; e += 64) {
    const int a = e % w, c = e / w;
    Ls[a + c * L1] = (double)M[a + (int64_t)c * d.n];
  }
  __syncthreads();
  T* out = inv + ioff[blockIdx.x];
  double x[64];
  bool bad = false;
  if (mode == LOWER_FWD) {
#pragma unroll
    for (int a = 0; a < 64; a++) {
      double v = (a == j) ? 1.0 : 0.0;
#pragma unroll
      for (int b = 0; b < a; b++) v -= Ls[a + b * L1] * x[b];
      double dg = a < w ? Ls[a + a * L1] : 1.0;
      if (a < w && !(dg != 0.0)) {
        bad = true;
        dg = 1.0;
      }
      x[a] = (a < j || a >= w || j >= w) ? 0.0 : v / dg;
    }
  } else {
#pragma unroll
    for (int a = 63; a >= 0; a--) {
      double v = (a == j) ? 1.0 : 0.0;
#pragma unroll
      for (int b = a + 1; b < 64; b++) v -= Ls[a + b * L1] * x[b];
      double dg = a < w ? Ls[a + a * L1] : 1.0;
      if (a < w && !(dg != 0.0)) {
        bad = true;
        dg = 1.0;
      }
      x[a] = (a > j || a >= w || j >= w) ? 0.0 : v / dg;
    }
  }
#pragma unroll
  for (int a = 0; a < 64; a++) out[a + 64 * j] = (T)x[a];
  if (bad) atomicOr(err, ERR_PIVOT);
}

}  // namespace

template <class T>
void batched_gemm(hipStream_t s, const std::vector<GemmDesc>& d, bool transA, bool transB, const T* A, const T* B,
                  T* C, T alpha, T beta) {
  std::vector<GemmDesc> dd;
  std::vector<int64_t> pref;
  int64_t tot = 0;
  for (const auto& g : d) {
    if (g.M <= 0 || g.N <= 0) continue;
    dd.push_back(g);
    pref.push_back(tot);
    tot += (int64_t)((g.M + 63) / 64) * ((g.N + 63) / 64);
  }
  if (tot == 0) return;
  pref.push_back(tot);
  DBuf<GemmDesc> ddesc;
  DBuf<int64_t> dpref;
  ddesc.upload(dd, s);
  dpref.upload(pref, s);
  const int nd = (int)dd.size();
  if (!transA && !transB)
    hipLaunchKernelGGL((k_gemm<T, false, false>), dim3((unsigned)tot), dim3(256), 0, s, ddesc.p, dpref.p, nd, A, B,
                       C, alpha, beta);
  else if (transA && !transB)
    hipLaunchKernelGGL((k_gemm<T, true, false>), dim3((unsigned)tot), dim3(256), 0, s, ddesc.p, dpref.p, nd, A, B,
                       C, alpha, beta);
  else if (!transA && transB)
    hipLaunchKernelGGL((k_gemm<T, false, true>), dim3((unsigned)tot), dim3(256), 0, s, ddesc.p, dpref.p, nd, A, B,
                       C, alpha, beta);
  else
    hipLaunchKernelGGL((k_gemm<T, true, true>), dim3((unsigned)tot), dim3(256), 0, s, ddesc.p, dpref.p, nd, A, B, C,
                       alpha, beta);
  TLS_LAUNCH_CHECK();
  TLS_HIP(hipStreamSynchronize(s));
}

void gemm_plan(GemmPlan& p, const std::vector<GemmDesc>& d, hipStream_t s) {
  std::vector<GemmDesc> dd;
  std::vector<int64_t> pref;
  int64_t tot = 0;
  for (const auto& g : d) {
    if (g.M <= 0 || g.N <= 0) continue;
    dd.push_back(g);
    pref.push_back(tot);
    tot += (int64_t)((g.M + 63) / 64) * ((g.N + 63) / 64);
  }
  pref.push_back(tot);
  if (p.desc.n < std::max<size_t>(dd.size(), 1)) p.desc.alloc(std::max<size_t>(dd.size(), 1));
  if (p.pref.n < pref.size()) p.pref.alloc(pref.size());
  if (!dd.empty()) TLS_HIP(hipMemcpyAsync(p.desc.p, dd.data(), sizeof(GemmDesc) * dd.size(), hipMemcpyHostToDevice, s));
  TLS_HIP(hipMemcpyAsync(p.pref.p, pref.data(), sizeof(int64_t) * pref.size(), hipMemcpyHostToDevice, s));
  TLS_HIP(hipStreamSynchronize(s));  // dd and pref are host temporaries
  p.nd = (int)dd.size();
  p.tiles = tot;
}

template <class T>
void gemm_run(hipStream_t s, const GemmPlan& p, bool transA, bool transB, const T* A, const T* B, T* C, T alpha,
              T beta) {
  if (p.tiles == 0) return;
  const dim3 g((unsigned)p.tiles);
  if (!transA && !transB)
    hipLaunchKernelGGL((k_gemm<T, false, false>), g, dim3(256), 0, s, p.desc.p, p.pref.p, p.nd, A, B, C, alpha, beta);
  else if (transA && !transB)
    hipLaunchKernelGGL((k_gemm<T, true, false>), g, dim3(256), 0, s, p.desc.p, p.pref.p, p.nd, A, B, C, alpha, beta);
  else if (!transA && transB)
    hipLaunchKernelGGL((k_gemm<T, false, true>), g, dim3(256), 0, s, p.desc.p, p.pref.p, p.nd, A, B, C, alpha, beta);
  else
    hipLaunchKernelGGL((k_gemm<T, true, true>), g, dim3(256), 0, s, p.desc.p, p.pref.p, p.nd, A, B, C, alpha, beta);
  TLS_LAUNCH_CHECK();
}

// Blocked triangular solve with many right-hand sides: the diagonal 64 x 64
// blocks are inverted once (k_tri_inv), then for each block row k (in the
// solve order) X_k = inv(M_kk) B_k and the rows still to solve get
// B -= M(:, k) X_k, both as batched MFMA GEMMs over all descriptors. The
// first GEMM writes X_k over B_k: it has a single 64-row output tile, so
// each workgroup reads all of its B columns before writing them.
template <class T>
void batched_trsm(hipStream_t s, const std::vector<TriDesc>& d, TriMode mode, const T* M, T* B, int* err) {
  std::vector<TriDesc> dd;
  for (const auto& t : d)
    if (t.nrhs > 0 && t.n > 0) dd.push_back(t);
  if (dd.empty()) return;
  std::vector<int2> blk;
  std::vector<int64_t> ioff;
  std::vector<int64_t> first(dd.size());
  int maxnb = 0;
  for (size_t q = 0; q < dd.size(); q++) {
    const int nb = (dd[q].n + 63) / 64;
    maxnb = std::max(maxnb, nb);
    first[q] = (int64_t)blk.size();
    for (int b = 0; b < nb; b++) {
      blk.push_back(make_int2((int)q, b));
      ioff.push_back((int64_t)(blk.size() - 1) * 4096);
    }
  }
  DBuf<TriDesc> ddesc;
  DBuf<int2> dblk;
  DBuf<int64_t> dioff;
  DBuf<T> inv;
  ddesc.upload(dd, s);
  dblk.upload(blk, s);
  dioff.upload(ioff, s);
  inv.alloc(blk.size() * 4096);
  hipLaunchKernelGGL(k_tri_inv<T>, dim3((unsigned)blk.size()), dim3(64), 0, s, ddesc.p, dblk.p, dioff.p, (int)mode, M,
                     inv.p, err);
  TLS_LAUNCH_CHECK();
  // inv and M are separate buffers: the GEMMs read the inverse blocks from
  // inv (A operand, offset into inv) and the off-diagonal blocks from M.
  // The block rows are taken in panels of PW: inside a panel each solved
  // block updates only the panel's rows still to solve; when the panel is
  // done, one GEMM with K = the panel's rows updates every row outside it,
  // so the right-hand sides are read and written once per panel instead of
  // once per block row.
  constexpr int PW = 8;
  GemmPlan p1, p2, p3;
  for (int step = 0; step < maxnb; step++) {
    std::vector<GemmDesc> g1, g2, g3;
    for (size_t q = 0; q < dd.size(); q++) {
      const TriDesc& t = dd[q];
      const int nb = (t.n + 63) / 64;
      if (step >= nb) continue;
      const int k = mode == LOWER_FWD ? step : nb - 1 - step;
      const int k0 = 64 * k, w = std::min(64, t.n - k0);
      // rows of this step's panel: steps [ps0, ps1) of the solve order
      const int ps0 = step / PW * PW, ps1 = std::min(ps0 + PW, nb);
      const int pr0 = mode == LOWER_FWD ? 64 * ps0 : 64 * (nb - ps1);
      const int pr1 = mode == LOWER_FWD ? std::min(t.n, 64 * ps1) : std::min(t.n, 64 * (nb - ps0));
      // X_k = inv(M_kk) B_k, written over B_k
      g1.push_back(GemmDesc{w, t.nrhs, w, 64, (int)t.ldb, (first[q] + k) * 4096, t.b_off + k0, t.b_off + k0, t.ldb});
      // the panel's rows still to solve: below (forward) or above (backward) the block
      const int r0 = mode == LOWER_FWD ? k0 + w : pr0;
      const int rn = mode == LOWER_FWD ? pr1 - k0 - w : k0 - pr0;
      if (rn > 0)
        g2.push_back(GemmDesc{rn, t.nrhs, w, t.n, (int)t.ldb, t.m_off + r0 + (int64_t)k0 * t.n, t.b_off + k0,
                              t.b_off + r0, t.ldb});
      // the panel is solved: the rows after it in the solve order
      if (step == ps1 - 1) {
        const int o0 = mode == LOWER_FWD ? pr1 : 0;
        const int on = mode == LOWER_FWD ? t.n - pr1 : pr0;
        if (on > 0)
          g3.push_back(GemmDesc{on, t.nrhs, pr1 - pr0, t.n, (int)t.ldb, t.m_off + o0 + (int64_t)pr0 * t.n,
                                t.b_off + pr0, t.b_off + o0, t.ldb});
      }
    }
    gemm_plan(p1, g1, s);
    gemm_run<T>(s, p1, false, false, inv.p, B, B, T(1), T(0));
    if (!g2.empty()) {
      gemm_plan(p2, g2, s);
      gemm_run<T>(s, p2, false, false, M, B, B, T(-1), T(1));
    }
    if (!g3.empty()) {
      gemm_plan(p3, g3, s);
      gemm_run<T>(s, p3, false, false, M, B, B, T(-1), T(1));
    }
  }
  TLS_HIP(hipStreamSynchronize(s));
}

template void batched_gemm<float>(hipStream_t, const std::vector<GemmDesc>&, bool, bool, const float*, const float*,
                                  float*, float, float);
template void batched_gemm<double>(hipStream_t, const std::vector<GemmDesc>&, bool, bool, const double*,
                                   const double*, double*, double, double);
template void gemm_run<float>(hipStream_t, const GemmPlan&, bool, bool, const float*, const float*, float*, float,
                              float);
template void gemm_run<double>(hipStream_t, const GemmPlan&, bool, bool, const double*, const double*, double*,
                               double, double);
template void batched_trsm<float>(hipStream_t, const std::vector<TriDesc>&, TriMode, const float*, float*, int*);
template void batched_trsm<double>(hipStream_t, const std::vector<TriDesc>&, TriMode, const double*, double*, int*);

}  // namespace tls
