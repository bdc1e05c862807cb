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
struct GemmPad;
template <>
struct GemmPad<float> {
  static constexpr int v = 16;
};
template <>
struct GemmPad<double> {
  static constexpr int v = 0;
};

// One 64x64 tile of C per 256-thread workgroup; K in chunks of 16.
template <class T, bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm(const GemmDesc* __restrict__ desc, const int64_t* __restrict__ pref,
                                              int nd, const T* __restrict__ A, const T* __restrict__ B, T* C,
                                              T alpha, T beta) {
  constexpr int KC = 16;
  constexpr int LD = 64 + GemmPad<T>::v;
  __shared__ T As[KC * LD];
  __shared__ T Bs[KC * LD];
  const int64_t bid = blockIdx.x;
  const int di = find_desc(pref, nd, bid);
  const GemmDesc g = desc[di];
  const int64_t t = bid - pref[di];
  const int tm = (g.M + 63) / 64;
  const int bm = (int)(t % tm) * 64, bn = (int)(t / tm) * 64;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) acc[x][y] = Mfma<T>::zero();
  for (int k0 = 0; k0 < g.K; k0 += KC) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      int e = tid + 256 * q;
      int m, k;
      if (!TA) {
        m = e & 63;
        k = e >> 6;
      } else {
        k = e & 15;
        m = e >> 4;
      }
      int gm = bm + m, gk = k0 + k;
      T v = T(0);
      if (gm < g.M && gk < g.K)
        v = TA ? A[g.a_off + gk + (int64_t)gm * g.lda] : A[g.a_off + gm + (int64_t)gk * g.lda];
      As[k * LD + m] = v;
      int n2, k2;
      if (!TB) {
        k2 = e & 15;
        n2 = e >> 4;
      } else {
        n2 = e & 63;
        k2 = e >> 6;
      }
      int gn = bn + n2, gk2 = k0 + k2;
      T w = T(0);
      if (gn < g.N && gk2 < g.K)
        w = TB ? B[g.b_off + gn + (int64_t)gk2 * g.ldb] : B[g.b_off + gk2 + (int64_t)gn * g.ldb];
      Bs[k2 * LD + n2] = w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      T a0 = As[(kk + lk) * LD + wr + li];
      T a1 = As[(kk + lk) * LD + wr + 16 + li];
      T b0 = Bs[(kk + lk) * LD + wc + li];
      T b1 = Bs[(kk + lk) * LD + wc + 16 + li];
      acc[0][0] = Mfma<T>::mac(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<T>::mac(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<T>::mac(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<T>::mac(a1, b1, acc[1][1]);
    }
    __syncthreads();
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

// One workgroup per (descriptor, group of RC right-hand sides); the group
// lives in LDS (dynamic, n * RC elements).
template <class T>
__global__ void __launch_bounds__(256) k_trsm_batched(const TriDesc* __restrict__ desc, const int64_t* __restrict__ pref,
                                                      int nd, int RC, int mode, const T* __restrict__ Mat, T* Bm,
                                                      int* err) {
  extern __shared__ unsigned char smem_raw[];
  T* Bs = reinterpret_cast<T*>(smem_raw);
  const int64_t bid = blockIdx.x;
  const int di = find_desc(pref, nd, bid);
  const TriDesc d = desc[di];
  const int g0 = (int)(bid - pref[di]) * RC;
  const int nc = min(RC, d.nrhs - g0);
  const int n = d.n;
  const T* M = Mat + d.m_off;
  T* B = Bm + d.b_off + (int64_t)g0 * d.ldb;
  const int tid = threadIdx.x;
  for (int e = tid; e < n * nc; e += 256) {
    int r = e % n, cc = e / n;
    Bs[r * RC + cc] = B[r + (int64_t)cc * d.ldb];
  }
  const int col = tid % RC, rslot = tid / RC, rstride = 256 / RC;
  bool bad = false;
  for (int s = 0; s < n; s++) {
    const int b = mode == LOWER_FWD ? s : n - 1 - s;
    __syncthreads();
    if (rslot == 0 && col < nc) {
      T dg = M[b + (int64_t)b * n];
      if (!(dg != T(0))) {
        bad = true;
        dg = T(1);
      }
      Bs[b * RC + col] /= dg;
    }
    __syncthreads();
    if (col < nc && rslot < rstride) {
      T xb = Bs[b * RC + col];
      if (mode == LOWER_FWD) {
        for (int a = b + 1 + rslot; a < n; a += rstride) Bs[a * RC + col] -= M[a + (int64_t)b * n] * xb;
      } else {
        for (int a = rslot; a < b; a += rstride) Bs[a * RC + col] -= M[a + (int64_t)b * n] * xb;
      }
    }
  }
  __syncthreads();
  if (bad) atomicOr(err, ERR_PIVOT);
  for (int e = tid; e < n * nc; e += 256) {
    int r = e % n, cc = e / n;
    B[r + (int64_t)cc * d.ldb] = Bs[r * RC + cc];
  }
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

template <class T>
void batched_trsm(hipStream_t s, const std::vector<TriDesc>& d, TriMode mode, const T* M, T* B, int* err) {
  int nmax = 0;
  for (const auto& t : d)
    if (t.nrhs > 0) nmax = std::max(nmax, t.n);
  if (nmax == 0) return;
  const int lds_cap = 64 * 1024;
  int RC = std::min<int64_t>(16, lds_cap / ((int64_t)nmax * sizeof(T)));
  if (RC < 1) fail(TLS_E_ARG, "local block too large for the batched triangular solve (" + std::to_string(nmax) + ")");
  // power of two dividing 256
  int rc = 1;
  while (rc * 2 <= RC) rc *= 2;
  RC = rc;
  std::vector<TriDesc> dd;
  std::vector<int64_t> pref;
  int64_t tot = 0;
  for (const auto& t : d) {
    if (t.nrhs <= 0 || t.n <= 0) continue;
    dd.push_back(t);
    pref.push_back(tot);
    tot += (t.nrhs + RC - 1) / RC;
  }
  if (tot == 0) return;
  pref.push_back(tot);
  DBuf<TriDesc> ddesc;
  DBuf<int64_t> dpref;
  ddesc.upload(dd, s);
  dpref.upload(pref, s);
  size_t shm = (size_t)nmax * RC * sizeof(T);
  hipLaunchKernelGGL(k_trsm_batched<T>, dim3((unsigned)tot), dim3(256), shm, s, ddesc.p, dpref.p, (int)dd.size(), RC,
                     (int)mode, M, B, err);
  TLS_LAUNCH_CHECK();
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
