// Iterative refinement of the local solves (option local_refine, FP32 mode).
//
// With FP32 local factors (or explicit inverses), x_i = A_ii^{-1} b_i of
// eq. onelevelasm carries a forward error of order cond(A_ii) u_32. One
// refinement step computes the residual b_i - A_ii x_i in FP64 with the
// sparse rows of A_ii = R_i A R_i^T (the entries of A whose row and column
// both lie in Omega_i, Section 2.3), solves for the correction with the
// same FP32 factor and adds it in FP64, so the error contracts by the
// factor rho(I - F_32 A_ii), F_32 the FP32 solve, at each step (mixed-
// precision iterative refinement). The refined local solutions are held in
// an FP64 padded vector that the apply's scatter reads.
//
// The local CSR is indexed by the position p of a row in the concatenated
// Omega lists; its columns are local indices b in [0, #Omega_i), so the
// padded address of a column is voff_i + b. With Jacobi scaling the stored
// values are s_a A_ab s_b, the matrix that was factored.
#include <algorithm>

#include "kernels.hpp"
#include "scan.hpp"

namespace tls {

namespace {

// mode 0: count the entries of row p of A_ii; mode 1: write them
__global__ void k_lref_rows(int mode, int total, const int* __restrict__ sub_idx, const int* __restrict__ sub_of_pos,
                            const int* __restrict__ sub_ptr, const int* __restrict__ layer_ptr, int stride, int nseg,
                            const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ val,
                            const double* __restrict__ scale, const int64_t* __restrict__ voff, int* cnt,
                            const int* __restrict__ lptr, int* lcol, double* lval) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  const int i = sub_of_pos[p];
  const int g = sub_idx[p];
  const int* lp = layer_ptr + (size_t)i * stride;
  const int p0 = sub_ptr[i];
  const double sa = scale ? scale[voff[i] + (p - p0)] : 1.0;
  int k = 0;
  const int base = mode ? lptr[p] : 0;
  for (int j = rp[g]; j < rp[g + 1]; j++) {
    const int q = find_local_pos(ci[j], sub_idx, lp, nseg);
    if (q < 0) continue;
    if (mode) {
      const int b = q - p0;
      lcol[base + k] = b;
      lval[base + k] = scale ? val[j] * sa * scale[voff[i] + b] : val[j];
    }
    k++;
  }
  if (!mode) cnt[p] = k;
}

// x64 = (first ? 0 : x64) + x at every real position of every subdomain
template <class T>
__global__ void k_refine_acc(int total, const int* __restrict__ sub_of_pos, const int* __restrict__ sub_ptr,
                             const int64_t* __restrict__ voff, const T* __restrict__ x, double* x64, int first,
                             const int* __restrict__ done) {
  if (*done) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  const int i = sub_of_pos[p];
  const int64_t pos = voff[i] + (p - sub_ptr[i]);
  const double v = (double)x[pos];
  x64[pos] = first ? v : x64[pos] + v;
}

// x = b64 - A_ii x64 (FP64 arithmetic), rounded to the local precision
template <class T>
__global__ void k_refine_res(int total, const int* __restrict__ sub_of_pos, const int* __restrict__ sub_ptr,
                             const int64_t* __restrict__ voff, const int* __restrict__ lptr,
                             const int* __restrict__ lcol, const double* __restrict__ lval,
                             const double* __restrict__ b64, const double* __restrict__ x64, T* x,
                             const int* __restrict__ done) {
  if (*done) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  const int i = sub_of_pos[p];
  const int64_t o = voff[i];
  const int64_t pos = o + (p - sub_ptr[i]);
  double s = b64[pos];
  for (int j = lptr[p]; j < lptr[p + 1]; j++) s -= lval[j] * x64[o + lcol[j]];
  x[pos] = (T)s;
}

}  // namespace

void build_refine(tls_ctx* c) {
  c->refine = 0;
  if (!c->fp32 || c->opt.local_refine <= 0) return;
  hipStream_t s = c->stream;
  const int total = c->h_sub_ptr[c->N];
  const int stride = c->delta + 2, nseg = c->delta + 1;
  const double* scale = c->opt.jacobi_scale ? c->scale.p : nullptr;
  DBuf<int> cnt;
  cnt.alloc((size_t)total + 1);
  const dim3 g(div_up(total, 256));
  hipLaunchKernelGGL(k_lref_rows, g, dim3(256), 0, s, 0, total, c->sub_idx.p, c->sub_of_pos.p, c->sub_ptr.p,
                     c->layer_ptr.p, stride, nseg, c->row_ptr.p, c->col_idx.p, c->val.p, scale, c->d_voff.p, cnt.p,
                     nullptr, nullptr, nullptr);
  TLS_LAUNCH_CHECK();
  TLS_HIP(hipMemsetAsync(cnt.p + total, 0, sizeof(int), s));
  c->lref_ptr.alloc((size_t)total + 1);
  scan_exclusive_i32(cnt.p, c->lref_ptr.p, total + 1, s);
  int nnz = 0;
  TLS_HIP(hipMemcpyAsync(&nnz, c->lref_ptr.p + total, sizeof(int), hipMemcpyDeviceToHost, s));
  TLS_HIP(hipStreamSynchronize(s));
  c->lref_col.alloc(std::max(nnz, 1));
  c->lref_val.alloc(std::max(nnz, 1));
  hipLaunchKernelGGL(k_lref_rows, g, dim3(256), 0, s, 1, total, c->sub_idx.p, c->sub_of_pos.p, c->sub_ptr.p,
                     c->layer_ptr.p, stride, nseg, c->row_ptr.p, c->col_idx.p, c->val.p, scale, c->d_voff.p, nullptr,
                     c->lref_ptr.p, c->lref_col.p, c->lref_val.p);
  TLS_LAUNCH_CHECK();
  c->xref64.alloc(c->sum_M);
  c->bref64.alloc(c->sum_M);
  TLS_HIP(hipMemsetAsync(c->xref64.p, 0, sizeof(double) * c->sum_M, s));
  TLS_HIP(hipMemsetAsync(c->bref64.p, 0, sizeof(double) * c->sum_M, s));
  TLS_HIP(hipStreamSynchronize(s));
  c->refine = std::min(c->opt.local_refine, 8);
}

bool local_solve_refined(tls_ctx* c, const int* done, hipEvent_t ev_begin, hipEvent_t ev_mid, hipEvent_t ev_end) {
  local_solve(c, done, ev_begin, ev_mid, ev_end);
  if (c->refine <= 0) return false;
  hipStream_t s = c->stream;
  const int total = c->h_sub_ptr[c->N];
  const dim3 g(div_up(total, 256));
  float* x = c->xloc32.p;
  for (int step = 0; step < c->refine; step++) {
    hipLaunchKernelGGL(k_refine_acc<float>, g, dim3(256), 0, s, total, c->sub_of_pos.p, c->sub_ptr.p, c->d_voff.p, x,
                       c->xref64.p, step == 0 ? 1 : 0, done);
    hipLaunchKernelGGL(k_refine_res<float>, g, dim3(256), 0, s, total, c->sub_of_pos.p, c->sub_ptr.p, c->d_voff.p,
                       c->lref_ptr.p, c->lref_col.p, c->lref_val.p, c->bref64.p, c->xref64.p, x, done);
    TLS_LAUNCH_CHECK();
    local_solve(c, done);
  }
  hipLaunchKernelGGL(k_refine_acc<float>, g, dim3(256), 0, s, total, c->sub_of_pos.p, c->sub_ptr.p, c->d_voff.p, x,
                     c->xref64.p, 0, done);
  TLS_LAUNCH_CHECK();
  return true;
}

}  // namespace tls
