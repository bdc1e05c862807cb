// The two-level preconditioner on the stream, Q = R_0^T A_00^{-1} R_0.
//
// Additive composition (Remark in Section 4.3, the operator M_2^{-1}):
//   z = sum_i R_i^T A_ii^{-1} R_i r + Q r
//   1. gather R_i r into the padded local vectors (cast to the local
//      precision, Jacobi-scaled if enabled); R_0 r = Z^T r and the coarse
//      solve run on a second stream meanwhile;
//   2. forward and backward local solves (persistent kernels);
//   3. z = sum over the owners of each row (fixed order, no atomics)
//      + Z y0 on the rows I_i.
//
// Restricted composition with deflated coarse correction (Section 7.2,
// eq. onelevelras): z = Q r + M_RAS^{-1} (r - A Q r)
//   1. y0 = A_00^{-1} Z^T r; t = Z y0; u = r - A t (one SpMV);
//   2. gather R_i u, local solves;
//   3. z = t + the value of each row's own subdomain (D_i keeps row g only
//      in the subdomain whose I_i holds it): a plain write, no sum.
#include "kernels.hpp"

namespace tls {

namespace {

template <class T>
__global__ void k_apply_gather(int total, const int* __restrict__ sub_idx, const int* __restrict__ sub_of_pos,
                               const int* __restrict__ sub_ptr, const int64_t* __restrict__ voff,
                               const double* __restrict__ scale, const double* __restrict__ r, T* xloc,
                               double* b64, const int* __restrict__ done) {
  if (*done) return;
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  int i = sub_of_pos[p];
  int64_t pos = voff[i] + (p - sub_ptr[i]);
  double v = r[sub_idx[p]];
  if (scale) v *= scale[pos];
  xloc[pos] = (T)v;
  if (b64) b64[pos] = v;  // FP64 right-hand side of the refinement steps
}

template <class T>
__global__ void k_apply_scatter(int n, const int* __restrict__ own_ptr, const int64_t* __restrict__ own_pos,
                                const T* __restrict__ xloc, const double* __restrict__ scale,
                                const int* __restrict__ part, const int* __restrict__ ipos,
                                const int* __restrict__ nI, const int* __restrict__ kz,
                                const int* __restrict__ zcol, const int64_t* __restrict__ zoff,
                                const double* __restrict__ Z, const double* __restrict__ y0, double* z,
                                const int* __restrict__ done) {
  if (*done) return;
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  double s = 0.0;
  for (int e = own_ptr[g]; e < own_ptr[g + 1]; e++) {
    int64_t pos = own_pos[e];
    double v = (double)xloc[pos];
    if (scale) v *= scale[pos];
    s += v;
  }
  if (y0) {
    int p = part[g];
    int k = kz[p];
    const double* zp = Z + zoff[p] + ipos[g];
    const double* yp = y0 + zcol[p];
    const int ld = nI[p];
    for (int a = 0; a < k; a++) s += zp[(int64_t)a * ld] * yp[a];
  }
  z[g] = s;
}

// t = Z y0: row g of the block of its own subdomain
__global__ void k_coarse_prolong(int n, const int* __restrict__ part, const int* __restrict__ ipos,
                                 const int* __restrict__ nI, const int* __restrict__ kz, const int* __restrict__ zcol,
                                 const int64_t* __restrict__ zoff, const double* __restrict__ Z,
                                 const double* __restrict__ y0, double* t, const int* __restrict__ done) {
  if (*done) return;
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int p = part[g];
  const int k = kz[p];
  const double* zp = Z + zoff[p] + ipos[g];
  const double* yp = y0 + zcol[p];
  const int ld = nI[p];
  double s = 0.0;
  for (int a = 0; a < k; a++) s += zp[(int64_t)a * ld] * yp[a];
  t[g] = s;
}

// z[g] = t[g] + x_p[position of g in Omega_p], p = part[g]; I_p comes first
// in Omega_p, so that position is ipos[g]
template <class T>
__global__ void k_apply_scatter_ras(int n, const int* __restrict__ part, const int* __restrict__ ipos,
                                    const int64_t* __restrict__ voff, const T* __restrict__ xloc,
                                    const double* __restrict__ scale, const double* __restrict__ t, double* z,
                                    const int* __restrict__ done) {
  if (*done) return;
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int64_t pos = voff[part[g]] + ipos[g];
  double v = (double)xloc[pos];
  if (scale) v *= scale[pos];
  z[g] = t ? t[g] + v : v;
}

template <class T>
void apply_impl(tls_ctx* c, const double* r, double* z, const int* done, T* xloc, bool profile) {
  hipStream_t s = c->stream;
  if (profile) {
    for (auto& e : c->prof_ev)
      if (!e) TLS_HIP(hipEventCreate(&e));
    TLS_HIP(hipEventRecord(c->prof_ev[0], s));
  }
  const int total = c->h_sub_ptr[c->N];
  const double* scale = c->opt.jacobi_scale ? c->scale.p : nullptr;
  double* b64 = c->refine > 0 ? c->bref64.p : nullptr;
  if (c->opt.composition == 1) {
    const bool coarse = c->nC > 0;
    const double* rl = r;
    if (coarse) {
      coarse_restrict(c, r, done);
      coarse_solve(c, done);
      hipLaunchKernelGGL(k_coarse_prolong, dim3(div_up(c->n, 256)), dim3(256), 0, s, c->n, c->part.p, c->ipos.p,
                         c->d_nI.p, c->kz_dev.p, c->zcol.p, c->zoff.p, c->Z.p, c->y0.p, c->ras_t.p, done);
      TLS_LAUNCH_CHECK();
      spmv_residual(c, r, c->ras_t.p, c->ras_u.p, done);
      rl = c->ras_u.p;
    }
    hipLaunchKernelGGL(k_apply_gather<T>, dim3(div_up(total, 256)), dim3(256), 0, s, total, c->sub_idx.p,
                       c->sub_of_pos.p, c->sub_ptr.p, c->d_voff.p, scale, rl, xloc, b64, done);
    TLS_LAUNCH_CHECK();
    const bool refined = local_solve_refined(c, done, profile ? c->prof_ev[1] : nullptr,
                                             profile ? c->prof_ev[4] : nullptr, profile ? c->prof_ev[2] : nullptr);
    if (refined)
      hipLaunchKernelGGL(k_apply_scatter_ras<double>, dim3(div_up(c->n, 256)), dim3(256), 0, s, c->n, c->part.p,
                         c->ipos.p, c->d_voff.p, c->xref64.p, scale, coarse ? c->ras_t.p : nullptr, z, done);
    else
      hipLaunchKernelGGL(k_apply_scatter_ras<T>, dim3(div_up(c->n, 256)), dim3(256), 0, s, c->n, c->part.p,
                         c->ipos.p, c->d_voff.p, xloc, scale, coarse ? c->ras_t.p : nullptr, z, done);
    TLS_LAUNCH_CHECK();
  } else {
    hipLaunchKernelGGL(k_apply_gather<T>, dim3(div_up(total, 256)), dim3(256), 0, s, total, c->sub_idx.p,
                       c->sub_of_pos.p, c->sub_ptr.p, c->d_voff.p, scale, r, xloc, b64, done);
    TLS_LAUNCH_CHECK();
    const bool coarse = c->nC > 0;
    if (coarse) {
      // the coarse restriction and solve run on a second stream, overlapped
      // with the local solves; joined before the final scatter
      TLS_HIP(hipEventRecord(c->ev_fork, s));
      TLS_HIP(hipStreamWaitEvent(c->stream2, c->ev_fork, 0));
      hipStream_t keep = c->stream;
      c->stream = c->stream2;
      coarse_restrict(c, r, done);
      coarse_solve(c, done);
      c->stream = keep;
      TLS_HIP(hipEventRecord(c->ev_join, c->stream2));
    }
    const bool refined = local_solve_refined(c, done, profile ? c->prof_ev[1] : nullptr,
                                             profile ? c->prof_ev[4] : nullptr, profile ? c->prof_ev[2] : nullptr);
    if (coarse) TLS_HIP(hipStreamWaitEvent(s, c->ev_join, 0));
    if (refined)
      hipLaunchKernelGGL(k_apply_scatter<double>, dim3(div_up(c->n, 256)), dim3(256), 0, s, c->n, c->own_ptr.p,
                         c->own_pos.p, c->xref64.p, scale, c->part.p, c->ipos.p, c->d_nI.p,
                         coarse ? c->kz_dev.p : nullptr, c->zcol.p, c->zoff.p, c->Z.p, coarse ? c->y0.p : nullptr, z,
                         done);
    else
      hipLaunchKernelGGL(k_apply_scatter<T>, dim3(div_up(c->n, 256)), dim3(256), 0, s, c->n, c->own_ptr.p,
                         c->own_pos.p, xloc, scale, c->part.p, c->ipos.p, c->d_nI.p, coarse ? c->kz_dev.p : nullptr,
                         c->zcol.p, c->zoff.p, c->Z.p, coarse ? c->y0.p : nullptr, z, done);
    TLS_LAUNCH_CHECK();
  }
  if (profile) {
    TLS_HIP(hipEventRecord(c->prof_ev[3], s));
    TLS_HIP(hipEventSynchronize(c->prof_ev[3]));
    float t_local = 0.f, t_fwd = 0.f, t_all = 0.f;
    TLS_HIP(hipEventElapsedTime(&t_local, c->prof_ev[1], c->prof_ev[2]));
    TLS_HIP(hipEventElapsedTime(&t_fwd, c->prof_ev[1], c->prof_ev[4]));
    TLS_HIP(hipEventElapsedTime(&t_all, c->prof_ev[0], c->prof_ev[3]));
    c->prof_local_ms += t_local;
    c->prof_fwd_ms += t_fwd;
    c->prof_apply_ms += t_all;
    c->prof_count++;
  }
}

}  // namespace

void apply_precond(tls_ctx* c, const double* r, double* z, const int* done, bool profile) {
  if (c->fp32)
    apply_impl<float>(c, r, z, done, c->xloc32.p, profile);
  else
    apply_impl<double>(c, r, z, done, c->xloc64.p, profile);
}

}  // namespace tls
