// CSR SpMV and the outer Krylov solver (FP64): preconditioned conjugate
// gradients from x0 = 0, stopping on ||r_k|| <= tol ||b|| (the recurrence
// residual), then reporting the true residual ||b - A x|| / ||b||.
//
// Every scalar lives on the device; each kernel of an iteration returns at
// once when the device "done" flag is set, so a chunk of iterations can be
// enqueued (or replayed as a captured hipGraph) and the host reads the flag
// once per chunk. Dot products use a fixed grid and a fixed reduction tree,
// so results are bitwise reproducible.
#include <chrono>
#include <cmath>

#include "kernels.hpp"

namespace tls {

namespace {

constexpr int RED_BLOCKS = 512;

// y = A x, or y = f - A x when f is given; G lanes per row
template <int G>
__global__ void __launch_bounds__(256) k_spmv(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                              const double* __restrict__ val, const double* __restrict__ x,
                                              double* __restrict__ y, const int* __restrict__ done,
                                              const double* __restrict__ f) {
  if (*done) return;
  const int lane = threadIdx.x % G;
  const int row = blockIdx.x * (256 / G) + threadIdx.x / G;
  double s = 0.0;
  if (row < n) {
    const int b = rp[row + 1];
    for (int j = rp[row] + lane; j < b; j += G) s += val[j] * x[ci[j]];
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
  if (row < n && lane == 0) y[row] = f ? f[row] - s : s;
}

__device__ inline void block_reduce_store(double v, double* out) {
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}

// Dot products in one launch of RED_BLOCKS blocks: each block stores its
// partial sum; the last block to finish (counted in *ctr, which it resets)
// adds the partials in index order and stores the result, so the value
// does not depend on the order in which the blocks ran.
__device__ inline bool last_block(unsigned* ctr) {
  __shared__ bool s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();  // this block's partial is visible before it is counted
    s_last = atomicAdd(ctr, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (s_last) {
    __threadfence();  // every counted partial is visible to the last block
    if (threadIdx.x == 0) *ctr = 0u;
  }
  return s_last;
}

__device__ inline void sum_partials(const double* partial, double* out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < RED_BLOCKS; i += 256) s += partial[i];
  block_reduce_store(s, out);
}

__global__ void __launch_bounds__(256) k_dot(int n, const double* __restrict__ a, const double* __restrict__ b,
                                             double* partial, unsigned* ctr, double* out,
                                             const int* __restrict__ done) {
  if (*done) return;
  double s = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += RED_BLOCKS * 256) s += a[i] * b[i];
  block_reduce_store(s, partial + blockIdx.x);
  if (last_block(ctr)) sum_partials(partial, out);
}

// pq = p.q into scal[2]; a non-positive pq stops the iteration (breakdown)
__global__ void __launch_bounds__(256) k_dot_pq(int n, const double* __restrict__ p, const double* __restrict__ q,
                                                double* partial, unsigned* ctr, double* scal, int* done) {
  if (done[0]) return;
  double s = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += RED_BLOCKS * 256) s += p[i] * q[i];
  block_reduce_store(s, partial + blockIdx.x);
  if (last_block(ctr)) {
    sum_partials(partial, scal + 2);
    if (threadIdx.x == 0 && !(scal[2] > 0.0)) {
      done[0] = 1;
      done[3] = 1;
    }
  }
}

// alpha = rz / pq; x += alpha p; r -= alpha q; r.r into scal[3]; then the
// last block records ||r||/||b|| and stops on the tolerance or the cap
__global__ void __launch_bounds__(256) k_pcg_update(int n, double* __restrict__ x, double* __restrict__ r,
                                                    const double* __restrict__ p, const double* __restrict__ q,
                                                    double* scal, double* partial, unsigned* ctr, int* done,
                                                    double* hist, int maxit, double tol2) {
  if (done[0]) return;
  const double alpha = scal[1] / scal[2];
  double s = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += RED_BLOCKS * 256) {
    x[i] += alpha * p[i];
    double ri = r[i] - alpha * q[i];
    r[i] = ri;
    s += ri * ri;
  }
  block_reduce_store(s, partial + blockIdx.x);
  if (last_block(ctr)) {
    sum_partials(partial, scal + 3);
    if (threadIdx.x == 0) {
      const int it = ++done[1];
      const double rr = scal[3], bb = scal[0];
      hist[it - 1] = sqrt(rr / bb);
      if (rr <= tol2 * bb) {
        done[0] = 1;
        done[2] = 1;
      } else if (it >= maxit) {
        done[0] = 1;
      }
    }
  }
}

__global__ void k_copy(int n, const double* __restrict__ a, double* __restrict__ b, const int* __restrict__ done) {
  if (*done) return;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) b[i] = a[i];
}

// beta = (r.z - [r.zold]) / rz_prev ; p = z + beta p
__global__ void k_pcg_p(int n, double* __restrict__ p, const double* __restrict__ z, const double* __restrict__ scal,
                        int flexible, const int* __restrict__ done) {
  if (*done) return;
  const double beta = (scal[4] - (flexible ? scal[5] : 0.0)) / scal[1];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = z[i] + beta * p[i];
}

__global__ void k_pcg_shift(double* scal, const int* __restrict__ done) {
  if (*done) return;
  scal[1] = scal[4];
}

__global__ void k_sub(int n, const double* __restrict__ b, const double* __restrict__ q, double* __restrict__ r) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) r[i] = b[i] - q[i];
}

}  // namespace

bool take_wait_flag(tls_ctx* c) {
  int err = 0;
  read_back(c->errflag.p, &err, 1, c->stream);
  if (!(err & ERR_WAIT)) return false;
  TLS_HIP(hipMemsetAsync(c->errflag.p, 0, sizeof(int), c->stream));
  TLS_HIP(hipStreamSynchronize(c->stream));
  return true;
}

namespace {

void dot(tls_ctx* c, const KWork& w, const double* a, const double* b, double* out, const int* done) {
  hipLaunchKernelGGL(k_dot, dim3(RED_BLOCKS), dim3(256), 0, c->stream, c->n, a, b, w.partial, w.redctr, out, done);
  TLS_LAUNCH_CHECK();
}

struct PcgVec {
  double *x, *r, *z, *p, *q, *zold, *b;
};

PcgVec vecs(const tls_ctx* c, const KWork& w) {
  const size_t n = c->n;
  double* k = w.kr;
  return PcgVec{k, k + n, k + 2 * n, k + 3 * n, k + 4 * n, k + 5 * n, k + 6 * n};
}

void pcg_iteration(tls_ctx* c, const KWork& w, const PcgVec& v, int maxit, double tol2, bool flexible) {
  hipStream_t s = c->stream;
  const int* done = w.done;
  const int n = c->n;
  const int vg = std::min(4096, div_up(n, 256));
  spmv(c, v.p, v.q, done);
  hipLaunchKernelGGL(k_dot_pq, dim3(RED_BLOCKS), dim3(256), 0, s, n, v.p, v.q, w.partial, w.redctr, w.scal, w.done);
  hipLaunchKernelGGL(k_pcg_update, dim3(RED_BLOCKS), dim3(256), 0, s, n, v.x, v.r, v.p, v.q, w.scal, w.partial,
                     w.redctr, w.done, w.hist, maxit, tol2);
  TLS_LAUNCH_CHECK();
  if (flexible) hipLaunchKernelGGL(k_copy, dim3(vg), dim3(256), 0, s, n, v.z, v.zold, done);
  apply_precond(c, v.r, v.z, done);
  dot(c, w, v.r, v.z, w.scal + 4, done);
  if (flexible) dot(c, w, v.r, v.zold, w.scal + 5, done);
  hipLaunchKernelGGL(k_pcg_p, dim3(vg), dim3(256), 0, s, n, v.p, v.z, w.scal, flexible ? 1 : 0, done);
  hipLaunchKernelGGL(k_pcg_shift, dim3(1), dim3(1), 0, s, w.scal, done);
  TLS_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Flexible GMRES(m), right preconditioned (general A). The Hessenberg matrix,
// Givens rotations, the inner index j and the stop flags live on the device.
// ---------------------------------------------------------------------------
constexpr int MD_BLOCKS = 128;
// gm layout (doubles): H[(m+1) m] | cs[m] | sn[m] | g[m+1] | y[m] | h1[m+1] | h2[m+1] | misc[8]
struct GmLayout {
  int m;
  int64_t H, cs, sn, g, y, h1, h2, misc, total;
  explicit GmLayout(int m_) : m(m_) {
    H = 0;
    cs = H + (int64_t)(m + 1) * m;
    sn = cs + m;
    g = sn + m;
    y = g + m + 1;
    h1 = y + m;
    h2 = h1 + m + 1;
    misc = h2 + m + 1;
    total = misc + 8;
  }
};
// gi: [0] j, [1] cycle end
__device__ inline bool gm_stop(const int* done, const int* gi) { return done[0] || gi[1]; }

__global__ void k_gm_cycle_init(double* gm, int* gi, GmLayout L, const double* __restrict__ rr) {
  // rr: ||r||^2 of the cycle's start residual
  gi[0] = 0;
  gi[1] = 0;
  double beta = sqrt(rr[0]);
  for (int k = 0; k <= L.m; k++) gm[L.g + k] = 0.0;
  gm[L.g] = beta;
  gm[L.misc + 0] = beta;
  if (!(beta > 0.0)) gi[1] = 1;
}

__global__ void k_gm_v0(int n, const double* __restrict__ r, double* V0, const double* __restrict__ gm, GmLayout L) {
  const double beta = gm[L.misc];
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) V0[i] = r[i] * inv;
}

// vj = V[:, j]  (or Zb[:, j] <- z)
__global__ void k_gm_take(int n, const double* __restrict__ V, double* vj, const int* __restrict__ gi,
                          const int* __restrict__ done) {
  if (gm_stop(done, gi)) return;
  const double* src = V + (int64_t)gi[0] * n;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) vj[i] = src[i];
}
__global__ void k_gm_put(int n, const double* __restrict__ z, double* Zb, const int* __restrict__ gi,
                         const int* __restrict__ done) {
  if (gm_stop(done, gi)) return;
  double* dst = Zb + (int64_t)gi[0] * n;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) dst[i] = z[i];
}

// partial dot products V[:, c] . w for c <= j
__global__ void __launch_bounds__(256) k_gm_multidot(int n, const double* __restrict__ V, const double* __restrict__ w,
                                                     double* partial, const int* __restrict__ gi,
                                                     const int* __restrict__ done) {
  if (gm_stop(done, gi)) return;
  const int c = blockIdx.y;
  if (c > gi[0]) return;
  const double* v = V + (int64_t)c * n;
  double s = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += MD_BLOCKS * 256) s += v[i] * w[i];
  block_reduce_store(s, partial + (int64_t)c * MD_BLOCKS + blockIdx.x);
}
__global__ void __launch_bounds__(256) k_gm_multidot_final(const double* __restrict__ partial, double* h,
                                                           const int* __restrict__ gi, const int* __restrict__ done) {
  if (gm_stop(done, gi)) return;
  const int c = blockIdx.x;
  if (c > gi[0]) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < MD_BLOCKS; i += 256) s += partial[(int64_t)c * MD_BLOCKS + i];
  block_reduce_store(s, h + c);
}
// w -= sum_{c <= j} h[c] V[:, c]
__global__ void k_gm_axpy(int n, const double* __restrict__ V, const double* __restrict__ h, double* w,
                          const int* __restrict__ gi, const int* __restrict__ done) {
  if (gm_stop(done, gi)) return;
  const int j = gi[0];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    double s = 0.0;
    for (int c = 0; c <= j; c++) s += h[c] * V[(int64_t)c * n + i];
    w[i] -= s;
  }
}
// V[:, j+1] = w / ||w||
__global__ void k_gm_vnext(int n, const double* __restrict__ w, double* V, const double* __restrict__ ww,
                           const int* __restrict__ gi, const int* __restrict__ done) {
  if (gm_stop(done, gi)) return;
  const double nw = sqrt(ww[0]);
  const double inv = nw > 0.0 ? 1.0 / nw : 0.0;
  double* dst = V + (int64_t)(gi[0] + 1) * n;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) dst[i] = w[i] * inv;
}
// column j of H (h1 + h2, ||w||), Givens update, residual check, j++
__global__ void k_gm_givens(double* gm, GmLayout L, const double* __restrict__ ww, int* gi, int* done, double* hist,
                            int maxit, double tol2, double bnorm2) {
  if (gm_stop(done, gi)) return;
  const int j = gi[0], m = L.m;
  double* H = gm + L.H;  // column-major (m+1) x m
  double* col = H + (int64_t)j * (m + 1);
  for (int k = 0; k <= j; k++) col[k] = gm[L.h1 + k] + gm[L.h2 + k];
  const double hn = sqrt(ww[0]);
  col[j + 1] = hn;
  for (int k = 0; k < j; k++) {
    const double c = gm[L.cs + k], s = gm[L.sn + k];
    const double a = col[k], b = col[k + 1];
    col[k] = c * a + s * b;
    col[k + 1] = -s * a + c * b;
  }
  const double a = col[j], b = col[j + 1];
  const double rr = sqrt(a * a + b * b);
  const double c = rr > 0.0 ? a / rr : 1.0, s = rr > 0.0 ? b / rr : 0.0;
  gm[L.cs + j] = c;
  gm[L.sn + j] = s;
  col[j] = rr;
  col[j + 1] = 0.0;
  const double gj = gm[L.g + j];
  gm[L.g + j] = c * gj;
  gm[L.g + j + 1] = -s * gj;
  const double res = fabs(gm[L.g + j + 1]);
  const int it = ++done[1];
  hist[it - 1] = sqrt(res * res / bnorm2);
  gi[0] = j + 1;
  if (res * res <= tol2 * bnorm2) {
    done[0] = 1;
    done[2] = 1;
  } else if (it >= maxit) {
    done[0] = 1;
  }
  if (j + 1 >= m || !(hn > 0.0)) gi[1] = 1;
}
// y = R^{-1} g for the jj = gi[0] completed columns; then x += Zb y
__global__ void k_gm_solve_y(double* gm, GmLayout L, const int* __restrict__ gi) {
  const int jj = gi[0], m = L.m;
  const double* H = gm + L.H;
  for (int k = jj - 1; k >= 0; k--) {
    double s = gm[L.g + k];
    for (int l = k + 1; l < jj; l++) s -= H[(int64_t)l * (m + 1) + k] * gm[L.y + l];
    gm[L.y + k] = s / H[(int64_t)k * (m + 1) + k];
  }
}
__global__ void k_gm_update_x(int n, double* x, const double* __restrict__ Zb, const double* __restrict__ gm, GmLayout L,
                              const int* __restrict__ gi) {
  const int jj = gi[0];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    double s = 0.0;
    for (int c = 0; c < jj; c++) s += gm[L.y + c] * Zb[(int64_t)c * n + i];
    x[i] += s;
  }
}

}  // namespace

void spmv_residual(tls_ctx* c, const double* f, const double* x, double* y, const int* done) {
  hipStream_t s = c->stream;
  const int n = c->n;
  const int G = c->spmv_group;
  const unsigned grid = div_up(n, 256 / G);
  switch (G) {
    case 4:
      hipLaunchKernelGGL(k_spmv<4>, dim3(grid), dim3(256), 0, s, n, c->row_ptr.p, c->col_idx.p, c->val.p, x, y, done, f);
      break;
    case 8:
      hipLaunchKernelGGL(k_spmv<8>, dim3(grid), dim3(256), 0, s, n, c->row_ptr.p, c->col_idx.p, c->val.p, x, y, done, f);
      break;
    case 16:
      hipLaunchKernelGGL(k_spmv<16>, dim3(grid), dim3(256), 0, s, n, c->row_ptr.p, c->col_idx.p, c->val.p, x, y, done,
                         f);
      break;
    case 32:
      hipLaunchKernelGGL(k_spmv<32>, dim3(grid), dim3(256), 0, s, n, c->row_ptr.p, c->col_idx.p, c->val.p, x, y, done,
                         f);
      break;
    default:
      hipLaunchKernelGGL(k_spmv<64>, dim3(grid), dim3(256), 0, s, n, c->row_ptr.p, c->col_idx.p, c->val.p, x, y, done,
                         f);
      break;
  }
  TLS_LAUNCH_CHECK();
}

void spmv(tls_ctx* c, const double* x, double* y, const int* done) { spmv_residual(c, nullptr, x, y, done); }

namespace {

bool use_pcg(const tls_ctx* c) { return c->kind == 0 && c->opt.composition == 0; }
int krylov_maxit(const tls_ctx* c) { return c->opt.maxit > 0 ? c->opt.maxit : (use_pcg(c) ? 1000 : 3000); }
int gmres_m(const tls_ctx* c) { return c->opt.restart > 0 ? c->opt.restart : 30; }

void pcg_run(tls_ctx* c, const KWork& w, const double* b, double* x, double tol, int* iters, double* relres,
             bool* converged) {
  hipStream_t s = c->stream;
  const int n = c->n;
  const int maxit = krylov_maxit(c);
  const bool flexible = c->opt.flexible != 0;
  TLS_HIP(hipMemsetAsync(w.redctr, 0, sizeof(unsigned), s));  // outside any captured graph
  if (take_wait_flag(c)) c->apply_wait_seen = true;  // from an earlier tls_apply: reported by tls_info
  PcgVec v = vecs(c, w);
  const double tol2 = tol * tol;
  auto t0 = std::chrono::steady_clock::now();
  TLS_HIP(hipMemsetAsync(w.done, 0, sizeof(int) * 4, s));
  TLS_HIP(hipMemsetAsync(v.x, 0, sizeof(double) * n, s));
  TLS_HIP(hipMemcpyAsync(v.b, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  TLS_HIP(hipMemcpyAsync(v.r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  TLS_HIP(hipMemsetAsync(v.zold, 0, sizeof(double) * n, s));
  dot(c, w, v.b, v.b, w.scal + 0, w.done);
  double bb = 0.0;
  read_back(w.scal, &bb, 1, s);
  int it = 0;
  bool conv = false;
  c->h_hist.clear();
  if (bb == 0.0) {
    TLS_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    TLS_HIP(hipStreamSynchronize(s));
    *iters = 0;
    *relres = 0.0;
    *converged = true;
    return;
  }
  apply_precond(c, v.r, v.z, w.done);
  dot(c, w, v.r, v.z, w.scal + 1, w.done);
  TLS_HIP(hipMemcpyAsync(v.p, v.z, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  const int chunk = 8;
  // the captured graph refers to the context's own work buffers
  const bool use_graph = c->opt.use_graph != 0 && w.context_bufs;
  if (use_graph && (!c->graph_exec || c->graph_chunk != chunk || c->graph_maxit != maxit ||
                    c->graph_tol2 != tol2 || c->graph_flex != flexible)) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
    hipGraph_t g;
    TLS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int j = 0; j < chunk; j++) pcg_iteration(c, w, v, maxit, tol2, flexible);
    TLS_HIP(hipStreamEndCapture(s, &g));
    TLS_HIP(hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    c->graph_chunk = chunk;
    c->graph_maxit = maxit;
    c->graph_tol2 = tol2;
    c->graph_flex = flexible;
  }
  int hd[4] = {0, 0, 0, 0};
  const int* zero = c->zero_int.p;
  double rr = 0.0;
  // The recurrence residual decides when to stop iterating; convergence is
  // only reported when the true residual b - A x meets the tolerance too.
  // Otherwise PCG restarts from the current x (at most kRestarts times).
  constexpr int kRestarts = 4;
  for (int restart = 0;; restart++) {
    for (int launched = 0; launched < maxit + chunk; launched += chunk) {
      if (use_graph)
        TLS_HIP(hipGraphLaunch(c->graph_exec, s));
      else
        for (int j = 0; j < chunk; j++) pcg_iteration(c, w, v, maxit, tol2, flexible);
      read_back(w.done, hd, 4, s);
      if (hd[0]) break;
    }
    it = hd[1];
    conv = hd[2] != 0;
    if (hd[3]) fail(TLS_E_NOT_SPD, "PCG breakdown: p^T A p <= 0 (A or M^{-1} not SPD)");
    // true residual r = b - A x
    spmv(c, v.x, v.q, zero);
    hipLaunchKernelGGL(k_sub, dim3(std::min(4096, div_up(n, 256))), dim3(256), 0, s, n, v.b, v.q, v.r);
    TLS_LAUNCH_CHECK();
    dot(c, w, v.r, v.r, w.scal + 7, zero);
    read_back(w.scal + 7, &rr, 1, s);
    if (!conv || rr <= tol2 * bb) break;
    if (restart == kRestarts || it >= maxit) {
      conv = false;
      break;
    }
    // restart from x with the true residual: z = M^{-1} r, p = z
    TLS_HIP(hipMemsetAsync(w.done, 0, sizeof(int), s));
    TLS_HIP(hipMemsetAsync(w.done + 2, 0, sizeof(int), s));
    TLS_HIP(hipMemsetAsync(v.zold, 0, sizeof(double) * n, s));
    apply_precond(c, v.r, v.z, w.done);
    dot(c, w, v.r, v.z, w.scal + 1, w.done);
    TLS_HIP(hipMemcpyAsync(v.p, v.z, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  }
  TLS_HIP(hipMemcpyAsync(x, v.x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  if (w.context_bufs) c->h_hist = download(w.hist, it, s);
  TLS_HIP(hipStreamSynchronize(s));
  auto t1 = std::chrono::steady_clock::now();
  c->t_solve = std::chrono::duration<double, std::milli>(t1 - t0).count();
  *iters = it;
  *relres = std::sqrt(rr / bb);
  *converged = conv;
  if (take_wait_flag(c)) fail(TLS_E_HIP, "a triangular-solve wait of this solve exceeded its spin limit");
}

struct GmBufs {
  double *x, *r, *w, *vj, *zj, *b, *V, *Zb;
};

void fgmres_inner(tls_ctx* c, const KWork& W, const GmBufs& B, const GmLayout& L, int maxit, double tol2,
                  double bnorm2) {
  hipStream_t s = c->stream;
  const int n = c->n;
  const int* done = W.done;
  double* gm = W.gm;
  int* gi = W.gi;
  double* mdpart = W.partial;
  const int vg = std::min(4096, div_up(n, 256));
  hipLaunchKernelGGL(k_gm_take, dim3(vg), dim3(256), 0, s, n, B.V, B.vj, gi, done);
  TLS_LAUNCH_CHECK();
  // the apply and the SpMV are gated by the done flag only; when the cycle has
  // ended they work on stale vectors whose results nothing reads
  apply_precond(c, B.vj, B.zj, done);
  hipLaunchKernelGGL(k_gm_put, dim3(vg), dim3(256), 0, s, n, B.zj, B.Zb, gi, done);
  spmv(c, B.zj, B.w, done);
  for (int pass = 0; pass < 2; pass++) {
    double* h = gm + (pass == 0 ? L.h1 : L.h2);
    hipLaunchKernelGGL(k_gm_multidot, dim3(MD_BLOCKS, L.m + 1), dim3(256), 0, s, n, B.V, B.w, mdpart, gi, done);
    hipLaunchKernelGGL(k_gm_multidot_final, dim3(L.m + 1), dim3(256), 0, s, mdpart, h, gi, done);
    hipLaunchKernelGGL(k_gm_axpy, dim3(vg), dim3(256), 0, s, n, B.V, h, B.w, gi, done);
    TLS_LAUNCH_CHECK();
  }
  dot(c, W, B.w, B.w, W.scal + 8, done);
  hipLaunchKernelGGL(k_gm_vnext, dim3(vg), dim3(256), 0, s, n, B.w, B.V, W.scal + 8, gi, done);
  hipLaunchKernelGGL(k_gm_givens, dim3(1), dim3(1), 0, s, gm, L, W.scal + 8, gi, W.done, W.hist, maxit, tol2,
                     bnorm2);
  TLS_LAUNCH_CHECK();
}

void fgmres_run(tls_ctx* c, const KWork& W, const double* b, double* x, double tol, int* iters, double* relres,
                bool* converged) {
  hipStream_t s = c->stream;
  const int n = c->n;
  const int m = gmres_m(c);
  const int maxit = krylov_maxit(c);
  const GmLayout L(m);
  TLS_HIP(hipMemsetAsync(W.redctr, 0, sizeof(unsigned), s));  // outside any captured graph
  if (take_wait_flag(c)) c->apply_wait_seen = true;  // from an earlier tls_apply: reported by tls_info
  double* k = W.kr;
  GmBufs B{k, k + n, k + 2 * (size_t)n, k + 3 * (size_t)n, k + 4 * (size_t)n, k + 5 * (size_t)n, k + 6 * (size_t)n,
           k + (6 + (size_t)(m + 1)) * n};
  auto t0 = std::chrono::steady_clock::now();
  TLS_HIP(hipMemsetAsync(W.done, 0, sizeof(int) * 4, s));
  TLS_HIP(hipMemsetAsync(B.x, 0, sizeof(double) * n, s));
  TLS_HIP(hipMemsetAsync(W.gm, 0, sizeof(double) * L.total, s));
  TLS_HIP(hipMemcpyAsync(B.b, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  const int* zero = c->zero_int.p;
  dot(c, W, B.b, B.b, W.scal + 0, zero);
  double bb = 0.0;
  read_back(W.scal, &bb, 1, s);
  c->h_hist.clear();
  if (bb == 0.0) {
    TLS_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    TLS_HIP(hipStreamSynchronize(s));
    *iters = 0;
    *relres = 0.0;
    *converged = true;
    return;
  }
  const double tol2 = tol * tol;
  const int vg = std::min(4096, div_up(n, 256));
  bool conv = false;
  int hd[4] = {0, 0, 0, 0};
  double rr = bb;
  for (int cycle = 0;; cycle++) {
    // r = b - A x
    spmv(c, B.x, B.w, zero);
    hipLaunchKernelGGL(k_sub, dim3(vg), dim3(256), 0, s, n, B.b, B.w, B.r);
    dot(c, W, B.r, B.r, W.scal + 9, zero);
    hipLaunchKernelGGL(k_gm_cycle_init, dim3(1), dim3(1), 0, s, W.gm, W.gi, L, W.scal + 9);
    hipLaunchKernelGGL(k_gm_v0, dim3(vg), dim3(256), 0, s, n, B.r, B.V, W.gm, L);
    TLS_LAUNCH_CHECK();
    for (int j = 0; j < m; j++) fgmres_inner(c, W, B, L, maxit, tol2, bb);
    hipLaunchKernelGGL(k_gm_solve_y, dim3(1), dim3(1), 0, s, W.gm, L, W.gi);
    hipLaunchKernelGGL(k_gm_update_x, dim3(vg), dim3(256), 0, s, n, B.x, B.Zb, W.gm, L, W.gi);
    TLS_LAUNCH_CHECK();
    // true residual of the new iterate
    spmv(c, B.x, B.w, zero);
    hipLaunchKernelGGL(k_sub, dim3(vg), dim3(256), 0, s, n, B.b, B.w, B.r);
    dot(c, W, B.r, B.r, W.scal + 7, zero);
    read_back(W.scal + 7, &rr, 1, s);
    read_back(W.done, hd, 4, s);
    if (rr <= tol2 * bb) {
      conv = true;
      break;
    }
    if (hd[1] >= maxit) break;
    // not converged by the true residual: clear the stop flag and restart
    TLS_HIP(hipMemsetAsync(W.done, 0, sizeof(int) * 1, s));
    TLS_HIP(hipMemsetAsync(W.done + 2, 0, sizeof(int) * 1, s));
  }
  TLS_HIP(hipMemcpyAsync(x, B.x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  const int it = hd[1];
  if (W.context_bufs) c->h_hist = download(W.hist, std::max(it, 0), s);
  TLS_HIP(hipStreamSynchronize(s));
  c->t_solve = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *iters = it;
  *relres = std::sqrt(rr / bb);
  *converged = conv;
  if (take_wait_flag(c)) fail(TLS_E_HIP, "a triangular-solve wait of this solve exceeded its spin limit");
}

}  // namespace

KrylovNeeds krylov_needs(const tls_ctx* c) {
  KrylovNeeds k;
  k.hist = krylov_maxit(c);
  if (use_pcg(c)) {
    k.kr = (size_t)7 * c->n;
    k.partial = RED_BLOCKS;
    k.gm = 0;
  } else {
    const int m = gmres_m(c);
    k.kr = (size_t)c->n * (6 + (m + 1) + m);
    k.partial = (size_t)std::max(RED_BLOCKS, MD_BLOCKS * (m + 1));
    k.gm = (size_t)GmLayout(m).total;
  }
  return k;
}

void krylov_run(tls_ctx* c, const KWork& w, const double* b, double* x, double tol, int* iters, double* relres,
                bool* converged) {
  // PCG needs a symmetric preconditioner: SPD A with the additive composition
  if (use_pcg(c))
    pcg_run(c, w, b, x, tol, iters, relres, converged);
  else
    fgmres_run(c, w, b, x, tol, iters, relres, converged);
}

void krylov_solve(tls_ctx* c, const double* b, double* x, double tol, int* iters, double* relres, bool* converged) {
  const KrylovNeeds k = krylov_needs(c);
  if (c->kr.n < k.kr) c->kr.alloc(k.kr);
  if (c->scal.n < 16) c->scal.alloc(16);
  if (c->partial.n < k.partial) c->partial.alloc(k.partial);
  if (c->done.n < 4) c->done.alloc(4);
  if (c->hist.n < (size_t)k.hist) c->hist.alloc(k.hist);
  if (c->redctr.n < 1) c->redctr.alloc(1);
  if (k.gm && c->gm_state.n < k.gm) c->gm_state.alloc(k.gm);
  if (c->gm_idx.n < 4) c->gm_idx.alloc(4);
  KWork w;
  w.kr = c->kr.p;
  w.scal = c->scal.p;
  w.partial = c->partial.p;
  w.redctr = c->redctr.p;
  w.done = c->done.p;
  w.hist = c->hist.p;
  w.gm = c->gm_state.p;
  w.gi = c->gm_idx.p;
  w.context_bufs = true;
  krylov_run(c, w, b, x, tol, iters, relres, converged);
}

}  // namespace tls
