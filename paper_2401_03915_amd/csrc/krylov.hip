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

// Reductions run on red_grid(n) <= RED_BLOCKS blocks of 256 threads (each
// thread with four loads in flight): the last block is found with one
// same-address atomic per block, and on this GPU those serialize at about
// 10 ns each (4096 of them cost ~37 us), so the grid is kept small.
constexpr int RED_BLOCKS = 512;
inline int red_grid(int n) { return std::max(1, std::min(RED_BLOCKS, (n + 2047) / 2048)); }

// SpMV by row blocks: a block of SPMV_ROWS consecutive rows streams its
// stored entries (values and columns) with consecutive threads on
// consecutive entries, keeps the products in LDS and then sums each row's
// products in the stored order; rows whose block holds more than CAP
// entries are done one thread per row instead. Short rows (the 5- and
// 7-point stencils) are read fully coalesced this way.
constexpr int SPMV_ROWS = 256;
// with p.q (PCG) the SpMV stores one partial per block (at most this many
// blocks, looping over row blocks beyond); k_pcg_update adds them
constexpr int SPMV_PQ_BLOCKS = 4096;
inline int spmv_blocks(int n) { return (n + SPMV_ROWS - 1) / SPMV_ROWS; }

__device__ inline void block_reduce_store(double v, double* out) {
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}

// Each reduction is one launch: every block stores its partial sum; the last
// block to finish (counted in *ctr, which it resets) adds the partials in
// index order and stores the result, so the value does not depend on the
// order in which the blocks ran. The partials and the counter are device-
// coherent accesses (relaxed agent-scope atomics, which bypass the per-XCD
// L2): a block waits for its partial's store to complete before it counts
// itself, and the last block reads the partials with coherent loads. No
// cache write-back or invalidation is needed (an agent-scope fence in every
// block wrote back the XCD's L2 each time and made a 4096-block SpMV with
// its dot product five times slower).
__device__ inline void block_reduce_partial(double v, double* partial) {
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_store(partial + blockIdx.x, (red[0] + red[1]) + (red[2] + red[3]), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);  // the coherent store has completed before the block is counted
  }
}

__device__ inline bool last_block(unsigned* ctr) {
  __shared__ bool s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    s_last = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
    if (s_last) __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  return s_last;
}

// the partials in index order (coherent loads), into *out
__device__ inline void sum_partials(const double* partial, int count, double* out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) s += __hip_atomic_load(partial + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  block_reduce_store(s, out);
}

// y = A x, or y = f - A x when f is given. With pq (PCG): also each block's
// part of p.q (x = p, y = q) into partial[blockIdx.x]; the next launch adds
// the partials (a plain store: no counter, no atomics).
// CAP (the LDS products of one row block) is the smallest of 1280, 1536,
// 2048 and 4096 that holds every row block's entries (chosen at setup): the
// less LDS, the more blocks per CU; each thread issues all of its CAP / 256
// value and column loads before its gathers from x.
template <int CAP>
__global__ void __launch_bounds__(256) k_spmv(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                              const double* __restrict__ val, const double* __restrict__ x,
                                              double* __restrict__ y, const int* __restrict__ done,
                                              const double* __restrict__ f, int pq, double* partial) {
  if (*done) return;
  constexpr int U = CAP / 256;
  __shared__ double prod[CAP];
  __shared__ int srp[SPMV_ROWS + 1];
  double mine = 0.0;  // this thread's rows (pq only)
  const int nblk = (n + SPMV_ROWS - 1) / SPMV_ROWS;
  for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int r0 = blk * SPMV_ROWS;
    const int nr = min(n - r0, SPMV_ROWS);
    __syncthreads();  // the previous row block is done with srp and prod
    for (int t = threadIdx.x; t <= nr; t += 256) srp[t] = rp[r0 + t];
    __syncthreads();
    const int j0 = srp[0], nz = srp[nr] - j0;
    if (nz <= CAP) {
      double vv[U];
      int cc[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int t = threadIdx.x + 256 * u;
        if (t < nz) {
          vv[u] = __builtin_nontemporal_load(val + j0 + t);
          cc[u] = __builtin_nontemporal_load(ci + j0 + t);
        }
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int t = threadIdx.x + 256 * u;
        if (t < nz) prod[t] = vv[u] * x[cc[u]];
      }
      __syncthreads();
      for (int r = threadIdx.x; r < nr; r += 256) {
        double s = 0.0;
        for (int t = srp[r] - j0; t < srp[r + 1] - j0; t++) s += prod[t];
        const double v = f ? f[r0 + r] - s : s;
        y[r0 + r] = v;
        if (pq) mine += x[r0 + r] * v;
      }
    } else {
      for (int r = threadIdx.x; r < nr; r += 256) {
        double s = 0.0;
        for (int j = srp[r]; j < srp[r + 1]; j++) s += val[j] * x[ci[j]];
        const double v = f ? f[r0 + r] - s : s;
        y[r0 + r] = v;
        if (pq) mine += x[r0 + r] * v;
      }
    }
  }
  if (pq) block_reduce_store(mine, partial + blockIdx.x);
}

// Longer rows: G lanes per row and a shuffle reduction.
template <int G>
__global__ void __launch_bounds__(256) k_spmv_group(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                    const double* __restrict__ val, const double* __restrict__ x,
                                                    double* __restrict__ y, const int* __restrict__ done,
                                                    const double* __restrict__ f, int pq, double* partial) {
  if (*done) return;
  const int lane = threadIdx.x % G;
  const int nrb = (n + 256 / G - 1) / (256 / G);
  double mine = 0.0;
  for (int rb = blockIdx.x; rb < nrb; rb += gridDim.x) {
    const int row = rb * (256 / G) + threadIdx.x / G;
    double s = 0.0;
    if (row < n) {
      const int b = rp[row + 1];
      for (int j = rp[row] + lane; j < b; j += G) s += val[j] * x[ci[j]];
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
    if (row < n && lane == 0) {
      const double v = f ? f[row] - s : s;
      y[row] = v;
      if (pq) mine += x[row] * v;
    }
  }
  if (pq) block_reduce_store(mine, partial + blockIdx.x);
}

__global__ void __launch_bounds__(256) k_dot(int n, const double* __restrict__ a, const double* __restrict__ b,
                                             double* partial, unsigned* ctr, double* out,
                                             const int* __restrict__ done) {
  if (*done) return;
  double s = 0.0;
  const int st = gridDim.x * 256;
  for (int i0 = blockIdx.x * 256 + threadIdx.x; i0 < n; i0 += 4 * st)
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int i = i0 + u * st;
      if (i < n) s += a[i] * b[i];
    }
  block_reduce_partial(s, partial);
  if (last_block(ctr)) sum_partials(partial, gridDim.x, out);
}

// r.z into scal[4] (its previous value moves to scal[1]) and, for the
// flexible variant, r.zold into scal[5], in one pass
__global__ void __launch_bounds__(256) k_dot_rz(int n, const double* __restrict__ r, const double* __restrict__ z,
                                                const double* __restrict__ zold, double* partial, unsigned* ctr,
                                                double* scal, const int* __restrict__ done) {
  if (*done) return;
  double s = 0.0, t = 0.0;
  const int st = gridDim.x * 256;
  for (int i0 = blockIdx.x * 256 + threadIdx.x; i0 < n; i0 += 4 * st)
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int i = i0 + u * st;
      if (i < n) {
        const double ri = r[i];
        s += ri * z[i];
        if (zold) t += ri * zold[i];
      }
    }
  block_reduce_partial(s, partial);
  __syncthreads();
  if (zold) block_reduce_partial(t, partial + RED_BLOCKS);
  if (last_block(ctr)) {
    if (threadIdx.x == 0) scal[1] = scal[4];  // the previous r.z, for beta
    __syncthreads();
    sum_partials(partial, gridDim.x, scal + 4);
    __syncthreads();
    if (zold) sum_partials(partial + RED_BLOCKS, gridDim.x, scal + 5);
  }
}

// p.q = the SpMV's partials added in index order (every block alike; a
// non-positive p.q stops the iteration: breakdown); alpha = r.z / p.q;
// x += alpha p; r -= alpha q; [zold = z]; r.r into scal[3]; then the last
// block records ||r||/||b|| and stops on the tolerance or the cap
__global__ void __launch_bounds__(256) k_pcg_update(int n, double* __restrict__ x, double* __restrict__ r,
                                                    const double* __restrict__ p, const double* __restrict__ q,
                                                    const double* __restrict__ z, double* __restrict__ zold,
                                                    const double* __restrict__ pqpart, int npq, double* scal,
                                                    double* partial, unsigned* ctr, int* done, double* hist,
                                                    int maxit, double tol2) {
  if (done[0]) return;
  __shared__ double s_pq;
  {
    double v = 0.0;
    for (int i = threadIdx.x; i < npq; i += 256) v += pqpart[i];
    block_reduce_store(v, &s_pq);
    __syncthreads();
  }
  const double pqv = s_pq;
  if (!(pqv > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      scal[2] = pqv;
      done[0] = 1;
      done[3] = 1;
    }
    return;
  }
  const double alpha = scal[4] / pqv;
  double s = 0.0;
  const int st = gridDim.x * 256;
  for (int i0 = blockIdx.x * 256 + threadIdx.x; i0 < n; i0 += 4 * st)
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int i = i0 + u * st;
      if (i < n) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        s += ri * ri;
        if (zold) zold[i] = z[i];
      }
    }
  block_reduce_partial(s, partial);
  if (last_block(ctr)) {
    sum_partials(partial, gridDim.x, scal + 3);
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

// beta = (r.z - [r.zold]) / rz_prev ; p = z + beta p
__global__ void k_pcg_p(int n, double* __restrict__ p, const double* __restrict__ z, const double* __restrict__ scal,
                        int flexible, const int* __restrict__ done) {
  if (*done) return;
  const double beta = (scal[4] - (flexible ? scal[5] : 0.0)) / scal[1];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = z[i] + beta * p[i];
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

// blocks of the SpMV launch; with p.q (its number of partial sums) the
// row-block kernel loops over row blocks on at most RED_BLOCKS blocks
int spmv_grid(const tls_ctx* c, bool pq) {
  const int nb = c->spmv_group == 0 ? spmv_blocks(c->n) : div_up(c->n, 256 / c->spmv_group);
  return pq ? std::min(nb, SPMV_PQ_BLOCKS) : nb;
}

// y = A x (or f - A x); with w (PCG): also p.q, the breakdown check and the r.z shift
void spmv_launch(tls_ctx* c, const double* f, const double* x, double* y, const int* done, const KWork* w) {
  hipStream_t s = c->stream;
  const int n = c->n;
  const dim3 grid(spmv_grid(c, w != nullptr));
  const int pq = w ? 1 : 0;
  double* partial = w ? w->partial + 2 * RED_BLOCKS : nullptr;  // after the dot partials
  const int *rp = c->row_ptr.p, *ci = c->col_idx.p;
  const double* val = c->val.p;
  switch (c->spmv_group) {
    case 0:
      switch (c->spmv_cap) {
        case 1280:
          hipLaunchKernelGGL(k_spmv<1280>, grid, dim3(256), 0, s, n, rp, ci, val, x, y, done, f, pq, partial);
          break;
        case 1536:
          hipLaunchKernelGGL(k_spmv<1536>, grid, dim3(256), 0, s, n, rp, ci, val, x, y, done, f, pq, partial);
          break;
        case 2048:
          hipLaunchKernelGGL(k_spmv<2048>, grid, dim3(256), 0, s, n, rp, ci, val, x, y, done, f, pq, partial);
          break;
        default:
          hipLaunchKernelGGL(k_spmv<4096>, grid, dim3(256), 0, s, n, rp, ci, val, x, y, done, f, pq, partial);
          break;
      }
      break;
    case 8:
      hipLaunchKernelGGL(k_spmv_group<8>, grid, dim3(256), 0, s, n, rp, ci, val, x, y, done, f, pq, partial);
      break;
    case 16:
      hipLaunchKernelGGL(k_spmv_group<16>, grid, dim3(256), 0, s, n, rp, ci, val, x, y, done, f, pq, partial);
      break;
    case 32:
      hipLaunchKernelGGL(k_spmv_group<32>, grid, dim3(256), 0, s, n, rp, ci, val, x, y, done, f, pq, partial);
      break;
    default:
      hipLaunchKernelGGL(k_spmv_group<64>, grid, dim3(256), 0, s, n, rp, ci, val, x, y, done, f, pq, partial);
      break;
  }
  TLS_LAUNCH_CHECK();
}

void dot(tls_ctx* c, const KWork& w, const double* a, const double* b, double* out, const int* done) {
  hipLaunchKernelGGL(k_dot, dim3(red_grid(c->n)), dim3(256), 0, c->stream, c->n, a, b, w.partial, w.redctr, out,
                     done);
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

// One PCG iteration in five launches besides the preconditioner:
//   q = A p with p.q (and rz <- rz_new) | alpha, x, r, r.r, convergence [, zold = z]
//   | z = M^{-1} r | r.z [, r.zold] | p = z + beta p
void pcg_iteration(tls_ctx* c, const KWork& w, const PcgVec& v, int maxit, double tol2, bool flexible) {
  hipStream_t s = c->stream;
  const int* done = w.done;
  const int n = c->n;
  const int vg = std::min(4096, div_up(n, 256));
  const dim3 rg(red_grid(n));
  spmv_launch(c, nullptr, v.p, v.q, done, &w);
  hipLaunchKernelGGL(k_pcg_update, rg, dim3(256), 0, s, n, v.x, v.r, v.p, v.q, v.z, flexible ? v.zold : nullptr,
                     w.partial + 2 * RED_BLOCKS, spmv_grid(c, true), w.scal, w.partial, w.redctr, w.done, w.hist,
                     maxit, tol2);
  TLS_LAUNCH_CHECK();
  apply_precond(c, v.r, v.z, done);
  hipLaunchKernelGGL(k_dot_rz, rg, dim3(256), 0, s, n, v.r, v.z, flexible ? v.zold : nullptr, w.partial, w.redctr,
                     w.scal, done);
  hipLaunchKernelGGL(k_pcg_p, dim3(vg), dim3(256), 0, s, n, v.p, v.z, w.scal, flexible ? 1 : 0, done);
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
  spmv_launch(c, f, x, y, done, nullptr);
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
  dot(c, w, v.r, v.z, w.scal + 4, w.done);  // the first SpMV makes it the current r.z
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
    dot(c, w, v.r, v.z, w.scal + 4, w.done);
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
    k.partial = (size_t)(2 * RED_BLOCKS + spmv_grid(c, true));
    k.gm = 0;
  } else {
    const int m = gmres_m(c);
    k.kr = (size_t)c->n * (6 + (m + 1) + m);
    k.partial = (size_t)std::max(2 * RED_BLOCKS + spmv_grid(c, true), MD_BLOCKS * (m + 1));
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
