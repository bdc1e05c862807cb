// Ingest, validation and the overlapping subdomains (Section 2.1):
//   * CSR / partition validation (device, error bits);
//   * pattern of A^T for nonsymmetric A (graph(A + A^T) is explored through
//     the rows of A and of A^T);
//   * delta-layer breadth-first overlap per subdomain, every layer in
//     ascending global order: Omega_i = [I_i, Gamma_{i,1}, .., Gamma_{i,delta}];
//   * the maps the apply needs (owners of every global row, interior
//     positions).
#include "context.hpp"
#include "kernels.hpp"
#include "scan.hpp"

namespace tls {

namespace {

constexpr uint8_t UNSEEN = 0xFF;

__global__ void k_validate(int n, int nnz, const int* __restrict__ rp, const int* __restrict__ ci,
                           const double* __restrict__ v, const int* __restrict__ part, int N,
                           int* err, int* part_count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (i == 0 && rp[0] != 0) atomicOr(err, ERR_CSR);
  if (i == n - 1 && rp[n] != nnz) atomicOr(err, ERR_CSR);
  int a = rp[i], b = rp[i + 1];
  if (a < 0 || b < a || b > nnz) {
    atomicOr(err, ERR_CSR);
  } else {
    int prev = -1;
    for (int j = a; j < b; j++) {
      int c = ci[j];
      if (c < 0 || c >= n || c <= prev) atomicOr(err, ERR_CSR);
      prev = c;
      if (!isfinite(v[j])) atomicOr(err, ERR_NAN);
    }
  }
  int p = part[i];
  if (p < 0 || p >= N)
    atomicOr(err, ERR_PART);
  else
    atomicAdd(&part_count[p], 1);
}

__global__ void k_count_cols(int nnz, const int* __restrict__ ci, int* cnt) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < nnz) atomicAdd(&cnt[ci[j]], 1);
}

__global__ void k_fill_transpose(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                 const int* __restrict__ trp, int* cursor, int* tci) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int j = rp[i]; j < rp[i + 1]; j++) {
    int c = ci[j];
    int pos = atomicAdd(&cursor[c], 1);
    tci[trp[c] + pos] = i;
  }
}

__global__ void k_mark_interior(int n, const int* __restrict__ part, uint8_t* dist) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) dist[(size_t)part[v] * n + v] = 0;
}

// Count entries of row i of dist equal to `level` (one block per subdomain).
__global__ void k_level_count(int n, const uint8_t* __restrict__ dist, uint8_t level, int* cnt) {
  const uint8_t* row = dist + (size_t)blockIdx.x * n;
  int c = 0;
  for (int v = threadIdx.x; v < n; v += blockDim.x) c += (row[v] == level);
  __shared__ int sh[256];
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) cnt[blockIdx.x] = sh[0];
}

// Ordered compaction of row i of dist: the global ids v with dist == level,
// ascending, written to out[off[i] ..]; the subdomain id goes to osub.
__global__ void k_level_fill(int n, const uint8_t* __restrict__ dist, uint8_t level,
                             const int* __restrict__ off, int* out, int* osub) {
  const int i = blockIdx.x;
  const uint8_t* row = dist + (size_t)i * n;
  constexpr int PER = 16;
  __shared__ int sh[256];
  int base_out = off[i];
  for (int64_t chunk = 0; chunk < n; chunk += 256 * PER) {
    int64_t start = chunk + (int64_t)threadIdx.x * PER;
    int c = 0;
    for (int j = 0; j < PER; j++) {
      int64_t v = start + j;
      if (v < n && row[v] == level) c++;
    }
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int s = 1; s < 256; s <<= 1) {
      int add = threadIdx.x >= s ? sh[threadIdx.x - s] : 0;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    int pos = base_out + sh[threadIdx.x] - c;
    int tot = sh[255];
    __syncthreads();
    for (int j = 0; j < PER; j++) {
      int64_t v = start + j;
      if (v < n && row[v] == level) {
        out[pos] = (int)v;
        osub[pos] = i;
        pos++;
      }
    }
    base_out += tot;
  }
}

// One breadth-first step: every neighbor (in A or A^T) of a level-(l-1) node
// of subdomain i that is still unseen for i gets level l. Concurrent writers
// store the same value.
__global__ void k_expand(int count, const int* __restrict__ lay, const int* __restrict__ lsub, int n,
                         const int* __restrict__ rp, const int* __restrict__ ci,
                         const int* __restrict__ trp, const int* __restrict__ tci, uint8_t level,
                         uint8_t* dist) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  int v = lay[e];
  size_t rowbase = (size_t)lsub[e] * n;
  for (int j = rp[v]; j < rp[v + 1]; j++) {
    int u = ci[j];
    if (dist[rowbase + u] == UNSEEN) dist[rowbase + u] = level;
  }
  if (trp) {
    for (int j = trp[v]; j < trp[v + 1]; j++) {
      int u = tci[j];
      if (dist[rowbase + u] == UNSEEN) dist[rowbase + u] = level;
    }
  }
}

// Copy level-l entries into their place in sub_idx.
__global__ void k_place_level(int count, const int* __restrict__ lay, const int* __restrict__ lsub,
                              const int* __restrict__ loff, const int* __restrict__ layer_ptr,
                              int stride, int l, int* sub_idx) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  int i = lsub[e];
  sub_idx[layer_ptr[i * stride + l] + (e - loff[i])] = lay[e];
}

__global__ void k_sub_maps(int N, const int* __restrict__ sub_ptr, const int* __restrict__ nI,
                           const int* __restrict__ sub_idx, int* sub_of_pos, int* ipos) {
  int i = blockIdx.x;
  for (int p = sub_ptr[i] + threadIdx.x; p < sub_ptr[i + 1]; p += blockDim.x) {
    sub_of_pos[p] = i;
    int j = p - sub_ptr[i];
    if (j < nI[i]) ipos[sub_idx[p]] = j;
  }
}

__global__ void k_owner_count(int total, const int* __restrict__ sub_idx, int* cnt) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < total) atomicAdd(&cnt[sub_idx[p]], 1);
}

__global__ void k_owner_fill(int total, const int* __restrict__ sub_idx, const int* __restrict__ sub_of_pos,
                             const int* __restrict__ sub_ptr, const int64_t* __restrict__ voff,
                             const int* __restrict__ own_ptr, int* cursor, int64_t* own_pos) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  int g = sub_idx[p];
  int i = sub_of_pos[p];
  int k = atomicAdd(&cursor[g], 1);
  own_pos[own_ptr[g] + k] = voff[i] + (p - sub_ptr[i]);
}

// Sort each owner list (a handful of entries) so sums run in a fixed order.
__global__ void k_owner_sort(int n, const int* __restrict__ own_ptr, int64_t* own_pos) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  int a = own_ptr[g], b = own_ptr[g + 1];
  for (int x = a + 1; x < b; x++) {
    int64_t key = own_pos[x];
    int y = x - 1;
    while (y >= a && own_pos[y] > key) {
      own_pos[y + 1] = own_pos[y];
      y--;
    }
    own_pos[y + 1] = key;
  }
}

}  // namespace

void validate_input(tls_ctx* c) {
  hipStream_t s = c->stream;
  DBuf<int> cnt;
  cnt.alloc(c->N);
  TLS_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int) * c->N, s));
  TLS_HIP(hipMemsetAsync(c->errflag.p, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_validate, dim3(div_up(c->n, 256)), dim3(256), 0, s, c->n, c->nnz, c->row_ptr.p,
                     c->col_idx.p, c->val.p, c->part.p, c->N, c->errflag.p, cnt.p);
  TLS_LAUNCH_CHECK();
  int err = download(c->errflag.p, 1, s)[0];
  if (err & ERR_CSR) fail(TLS_E_ARG, "malformed CSR (row_ptr, column range or column order)");
  if (err & ERR_NAN) fail(TLS_E_ARG, "non-finite matrix value");
  if (err & ERR_PART) fail(TLS_E_ARG, "partition value out of range");
  auto h = download(cnt.p, c->N, s);
  for (int i = 0; i < c->N; i++)
    if (h[i] == 0) fail(TLS_E_ARG, "part " + std::to_string(i) + " is empty");
}

void build_transpose(tls_ctx* c) {
  hipStream_t s = c->stream;
  DBuf<int> cnt, cursor;
  cnt.alloc(c->n);
  cursor.alloc(c->n);
  c->trow_ptr.alloc(c->n + 1);
  c->tcol_idx.alloc(c->nnz);
  TLS_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int) * c->n, s));
  TLS_HIP(hipMemsetAsync(cursor.p, 0, sizeof(int) * c->n, s));
  hipLaunchKernelGGL(k_count_cols, dim3(div_up(c->nnz, 256)), dim3(256), 0, s, c->nnz, c->col_idx.p, cnt.p);
  TLS_LAUNCH_CHECK();
  scan_exclusive_i32(cnt.p, c->trow_ptr.p, c->n, s);
  hipLaunchKernelGGL(k_fill_transpose, dim3(div_up(c->n, 256)), dim3(256), 0, s, c->n, c->row_ptr.p,
                     c->col_idx.p, c->trow_ptr.p, cursor.p, c->tcol_idx.p);
  TLS_LAUNCH_CHECK();
  TLS_HIP(hipStreamSynchronize(s));
}

void build_overlap(tls_ctx* c, DBuf<uint8_t>& dist) {
  hipStream_t s = c->stream;
  const int n = c->n, N = c->N, L = c->delta;
  const int stride = L + 2;
  dist.alloc((size_t)N * n);
  TLS_HIP(hipMemsetAsync(dist.p, UNSEEN, (size_t)N * n, s));
  hipLaunchKernelGGL(k_mark_interior, dim3(div_up(n, 256)), dim3(256), 0, s, n, c->part.p, dist.p);
  TLS_LAUNCH_CHECK();

  std::vector<std::vector<int>> cnt(L + 1, std::vector<int>(N));
  std::vector<DBuf<int>> lay(L + 1), lsub(L + 1), loff(L + 1);
  DBuf<int> dcnt;
  dcnt.alloc(N);
  const int* trp = c->kind == 1 ? c->trow_ptr.p : nullptr;
  const int* tci = c->kind == 1 ? c->tcol_idx.p : nullptr;
  for (int l = 0; l <= L; l++) {
    if (l > 0) {
      int prev = (int)lay[l - 1].n;
      if (prev > 0 && lay[l - 1].p) {
        int count = 0;
        for (int i = 0; i < N; i++) count += cnt[l - 1][i];
        if (count > 0)
          hipLaunchKernelGGL(k_expand, dim3(div_up(count, 256)), dim3(256), 0, s, count, lay[l - 1].p,
                             lsub[l - 1].p, n, c->row_ptr.p, c->col_idx.p, trp, tci, (uint8_t)l, dist.p);
        TLS_LAUNCH_CHECK();
      }
    }
    hipLaunchKernelGGL(k_level_count, dim3(N), dim3(256), 0, s, n, dist.p, (uint8_t)l, dcnt.p);
    TLS_LAUNCH_CHECK();
    cnt[l] = download(dcnt.p, N, s);
    std::vector<int> off(N + 1, 0);
    for (int i = 0; i < N; i++) off[i + 1] = off[i] + cnt[l][i];
    lay[l].alloc(off[N]);
    lsub[l].alloc(off[N]);
    loff[l].upload(off, s);
    hipLaunchKernelGGL(k_level_fill, dim3(N), dim3(256), 0, s, n, dist.p, (uint8_t)l, loff[l].p, lay[l].p,
                       lsub[l].p);
    TLS_LAUNCH_CHECK();
  }

  // layout of Omega_i
  c->h_sub_ptr.assign(N + 1, 0);
  c->h_layer_ptr.assign((size_t)N * stride, 0);
  c->h_m.resize(N);
  c->h_nI.resize(N);
  c->h_nP.resize(N);
  for (int i = 0; i < N; i++) {
    int pos = c->h_sub_ptr[i];
    for (int l = 0; l <= L; l++) {
      c->h_layer_ptr[(size_t)i * stride + l] = pos;
      pos += cnt[l][i];
    }
    c->h_layer_ptr[(size_t)i * stride + L + 1] = pos;
    c->h_sub_ptr[i + 1] = pos;
    c->h_m[i] = pos - c->h_sub_ptr[i];
    c->h_nI[i] = cnt[0][i];
    int np = 0;
    for (int l = 0; l < L; l++) np += cnt[l][i];
    c->h_nP[i] = L == 0 ? cnt[0][i] : np;
  }
  int total = c->h_sub_ptr[N];
  c->sub_ptr.upload(c->h_sub_ptr, s);
  c->layer_ptr.upload(c->h_layer_ptr, s);
  c->sub_idx.alloc(total);
  for (int l = 0; l <= L; l++) {
    int count = (int)lay[l].n;
    int real = 0;
    for (int i = 0; i < N; i++) real += cnt[l][i];
    if (real == 0) continue;
    (void)count;
    hipLaunchKernelGGL(k_place_level, dim3(div_up(real, 256)), dim3(256), 0, s, real, lay[l].p, lsub[l].p,
                       loff[l].p, c->layer_ptr.p, stride, l, c->sub_idx.p);
    TLS_LAUNCH_CHECK();
  }
  TLS_HIP(hipStreamSynchronize(s));
}

void build_layout(tls_ctx* c) {
  hipStream_t s = c->stream;
  const int N = c->N;
  c->h_nt.resize(N);
  c->h_foff.assign(N + 1, 0);
  c->h_voff.assign(N + 1, 0);
  c->h_toff.assign(N + 1, 0);
  c->sum_m = c->sum_m2 = 0;
  c->max_nt = 0;
  for (int i = 0; i < N; i++) {
    int m = c->h_m[i];
    int nt = div_up(m, TS);
    c->h_nt[i] = nt;
    c->max_nt = std::max(c->max_nt, nt);
    c->h_foff[i + 1] = c->h_foff[i] + tiles_of(c->kind, nt) * TS2;
    c->h_voff[i + 1] = c->h_voff[i] + (int64_t)nt * TS;
    c->h_toff[i + 1] = c->h_toff[i] + nt;
    c->sum_m += m;
    c->sum_m2 += (int64_t)m * m;
  }
  c->fac_elems = c->h_foff[N];
  c->sum_M = c->h_voff[N];
  c->sum_nt = c->h_toff[N];
  c->d_m.upload(c->h_m, s);
  c->d_nI.upload(c->h_nI, s);
  c->d_nP.upload(c->h_nP, s);
  c->d_nt.upload(c->h_nt, s);
  c->d_foff.upload(c->h_foff, s);
  c->d_voff.upload(c->h_voff, s);
  c->d_toff.upload(c->h_toff, s);

  // maps
  int total = c->h_sub_ptr[N];
  c->sub_of_pos.alloc(total);
  c->ipos.alloc(c->n);
  hipLaunchKernelGGL(k_sub_maps, dim3(N), dim3(256), 0, s, N, c->sub_ptr.p, c->d_nI.p, c->sub_idx.p,
                     c->sub_of_pos.p, c->ipos.p);
  TLS_LAUNCH_CHECK();
  DBuf<int> cnt, cursor;
  cnt.alloc(c->n);
  cursor.alloc(c->n);
  TLS_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int) * c->n, s));
  TLS_HIP(hipMemsetAsync(cursor.p, 0, sizeof(int) * c->n, s));
  hipLaunchKernelGGL(k_owner_count, dim3(div_up(total, 256)), dim3(256), 0, s, total, c->sub_idx.p, cnt.p);
  TLS_LAUNCH_CHECK();
  c->own_ptr.alloc(c->n + 1);
  scan_exclusive_i32(cnt.p, c->own_ptr.p, c->n, s);
  c->own_pos.alloc(total);
  hipLaunchKernelGGL(k_owner_fill, dim3(div_up(total, 256)), dim3(256), 0, s, total, c->sub_idx.p,
                     c->sub_of_pos.p, c->sub_ptr.p, c->d_voff.p, c->own_ptr.p, cursor.p, c->own_pos.p);
  TLS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_owner_sort, dim3(div_up(c->n, 256)), dim3(256), 0, s, c->n, c->own_ptr.p,
                     c->own_pos.p);
  TLS_LAUNCH_CHECK();
  TLS_HIP(hipStreamSynchronize(s));
}

}  // namespace tls
