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
#include "sort.hpp"

namespace tls {

namespace {

__global__ void k_validate(int n, int nnz, const int* __restrict__ rp, const int* __restrict__ ci,
                           const double* __restrict__ v, const int* __restrict__ part, int N,
                           int* err, int* part_count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int p = -1;
  if (i < n) {
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
    p = part[i];
    if (p < 0 || p >= N) {
      atomicOr(err, ERR_PART);
      p = -1;
    }
  }
  // rows of one wave mostly share their part: one atomic per distinct part
  // of the wave instead of one per row (the counters are few and hot)
  const int lane = threadIdx.x & 63;
  uint64_t left = __ballot(p >= 0);
  while (left) {
    const int lead = __builtin_ctzll(left);
    const int pl = __shfl(p, lead);
    const uint64_t same = __ballot(p == pl) & left;
    if (lane == lead) atomicAdd(&part_count[pl], __popcll(same));
    left &= ~same;
  }
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

// Level 0 keys: (part[v], v); v ascending on input, so a stable sort on
// the subdomain bits alone orders them by (subdomain, v).
__global__ void k_interior_keys(int n, const int* __restrict__ part, int sh, uint64_t* keys) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) keys[v] = ((uint64_t)part[v] << sh) | (uint64_t)v;
}

// Is u already in Omega_i at a level below the one being built? Level 0 is
// part[u] == i; levels 1 .. l-1 are ascending segments of their layer
// arrays (binary search).
__device__ inline bool already_in(int u, int i, const int* __restrict__ part, int levels,
                                  const int* const* __restrict__ lays, const int* const* __restrict__ offs) {
  if (part[u] == i) return true;
  for (int lv = 1; lv < levels; lv++) {
    const int* lay = lays[lv];
    int lo = offs[lv][i], hi = offs[lv][i + 1] - 1;
    if (lo > hi || u < lay[lo] || u > lay[hi]) continue;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (lay[mid] < u)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lay[lo] == u) return true;
  }
  return false;
}

// Breadth-first candidates of level l: every neighbor u (in A, and in A^T
// for general A) of a level-(l-1) entry (v, i) that is not yet in Omega_i,
// as the key (i, u). The first pass counts them per entry, the second
// writes them at the scanned offsets; duplicates are removed after the sort.
template <bool FILL>
__global__ void k_candidates(int count, const int* __restrict__ lay, const int* __restrict__ lsub,
                             const int* __restrict__ rp, const int* __restrict__ ci,
                             const int* __restrict__ trp, const int* __restrict__ tci,
                             const int* __restrict__ part, int levels, const int* const* __restrict__ lays,
                             const int* const* __restrict__ offs, int sh, int64_t* cnt,
                             const int64_t* __restrict__ cpos, uint64_t* keys) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const int v = lay[e], i = lsub[e];
  const uint64_t hi = (uint64_t)i << sh;
  int c = 0;
  int64_t at = FILL ? cpos[e] : 0;
  for (int j = rp[v]; j < rp[v + 1]; j++) {
    int u = ci[j];
    if (already_in(u, i, part, levels, lays, offs)) continue;
    if (FILL) keys[at + c] = hi | (uint64_t)u;
    c++;
  }
  if (trp) {
    for (int j = trp[v]; j < trp[v + 1]; j++) {
      int u = tci[j];
      if (already_in(u, i, part, levels, lays, offs)) continue;
      if (FILL) keys[at + c] = hi | (uint64_t)u;
      c++;
    }
  }
  if (!FILL) cnt[e] = c;
}

// 1 where a sorted key differs from its predecessor
__global__ void k_first_of_run(int count, const uint64_t* __restrict__ keys, int* flag) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) flag[k] = (k == 0 || keys[k] != keys[k - 1]) ? 1 : 0;
}

// Distinct sorted keys -> the layer (u ascending within each subdomain) and
// its subdomain ids.
__global__ void k_unpack_runs(int count, const uint64_t* __restrict__ keys, const int* __restrict__ pos, int sh,
                              int* lay, int* lsub) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  if (k == 0 || keys[k] != keys[k - 1]) {
    lay[pos[k]] = (int)(keys[k] & ((1ull << sh) - 1));
    lsub[pos[k]] = (int)(keys[k] >> sh);
  }
}

// Segment offsets of a layer grouped by ascending subdomain id:
// off[j] = first position with lsub >= j, off[N] = total.
__global__ void k_segment_offsets(int total, int N, const int* __restrict__ lsub, int* off) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  int prev = p == 0 ? -1 : lsub[p - 1];
  for (int j = prev + 1; j <= lsub[p]; j++) off[j] = p;
  if (p == total - 1)
    for (int j = lsub[p] + 1; j <= N; j++) off[j] = total;
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

namespace {

int bit_length(uint64_t x) {
  int b = 0;
  while (x) {
    b++;
    x >>= 1;
  }
  return b;
}

// Sorted keys -> one layer: distinct entries, their subdomain ids and the
// per-subdomain segment offsets (off has N + 1 entries). Returns the size.
int keys_to_layer(const uint64_t* keys, int count, int sh, int N, DBuf<int>& lay, DBuf<int>& lsub,
                  DBuf<int>& off, hipStream_t s) {
  off.alloc(N + 1);
  if (count == 0) {
    TLS_HIP(hipMemsetAsync(off.p, 0, sizeof(int) * (N + 1), s));
    lay.alloc(0);
    lsub.alloc(0);
    return 0;
  }
  DBuf<int> flag, pos;
  flag.alloc(count);
  pos.alloc((size_t)count + 1);
  hipLaunchKernelGGL(k_first_of_run, dim3(div_up(count, 256)), dim3(256), 0, s, count, keys, flag.p);
  TLS_LAUNCH_CHECK();
  scan_exclusive_i32(flag.p, pos.p, count, s);
  int total = 0;
  read_back(pos.p + count, &total, 1, s);
  lay.alloc(total);
  lsub.alloc(total);
  hipLaunchKernelGGL(k_unpack_runs, dim3(div_up(count, 256)), dim3(256), 0, s, count, keys, pos.p, sh, lay.p,
                     lsub.p);
  TLS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_segment_offsets, dim3(div_up(total, 256)), dim3(256), 0, s, total, N, lsub.p, off.p);
  TLS_LAUNCH_CHECK();
  TLS_HIP(hipStreamSynchronize(s));
  return total;
}

}  // namespace

// Omega_i layer by layer with O(sum_i #Omega_i) work and memory: a layer is
// the sorted, de-duplicated list of (i, u) keys generated from the previous
// layer's neighbors, less the entries already in Omega_i.
void build_overlap(tls_ctx* c) {
  hipStream_t s = c->stream;
  const int n = c->n, N = c->N, L = c->delta;
  const int stride = L + 2;
  const int sh = std::max(1, bit_length((uint64_t)(n - 1)));
  const int top = sh + std::max(1, bit_length((uint64_t)(N - 1)));

  std::vector<std::vector<int>> cnt(L + 1, std::vector<int>(N));
  std::vector<DBuf<int>> lay(L + 1), lsub(L + 1), loff(L + 1);
  std::vector<int> size(L + 1, 0);
  std::vector<int> h_off;
  const int* trp = c->kind == 1 ? c->trow_ptr.p : nullptr;
  const int* tci = c->kind == 1 ? c->tcol_idx.p : nullptr;
  // device tables of the layer arrays built so far (entry 0 unused)
  DBuf<const int*> lays_d, offs_d;
  std::vector<const int*> lays_h(L + 1, nullptr), offs_h(L + 1, nullptr);
  for (int l = 0; l <= L; l++) {
    DBuf<uint64_t> ka, kb;
    int count = 0;
    if (l == 0) {
      count = n;
      ka.alloc(n);
      kb.alloc(n);
      hipLaunchKernelGGL(k_interior_keys, dim3(div_up(n, 256)), dim3(256), 0, s, n, c->part.p, sh, ka.p);
      TLS_LAUNCH_CHECK();
    } else if (size[l - 1] > 0) {
      const int F = size[l - 1];
      lays_d.upload(lays_h, s);
      offs_d.upload(offs_h, s);
      DBuf<int64_t> ccnt, cpos;
      ccnt.alloc(F);
      cpos.alloc((size_t)F + 1);
      hipLaunchKernelGGL(k_candidates<false>, dim3(div_up(F, 256)), dim3(256), 0, s, F, lay[l - 1].p,
                         lsub[l - 1].p, c->row_ptr.p, c->col_idx.p, trp, tci, c->part.p, l, lays_d.p, offs_d.p,
                         sh, ccnt.p, nullptr, nullptr);
      TLS_LAUNCH_CHECK();
      scan_exclusive_i64(ccnt.p, cpos.p, F, s);
      int64_t total = 0;
      read_back(cpos.p + F, &total, 1, s);
      if (total >= INT32_MAX) fail(TLS_E_ARG, "overlap candidates exceed 2^31 entries");
      count = (int)total;
      ka.alloc(count);
      kb.alloc(count);
      if (count > 0) {
        hipLaunchKernelGGL(k_candidates<true>, dim3(div_up(F, 256)), dim3(256), 0, s, F, lay[l - 1].p,
                           lsub[l - 1].p, c->row_ptr.p, c->col_idx.p, trp, tci, c->part.p, l, lays_d.p,
                           offs_d.p, sh, nullptr, cpos.p, ka.p);
        TLS_LAUNCH_CHECK();
      }
    }
    // level 0 is ascending in u already: sort on the subdomain bits only
    uint64_t* sorted = radix_sort_u64(ka.p, kb.p, count, l == 0 ? sh : 0, top, s);
    size[l] = keys_to_layer(sorted, count, sh, N, lay[l], lsub[l], loff[l], s);
    h_off = download(loff[l].p, N + 1, s);
    for (int i = 0; i < N; i++) cnt[l][i] = h_off[i + 1] - h_off[i];
    lays_h[l] = lay[l].p;
    offs_h[l] = loff[l].p;
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
    if (size[l] == 0) continue;
    hipLaunchKernelGGL(k_place_level, dim3(div_up(size[l], 256)), dim3(256), 0, s, size[l], lay[l].p,
                       lsub[l].p, loff[l].p, c->layer_ptr.p, stride, l, c->sub_idx.p);
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
