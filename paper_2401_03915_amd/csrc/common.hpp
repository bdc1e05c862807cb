// Shared definitions of the two-level Schwarz library (gfx950, HIP).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "tls.h"

namespace tls {

// ---------------------------------------------------------------------------
// Errors. Internal code throws TlsError; the C ABI converts it to a status.
// ---------------------------------------------------------------------------
struct TlsError {
  tls_status code;
  std::string msg;
};

[[noreturn]] inline void fail(tls_status code, const std::string& msg) { throw TlsError{code, msg}; }

#define TLS_HIP(call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      ::tls::fail(TLS_E_HIP, std::string(#call) + " failed: " + hipGetErrorString(e_));    \
  } while (0)

#define TLS_LAUNCH_CHECK() TLS_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// Large device blocks (>= 32 MiB) are kept for reuse instead of being freed.
// Freeing and allocating again the tens of GB a setup uses slowed the
// kernels of the following setups several-fold (freed device memory is
// cleared in the background and mapped again on the next allocation). The
// blocks are kept per device. A request takes the smallest kept block that
// holds it and is at most 1.25 times its size, else new memory; when the
// device has no room left it takes any kept block that holds it (the set-up
// that freed the blocks of one size often asks for slightly different
// sizes next time), and only then are kept blocks freed, the largest first,
// until the allocation succeeds. Each block handed out remembers its real
// size, so a larger block returns to the pool whole. Releasing a large
// block waits for the device, as freeing it would, so no queued work still
// uses it when it is handed out again.
// ---------------------------------------------------------------------------
namespace devmem {
constexpr size_t kMin = size_t(32) << 20;
constexpr size_t kGrain = size_t(2) << 20;

struct Pool {
  std::mutex mu;
  std::map<int, std::multimap<size_t, void*>> free;  // device -> (size, block)
  std::map<void*, size_t> used;                      // large block in use -> its real size
};
inline Pool& pool() {
  static Pool* p = new Pool;  // never destroyed: buffers may be released during process teardown
  return *p;
}
// Sizes of 1 GiB and more are rounded up to whole 256 MiB: a set-up run
// again asks for sizes that differ by a fraction of a percent (its groups
// of subdomains can shift by one), which then still match the kept blocks.
inline size_t rounded(size_t bytes) {
  const size_t g = bytes >= (size_t(1) << 30) ? size_t(256) << 20 : kGrain;
  return (bytes + g - 1) / g * g;
}

inline void trim() {
  Pool& pl = pool();
  std::lock_guard<std::mutex> lock(pl.mu);
  for (auto& d : pl.free)
    for (auto& b : d.second) (void)hipFree(b.second);
  pl.free.clear();
}

inline hipError_t alloc(void** p, size_t bytes) {
  if (bytes < kMin) return hipMalloc(p, bytes);
  const size_t want = rounded(bytes);
  int dev = 0;
  (void)hipGetDevice(&dev);
  Pool& pl = pool();
  // a kept block of at least `want` bytes and at most `most` (under the lock)
  auto take = [&](size_t most) {
    auto& fl = pl.free[dev];
    auto it = fl.lower_bound(want);
    if (it == fl.end() || it->first > most) return false;
    *p = it->second;
    pl.used[it->second] = it->first;
    fl.erase(it);
    return true;
  };
  {
    std::lock_guard<std::mutex> lock(pl.mu);
    if (take(want + want / 4)) return hipSuccess;  // no large block for a much smaller request
  }
  hipError_t e = hipMalloc(p, want);
  while (e != hipSuccess) {
    (void)hipGetLastError();
    std::lock_guard<std::mutex> lock(pl.mu);
    if (take(SIZE_MAX)) return hipSuccess;
    auto& fl = pl.free[dev];
    if (fl.empty()) break;
    auto last = std::prev(fl.end());
    (void)hipFree(last->second);
    fl.erase(last);
    e = hipMalloc(p, want);
  }
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> lock(pl.mu);
    pl.used[*p] = want;
  }
  return e;
}

// Free kept blocks of the current device, the smallest first, until the
// driver has `frac` of the device's memory free again (or none are kept):
// other allocators of the process (the framework that holds the inputs)
// must still find room after a context is gone.
inline void keep_headroom(double frac) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  Pool& pl = pool();
  std::lock_guard<std::mutex> lock(pl.mu);
  auto& fl = pl.free[dev];
  while (!fl.empty()) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();
      return;
    }
    if ((double)fr >= frac * (double)tot) return;
    (void)hipFree(fl.begin()->second);
    fl.erase(fl.begin());
  }
}

// Bytes that allocations on the current device can still obtain: what the
// driver reports free plus the blocks kept here for reuse, capped by the
// environment variable TLS_MEMORY_LIMIT (bytes) when it is set. Set-up steps
// that can work on groups of subdomains size their groups by it.
inline size_t available() {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  {
    Pool& pl = pool();
    std::lock_guard<std::mutex> lock(pl.mu);
    for (const auto& b : pl.free[dev]) fr += b.first;
  }
  if (const char* lim = std::getenv("TLS_MEMORY_LIMIT")) {
    const unsigned long long v = std::strtoull(lim, nullptr, 10);
    if (v > 0 && v < fr) fr = (size_t)v;
  }
  return fr;
}

// The memory a step that works on groups of subdomains may plan for: 90%
// of available(), rounded down to whole 8 GiB once that is 64 GiB or more,
// so that a set-up run again in the same process cuts the same groups
// (and finds its kept blocks) though other allocators hold a little more.
inline size_t budget() {
  const double b = 0.9 * (double)available();
  const double q = (double)(size_t(8) << 30);
  return b >= 8.0 * q ? (size_t)(std::floor(b / q) * q) : (size_t)b;
}

inline void release(void* p, size_t bytes) {
  if (bytes < kMin) {
    (void)hipFree(p);
    return;
  }
  (void)hipDeviceSynchronize();
  int dev = 0;
  (void)hipGetDevice(&dev);
  Pool& pl = pool();
  std::lock_guard<std::mutex> lock(pl.mu);
  auto it = pl.used.find(p);
  size_t size = rounded(bytes);
  if (it != pl.used.end()) {
    size = it->second;
    pl.used.erase(it);
  }
  pl.free[dev].insert({size, p});
}
}  // namespace devmem

// ---------------------------------------------------------------------------
// Device buffer owned by a context (released on destruction).
// ---------------------------------------------------------------------------
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) devmem::release(p, n * sizeof(T));
    p = nullptr;
    n = 0;
  }
  void swap(DBuf& o) {
    std::swap(p, o.p);
    std::swap(n, o.n);
  }
  void alloc(size_t count) {
    release();
    if (count == 0) count = 1;
    hipError_t e = devmem::alloc(reinterpret_cast<void**>(&p), count * sizeof(T));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      fail(TLS_E_NOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    n = count;
  }
  void upload(const std::vector<T>& h, hipStream_t s) {
    alloc(h.size());
    if (!h.empty()) TLS_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  }
  operator T*() const { return p; }
};

template <class T>
inline void read_back(const T* d, T* h, size_t count, hipStream_t s) {
  if (count) {
    TLS_HIP(hipMemcpyAsync(h, d, count * sizeof(T), hipMemcpyDeviceToHost, s));
    TLS_HIP(hipStreamSynchronize(s));
  }
}

template <class T>
inline std::vector<T> download(const T* d, size_t count, hipStream_t s) {
  std::vector<T> h(count);
  if (count) {
    TLS_HIP(hipMemcpyAsync(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, s));
    TLS_HIP(hipStreamSynchronize(s));
  }
  return h;
}

// ---------------------------------------------------------------------------
// Dense tile storage of the local factors.
//
// Subdomain i of padded size M_i = nt_i * TS is stored as square TS x TS
// tiles, column-major inside a tile. SPD (Cholesky): only the lower tiles
// (r >= c), packed row by row: tile (r, c) has index r(r+1)/2 + c. General
// (LU): all nt_i^2 tiles, index r * nt_i + c. The padding rows/columns hold
// the identity, so the factor of the padded matrix is diag(L, I).
// ---------------------------------------------------------------------------
constexpr int TS = 64;
constexpr int TS2 = TS * TS;

__host__ __device__ inline int64_t tile_index(int kind, int nt, int r, int c) {
  return kind == 0 ? (int64_t)r * (r + 1) / 2 + c : (int64_t)r * nt + c;
}
__host__ __device__ inline int64_t tiles_of(int kind, int nt) {
  return kind == 0 ? (int64_t)nt * (nt + 1) / 2 : (int64_t)nt * nt;
}
// element (a, b) of the padded local matrix stored at base
template <class T>
__device__ inline T* elem_ptr(T* base, int kind, int nt, int a, int b) {
  return base + tile_index(kind, nt, a / TS, b / TS) * TS2 + (b % TS) * TS + (a % TS);
}

// Position of global row g in the concatenated Omega lists of one
// subdomain, given the absolute starts of its nseg ascending segments
// (I_i, Gamma_1, ..., Gamma_delta) in lp[0..nseg]; -1 if g is not in Omega_i.
__device__ inline int find_local_pos(int g, const int* __restrict__ sub_idx, const int* __restrict__ lp, int nseg) {
  for (int d = 0; d < nseg; d++) {
    int lo = lp[d], hi = lp[d + 1] - 1;
    if (lo > hi) continue;
    if (g < sub_idx[lo] || g > sub_idx[hi]) continue;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (sub_idx[mid] < g)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (sub_idx[lo] == g) return lo;
  }
  return -1;
}

// Per-subdomain layout table shared by the factor, the solves and the
// eigensolver (device copy of host vectors).
struct LocalLayout {
  const int* m;        // #Omega_i
  const int* nI;       // #I_i
  const int* nP;       // #Omega_{i,1:delta-1}
  const int* nt;       // tiles per side
  const int64_t* foff; // element offset of the factor of i
  const int64_t* voff; // offset of i's padded vector (M_i entries)
  const int64_t* toff; // offset of i's first tile row in the flag arrays (= sum nt_j)
  // Profile storage (null: every tile of the packed lower triangle, or of
  // the full square for LU, is stored). With it, tile row r keeps only its
  // tiles from column prof[toff_i + r] to the diagonal, tile (r, c) at tile
  // trow[toff_i + r] + c of the subdomain's storage; for LU the tiles
  // strictly above the diagonal are kept by columns, column c from row
  // profc[toff_i + c], tile (r, c) at tile tcol[toff_i + c] + r.
  const int64_t* trow = nullptr;
  const int64_t* tcol = nullptr;
  const int* prof = nullptr;
  const int* profc = nullptr;
};

// Element offset of tile (r, c) inside subdomain i's factor storage (the
// tile must be stored: inside the profiles, or any tile without them).
__device__ inline int64_t tile_off(const LocalLayout& lay, int i, int kind, int nt, int r, int c) {
  if (!lay.trow) return tile_index(kind, nt, r, c) * TS2;
  const int64_t t0 = lay.toff[i];
  if (kind == 0 || r >= c) return (lay.trow[t0 + r] + c) * TS2;
  return (lay.tcol[t0 + c] + r) * TS2;
}
// Is tile (r, c) stored (always, without profile storage)?
__device__ inline bool tile_in(const LocalLayout& lay, int i, int kind, int r, int c) {
  if (!lay.trow) return true;
  const int64_t t0 = lay.toff[i];
  if (kind == 0 || r >= c) return c >= lay.prof[t0 + r];
  return r >= lay.profc[t0 + c];
}
// element (a, b) of subdomain i's padded local matrix (its tile must be stored)
template <class T>
__device__ inline T* elem_ptr_l(T* base, const LocalLayout& lay, int i, int kind, int nt, int a, int b) {
  return base + tile_off(lay, i, kind, nt, a / TS, b / TS) + (b % TS) * TS + (a % TS);
}

// Work list of the symmetric product with explicit inverses (block and row
// descriptors in 16-byte words) and its row and column partial sums.
struct SymvWork {
  DBuf<int4> blocks, rows;
  int64_t nblocks = 0, nrows = 0;
  int block = 8;  // block side in tiles (8, or 4 for a single matrix that needs more workgroups)
  DBuf<float> RP32, CP32;
  DBuf<double> RP64, CP64;
};

// Work list of one persistent triangular-solve launch: task (x = i, y = r)
// is block row r of subdomain i; flags[toff_i + r] holds the epoch of the
// last solve that finished that block row. `order` records the ordering.
struct SolvePlan {
  DBuf<int4> tasks;
  int ntasks = 0;
  DBuf<int> flags;
  int order = 0;
  int rows = 1;   // block rows per task (1: k_trsv, more: k_trsv_sr)
  int early = 0;  // tasks handed out ahead of their dependencies (the grid exceeds this)
};

// Error bits reported by kernels into a device int.
enum : int {
  ERR_CSR = 1,
  ERR_PART = 2,
  ERR_NAN = 4,
  ERR_PIVOT = 8,
  ERR_WAIT = 16,
  ERR_EIG = 32,
};

inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace tls
