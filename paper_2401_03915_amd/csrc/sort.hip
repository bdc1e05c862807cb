// Stable LSD radix sort of 64-bit keys, one 8-bit digit per pass.
//
// A pass is three launches: per-tile digit histograms (digit-major, so the
// exclusive scan of the table gives every tile its output offset per
// digit), that scan, and a stable scatter. In the scatter each 64-wide
// wavefront ranks its keys among equal digits with eight ballots (the lanes
// that agree with a lane on every digit bit), the four waves of the block
// add their per-digit counts in LDS, and a running offset per digit carries
// the order from one 256-key round of the tile to the next, so keys leave
// in input order within each digit.
#include "sort.hpp"
#include "scan.hpp"

namespace tls {

namespace {

constexpr int RS_T = 256;                // threads per block (four waves)
constexpr int RS_PER = 16;               // rounds of 256 keys per tile
constexpr int RS_TILE = RS_T * RS_PER;   // keys per tile
constexpr int RS_BINS = 256;             // 8-bit digits

__global__ void __launch_bounds__(RS_T) k_radix_hist(const uint64_t* __restrict__ keys, int count, int shift,
                                                     int nb, int* __restrict__ hist) {
  __shared__ int h[RS_BINS];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_PER; r++) {
    const int64_t k = base + r * RS_T + threadIdx.x;
    if (k < count) atomicAdd(&h[(int)((keys[k] >> shift) & 0xFF)], 1);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(RS_T) k_radix_scatter(const uint64_t* __restrict__ in,
                                                        uint64_t* __restrict__ out, int count, int shift,
                                                        int nb, const int* __restrict__ off) {
  __shared__ int run[RS_BINS];
  __shared__ int wc[RS_T / 64][RS_BINS];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  run[t] = off[(size_t)t * nb + blockIdx.x];
#pragma unroll
  for (int q = 0; q < RS_T / 64; q++) wc[q][t] = 0;
  __syncthreads();
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_PER; r++) {
    const int64_t k = base + r * RS_T + t;
    const bool valid = k < count;
    const uint64_t key = valid ? in[k] : 0ull;
    const int d = (int)((key >> shift) & 0xFF);
    // lanes of this wave holding a valid key with the same digit
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; bit++) {
      const int set = (d >> bit) & 1;
      const uint64_t on = __ballot(set);
      same &= set ? on : ~on;
    }
    const int rank = __popcll(same & below);
    if (valid && rank == 0) wc[w][d] = __popcll(same);
    __syncthreads();
    if (valid) {
      int pos = run[d] + rank;
      for (int q = 0; q < w; q++) pos += wc[q][d];
      out[pos] = key;
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int q = 0; q < RS_T / 64; q++) {
      add += wc[q][t];
      wc[q][t] = 0;
    }
    run[t] += add;
    __syncthreads();
  }
}

}  // namespace

uint64_t* radix_sort_u64(uint64_t* a, uint64_t* b, int count, int lo_bit, int hi_bit, hipStream_t s) {
  if (count <= 1 || hi_bit <= lo_bit) return a;
  const int nb = div_up(count, RS_TILE);
  if ((int64_t)nb * RS_BINS >= INT32_MAX) fail(TLS_E_ARG, "sort too large");
  DBuf<int> hist, off;
  hist.alloc((size_t)nb * RS_BINS);
  off.alloc((size_t)nb * RS_BINS + 1);
  for (int shift = lo_bit; shift < hi_bit; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(RS_T), 0, s, a, count, shift, nb, hist.p);
    TLS_LAUNCH_CHECK();
    scan_exclusive_i32(hist.p, off.p, nb * RS_BINS, s);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(RS_T), 0, s, a, b, count, shift, nb, off.p);
    TLS_LAUNCH_CHECK();
    std::swap(a, b);
  }
  TLS_HIP(hipStreamSynchronize(s));
  return a;
}

}  // namespace tls
