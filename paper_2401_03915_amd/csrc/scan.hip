// Device exclusive prefix sums.
#include "scan.hpp"

namespace tls {

namespace {

constexpr int SCAN_T = 256;
constexpr int SCAN_PER = 4;
constexpr int SCAN_BLOCK = SCAN_T * SCAN_PER;  // elements per block

template <class T>
__device__ T block_exclusive_scan(T v, T* sh, T* total) {
  // Hillis-Steele over the 256 thread values in shared memory.
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_T; off <<= 1) {
    T add = (t >= off) ? sh[t - off] : T(0);
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  T incl = sh[t];
  if (total) *total = sh[SCAN_T - 1];
  __syncthreads();
  return incl - v;
}

template <class T>
__global__ void k_scan_blocks(const T* in, T* out, T* block_tot, int count) {
  __shared__ T sh[SCAN_T];
  int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_PER;
  T loc[SCAN_PER];
  T sum = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER; j++) {
    int64_t idx = base + j;
    loc[j] = idx < count ? in[idx] : T(0);
    sum += loc[j];
  }
  __shared__ T tot;
  T ex = block_exclusive_scan<T>(sum, sh, &tot);
#pragma unroll
  for (int j = 0; j < SCAN_PER; j++) {
    int64_t idx = base + j;
    if (idx < count) out[idx] = ex;
    ex += loc[j];
  }
  if (threadIdx.x == 0) block_tot[blockIdx.x] = tot;
}

template <class T>
__global__ void k_scan_add(T* out, const T* block_off, int count) {
  int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_PER;
  T add = block_off[blockIdx.x];
#pragma unroll
  for (int j = 0; j < SCAN_PER; j++) {
    int64_t idx = base + j;
    if (idx < count) out[idx] += add;
  }
}

template <class T>
__global__ void k_set_total(T* out, const T* block_off, int nblocks, int count) {
  out[count] = block_off[nblocks];
}

template <class T>
void scan_impl(const T* in, T* out, int count, hipStream_t s) {
  if (count <= 0) {
    TLS_HIP(hipMemsetAsync(out, 0, sizeof(T), s));
    return;
  }
  int nb = div_up(count, SCAN_BLOCK);
  DBuf<T> tot, off;
  tot.alloc(nb);
  off.alloc(nb + 1);
  hipLaunchKernelGGL(k_scan_blocks<T>, dim3(nb), dim3(SCAN_T), 0, s, in, out, tot.p, count);
  TLS_LAUNCH_CHECK();
  // block totals: recursive scan (nb < count / 1024)
  if (nb > 1)
    scan_impl<T>(tot.p, off.p, nb, s);
  else {
    TLS_HIP(hipMemsetAsync(off.p, 0, sizeof(T), s));
    TLS_HIP(hipMemcpyAsync(off.p + 1, tot.p, sizeof(T), hipMemcpyDeviceToDevice, s));
  }
  hipLaunchKernelGGL(k_scan_add<T>, dim3(nb), dim3(SCAN_T), 0, s, out, off.p, count);
  TLS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_set_total<T>, dim3(1), dim3(1), 0, s, out, off.p, nb, count);
  TLS_LAUNCH_CHECK();
  TLS_HIP(hipStreamSynchronize(s));  // temporaries are freed on return
}

}  // namespace

void scan_exclusive_i32(const int* in, int* out, int count, hipStream_t s) {
  scan_impl<int>(in, out, count, s);
}
void scan_exclusive_i64(const int64_t* in, int64_t* out, int count, hipStream_t s) {
  scan_impl<int64_t>(in, out, count, s);
}

}  // namespace tls
