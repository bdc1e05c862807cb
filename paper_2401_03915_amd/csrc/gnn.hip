// Learned warm start of the local eigensolver (not part of the paper).
//
// A small message-passing network on the graph of every local matrix A_ii
// guesses the dominant eigenvectors of eq. gevpsvd restricted to
// Gamma_{i,delta}; the subspace iteration then starts from that guess
// instead of a random block and still converges to the same tolerance.
//
// Network (all FP32), Omega_i in its local order [I, Gamma_1, .., Gamma_delta]:
//   edges   e_ab = |a_ab| / sqrt(|a_aa| |a_bb|) for a != b, (A_ii)_ab != 0
//   H_0     = [1, 1{a in I_i}, 1{a in Gamma_{i,delta}}, log10(|a_aa| / mean |a_bb|),
//              r_a0 .. r_a7], r_aj = 2 u - 1, u = (z >> 11) 2^-53, z = output
//              8a + j + 1 of SplitMix64 from state 0 (a = local index)
//   H_l     = tanh(E H_{l-1} Theta_l + H_{l-1} Phi_l + b_l),  l = 1..4, width 32
//   X       = H_4 Omega  (c_out columns)
// Loss of subdomain i against an orthonormal basis Q_i (#T x k_i) of the
// rows T = Gamma_{i,delta} of its top-k eigenvectors:
//   f_i = -(1/k_i) tr(G^{-1} B),  G = X_T^T X_T + EPS (tr(X_T^T X_T) / c) I,
//   B = X_T^T Q Q^T X_T,  EPS = 1e-3,
//   df_i/dX_T = -(2/k_i) (Q Q^T X_T G^{-1} - X_T T2 - (EPS / c) tr(T2) X_T),
//   T2 = G^{-1} B G^{-1}.
//
// Data layout: every node of every subdomain is one "position" p of the
// concatenated Omega lists (sub_idx order); node features and hidden
// states are row-major (p, channel). The graph is a CSR over positions.
// Kernels: the message (E H) is a gather over the node's CSR row, 32 lanes
// per node reading one 128-byte row of H per neighbour; the two 32 x 32
// products use weights staged in LDS. Weight gradients are reduced over
// nodes per workgroup, then over workgroups in a fixed order.
#include <algorithm>
#include <cmath>

#include "kernels.hpp"
#include "scan.hpp"

namespace tls {

namespace {

constexpr int HID = TLS_GNN_HIDDEN;
constexpr int NF = TLS_GNN_FEATURES;
constexpr int NR = TLS_GNN_RANDOM;  // random input channels (the last NR features)
constexpr double EPS = 1e-3;        // loss regularization
constexpr int NL = TLS_GNN_LAYERS;
constexpr int SLOTS = 256 / HID;  // nodes per workgroup pass
constexpr int GNN_BLOCKS = 1024;  // persistent workgroups of the node kernels
constexpr int CMAX = 64;          // largest c_out

// offsets of the weight blocks in the flat vector (see tls.h)
struct WOff {
  int th[NL], ph[NL], b[NL], om, total;
};
inline WOff woff(int c_out) {
  WOff o{};
  int x = 0, cin = NF;
  for (int l = 0; l < NL; l++) {
    o.th[l] = x;
    x += cin * HID;
    o.ph[l] = x;
    x += cin * HID;
    o.b[l] = x;
    x += HID;
    cin = HID;
  }
  o.om = x;
  o.total = x + HID * c_out;
  return o;
}

// position of global row g inside Omega_i (segments ascending), or -1
__global__ void k_gnn_diag(int total, const int* __restrict__ sub_idx, const int* __restrict__ rp,
                           const int* __restrict__ ci, const double* __restrict__ val, float* dg) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  int g = sub_idx[p];
  double d = 0.0;
  for (int j = rp[g]; j < rp[g + 1]; j++)
    if (ci[j] == g) d = fabs(val[j]);
  dg[p] = (float)d;
}

// mode 0: count the neighbours of each position; mode 1: write them
__global__ void k_gnn_edges(int mode, int total, const int* __restrict__ sub_idx, const int* __restrict__ sub_of_pos,
                            const int* __restrict__ layer_ptr, int stride, int nseg, const int* __restrict__ rp,
                            const int* __restrict__ ci, const double* __restrict__ val, const float* __restrict__ dg,
                            int* cnt, const int* __restrict__ gptr, int* gcol, float* gw) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  const int i = sub_of_pos[p];
  const int g = sub_idx[p];
  const int* lp = layer_ptr + (size_t)i * stride;
  int k = 0;
  const int base = mode ? gptr[p] : 0;
  const float sa = dg[p];
  for (int j = rp[g]; j < rp[g + 1]; j++) {
    const int c = ci[j];
    if (c == g) continue;
    const int q = find_local_pos(c, sub_idx, lp, nseg);
    if (q < 0) continue;
    if (mode) {
      const float sb = dg[q];
      gcol[base + k] = q;
      gw[base + k] = (sa > 0.f && sb > 0.f) ? (float)(fabs(val[j]) / sqrt((double)sa * (double)sb)) : 0.f;
    }
    k++;
  }
  if (!mode) cnt[p] = k;
}

// output counter + 1 of SplitMix64 started from state 0
__device__ inline uint64_t splitmix64(uint64_t counter) {
  uint64_t z = (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// features of every position of subdomain i (one workgroup per subdomain)
__global__ void k_gnn_features(const int* __restrict__ sub_ptr, const int* __restrict__ nI_,
                               const int* __restrict__ nP_, const float* __restrict__ dg, float* feat) {
  __shared__ double red[4];
  const int i = blockIdx.x;
  const int p0 = sub_ptr[i], m = sub_ptr[i + 1] - p0;
  const int nI = nI_[i], nP = nP_[i];
  double s = 0.0;
  for (int a = threadIdx.x; a < m; a += blockDim.x) s += (double)dg[p0 + a];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double mean = (red[0] + red[1] + red[2] + red[3]) / (double)max(m, 1);
  for (int a = threadIdx.x; a < m; a += blockDim.x) {
    float* f = feat + (int64_t)(p0 + a) * NF;
    const double d = (double)dg[p0 + a];
    f[0] = 1.f;
    f[1] = a < nI ? 1.f : 0.f;
    f[2] = a >= nP ? 1.f : 0.f;
    f[3] = (d > 0.0 && mean > 0.0) ? (float)log10(d / mean) : 0.f;
    for (int j = 0; j < NR; j++) {
      const uint64_t z = splitmix64((uint64_t)a * NR + j);
      f[NF - NR + j] = (float)((double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0);
    }
  }
}

// H_out = tanh(E H_in Theta + H_in Phi + b); M_out = E H_in (training)
template <int CIN>
__global__ void __launch_bounds__(256) k_gnn_layer(int total, const int* __restrict__ gptr,
                                                   const int* __restrict__ gcol, const float* __restrict__ gw,
                                                   const float* __restrict__ Hin, const float* __restrict__ W,
                                                   int oth, int oph, int ob, float* Mout, float* Hout) {
  __shared__ float sTh[CIN * HID], sPh[CIN * HID], sb[HID];
  __shared__ float sm[SLOTS][CIN], sh[SLOTS][CIN];
  const int tid = threadIdx.x, slot = tid / HID, o = tid % HID;
  for (int e = tid; e < CIN * HID; e += 256) {
    sTh[e] = W[oth + e];
    sPh[e] = W[oph + e];
  }
  if (tid < HID) sb[tid] = W[ob + tid];
  for (int g0 = blockIdx.x * SLOTS; g0 < total; g0 += gridDim.x * SLOTS) {
    const int p = g0 + slot;
    __syncthreads();
    if (p < total && o < CIN) {
      float msg = 0.f;
      for (int e = gptr[p]; e < gptr[p + 1]; e++) msg += gw[e] * Hin[(int64_t)gcol[e] * CIN + o];
      sm[slot][o] = msg;
      sh[slot][o] = Hin[(int64_t)p * CIN + o];
      if (Mout) Mout[(int64_t)p * CIN + o] = msg;
    }
    __syncthreads();
    if (p < total) {
      float z = sb[o];
#pragma unroll
      for (int c = 0; c < CIN; c++) z += sm[slot][c] * sTh[c * HID + o] + sh[slot][c] * sPh[c * HID + o];
      Hout[(int64_t)p * HID + o] = tanhf(z);
    }
  }
}

// X = H_4 Omega
__global__ void k_gnn_out(int total, int c_out, const float* __restrict__ H, const float* __restrict__ W, int oom,
                          float* X) {
  __shared__ float sOm[HID * CMAX];
  for (int e = threadIdx.x; e < HID * c_out; e += blockDim.x) sOm[e] = W[oom + e];
  __syncthreads();
  const int64_t n = (int64_t)total * c_out;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = x / c_out;
    const int j = (int)(x % c_out);
    const float* h = H + p * HID;
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < HID; c++) s += h[c] * sOm[c * c_out + j];
    X[x] = s;
  }
}

// dH_4 = dX Omega^T; partial dOmega = H_4^T dX per workgroup
__global__ void __launch_bounds__(256) k_gnn_out_bwd(int total, int c_out, const float* __restrict__ H,
                                                     const float* __restrict__ dX, const float* __restrict__ W,
                                                     int oom, float* dH, float* part) {
  __shared__ float sOm[HID * CMAX];
  __shared__ float sH[SLOTS][HID], sX[SLOTS][CMAX];
  const int tid = threadIdx.x, slot = tid / HID, o = tid % HID;
  for (int e = tid; e < HID * c_out; e += 256) sOm[e] = W[oom + e];
  constexpr int PER = HID * CMAX / 256;
  float acc[PER];
#pragma unroll
  for (int q = 0; q < PER; q++) acc[q] = 0.f;
  for (int g0 = blockIdx.x * SLOTS; g0 < total; g0 += gridDim.x * SLOTS) {
    const int p = g0 + slot;
    __syncthreads();
    sH[slot][o] = p < total ? H[(int64_t)p * HID + o] : 0.f;
    for (int j = o; j < c_out; j += HID) sX[slot][j] = p < total ? dX[(int64_t)p * c_out + j] : 0.f;
    __syncthreads();
    if (p < total) {
      float s = 0.f;
      for (int j = 0; j < c_out; j++) s += sX[slot][j] * sOm[o * c_out + j];
      dH[(int64_t)p * HID + o] = s;
    }
#pragma unroll
    for (int q = 0; q < PER; q++) {
      const int e = tid + 256 * q;  // entry (c, j) of the HID x c_out block
      if (e < HID * c_out) {
        const int c = e / c_out, j = e % c_out;
        float s = 0.f;
#pragma unroll
        for (int t = 0; t < SLOTS; t++) s += sH[t][c] * sX[t][j];
        acc[q] += s;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < PER; q++) {
    const int e = tid + 256 * q;
    if (e < HID * c_out) part[(int64_t)blockIdx.x * HID * c_out + e] = acc[q];
  }
}

// Backward of one layer. Given dH (of this layer's output H), writes
// dM = dZ Theta^T and dL = dZ Phi^T (the local part of dH_in), and per
// workgroup partial sums of dTheta = M^T dZ, dPhi = H_in^T dZ, db = sum dZ.
template <int CIN>
__global__ void __launch_bounds__(256) k_gnn_layer_bwd(int total, const float* __restrict__ dH,
                                                       const float* __restrict__ H, const float* __restrict__ M,
                                                       const float* __restrict__ Hin, const float* __restrict__ W,
                                                       int oth, int oph, float* dM, float* dL, float* part) {
  __shared__ float sTh[CIN * HID], sPh[CIN * HID];
  __shared__ float sdz[SLOTS][HID], sm[SLOTS][CIN], sh[SLOTS][CIN];
  __shared__ float sred[SLOTS][CIN][HID + 1];
  const int tid = threadIdx.x, slot = tid / HID, o = tid % HID;
  for (int e = tid; e < CIN * HID; e += 256) {
    sTh[e] = W[oth + e];
    sPh[e] = W[oph + e];
  }
  float aT[CIN], aP[CIN], aB = 0.f;
#pragma unroll
  for (int c = 0; c < CIN; c++) aT[c] = aP[c] = 0.f;
  for (int g0 = blockIdx.x * SLOTS; g0 < total; g0 += gridDim.x * SLOTS) {
    const int p = g0 + slot;
    __syncthreads();
    float dz = 0.f;
    if (p < total) {
      const float h = H[(int64_t)p * HID + o];
      dz = dH[(int64_t)p * HID + o] * (1.f - h * h);
    }
    sdz[slot][o] = dz;
    if (o < CIN) {
      sm[slot][o] = p < total ? M[(int64_t)p * CIN + o] : 0.f;
      sh[slot][o] = p < total ? Hin[(int64_t)p * CIN + o] : 0.f;
    }
    __syncthreads();
    if (p < total && o < CIN) {
      float s1 = 0.f, s2 = 0.f;
#pragma unroll
      for (int q = 0; q < HID; q++) {
        s1 += sdz[slot][q] * sTh[o * HID + q];
        s2 += sdz[slot][q] * sPh[o * HID + q];
      }
      dM[(int64_t)p * CIN + o] = s1;
      dL[(int64_t)p * CIN + o] = s2;
    }
#pragma unroll
    for (int c = 0; c < CIN; c++) {
      aT[c] += sm[slot][c] * dz;
      aP[c] += sh[slot][c] * dz;
    }
    aB += dz;
  }
  // reduce over the slots: dTheta, then dPhi, then db
  float* out = part + (int64_t)blockIdx.x * (2 * CIN * HID + HID);
  for (int which = 0; which < 2; which++) {
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CIN; c++) sred[slot][c][o] = which == 0 ? aT[c] : aP[c];
    __syncthreads();
    for (int e = tid; e < CIN * HID; e += 256) {
      const int c = e / HID, q = e % HID;
      float s = 0.f;
#pragma unroll
      for (int t = 0; t < SLOTS; t++) s += sred[t][c][q];
      out[which * CIN * HID + e] = s;
    }
  }
  __syncthreads();
  sred[slot][0][o] = aB;
  __syncthreads();
  if (tid < HID) {
    float s = 0.f;
#pragma unroll
    for (int t = 0; t < SLOTS; t++) s += sred[t][0][tid];
    out[2 * CIN * HID + tid] = s;
  }
}

// dH_in = dL + E^T dM (E is symmetric for the SPD matrices this runs on)
template <int CIN>
__global__ void k_gnn_spmm_add(int total, const int* __restrict__ gptr, const int* __restrict__ gcol,
                               const float* __restrict__ gw, const float* __restrict__ dM,
                               const float* __restrict__ dL, float* dHin) {
  const int64_t n = (int64_t)total * CIN;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = x / CIN;
    const int c = (int)(x % CIN);
    float s = dL[x];
    for (int e = gptr[p]; e < gptr[p + 1]; e++) s += gw[e] * dM[(int64_t)gcol[e] * CIN + c];
    dHin[x] = s;
  }
}

// out[e] (+)= sum over blocks of part[b * stride + e], fixed order
__global__ void k_gnn_reduce(int nblocks, int count, int64_t stride, const float* __restrict__ part, float* out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; b++) s += (double)part[(int64_t)b * stride + e];
  out[e] = (float)s;
}

// Loss and dX of one subdomain per workgroup (FP64 inside). Q_i is nT x k
// column-major at toff[i]; X rows T are the last nT positions of Omega_i.
// Work matrices (CMAX x CMAX, FP64) live in per-subdomain global scratch.
__global__ void __launch_bounds__(256) k_gnn_loss(const int* __restrict__ sub_ptr, const int* __restrict__ nT_,
                                                  const int* __restrict__ k_, const int64_t* __restrict__ toff,
                                                  const double* __restrict__ Q, const float* __restrict__ X, int c,
                                                  double scale, double* work, float* dX, double* floss, int* bad) {
  __shared__ int s_ok;
  const int i = blockIdx.x;
  double* G = work + (int64_t)i * 4 * CMAX * CMAX;  // G, then its inverse
  double* B = G + CMAX * CMAX;                      // B = A1^T A1, then G^{-1} B G^{-1}
  double* T2 = B + CMAX * CMAX;                     // B G^{-1}, then A1 G^{-1}
  double* A1 = T2 + CMAX * CMAX;                    // Q^T X_T (k x c)
  const int tid = threadIdx.x;
  const int nT = nT_[i], k = k_[i];
  if (k <= 0 || nT <= 0) {
    if (tid == 0) floss[i] = 0.0;
    return;
  }
  const int64_t r0 = sub_ptr[i + 1] - nT;  // first position of Gamma_{i,delta}
  const double* Qi = Q + toff[i];
  // G = X_T^T X_T, A1 = Q^T X_T
  for (int e = tid; e < c * c; e += 256) {
    const int a = e % c, b = e / c;
    double s = 0.0;
    for (int r = 0; r < nT; r++) s += (double)X[(r0 + r) * c + a] * (double)X[(r0 + r) * c + b];
    G[a + b * CMAX] = s;
  }
  for (int e = tid; e < k * c; e += 256) {
    const int a = e % k, b = e / k;
    double s = 0.0;
    for (int r = 0; r < nT; r++) s += Qi[r + (int64_t)a * nT] * (double)X[(r0 + r) * c + b];
    A1[a + b * CMAX] = s;
  }
  __syncthreads();
  for (int e = tid; e < c * c; e += 256) {
    const int a = e % c, b = e / c;
    double s = 0.0;
    for (int q = 0; q < k; q++) s += A1[q + a * CMAX] * A1[q + b * CMAX];
    B[a + b * CMAX] = s;
  }
  __syncthreads();
  // G <- G + EPS (tr G / c) I
  if (tid == 0) {
    double tr = 0.0;
    for (int a = 0; a < c; a++) tr += G[a + a * CMAX];
    for (int a = 0; a < c; a++) G[a + a * CMAX] += EPS * tr / c;
  }
  __syncthreads();
  // G^{-1} by Gauss-Jordan on the SPD matrix (no pivoting needed), one thread
  if (tid == 0) {
    int ok = 1;
    for (int j = 0; j < c && ok; j++) {
      const double d = G[j + j * CMAX];
      if (!(d > 0.0)) {
        ok = 0;
        break;
      }
      const double inv = 1.0 / d;
      for (int x = 0; x < c; x++) G[j + x * CMAX] *= inv;
      G[j + j * CMAX] = inv;
      for (int r = 0; r < c; r++) {
        if (r == j) continue;
        const double f = G[r + j * CMAX];
        if (f == 0.0) continue;
        for (int x = 0; x < c; x++) G[r + x * CMAX] -= f * G[j + x * CMAX];
        G[r + j * CMAX] = -f * inv;
      }
    }
    s_ok = ok;
  }
  __syncthreads();
  if (!s_ok) {
    for (int64_t x = tid; x < (int64_t)nT * c; x += 256) dX[r0 * c + x] = 0.f;
    if (tid == 0) {
      floss[i] = 0.0;
      atomicAdd(bad, 1);
    }
    return;
  }
  // T2 = G^{-1} B G^{-1}: first T2 = B G^{-1}, then G^{-1} T2 (into B)
  for (int e = tid; e < c * c; e += 256) {
    const int a = e % c, b = e / c;
    double s = 0.0;
    for (int q = 0; q < c; q++) s += B[a + q * CMAX] * G[q + b * CMAX];
    T2[a + b * CMAX] = s;
  }
  __syncthreads();
  // f = -(1/k) tr(G^{-1} B)
  if (tid == 0) {
    double tr = 0.0;
    for (int a = 0; a < c; a++)
      for (int q = 0; q < c; q++) tr += G[a + q * CMAX] * B[q + a * CMAX];
    floss[i] = -tr / k;
  }
  __syncthreads();
  for (int e = tid; e < c * c; e += 256) {
    const int a = e % c, b = e / c;
    double s = 0.0;
    for (int q = 0; q < c; q++) s += G[a + q * CMAX] * T2[q + b * CMAX];
    B[a + b * CMAX] = s;  // G^{-1} B G^{-1}
  }
  __syncthreads();
  for (int e = tid; e < k * c; e += 256) {
    const int a = e % k, b = e / k;
    double s = 0.0;
    for (int q = 0; q < c; q++) s += A1[a + q * CMAX] * G[q + b * CMAX];
    T2[a + b * CMAX] = s;  // A1 G^{-1} (k x c)
  }
  __syncthreads();
  // dX_T = -(2/k) scale (Q A1 G^{-1} - X_T G^{-1} B G^{-1} - (EPS/c) tr(G^{-1} B G^{-1}) X_T)
  double trT = 0.0;
  for (int a = 0; a < c; a++) trT += B[a + a * CMAX];
  const double f2 = -2.0 * scale / k;
  for (int64_t x = tid; x < (int64_t)nT * c; x += 256) {
    const int r = (int)(x / c), b = (int)(x % c);
    double s = 0.0;
    for (int q = 0; q < k; q++) s += Qi[r + (int64_t)q * nT] * T2[q + b * CMAX];
    for (int q = 0; q < c; q++) s -= (double)X[(r0 + r) * c + q] * B[q + b * CMAX];
    s -= (EPS / c) * trT * (double)X[(r0 + r) * c + b];
    dX[(r0 + r) * c + b] = (float)(f2 * s);
  }
}

// Orthonormalize each subdomain's target block (nT x k, column-major) by
// modified Gram-Schmidt, twice. Columns that vanish are set to zero and
// counted out of k.
__global__ void __launch_bounds__(256) k_gnn_orth_targets(const int* __restrict__ nT_, int* k_,
                                                          const int64_t* __restrict__ toff, double* Q) {
  __shared__ double red[4];
  const int i = blockIdx.x, tid = threadIdx.x;
  const int nT = nT_[i], k = k_[i];
  double* Qi = Q + toff[i];
  auto bsum = [&](double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
  };
  int kept = 0;
  for (int a = 0; a < k; a++) {
    double* v = Qi + (int64_t)a * nT;
    double n0 = 0.0;
    for (int r = tid; r < nT; r += 256) n0 += v[r] * v[r];
    n0 = sqrt(bsum(n0));
    for (int pass = 0; pass < 2; pass++)
      for (int b = 0; b < kept; b++) {
        const double* q = Qi + (int64_t)b * nT;
        double d = 0.0;
        for (int r = tid; r < nT; r += 256) d += q[r] * v[r];
        d = bsum(d);
        for (int r = tid; r < nT; r += 256) v[r] -= d * q[r];
        __syncthreads();
      }
    double nr = 0.0;
    for (int r = tid; r < nT; r += 256) nr += v[r] * v[r];
    nr = sqrt(bsum(nr));
    if (nr > 1e-8 * n0 && nr > 0.0) {
      double* dst = Qi + (int64_t)kept * nT;
      for (int r = tid; r < nT; r += 256) dst[r] = v[r] / nr;
      kept++;
    }
    __syncthreads();
  }
  if (tid == 0) k_[i] = kept;
}

// rows T of X (first c0 columns) -> fp64 block nT x c0 (column-major) at off[i]
__global__ void k_gnn_take_rows(const int* __restrict__ sub_ptr, const int* __restrict__ nT_,
                                const int* __restrict__ act, const int64_t* __restrict__ off,
                                const float* __restrict__ X, int c_out, int c0, double* out) {
  const int i = blockIdx.y;
  if (act[i] <= 0) return;
  const int nT = nT_[i];
  const int64_t r0 = sub_ptr[i + 1] - nT;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < (int64_t)nT * c0;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(x % nT), j = (int)(x / nT);
    out[off[i] + x] = (double)X[(r0 + r) * c_out + j];
  }
}

}  // namespace

void gnn_check_weights(int c_out) {
  // X = H_4 Omega has rank <= HIDDEN: more columns would be dependent
  if (c_out < 1 || c_out > HID) fail(TLS_E_ARG, "gnn c_out must be in [1, TLS_GNN_HIDDEN]");
}

int gnn_n_weights(int c_out) { return woff(c_out).total; }

void gnn_build_graph(tls_ctx* c) {
  if (c->gnn_graph) return;
  hipStream_t s = c->stream;
  const int total = c->h_sub_ptr[c->N];
  const int stride = c->delta + 2, nseg = c->delta + 1;
  DBuf<float> dg;
  DBuf<int> cnt;
  dg.alloc(total);
  cnt.alloc(total + 1);
  const dim3 g(div_up(total, 256));
  hipLaunchKernelGGL(k_gnn_diag, g, dim3(256), 0, s, total, c->sub_idx.p, c->row_ptr.p, c->col_idx.p, c->val.p,
                     dg.p);
  hipLaunchKernelGGL(k_gnn_edges, g, dim3(256), 0, s, 0, total, c->sub_idx.p, c->sub_of_pos.p, c->layer_ptr.p,
                     stride, nseg, c->row_ptr.p, c->col_idx.p, c->val.p, dg.p, cnt.p, nullptr, nullptr, nullptr);
  TLS_LAUNCH_CHECK();
  TLS_HIP(hipMemsetAsync(cnt.p + total, 0, sizeof(int), s));
  c->gnn_ptr.alloc(total + 1);
  scan_exclusive_i32(cnt.p, c->gnn_ptr.p, total + 1, s);
  int nnz = 0;
  TLS_HIP(hipMemcpyAsync(&nnz, c->gnn_ptr.p + total, sizeof(int), hipMemcpyDeviceToHost, s));
  TLS_HIP(hipStreamSynchronize(s));
  c->gnn_col.alloc(std::max(nnz, 1));
  c->gnn_w.alloc(std::max(nnz, 1));
  hipLaunchKernelGGL(k_gnn_edges, g, dim3(256), 0, s, 1, total, c->sub_idx.p, c->sub_of_pos.p, c->layer_ptr.p,
                     stride, nseg, c->row_ptr.p, c->col_idx.p, c->val.p, dg.p, nullptr, c->gnn_ptr.p, c->gnn_col.p,
                     c->gnn_w.p);
  TLS_LAUNCH_CHECK();
  c->gnn_feat.alloc((size_t)total * NF);
  hipLaunchKernelGGL(k_gnn_features, dim3(c->N), dim3(256), 0, s, c->sub_ptr.p, c->d_nI.p, c->d_nP.p, dg.p,
                     c->gnn_feat.p);
  TLS_LAUNCH_CHECK();
  TLS_HIP(hipStreamSynchronize(s));
  c->gnn_graph = true;
}

void gnn_forward(tls_ctx* c, const float* w_host, int c_out, bool keep) {
  gnn_check_weights(c_out);
  gnn_build_graph(c);
  hipStream_t s = c->stream;
  const int total = c->h_sub_ptr[c->N];
  const WOff o = woff(c_out);
  const std::vector<float> wv(w_host, w_host + o.total);
  c->gnn_wdev.upload(wv, s);
  TLS_HIP(hipStreamSynchronize(s));  // wv is a host temporary
  c->gnn_H.alloc((size_t)NL * total * HID);
  if (keep) c->gnn_M.alloc((size_t)NL * total * HID);
  c->gnn_X.alloc((size_t)total * c_out);
  const dim3 g(GNN_BLOCKS);
  for (int l = 0; l < NL; l++) {
    const float* Hin = l == 0 ? c->gnn_feat.p : c->gnn_H.p + (size_t)(l - 1) * total * HID;
    float* Hout = c->gnn_H.p + (size_t)l * total * HID;
    float* M = keep ? c->gnn_M.p + (size_t)l * total * HID : nullptr;
    if (l == 0)
      hipLaunchKernelGGL(k_gnn_layer<NF>, g, dim3(256), 0, s, total, c->gnn_ptr.p, c->gnn_col.p, c->gnn_w.p, Hin,
                         c->gnn_wdev.p, o.th[l], o.ph[l], o.b[l], M, Hout);
    else
      hipLaunchKernelGGL(k_gnn_layer<HID>, g, dim3(256), 0, s, total, c->gnn_ptr.p, c->gnn_col.p, c->gnn_w.p, Hin,
                         c->gnn_wdev.p, o.th[l], o.ph[l], o.b[l], M, Hout);
    TLS_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_gnn_out, g, dim3(256), 0, s, total, c_out, c->gnn_H.p + (size_t)(NL - 1) * total * HID,
                     c->gnn_wdev.p, o.om, c->gnn_X.p);
  TLS_LAUNCH_CHECK();
  c->gnn_cout = c_out;
}

void gnn_keep_targets(tls_ctx* c, const std::vector<int>& nT, const std::vector<int>& k, const double* wT,
                      const std::vector<int64_t>& woff_) {
  hipStream_t s = c->stream;
  const int N = c->N;
  c->h_gnn_toff.assign(N + 1, 0);
  for (int i = 0; i < N; i++) c->h_gnn_toff[i + 1] = c->h_gnn_toff[i] + (int64_t)nT[i] * k[i];
  c->gnn_tgt.alloc(std::max<int64_t>(c->h_gnn_toff[N], 1));
  for (int i = 0; i < N; i++)
    if (k[i] > 0)
      TLS_HIP(hipMemcpyAsync(c->gnn_tgt.p + c->h_gnn_toff[i], wT + woff_[i], sizeof(double) * nT[i] * k[i],
                             hipMemcpyDeviceToDevice, s));
  c->gnn_nT.upload(nT, s);
  c->gnn_k.upload(k, s);
  c->gnn_toff.upload(c->h_gnn_toff, s);
  hipLaunchKernelGGL(k_gnn_orth_targets, dim3(N), dim3(256), 0, s, c->gnn_nT.p, c->gnn_k.p, c->gnn_toff.p,
                     c->gnn_tgt.p);
  TLS_LAUNCH_CHECK();
  TLS_HIP(hipStreamSynchronize(s));
}

double gnn_loss_grad(tls_ctx* c, const float* w_host, int c_out, float* grad_host) {
  if (c->h_gnn_toff.empty()) fail(TLS_E_STATE, "no eq. gevpsvd targets: set up the context with gnn_train = 1");
  gnn_forward(c, w_host, c_out, true);
  hipStream_t s = c->stream;
  const int N = c->N;
  const int total = c->h_sub_ptr[N];
  const WOff o = woff(c_out);
  auto kk = download(c->gnn_k.p, N, s);
  int nact = 0;
  for (int v : kk) nact += v > 0;
  if (nact == 0) fail(TLS_E_STATE, "no subdomain has eq. gevpsvd targets");
  DBuf<float> dX, dH, dH2, dM, dL, part, grad;
  DBuf<double> floss;
  DBuf<int> bad;
  dX.alloc((size_t)total * c_out);
  TLS_HIP(hipMemsetAsync(dX.p, 0, sizeof(float) * total * c_out, s));
  floss.alloc(N);
  bad.alloc(1);
  TLS_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
  DBuf<double> work;
  work.alloc((size_t)N * 4 * CMAX * CMAX);
  hipLaunchKernelGGL(k_gnn_loss, dim3(N), dim3(256), 0, s, c->sub_ptr.p, c->gnn_nT.p, c->gnn_k.p, c->gnn_toff.p,
                     c->gnn_tgt.p, c->gnn_X.p, c_out, 1.0 / nact, work.p, dX.p, floss.p, bad.p);
  TLS_LAUNCH_CHECK();
  grad.alloc(o.total);
  const dim3 g(GNN_BLOCKS);
  const int64_t pstride = 2 * HID * HID + HID;  // largest per-block partial
  part.alloc((size_t)GNN_BLOCKS * std::max<int64_t>(pstride, (int64_t)HID * c_out));
  dH.alloc((size_t)total * HID);
  dH2.alloc((size_t)total * HID);
  dM.alloc((size_t)total * HID);
  dL.alloc((size_t)total * HID);
  const float* H4 = c->gnn_H.p + (size_t)(NL - 1) * total * HID;
  hipLaunchKernelGGL(k_gnn_out_bwd, g, dim3(256), 0, s, total, c_out, H4, dX.p, c->gnn_wdev.p, o.om, dH.p, part.p);
  TLS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gnn_reduce, dim3(div_up(HID * c_out, 256)), dim3(256), 0, s, GNN_BLOCKS, HID * c_out,
                     (int64_t)HID * c_out, part.p, grad.p + o.om);
  TLS_LAUNCH_CHECK();
  float* dHcur = dH.p;
  float* dHnext = dH2.p;
  for (int l = NL - 1; l >= 0; l--) {
    const float* H = c->gnn_H.p + (size_t)l * total * HID;
    const float* M = c->gnn_M.p + (size_t)l * total * HID;
    const float* Hin = l == 0 ? c->gnn_feat.p : c->gnn_H.p + (size_t)(l - 1) * total * HID;
    const int cin = l == 0 ? NF : HID;
    const int64_t ps = 2 * cin * HID + HID;
    if (l == 0)
      hipLaunchKernelGGL(k_gnn_layer_bwd<NF>, g, dim3(256), 0, s, total, dHcur, H, M, Hin, c->gnn_wdev.p, o.th[l],
                         o.ph[l], dM.p, dL.p, part.p);
    else
      hipLaunchKernelGGL(k_gnn_layer_bwd<HID>, g, dim3(256), 0, s, total, dHcur, H, M, Hin, c->gnn_wdev.p, o.th[l],
                         o.ph[l], dM.p, dL.p, part.p);
    TLS_LAUNCH_CHECK();
    // partial layout per block: dTheta (cin x HID), dPhi (cin x HID), db (HID)
    // -- the same order as the flat weights th, ph, b of layer l
    hipLaunchKernelGGL(k_gnn_reduce, dim3(div_up(ps, 256)), dim3(256), 0, s, GNN_BLOCKS, (int)ps, ps, part.p,
                       grad.p + o.th[l]);
    TLS_LAUNCH_CHECK();
    if (l > 0) {
      hipLaunchKernelGGL(k_gnn_spmm_add<HID>, g, dim3(256), 0, s, total, c->gnn_ptr.p, c->gnn_col.p, c->gnn_w.p,
                         dM.p, dL.p, dHnext);
      TLS_LAUNCH_CHECK();
      std::swap(dHcur, dHnext);
    }
  }
  auto h_loss = download(floss.p, N, s);
  auto h_grad = download(grad.p, o.total, s);
  std::copy(h_grad.begin(), h_grad.end(), grad_host);
  double L = 0.0;
  for (double v : h_loss) L += v;
  return L / nact;
}

void gnn_take_rows(tls_ctx* c, const std::vector<int>& nT, const std::vector<int>& act, const std::vector<int64_t>& off,
                   int c0, double* out) {
  hipStream_t s = c->stream;
  DBuf<int> d_nT, d_act;
  DBuf<int64_t> d_off;
  d_nT.upload(nT, s);
  d_act.upload(act, s);
  d_off.upload(off, s);
  hipLaunchKernelGGL(k_gnn_take_rows, dim3(64, c->N), dim3(256), 0, s, c->sub_ptr.p, d_nT.p, d_act.p, d_off.p,
                     c->gnn_X.p, c->gnn_cout, c0, out);
  TLS_LAUNCH_CHECK();
  TLS_HIP(hipStreamSynchronize(s));
}

}  // namespace tls
