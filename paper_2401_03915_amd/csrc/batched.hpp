// Batched small dense kernels shared by the coarse-basis and coarse-operator
// builders: variable-size MFMA GEMM and triangular solves with many
// right-hand sides.
#pragma once

#include "common.hpp"

namespace tls {

// C[m + n*ldc] = alpha * sum_k opA(m,k) opB(k,n) + beta * C[m + n*ldc]
// opA(m,k) = transA ? A[k + m*lda] : A[m + k*lda] (same for B).
// syrk = 1: only the output tiles on or below the block diagonal are formed
// (C symmetric; the caller mirrors the rest). kstart (device, optional):
// per 64-wide block b of the output's rows and columns, the first k with a
// nonzero in that block's operand column (opA(m, k) = opB(k, m) = 0 for
// k < kstart[m / 64]); a tile's K loop starts at the larger of its two.
struct GemmDesc {
  int M, N, K;
  int lda, ldb;
  int64_t a_off, b_off, c_off;
  int64_t ldc;
  int syrk = 0;
  const int* kstart = nullptr;
};

template <class T>
void batched_gemm(hipStream_t s, const std::vector<GemmDesc>& d, bool transA, bool transB, const T* A,
                  const T* B, T* C, T alpha, T beta);

// A descriptor list kept on the device for repeated launches (the buffers
// grow as needed and are reused). gemm_run does not synchronize.
struct GemmPlan {
  DBuf<GemmDesc> desc;
  DBuf<int64_t> pref;
  int nd = 0;
  int64_t tiles = 0;
};
void gemm_plan(GemmPlan& p, const std::vector<GemmDesc>& d, hipStream_t s);
template <class T>
void gemm_run(hipStream_t s, const GemmPlan& p, bool transA, bool transB, const T* A, const T* B, T* C, T alpha,
              T beta);

// In-place triangular solves with a column-major n x n triangular matrix
// (leading dimension n) and nrhs right-hand sides (leading dimension ldb):
//   LOWER_FWD: M lower, solve M X = B (forward substitution)
//   UPPER_BWD: M upper, solve M X = B (backward substitution)
enum TriMode { LOWER_FWD = 0, UPPER_BWD = 1 };
struct TriDesc {
  int n, nrhs;
  int64_t m_off, b_off;
  int64_t ldb;
};

template <class T>
void batched_trsm(hipStream_t s, const std::vector<TriDesc>& d, TriMode mode, const T* M, T* B, int* err);

}  // namespace tls
