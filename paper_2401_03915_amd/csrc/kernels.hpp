// Internal entry points between the library's translation units.
#pragma once

#include "context.hpp"

namespace tls {

// setup_index.hip: validation, A^T pattern, overlap layers and maps
void validate_input(tls_ctx* c);
void build_transpose(tls_ctx* c);
void build_overlap(tls_ctx* c);
void build_layout(tls_ctx* c);

// dense.hip: local matrices, batched factorization, triangular solves
void gather_local(tls_ctx* c);
void factor_local(tls_ctx* c);
void build_solve_tasks(tls_ctx* c);
// local solves on the padded vector buffer x (fp64 or fp32 per c->fp32)
// ev_begin / ev_mid / ev_end (may be null) are recorded right before the
// forward, between the forward and the backward, and right after the
// backward triangular-solve kernel
// option local_inverse: replace every local Cholesky factor by A_ii^{-1}
// (lower tiles, full symmetric diagonal tiles) and build the symmetric-product
// work list; local_solve uses it from then on
void form_local_inverse(tls_ctx* c);
// tiles read by one forward and one backward substitution (inside the
// profiles), and the lower tiles of all local factors
void solve_tile_counts(const tls_ctx* c, int64_t* fwd, int64_t* bwd, int64_t* lower);
// option local_inverse = 2: form the explicit inverses when the two
// substitutions would read more tiles than the product (all lower tiles)
bool inverse_pays(const tls_ctx* c);
// the same for N FP64 Cholesky factors in any tile layout (A_0), and the
// work list and product of the symmetric product over them
void form_inverse_f64(hipStream_t s, int N, const std::vector<int>& nt, const LocalLayout& lay, double* fac,
                      const double* dinv);
void build_symv_work(SymvWork& w, hipStream_t s, int N, const std::vector<int>& nt,
                     const std::vector<int64_t>& foff, const std::vector<int64_t>& voff, bool fp32, int block = 8);
void symv_solve_f64(hipStream_t s, SymvWork& w, const double* S, double* x, const int* done);
void local_solve(tls_ctx* c, const int* done, hipEvent_t ev_begin = nullptr, hipEvent_t ev_mid = nullptr,
                 hipEvent_t ev_end = nullptr);
// X_i <- U_II^{-1} X_i with the leading block (rows and columns I_i) of the
// local factor: U_II of the LU factor (general A) or L_II^T of the Cholesky
// factor (SPD), many right-hand sides. X_i (64 nq_i columns, column-major
// with leading dimension ldx, or M_i when ldx = 0, at xoff[i]) is
// overwritten on its rows I_i; rows beyond I_i must be zero in the tile that
// holds the last rows of I_i
void local_bsolve_interior(tls_ctx* c, float* X, const std::vector<int>& nq, const std::vector<int64_t>& xoff,
                           int64_t ldx);
void local_bsolve_interior(tls_ctx* c, double* X, const std::vector<int>& nq, const std::vector<int64_t>& xoff,
                           int64_t ldx);
// generic pieces reused for the coarse factor (always fp64)
// (dinv: inverses of the diagonal tiles, one per tile row, written as it goes)
void factor_tiles_f64(hipStream_t s, int N, const std::vector<int>& nt, const LocalLayout& lay,
                      double* fac, double* dinv, int* err);
// work list of one direction (bwd = descending block rows) in one of the
// dependency-safe task orderings (1 level, 2 normalized progress,
// 3 longest chain first)
void build_plan(SolvePlan& p, bool bwd, const std::vector<int>& nt, const std::vector<int64_t>& toff, int order,
                hipStream_t s, int rows = 1, const std::vector<int>* width = nullptr);
// mode: 0 L y = b (Cholesky), 1 L^T x = y, 2 unit-lower L y = b (LU), 3 U x = y
void trsv_f64(hipStream_t s, int mode, SolvePlan& p, int* counter, const int* epoch, const LocalLayout& lay,
              const double* fac, const double* dinv, double* x, int* err, const int* done, int grid);
// (re)build the local plans for a task ordering (order_b: the backward
// plan's, 0 = the same as the forward's)
void build_local_plans(tls_ctx* c, int order, int rows, int order_b = 0);
void solve_begin(hipStream_t s, int* counters, const int* done);

// eigen.hip: coarse basis (eq. gevpsvd / Section 6)
void build_coarse_basis(tls_ctx* c);

// coarse.hip: A_0 = Z^T A Z, its factorization, coarse correction
void build_coarse_operator(tls_ctx* c);
void coarse_restrict(tls_ctx* c, const double* r, const int* done);
void coarse_solve(tls_ctx* c, const int* done);

// gnn.hip: learned warm start of the eigensolver
void gnn_check_weights(int c_out);
int gnn_n_weights(int c_out);
void gnn_build_graph(tls_ctx* c);
// X (positions x c_out, FP32) into c->gnn_X; keep = also keep the messages for training
void gnn_forward(tls_ctx* c, const float* w_host, int c_out, bool keep);
// keep orthonormal bases of the eq. gevpsvd eigenvectors' rows Gamma_{i,delta}
void gnn_keep_targets(tls_ctx* c, const std::vector<int>& nT, const std::vector<int>& k, const double* wT,
                      const std::vector<int64_t>& woff);
double gnn_loss_grad(tls_ctx* c, const float* w_host, int c_out, float* grad_host);
// rows Gamma_{i,delta} of c->gnn_X (first c0 columns) -> FP64 nT_i x c0 blocks at off[i] (act[i] > 0 only)
void gnn_take_rows(tls_ctx* c, const std::vector<int>& nT, const std::vector<int>& act,
                   const std::vector<int64_t>& off, int c0, double* out);

// tune.hip: autotuned launch shapes (default / timed / cached)
// workgroup count and task order of the persistent solves
void choose_solve_grid(tls_ctx* c);
// block side of the symmetric product with the local inverses (after form_local_inverse)
void choose_symv_block(tls_ctx* c);
// the batched factorization with its panel width picked (gathers again per candidate)
void factor_local_tuned(tls_ctx* c);

// refine.hip: iterative refinement of the FP32 local solves (option local_refine)
void build_refine(tls_ctx* c);
// local_solve on xloc32/xloc64, then c->refine refinement steps against the
// FP64 right-hand sides in c->bref64; returns true when the solutions are in
// c->xref64 (FP64) instead of the local-precision buffer
bool local_solve_refined(tls_ctx* c, const int* done, hipEvent_t ev_begin = nullptr, hipEvent_t ev_mid = nullptr,
                         hipEvent_t ev_end = nullptr);

// apply.hip: z = M^{-1} r
void apply_precond(tls_ctx* c, const double* r, double* z, const int* done, bool profile = false);

// krylov.hip
void spmv(tls_ctx* c, const double* x, double* y, const int* done);
// y = f - A x
void spmv_residual(tls_ctx* c, const double* f, const double* x, double* y, const int* done);
// Reads the device error word (synchronizing the stream); if a triangular-solve
// wait ran past its spin limit since the last call, clears it and returns true.
bool take_wait_flag(tls_ctx* c);
// Device work of one Krylov solve: tls_solve takes it from buffers that the
// context keeps (allocated on first use), tls_solve_noalloc from a fixed
// scratch area.
struct KWork {
  double* kr = nullptr;        // vectors
  double* scal = nullptr;      // 16 scalars
  double* partial = nullptr;   // reduction partials
  unsigned* redctr = nullptr;  // blocks done in the current one-launch reduction (0 between launches)
  int* done = nullptr;         // [0] stop, [1] iterations, [2] converged, [3] breakdown
  double* hist = nullptr;      // ||r_k|| / ||b|| per iteration
  double* gm = nullptr;        // FGMRES Hessenberg matrix, rotations, g, y and partial columns
  int* gi = nullptr;           // FGMRES inner index and cycle end (4 ints)
  bool context_bufs = false;   // the context's own buffers: the captured graph and history apply
};
// Element counts of each KWork part for the context's solver and options.
struct KrylovNeeds {
  size_t kr = 0, partial = 0, gm = 0;
  int hist = 0;
};
KrylovNeeds krylov_needs(const tls_ctx* c);
void krylov_run(tls_ctx* c, const KWork& w, const double* b, double* x, double tol, int* iters, double* relres,
                bool* converged);
void krylov_solve(tls_ctx* c, const double* b, double* x, double tol, int* iters, double* relres,
                  bool* converged);

}  // namespace tls
