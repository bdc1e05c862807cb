/*
 * tls.h - C ABI of the two-level additive Schwarz library for MI355X (gfx950).
 *
 * Method: Al Daas, Jolivet, Nataf, Tournier, "A robust two-level Schwarz
 * preconditioner for sparse matrices" (arXiv 2401.03915). The library builds,
 * for a sparse A, a nonoverlapping partition and an overlap width delta, the
 * preconditioner
 *
 *     M^{-1} r = sum_i R_i^T A_ii^{-1} R_i r + R_0^T A_00^{-1} R_0 r
 *
 * (Remark in Section 4.3; one-level part eq. onelevelasm), with the
 * coarse space of eq. coarse_space_2 for SPD A (dominant eigenvectors of
 * eq. gevpsvd, optionally of eq. uppergevp) or of Section 6 for general A
 * (dominant left singular vectors of D_i Pi_i), and applies it inside PCG or
 * right-preconditioned flexible GMRES (Section 7.2).
 *
 * Conventions for every entry point:
 *  - Indices are 0-based int32. CSR columns are sorted and unique in every
 *    row; A is square n x n; part[j] is in [0, n_parts) and every part is
 *    non-empty.
 *  - Matrix and vector pointers passed to tls_setup, tls_apply, tls_solve
 *    and tls_spmv are DEVICE pointers (memory allocated on the current HIP
 *    device, e.g. by PyTorch). The library never frees caller memory and
 *    keeps no pointer to it after the call returns: tls_setup deep-copies A
 *    and part.
 *  - All work is ordered on tls_options.stream (a hipStream_t). NULL makes
 *    the context create its own blocking stream, which the legacy default
 *    stream waits for and vice versa. tls_setup and tls_solve return after the stream
 *    has finished their work; tls_apply and tls_spmv are asynchronous on the
 *    stream.
 *  - Errors: every call returns a tls_status; no C++ exception crosses the
 *    ABI. A per-context message is available from tls_last_error. On a
 *    setup failure *out is set to NULL and the reason is available from
 *    tls_last_error(NULL) (thread-local).
 *  - The context is not thread safe: calls on one context must not overlap.
 */
#ifndef TLS_H
#define TLS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tls_ctx tls_ctx;

/* Learned warm start of the local eigensolver (not part of the paper).
 * A message-passing network on the graph of each A_ii (edges
 * e_ab = |a_ab| / sqrt(|a_aa| |a_bb|), 12 input features per node: 1,
 * in I_i, in Gamma_{i,delta}, log10 of the relative diagonal, and
 * TLS_GNN_RANDOM uniform [-1, 1) channels from SplitMix64: channel j of
 * local node a is 2 (z >> 11) 2^-53 - 1 with z the output 8a + j + 1 from
 * state 0) with
 * TLS_GNN_LAYERS layers of width TLS_GNN_HIDDEN,
 * H_l = tanh(E H_{l-1} Theta_l + H_{l-1} Phi_l + b_l), and a linear read-out
 * X = H_L Omega of c_out columns, predicts the rows Gamma_{i,delta} of the
 * eq. gevpsvd eigenvectors; the subspace iteration starts from it.
 * Weights are one FP32 vector: for each layer Theta_l (c_{l-1} x HIDDEN,
 * row major), Phi_l (same), b_l (HIDDEN); then Omega (HIDDEN x c_out);
 * c_0 = TLS_GNN_FEATURES. */
#define TLS_GNN_LAYERS 4
#define TLS_GNN_RANDOM 8
#define TLS_GNN_FEATURES 12
#define TLS_GNN_HIDDEN 32
#define TLS_GNN_NWEIGHTS(c_out)                                              \
  (2 * TLS_GNN_FEATURES * TLS_GNN_HIDDEN + TLS_GNN_HIDDEN +                  \
   (TLS_GNN_LAYERS - 1) * (2 * TLS_GNN_HIDDEN * TLS_GNN_HIDDEN + TLS_GNN_HIDDEN) + \
   TLS_GNN_HIDDEN * (c_out))

typedef enum {
  TLS_OK = 0,
  TLS_E_ARG = 1,       /* invalid argument or malformed input              */
  TLS_E_NOT_SPD = 2,   /* non-positive pivot in a Cholesky factorization    */
  TLS_E_SINGULAR = 3,  /* zero (or non-finite) pivot in an LU factorization */
  TLS_E_NOCONV = 4,    /* Krylov solver hit maxit; best iterate returned    */
  TLS_E_NOMEM = 5,     /* device allocation failed                          */
  TLS_E_HIP = 6,       /* a HIP runtime call failed                         */
  TLS_E_STATE = 7      /* call not valid for this context (e.g. NULL ctx)   */
} tls_status;

typedef struct {
  /* 0: every local and global quantity in FP64.
   * 1: local factorizations, triangular solves and the local eigensolver in
   *    FP32 (FP32 accumulation); SpMV, Krylov vectors, dot products, the
   *    coarse basis, A_0 and its factor stay FP64. */
  int32_t precision;
  /* 0: A is SPD: Cholesky, eq. gevpsvd (+ eq. uppergevp if nev1 > 0), PCG.
   * 1: general A: local LU without pivoting (nonzero pivots are needed:
   *    e.g. M-matrices, or quasi-definite saddle points [[A, B^T], [B, -C]]
   *    with A and C positive definite), LU with partial pivoting for A_0,
   *    Section 6 SVD variant, FGMRES.                                     */
  int32_t matrix_kind;
  /* eq. uppergevp vectors kept per subdomain (those with lambda > nu),
   * SPD only (TLS_E_ARG with matrix_kind 1). The paper's SPD experiments
   * use none (Section 7); default 0. */
  int32_t nev1;
  /* Thresholds: keep lambda^2 > tau^2 (eq. gevpsvd) or sigma > tau
   * (Section 6), and lambda > nu (eq. uppergevp), each capped by the
   * count. tau <= 0 means "count only"; nu defaults to 1. */
  double tau;
  double nu;
  int32_t restart;      /* FGMRES restart length m (default 30)            */
  int32_t maxit;        /* Krylov iteration cap (default 1000; 3000 general) */
  int32_t eig_maxit;    /* local subspace-iteration cap (default 300)      */
  double eig_tol;       /* relative eigen-residual tolerance (default 1e-9 FP64, 1e-5 FP32);
                           a residual below 10x that which stalls is accepted */
  int32_t eig_oversample; /* subspace block p = min(k + oversample, 48), k = min(nev, 40)
                             (eq. gevpsvd) or min(nev1, 40) (eq. uppergevp), so at most
                             40 vectors per subdomain and eigenproblem; default (-1): k */
  uint64_t seed;        /* seed of the counter-based start vectors         */
  int32_t use_graph;    /* capture Krylov iteration chunks in a hipGraph   */
  int32_t flexible;     /* PCG: Polak-Ribiere beta (default: 1 iff precision == 1) */
  int32_t jacobi_scale; /* symmetric diagonal scaling of each A_ii before factoring */
  int32_t profile;      /* tls_apply times its local triangular-solve kernels with HIP
                           events (and then waits for them); see tls_info_t */
  int32_t solve_wgs;    /* workgroups of the persistent triangular solves (0 = default) */
  int32_t solve_order;  /* task order of those solves: 1 level by level, 2 by the fraction of
                           the subdomain's rows done, 3 longest chain first, 4 / 5 as 2 with a
                           lead of 0.3 / 0.6 x nt_i / max nt for large subdomains; 0 = default (4);
                           when set, both directions use it */
  int32_t autotune;     /* 1: at setup, time candidates and keep the fastest: the panel width of
                           the batched factorization (4, 8 or 16 tiles), the block side of the
                           product with the local inverses (4, 6 or 8 tiles), and the workgroup
                           count, rows per task and, per direction, the task order of the
                           persistent solves (not when solve_wgs or solve_order is set) */
  const char* tune_cache; /* text file of earlier autotune picks (read, then appended);
                             NULL = no persistence. A cached pick is reused without timing. */
  /* Learned warm start (SPD only): host array of TLS_GNN_NWEIGHTS(gnn_c_out)
   * floats, read during tls_setup; NULL = random start (default). The first
   * min(gnn_c_out, p) columns of the eq. gevpsvd start block come from the
   * network, the rest are random. gnn_c_out in [1, TLS_GNN_HIDDEN] (the
   * read-out has rank <= TLS_GNN_HIDDEN). */
  const float* gnn_weights;
  int32_t gnn_c_out;
  /* 1: keep what tls_gnn_forward / tls_gnn_loss_grad need (the local graphs
   * and the eq. gevpsvd eigenvectors as training targets). SPD, nev > 0. */
  int32_t gnn_train;
  /* How the one-level and coarse parts combine (Q = R_0^T A_00^{-1} R_0):
   * 0: additive, z = sum_i R_i^T A_ii^{-1} R_i r + Q r (eq. onelevelasm plus
   *    the coarse correction, the operator of the theory; symmetric for SPD
   *    A, so PCG is used there);
   * 1: restricted additive Schwarz (eq. onelevelras) with the deflated
   *    coarse correction the experiments of Section 7.2 use,
   *    z = Q r + M_RAS^{-1} (r - A Q r); not symmetric, so tls_solve runs
   *    FGMRES for every matrix_kind. Default 0. */
  int32_t composition;
  /* 1 (SPD only): after the coarse basis is built, replace each Cholesky
   * factor by the explicit inverse A_ii^{-1} = L^{-T} L^{-1} (lower tiles,
   * same storage), so that a local solve is one symmetric product that reads
   * the stored triangle once instead of two substitutions that read it
   * twice. Costs about 2 #Omega_i^3 / 3 more flops per subdomain at setup.
   * A_0 is inverted the same way, so the coarse solve is one product too.
   * 0 (default): forward and backward substitution with the factors.
   * 2 (SPD only): choose. The substitutions read only the tiles inside each
   * factor's tile profile (twice); the product reads every lower tile once.
   * The inverse is formed when the two substitutions would read more than
   * the product (2 P > D, P the profile tiles, D the lower tiles, summed
   * over the subdomains); tls_info reports the choice. */
  int32_t local_inverse;
  /* FP32 mode (precision 1) only: steps of iterative refinement after each
   * local solve, in [0, 8]. A step forms the residual b_i - A_ii x_i in FP64
   * from the sparse rows of A_ii, solves for the correction with the same
   * FP32 factor (or explicit inverse) and adds it in FP64; each step costs
   * one more pass over the local factors. 0 (default): none. Ignored in
   * FP64 mode. */
  int32_t local_refine;
  /* Block rows per task of the persistent substitutions: 1 to 4 with FP32
   * local solves (precision 1), 1 or 2 in FP64. A task of S rows solves
   * them in sequence with the earlier rows' values from LDS, so a long
   * dependency chain makes S times fewer round trips through memory.
   * 0 (default): 1, or the autotuner's pick with autotune = 1 (which
   * still tunes the workgroup count and order for a rows value set here). */
  int32_t solve_rows;
  void* stream;         /* hipStream_t */
} tls_options;

typedef struct {
  int32_t n;
  int32_t n_parts;
  int32_t n_coarse;           /* n_C = number of columns of R_0^T            */
  double gc;                  /* grid complexity 1 + n_C / n (Section 7)     */
  double oc;                  /* operator complexity 1 + nnz(A_0) / nnz(A)   */
  int64_t local_sum_m;        /* sum_i #Omega_i                              */
  int64_t local_sum_m2;       /* sum_i #Omega_i^2                            */
  int64_t factor_bytes;       /* bytes of the stored local factors           */
  int32_t max_m;              /* max_i #Omega_i                              */
  int32_t min_m;              /* min_i #Omega_i                              */
  double t_setup[8];          /* ms: [0] overlap, [1] gather, [2] factorization and solve
                                 plans, [3] coarse basis (eigensolves, orthonormalization),
                                 [4] learned warm start (inside [3]), [5] A_0 and its
                                 factorization, [6] batched factorization with the
                                 diagonal-tile inverses (inside [2]), [7] total */
  double t_solve;             /* ms of the last tls_solve                    */
  int32_t iters;              /* iterations of the last tls_solve            */
  double relres;              /* true relative residual of the last solve    */
  double eig_resid_max;       /* max relative eigen-residual over subdomains */
  int32_t eig_iters_max;      /* max subspace iterations over subdomains     */
  double eig_iters_mean;      /* mean subspace iterations over subdomains    */
  int32_t n_res_history;      /* entries in res_history                      */
  int32_t n_profiled;         /* tls_apply calls timed with profile = 1       */
  double t_local_solve_ms;    /* mean duration of their local-solve kernels (HIP
                                 events): forward + backward substitution, or
                                 the symmetric product + its reduction       */
  double t_apply_ms;          /* mean duration of those whole applies         */
  double t_local_fwd_ms;      /* mean duration of their forward-substitution (or
                                 symmetric-product) kernel alone             */
  int32_t solve_wgs;          /* workgroups used by the persistent solves     */
  int32_t solve_order;        /* task order of the forward solves (1 .. 5)    */
  int32_t tuned;              /* 0 default, 1 timed at setup, 2 read from the cache */
  const double* res_history;  /* host array: ||r_k|| / ||b|| per iteration   */
  int32_t local_inverse;      /* 1 if the local solves use explicit inverses  */
  double t_inverse_ms;        /* setup ms spent forming them (inside t_setup[7]; the
                                 inverse of A_0 is inside t_setup[5]) */
  int32_t wait_timeout;       /* 1 if a tls_apply since the previous tls_info or tls_solve
                                 of this context ran a triangular-solve wait past its spin
                                 limit (its z is not valid); reading it clears it. tls_info
                                 waits for the context's stream to read it. */
  int32_t local_refine;       /* refinement steps of each local solve (option local_refine) */
  int32_t symv_block;         /* block side (tiles) of the product with the local inverses
                                 (4, 6 or 8; autotuned; 0 without local_inverse) */
  int32_t factor_panel;       /* panel width (tiles) of the batched factorization
                                 (4, 8 or 16; autotuned) */
  double factor_flops;        /* arithmetic of the local factorization as run (2 per
                                 multiply-add): for SPD matrices only the tiles inside
                                 each A_ii's tile profile (its envelope, where all fill
                                 stays), else 2/3 (64 nt_i)^3 per subdomain */
  double inverse_flops;       /* the same for forming the explicit local inverses
                                 (0 without local_inverse) */
  int64_t solve_tiles_fwd;    /* 64 x 64 tiles one forward substitution reads (all
                                 subdomains; the tiles inside the row profiles) */
  int64_t solve_tiles_bwd;    /* the same for the backward substitution (Cholesky: the
                                 same tiles read by columns; LU: the tiles of U inside
                                 its column profiles) */
  int64_t lower_tiles;        /* lower tiles of all local factors, sum nt_i (nt_i + 1) / 2
                                 (what the product with explicit inverses reads) */
  int32_t solve_rows;         /* block rows per task of the persistent substitutions */
  int32_t solve_order_bwd;    /* task order of the backward solves (1 .. 5; the
                                 autotuner picks each direction's own)        */
} tls_info_t;

/* Fill *opt with the defaults listed above. */
void tls_default_options(tls_options* opt);

/* Build the preconditioner (Sections 2-6): overlap layers, local matrices
 * A_ii = R_i A R_i^T, their factorization, the coarse basis Z, A_0 = Z^T A Z
 * and its factorization.
 *   n, nnz        : size and number of stored entries of A
 *   row_ptr[n+1], col_idx[nnz], val[nnz] : CSR of A (device)
 *   part[n]       : nonoverlapping partition (device), values in [0, n_parts)
 *   overlap       : delta >= 0 layers; 0 allows nev = 0 only
 *   nev           : eq. gevpsvd (SPD) / Section 6 (general) vectors kept per subdomain
 *   opt           : options (NULL = defaults)
 *   out           : receives the new context; NULL on failure
 * Errors: TLS_E_ARG (malformed CSR/partition, overlap 0 with nev > 0, NaN),
 * TLS_E_NOT_SPD, TLS_E_SINGULAR, TLS_E_NOMEM, TLS_E_HIP. */
tls_status tls_setup(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                     const double* val, const int32_t* part, int32_t n_parts, int32_t overlap,
                     int32_t nev, const tls_options* opt, tls_ctx** out);

/* z = M^{-1} r (device vectors of length n, r != z): the two-level operator
 * M_2^{-1} of the Remark in Section 4.3 (one-level part eq. onelevelasm), or
 * with composition = 1 the restricted one-level part of eq. onelevelras
 * with the deflated coarse correction of Section 7.2. Asynchronous: errors
 * that only the device sees (a wait past its spin limit) are reported by
 * the next tls_info (wait_timeout) and do not fail later solves. */
tls_status tls_apply(tls_ctx* c, const double* r, double* z);

/* y = A x with the stored CSR copy (device vectors, x != y). Asynchronous. */
tls_status tls_spmv(tls_ctx* c, const double* x, double* y);

/* Solve A x = b (eq. Ax=b, Section 1) from x0 = 0 with PCG (SPD A, additive
 * composition: Section 1 and its CG bound) or right-preconditioned flexible
 * GMRES(restart) (general A or composition = 1: Section 7.2), until the
 * true relative residual ||b - A x|| / ||b|| <= tol (Section 7.2 stops at
 * 1e-8). PCG stops on its recurrence residual, then restarts from x (at most
 * four times) while the true residual is above tol.
 * b, x: device vectors (b != x). iters, relres (true residual at exit) may
 * be NULL. Returns TLS_E_NOCONV with the last iterate if maxit is reached. */
tls_status tls_solve(tls_ctx* c, const double* b, double* x, double tol, int32_t* iters,
                     double* relres);

/* For callers that cannot allocate device memory (code running while another
 * stream of the process is under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the solve of tls_solve (same solver,
 * same arguments, same results as tls_solve with use_graph = 0) with no
 * device allocation and no hipFree. Its Krylov vectors, reduction partials,
 * flags and residual history live in a fixed device array of
 * TLS_NOALLOC_SCRATCH_BYTES that every GPU the library runs on holds until
 * the process ends; the context must have been set up (its own buffers come
 * from tls_setup) and its device must be current. The work needed is
 * 56 n bytes for PCG and 8 n (2 restart + 7) bytes for FGMRES, plus a few
 * tens of KB; a solve that needs more than the array returns TLS_E_ARG
 * (tls_solve has no such limit). Always eager (no captured graph); keeps no
 * residual history (tls_info reports none). Calls on one GPU share the
 * array: calls that overlap on one GPU race. */
#define TLS_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
tls_status tls_solve_noalloc(tls_ctx* c, const double* b, double* x, double tol, int32_t* iters,
                             double* relres);

/* Statistics of the context (host struct; res_history stays valid until
 * the next tls_solve or tls_destroy). */
tls_status tls_info(const tls_ctx* c, tls_info_t* info);

/* Copy internal setup products to host buffers for inspection (testing and
 * diagnostics). Each pointer may be NULL to skip it.
 *   sub_ptr[n_parts+1], sub_idx[sum #Omega_i] : ordered Omega_i lists
 *   layer_ptr[n_parts*(overlap+2)]            : per subdomain, offsets of I_i,
 *                                               Gamma_1 .. Gamma_delta, end
 *   zcol_ptr[n_parts+1]                       : first coarse column per subdomain
 *   eigvals[n_coarse]                         : per kept column, its eigenvalue: lambda^2
 *                                               (eq. gevpsvd), lambda (eq. uppergevp) or
 *                                               sigma (general A, Section 6)
 *   zsrc[n_coarse]                            : per kept column, where it came from:
 *                                               0 eq. gevpsvd, 1 eq. uppergevp, 2 Section 6
 *   Z[n * n_coarse]                           : dense column-major coarse basis
 *   A0[n_coarse * n_coarse]                   : dense column-major A_0          */
tls_status tls_export(const tls_ctx* c, int32_t* sub_ptr, int32_t* sub_idx, int32_t* layer_ptr,
                      int32_t* zcol_ptr, double* eigvals, int32_t* zsrc, double* Z, double* A0);

/* Copy the coarse basis in its compact form to a host buffer: for each
 * subdomain i in order, its k_i = zcol_ptr[i+1] - zcol_ptr[i] columns
 * restricted to the rows I_i, column-major (#I_i x k_i), rows in the order
 * of sub_idx[sub_ptr[i] .. sub_ptr[i] + #I_i). blocks must hold
 * sum_i #I_i k_i doubles (Z is zero outside these blocks). */
tls_status tls_export_zblocks(const tls_ctx* c, double* blocks);

/* Solve with one local factor: x = A_ii^{-1} b for subdomain i (host
 * vectors of length #Omega_i, in the Omega_i order). Diagnostics. */
tls_status tls_local_solve(tls_ctx* c, int32_t i, const double* b, double* x);

/* Last error message of the context (or of the calling thread's last failed
 * tls_setup when c is NULL). Never NULL. */
const char* tls_last_error(const tls_ctx* c);

/* Learned warm start, forward pass: X = network output on every local
 * graph of the context. weights: host, TLS_GNN_NWEIGHTS(c_out) floats.
 * X: host, (sum #Omega_i) x c_out floats, row-major, rows in the order of
 * tls_export's sub_idx. Needs a context set up with gnn_train = 1 or with
 * gnn_weights. */
tls_status tls_gnn_forward(tls_ctx* c, const float* weights, int32_t c_out, float* X);

/* Learned warm start, training step: the mean over subdomains of
 *   f_i = -(1/k_i) tr(G^{-1} X_T^T Q_i Q_i^T X_T),
 *   G = X_T^T X_T + 1e-3 (tr(X_T^T X_T) / c_out) I,
 * where X_T are the rows Gamma_{i,delta} of the network output and Q_i an
 * orthonormal basis of the same rows of the context's own top-k_i
 * eq. gevpsvd eigenvectors (kept by a setup with gnn_train = 1), and its
 * gradient with respect to the weights (forward and backward passes on the
 * device). weights, grad: host arrays of TLS_GNN_NWEIGHTS(c_out) floats;
 * loss: host scalar. TLS_E_STATE without targets. */
tls_status tls_gnn_loss_grad(tls_ctx* c, const float* weights, int32_t c_out, float* grad, double* loss);

/* Free everything the context owns. NULL is ignored. Device blocks of
 * 32 MiB and more are not handed back to the driver but kept for the next
 * contexts of the process (freeing and mapping tens of GB per setup slowed
 * the following setups several-fold), except that the smallest kept blocks
 * are handed back until 5% of the device's memory is free, so that other
 * allocators of the process still find room; tls_trim hands them all
 * back. */
void tls_destroy(tls_ctx* c);

/* Free the device blocks kept for reuse (all devices). Safe at any time:
 * blocks in use by live contexts are not affected. */
void tls_trim(void);

/* Memory planning. tls_setup runs the local eigen passes and the formation
 * of the explicit inverses on groups of subdomains whose buffers fit in 90%
 * of the device memory still available (free memory plus the kept blocks);
 * the results do not depend on the grouping. The environment variable
 * TLS_MEMORY_LIMIT (bytes, read at each setup) lowers that figure. */

#ifdef __cplusplus
}
#endif

#endif /* TLS_H */
