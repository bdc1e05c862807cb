// Library context: everything tls_setup builds and tls_apply / tls_solve use.
#pragma once

#include "common.hpp"

struct tls_ctx {
  tls_options opt{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;                            // HIP device current at tls_setup
  hipStream_t stream2 = nullptr;             // coarse solve, overlapped with the local solves
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int tuned = 0;
  std::string err;

  // problem
  int n = 0, nnz = 0, N = 0, delta = 0, nev = 0;
  int kind = 0;  // 0 SPD / Cholesky, 1 general / LU
  bool fp32 = false;
  tls::DBuf<int> row_ptr, col_idx, part;
  tls::DBuf<double> val;
  tls::DBuf<int> trow_ptr, tcol_idx;  // pattern of A^T (general matrices)
  int spmv_group = 0;  // 0: row-block SpMV through LDS; G > 0: G lanes per row
  int spmv_cap = 2048;  // LDS products per row block of the row-block SpMV

  // overlap: Omega_i lists (global ids) in [I, Gamma_1, .., Gamma_delta] order
  std::vector<int> h_sub_ptr;    // N+1
  std::vector<int> h_layer_ptr;  // N*(delta+2): per subdomain segment starts (absolute) and end
  std::vector<int> h_m, h_nI, h_nP, h_nt;
  std::vector<int64_t> h_foff, h_voff, h_toff;
  tls::DBuf<int> sub_ptr, sub_idx, layer_ptr, sub_of_pos;
  tls::DBuf<int> d_m, d_nI, d_nP, d_nt;
  tls::DBuf<int64_t> d_foff, d_voff, d_toff;
  int64_t sum_m = 0, sum_m2 = 0, sum_M = 0, sum_nt = 0, fac_elems = 0;
  int max_nt = 0;
  tls::DBuf<int> ipos;  // position of each global row inside its interior list

  // scatter map: for each global row, the padded positions holding it
  tls::DBuf<int> own_ptr;
  tls::DBuf<int64_t> own_pos;

  // local factors (fp64 or fp32 depending on the precision option)
  tls::DBuf<double> fac64;
  tls::DBuf<float> fac32;
  tls::DBuf<double> scale;  // Jacobi scaling per padded position (or empty)
  // tile profile (SPD): first tile column of tile row r of A_ii that holds
  // a nonzero, at toff_i + r. The Cholesky factor has no fill left of it,
  // so the factorization, the inverse and the substitutions skip those tiles.
  tls::DBuf<int> prof;
  std::vector<int> h_prof;
  // profile storage of the local factors: only the tiles inside the
  // profiles are stored (offsets trow / tcol, see LocalLayout); h_soff keeps
  // the offsets of the full packed storage, which the explicit inverses use
  bool prof_store = false;
  std::vector<int64_t> h_trow, h_tcol, h_soff;
  tls::DBuf<int64_t> d_trow, d_tcol;
  double flops_factor = 0, flops_inverse = 0;  // their arithmetic with the profile (2 per multiply-add)
  // inverses of the diagonal tiles (one per tile row, at (toff_i + r) * 64^2)
  tls::DBuf<double> dinv64;
  tls::DBuf<float> dinv32;
  // explicit inverses (option local_inverse): the symmetric-product work
  // lists of the local matrices and of A_0
  bool inv_formed = false, inv0_formed = false;
  int symv_block = 8;      // block side (tiles) of the symmetric product with the local inverses
  int factor_panel = 8;    // panel width (tiles) of the batched factorization
  double t_inverse = 0.0;
  tls::SymvWork inv_work, inv0_work;

  // factorization schedule: subdomains sorted by nt (desc); per step prefix tables
  std::vector<int> h_order;
  tls::DBuf<int> order;
  std::vector<int> h_active;  // number of active subdomains at step k
  std::vector<int64_t> h_pref_off;  // offset into the prefix tables for step k
  tls::DBuf<int64_t> pref_trsm, pref_upd;
  std::vector<int64_t> h_cnt_trsm, h_cnt_upd;

  // triangular-solve work lists
  tls::SolvePlan plan_fwd, plan_bwd;
  tls::DBuf<int> counters;  // [0] fwd task counter, [1] bwd task counter, [2] epoch
  int solve_grid = 1024;
  int solve_order = 4;    // task order of the forward plan
  int solve_order_b = 4;  // and of the backward plan
  int solve_rows = 1;     // block rows per substitution task

  // work vectors for the apply (padded local layout)
  tls::DBuf<double> xloc64;
  tls::DBuf<float> xloc32;
  // iterative refinement of the FP32 local solves (option local_refine):
  // sparse rows of every A_ii (CSR over the positions of the Omega lists,
  // local column indices), the FP64 local right-hand sides and solutions
  int refine = 0;
  tls::DBuf<int> lref_ptr, lref_col;
  tls::DBuf<double> lref_val, bref64, xref64;

  // coarse space
  int nC = 0, M0 = 0, nt0 = 0;
  std::vector<int> h_zcol;  // N+1 column offsets
  std::vector<double> h_eig;
  std::vector<int> h_zsrc;  // per coarse column: 0 eq. gevpsvd, 1 eq. uppergevp, 2 Section 6
  tls::DBuf<int> zcol;
  tls::DBuf<double> Z;      // per subdomain #I_i x k_i column-major, concatenated
  std::vector<int64_t> h_zoff;
  tls::DBuf<int64_t> zoff;
  tls::DBuf<double> A0;     // tile storage of A_0 (then its factor)
  tls::DBuf<double> A0_orig;  // lower tiles of A_0 before factorization (export)
  tls::DBuf<double> dinv0;    // inverses of the diagonal tiles of the factor of A_0
  tls::DBuf<int> perm0;       // general A: row order of the pivoted LU of A_0 (P r)[i] = r[perm0[i]]
  tls::DBuf<double> y0t;      // general A: the permuted coarse right-hand side
  tls::DBuf<int> kz_dev;    // coarse columns per subdomain
  tls::DBuf<double> y0;     // coarse vector (padded to M0)
  tls::DBuf<double> ras_t;  // composition 1: Q r (n)
  tls::DBuf<double> ras_u;  // composition 1: r - A Q r (n)
  tls::SolvePlan plan0_fwd, plan0_bwd;
  tls::DBuf<int> counters0;
  tls::DBuf<int> one_m, one_nI, one_nP, one_nt;
  tls::DBuf<int64_t> one_foff, one_voff, one_toff;
  double eig_resid_max = 0;
  int eig_iters_max = 0;
  double eig_iters_mean = 0;
  int64_t nnz0 = 0;

  // learned warm start of the eigensolver: local graphs (CSR over the
  // positions of the concatenated Omega lists), features, weights, hidden
  // states (4 layers x positions x 32) and the training targets
  bool gnn_graph = false;
  tls::DBuf<int> gnn_ptr, gnn_col;
  tls::DBuf<float> gnn_w, gnn_feat, gnn_wdev, gnn_H, gnn_M, gnn_X;
  int gnn_cout = 0;
  tls::DBuf<double> gnn_tgt;  // orthonormal bases (nT_i x k_i, column-major)
  std::vector<int64_t> h_gnn_toff;
  tls::DBuf<int> gnn_nT, gnn_k;
  tls::DBuf<int64_t> gnn_toff;

  // Krylov work
  tls::DBuf<double> kr;        // vectors
  tls::DBuf<double> scal;      // device scalars
  tls::DBuf<double> partial;   // reduction partials
  tls::DBuf<unsigned> redctr;  // blocks done in the current one-launch reduction (0 between launches)
  tls::DBuf<int> done;         // [0]: converged flag, [1]: iterations
  tls::DBuf<double> hist;      // residual history
  tls::DBuf<double> gm_state;  // FGMRES Hessenberg matrix and rotations
  tls::DBuf<int> gm_idx;       // FGMRES inner index and cycle end
  std::vector<double> h_hist;
  tls::DBuf<int> zero_int;     // constant 0 for "not done"
  hipGraphExec_t graph_exec = nullptr;
  int graph_chunk = 0, graph_maxit = 0;
  double graph_tol2 = 0;
  bool graph_flex = false;

  // diagnostics
  hipEvent_t prof_ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int prof_count = 0;
  double prof_local_ms = 0, prof_fwd_ms = 0, prof_apply_ms = 0;
  tls::DBuf<int> errflag;
  bool apply_wait_seen = false;  // a wait of an earlier tls_apply timed out (reported once by tls_info)
  double t_setup[8] = {0};
  double t_solve = 0;
  int last_iters = 0;
  double last_relres = 0;

  tls::LocalLayout layout() const {
    tls::LocalLayout l{d_m, d_nI, d_nP, d_nt, d_foff, d_voff, d_toff};
    if (prof_store) {
      l.trow = d_trow.p;
      l.tcol = kind == 1 ? d_tcol.p : nullptr;
      l.prof = prof.p;
      l.profc = kind == 1 ? prof.p + sum_nt : nullptr;
    }
    return l;
  }
  tls::LocalLayout layout0() const {
    return tls::LocalLayout{one_m, one_nI, one_nP, one_nt, one_foff, one_voff, one_toff};
  }
  ~tls_ctx() {
    // work may still be queued when setup fails part-way; wait for it before
    // the buffers are freed
    if (stream2) (void)hipStreamSynchronize(stream2);
    if (stream) (void)hipStreamSynchronize(stream);
    for (auto& e : prof_ev)
      if (e) (void)hipEventDestroy(e);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (stream2) (void)hipStreamDestroy(stream2);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};
