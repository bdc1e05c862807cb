// The C ABI declared in include/tls.h.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <functional>
#include <memory>

#include "kernels.hpp"

using tls::DBuf;
using tls::TlsError;

namespace {

thread_local std::string g_thread_err;

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) { return std::chrono::duration<double, std::milli>(clk::now() - t0).count(); }

tls_status guard(tls_ctx* c, const std::function<void()>& f) {
  try {
    f();
    return TLS_OK;
  } catch (const TlsError& e) {
    if (c) c->err = e.msg;
    g_thread_err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    if (c) c->err = e.what();
    g_thread_err = e.what();
    return TLS_E_HIP;
  }
}

}  // namespace

extern "C" {

void tls_default_options(tls_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = 0;
  o->matrix_kind = 0;
  o->nev1 = 0;
  o->tau = 0.0;
  o->nu = 1.0;
  o->restart = 30;
  o->maxit = 0;
  o->eig_maxit = 300;
  o->eig_tol = 0.0;
  o->eig_oversample = -1;
  o->seed = 0;
  o->use_graph = 0;
  o->flexible = -1;
  o->jacobi_scale = 0;
  o->profile = 0;
  o->solve_wgs = 0;
  o->solve_order = 0;
  o->autotune = 0;
  o->tune_cache = nullptr;
  o->gnn_weights = nullptr;
  o->gnn_c_out = 0;
  o->gnn_train = 0;
  o->composition = 0;
  o->local_inverse = 0;
  o->local_refine = 0;
  o->stream = nullptr;
}

tls_status tls_setup(int32_t n, int32_t nnz, const int32_t* row_ptr, const int32_t* col_idx, const double* val,
                     const int32_t* part, int32_t n_parts, int32_t overlap, int32_t nev, const tls_options* opt,
                     tls_ctx** out) {
  if (!out) {
    g_thread_err = "out must not be NULL";
    return TLS_E_ARG;
  }
  *out = nullptr;
  std::unique_ptr<tls_ctx> c(new tls_ctx());
  tls_status st = guard(c.get(), [&]() {
    auto t_all = clk::now();
    tls_default_options(&c->opt);
    if (opt) c->opt = *opt;
    if (n <= 0 || nnz < 0 || !row_ptr || !col_idx || !val || !part)
      tls::fail(TLS_E_ARG, "n must be positive and every pointer non-NULL");
    if (n_parts < 1 || n_parts > n) tls::fail(TLS_E_ARG, "n_parts must be in [1, n]");
    if (overlap < 0 || overlap > 200) tls::fail(TLS_E_ARG, "overlap must be in [0, 200]");
    if (nev < 0) tls::fail(TLS_E_ARG, "nev must be >= 0");
    if (overlap == 0 && nev > 0) tls::fail(TLS_E_ARG, "overlap 0 leaves Gamma_{i,delta} empty: nev must be 0");
    if (c->opt.precision != 0 && c->opt.precision != 1) tls::fail(TLS_E_ARG, "precision must be 0 or 1");
    if (c->opt.matrix_kind != 0 && c->opt.matrix_kind != 1) tls::fail(TLS_E_ARG, "matrix_kind must be 0 or 1");
    if (c->opt.nev1 < 0) tls::fail(TLS_E_ARG, "nev1 must be >= 0");
    if (c->opt.nev1 > 0 && c->opt.matrix_kind != 0)
      tls::fail(TLS_E_ARG, "nev1 (eq. uppergevp vectors) applies to SPD matrices only");
    if (c->opt.nev1 > 0 && overlap == 0) tls::fail(TLS_E_ARG, "overlap 0: nev1 must be 0");
    if (c->opt.solve_order < 0 || c->opt.solve_order > 5) tls::fail(TLS_E_ARG, "solve_order must be in [0, 5]");
    if (c->opt.solve_wgs < 0) tls::fail(TLS_E_ARG, "solve_wgs must be >= 0");
    if (c->opt.composition != 0 && c->opt.composition != 1) tls::fail(TLS_E_ARG, "composition must be 0 or 1");
    if (c->opt.local_inverse < 0 || c->opt.local_inverse > 2) tls::fail(TLS_E_ARG, "local_inverse must be 0, 1 or 2");
    if (c->opt.local_inverse && c->opt.matrix_kind != 0)
      tls::fail(TLS_E_ARG, "local_inverse applies to SPD matrices only");
    if (c->opt.local_refine < 0 || c->opt.local_refine > 8) tls::fail(TLS_E_ARG, "local_refine must be in [0, 8]");
    if (c->opt.solve_rows < 0 || c->opt.solve_rows > (c->opt.precision == 1 ? 4 : 2))
      tls::fail(TLS_E_ARG, "solve_rows must be in [0, 4] (FP32 local solves) or [0, 2] (FP64)");
    if (c->opt.gnn_weights || c->opt.gnn_train) {
      if (c->opt.matrix_kind != 0) tls::fail(TLS_E_ARG, "the learned warm start applies to SPD matrices only");
      if (c->opt.gnn_weights) tls::gnn_check_weights(c->opt.gnn_c_out);
    }
    if (c->opt.flexible < 0) c->opt.flexible = c->opt.precision == 1 ? 1 : 0;
    if (c->opt.eig_maxit <= 0) c->opt.eig_maxit = 300;
    if (c->opt.restart <= 0) c->opt.restart = 30;
    if ((size_t)n_parts * (size_t)n > ((size_t)1 << 36))
      tls::fail(TLS_E_ARG, "n_parts * n too large for the overlap marker array");
    c->n = n;
    c->nnz = nnz;
    c->N = n_parts;
    c->delta = overlap;
    c->nev = nev;
    c->kind = c->opt.matrix_kind;
    c->fp32 = c->opt.precision == 1;
    TLS_HIP(hipGetDevice(&c->device));
    if (c->opt.stream) {
      c->stream = reinterpret_cast<hipStream_t>(c->opt.stream);
    } else {
      // a blocking stream: ordered with the legacy default stream, on which
      // callers that pass no stream usually work
      TLS_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamDefault));
      c->own_stream = true;
    }
    hipStream_t s = c->stream;
    TLS_HIP(hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking));
    TLS_HIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    TLS_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    c->errflag.alloc(4);
    c->zero_int.alloc(4);
    TLS_HIP(hipMemsetAsync(c->zero_int.p, 0, sizeof(int) * 4, s));
    c->row_ptr.alloc(n + 1);
    c->col_idx.alloc(std::max(nnz, 1));
    c->val.alloc(std::max(nnz, 1));
    c->part.alloc(n);
    TLS_HIP(hipMemcpyAsync(c->row_ptr.p, row_ptr, sizeof(int) * (n + 1), hipMemcpyDeviceToDevice, s));
    if (nnz) {
      TLS_HIP(hipMemcpyAsync(c->col_idx.p, col_idx, sizeof(int) * nnz, hipMemcpyDeviceToDevice, s));
      TLS_HIP(hipMemcpyAsync(c->val.p, val, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s));
    }
    TLS_HIP(hipMemcpyAsync(c->part.p, part, sizeof(int) * n, hipMemcpyDeviceToDevice, s));
    double avg = (double)nnz / n;
    // short rows: row blocks streamed through LDS (0); longer ones: G lanes per row
    c->spmv_group = avg <= 12 ? 0 : avg <= 24 ? 16 : avg <= 48 ? 32 : 64;
    if (c->spmv_group == 0) {
      // the most entries in one block of 256 rows picks the row-block kernel's LDS size
      std::vector<int> hrp(n + 1);
      TLS_HIP(hipMemcpyAsync(hrp.data(), row_ptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, s));
      TLS_HIP(hipStreamSynchronize(s));
      int most = 0;
      for (int r0 = 0; r0 < n; r0 += 256) most = std::max(most, hrp[std::min(n, r0 + 256)] - hrp[r0]);
      c->spmv_cap = most <= 1280 ? 1280 : most <= 1536 ? 1536 : most <= 2048 ? 2048 : 4096;
    }

    auto t = clk::now();
    tls::validate_input(c.get());
    if (c->kind == 1) tls::build_transpose(c.get());
    tls::build_overlap(c.get());
    tls::build_layout(c.get());
    c->t_setup[0] = ms_since(t);
    t = clk::now();
    tls::gather_local(c.get());
    c->t_setup[1] = ms_since(t);
    t = clk::now();
    tls::factor_local_tuned(c.get());
    c->t_setup[6] = ms_since(t);
    tls::build_solve_tasks(c.get());
    c->t_setup[2] = ms_since(t);
    t = clk::now();
    tls::build_coarse_basis(c.get());
    c->t_setup[3] = ms_since(t);
    t = clk::now();
    tls::build_coarse_operator(c.get());
    c->t_setup[5] = ms_since(t);
    if (c->opt.composition == 1) {
      c->ras_t.alloc(n);
      c->ras_u.alloc(n);
    }
    if (c->opt.local_inverse == 1 || (c->opt.local_inverse == 2 && tls::inverse_pays(c.get()))) {
      t = clk::now();
      tls::form_local_inverse(c.get());
      c->t_inverse = ms_since(t);
    }
    tls::build_refine(c.get());
    tls::choose_solve_grid(c.get());
    tls::choose_symv_block(c.get());
    TLS_HIP(hipStreamSynchronize(s));
    c->t_setup[7] = ms_since(t_all);
  });
  c->opt.gnn_weights = nullptr;  // caller memory: read during setup only
  if (st != TLS_OK) return st;
  *out = c.release();
  return TLS_OK;
}

tls_status tls_apply(tls_ctx* c, const double* r, double* z) {
  if (!c) return TLS_E_STATE;
  if (!r || !z || r == z) {
    c->err = "r and z must be distinct non-NULL device vectors";
    return TLS_E_ARG;
  }
  return guard(c, [&]() { tls::apply_precond(c, r, z, c->zero_int.p, c->opt.profile != 0); });
}

tls_status tls_spmv(tls_ctx* c, const double* x, double* y) {
  if (!c) return TLS_E_STATE;
  if (!x || !y || x == y) {
    c->err = "x and y must be distinct non-NULL device vectors";
    return TLS_E_ARG;
  }
  return guard(c, [&]() { tls::spmv(c, x, y, c->zero_int.p); });
}

tls_status tls_solve(tls_ctx* c, const double* b, double* x, double tol, int32_t* iters, double* relres) {
  if (!c) return TLS_E_STATE;
  if (!b || !x || b == x || !(tol > 0.0)) {
    c->err = "b and x must be distinct non-NULL device vectors and tol > 0";
    return TLS_E_ARG;
  }
  bool conv = false;
  tls_status st = guard(c, [&]() {
    int it = 0;
    double rr = 0;
    tls::krylov_solve(c, b, x, tol, &it, &rr, &conv);
    c->last_iters = it;
    c->last_relres = rr;
  });
  if (iters) *iters = c->last_iters;
  if (relres) *relres = c->last_relres;
  if (st != TLS_OK) return st;
  if (!conv) {
    c->err = "maximum number of iterations reached";
    return TLS_E_NOCONV;
  }
  return TLS_OK;
}

tls_status tls_info(const tls_ctx* c, tls_info_t* info) {
  if (!c || !info) return TLS_E_STATE;
  std::memset(info, 0, sizeof(*info));
  info->n = c->n;
  info->n_parts = c->N;
  info->n_coarse = c->nC;
  info->gc = 1.0 + (double)c->nC / c->n;
  info->oc = 1.0 + (double)c->nnz0 / std::max(c->nnz, 1);
  info->local_sum_m = c->sum_m;
  info->local_sum_m2 = c->sum_m2;
  info->factor_bytes = c->fac_elems * (c->fp32 ? 4 : 8);
  int mx = 0, mn = c->N ? c->h_m[0] : 0;
  for (int m : c->h_m) {
    mx = std::max(mx, m);
    mn = std::min(mn, m);
  }
  info->max_m = mx;
  info->min_m = mn;
  for (int k = 0; k < 8; k++) info->t_setup[k] = c->t_setup[k];
  info->t_solve = c->t_solve;
  info->iters = c->last_iters;
  info->relres = c->last_relres;
  info->eig_resid_max = c->eig_resid_max;
  info->eig_iters_max = c->eig_iters_max;
  info->eig_iters_mean = c->eig_iters_mean;
  info->n_res_history = (int32_t)c->h_hist.size();
  info->res_history = c->h_hist.empty() ? nullptr : c->h_hist.data();
  info->n_profiled = c->prof_count;
  info->t_local_solve_ms = c->prof_count ? c->prof_local_ms / c->prof_count : 0.0;
  info->t_apply_ms = c->prof_count ? c->prof_apply_ms / c->prof_count : 0.0;
  info->t_local_fwd_ms = c->prof_count ? c->prof_fwd_ms / c->prof_count : 0.0;
  info->local_inverse = c->inv_formed ? 1 : 0;
  info->t_inverse_ms = c->t_inverse;
  info->solve_wgs = c->solve_grid;
  info->solve_order = c->solve_order;
  info->tuned = c->tuned;
  info->local_refine = c->refine;
  info->symv_block = c->inv_formed ? c->symv_block : 0;
  info->factor_panel = c->factor_panel;
  info->factor_flops = c->flops_factor;
  info->inverse_flops = c->inv_formed ? c->flops_inverse : 0.0;
  tls::solve_tile_counts(c, &info->solve_tiles_fwd, &info->solve_tiles_bwd, &info->lower_tiles);
  info->solve_rows = c->solve_rows;
  info->solve_order_bwd = c->solve_order_b;
  tls_ctx* cm = const_cast<tls_ctx*>(c);
  bool wt = cm->apply_wait_seen;
  if (guard(cm, [&]() { wt = tls::take_wait_flag(cm) || wt; }) != TLS_OK) return TLS_E_HIP;
  cm->apply_wait_seen = false;
  info->wait_timeout = wt ? 1 : 0;
  return TLS_OK;
}

tls_status tls_export(const tls_ctx* cc, int32_t* sub_ptr, int32_t* sub_idx, int32_t* layer_ptr, int32_t* zcol_ptr,
                      double* eigvals, int32_t* zsrc, double* Z, double* A0) {
  tls_ctx* c = const_cast<tls_ctx*>(cc);
  if (!c) return TLS_E_STATE;
  return guard(c, [&]() {
    hipStream_t s = c->stream;
    const int N = c->N;
    if (sub_ptr) std::copy(c->h_sub_ptr.begin(), c->h_sub_ptr.end(), sub_ptr);
    std::vector<int> h_idx;
    if (sub_idx || Z) h_idx = tls::download(c->sub_idx.p, c->h_sub_ptr[N], s);
    if (sub_idx) std::copy(h_idx.begin(), h_idx.end(), sub_idx);
    if (layer_ptr) std::copy(c->h_layer_ptr.begin(), c->h_layer_ptr.end(), layer_ptr);
    if (zcol_ptr) std::copy(c->h_zcol.begin(), c->h_zcol.end(), zcol_ptr);
    if (eigvals) std::copy(c->h_eig.begin(), c->h_eig.end(), eigvals);
    if (zsrc) std::copy(c->h_zsrc.begin(), c->h_zsrc.end(), zsrc);
    if (Z && c->nC > 0) {
      int64_t tot = c->h_zoff.empty() ? 0 : c->h_zoff[N];
      auto hz = tls::download(c->Z.p, std::max<int64_t>(tot, 1), s);
      std::memset(Z, 0, sizeof(double) * (size_t)c->n * c->nC);
      for (int p = 0; p < N; p++) {
        int nI = c->h_nI[p];
        for (int a = 0; a < c->h_zcol[p + 1] - c->h_zcol[p]; a++)
          for (int j = 0; j < nI; j++)
            Z[(size_t)(c->h_zcol[p] + a) * c->n + h_idx[c->h_sub_ptr[p] + j]] = hz[c->h_zoff[p] + (int64_t)a * nI + j];
      }
    }
    if (A0 && c->nC > 0) {
      auto ht = tls::download(c->A0_orig.p, c->A0_orig.n, s);
      const int nC = c->nC, nt = c->nt0, kind = c->kind;
      for (int b = 0; b < nC; b++)
        for (int a = (kind == 0 ? b : 0); a < nC; a++) {
          double v = ht[tls::tile_index(kind, nt, a / tls::TS, b / tls::TS) * tls::TS2 + (b % tls::TS) * tls::TS +
                        (a % tls::TS)];
          A0[(size_t)b * nC + a] = v;
          if (kind == 0) A0[(size_t)a * nC + b] = v;
        }
    }
  });
}

tls_status tls_export_zblocks(const tls_ctx* cc, double* blocks) {
  tls_ctx* c = const_cast<tls_ctx*>(cc);
  if (!c) return TLS_E_STATE;
  if (!blocks) {
    c->err = "blocks must not be NULL";
    return TLS_E_ARG;
  }
  return guard(c, [&]() {
    const int64_t tot = c->h_zoff.empty() ? 0 : c->h_zoff[c->N];
    if (tot > 0) {
      // stored blocks may hold room for columns dropped by the orthonormalization
      auto hz = tls::download(c->Z.p, tot, c->stream);
      int64_t o = 0;
      for (int i = 0; i < c->N; i++) {
        const int64_t len = (int64_t)c->h_nI[i] * (c->h_zcol[i + 1] - c->h_zcol[i]);
        std::copy(hz.begin() + c->h_zoff[i], hz.begin() + c->h_zoff[i] + len, blocks + o);
        o += len;
      }
    }
  });
}

tls_status tls_gnn_forward(tls_ctx* c, const float* weights, int32_t c_out, float* X) {
  if (!c) return TLS_E_STATE;
  if (!weights || !X) {
    c->err = "weights and X must not be NULL";
    return TLS_E_ARG;
  }
  return guard(c, [&]() {
    if (c->kind != 0) tls::fail(TLS_E_ARG, "the learned warm start applies to SPD matrices only");
    tls::gnn_forward(c, weights, c_out, false);
    const size_t total = (size_t)c->h_sub_ptr[c->N];
    auto h = tls::download(c->gnn_X.p, total * c_out, c->stream);
    std::copy(h.begin(), h.end(), X);
  });
}

tls_status tls_gnn_loss_grad(tls_ctx* c, const float* weights, int32_t c_out, float* grad, double* loss) {
  if (!c) return TLS_E_STATE;
  if (!weights || !grad || !loss) {
    c->err = "weights, grad and loss must not be NULL";
    return TLS_E_ARG;
  }
  return guard(c, [&]() { *loss = tls::gnn_loss_grad(c, weights, c_out, grad); });
}

tls_status tls_local_solve(tls_ctx* c, int32_t i, const double* b, double* x) {
  if (!c) return TLS_E_STATE;
  if (i < 0 || i >= c->N || !b || !x) {
    c->err = "subdomain index out of range or NULL vector";
    return TLS_E_ARG;
  }
  return guard(c, [&]() {
    hipStream_t s = c->stream;
    const int m = c->h_m[i];
    const int64_t off = c->h_voff[i];
    std::vector<double> sc(m, 1.0);
    if (c->opt.jacobi_scale) {
      sc = tls::download(c->scale.p + off, m, s);
    }
    if (c->fp32) {
      std::vector<float> hb(c->sum_M, 0.f);
      for (int j = 0; j < m; j++) hb[off + j] = (float)(b[j] * sc[j]);
      TLS_HIP(hipMemcpyAsync(c->xloc32.p, hb.data(), sizeof(float) * c->sum_M, hipMemcpyHostToDevice, s));
      if (c->refine > 0) {
        std::vector<double> hb64(c->sum_M, 0.0);
        for (int j = 0; j < m; j++) hb64[off + j] = b[j] * sc[j];
        TLS_HIP(hipMemcpyAsync(c->bref64.p, hb64.data(), sizeof(double) * c->sum_M, hipMemcpyHostToDevice, s));
      }
      if (tls::local_solve_refined(c, c->zero_int.p)) {
        auto hx = tls::download(c->xref64.p + off, m, s);
        for (int j = 0; j < m; j++) x[j] = hx[j] * sc[j];
      } else {
        auto hx = tls::download(c->xloc32.p + off, m, s);
        for (int j = 0; j < m; j++) x[j] = (double)hx[j] * sc[j];
      }
    } else {
      std::vector<double> hb(c->sum_M, 0.0);
      for (int j = 0; j < m; j++) hb[off + j] = b[j] * sc[j];
      TLS_HIP(hipMemcpyAsync(c->xloc64.p, hb.data(), sizeof(double) * c->sum_M, hipMemcpyHostToDevice, s));
      tls::local_solve(c, c->zero_int.p);
      auto hx = tls::download(c->xloc64.p + off, m, s);
      for (int j = 0; j < m; j++) x[j] = hx[j] * sc[j];
    }
  });
}

const char* tls_last_error(const tls_ctx* c) {
  if (c) return c->err.c_str();
  return g_thread_err.c_str();
}

void tls_destroy(tls_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  delete c;
  tls::devmem::keep_headroom(0.05);
}

void tls_trim(void) { tls::devmem::trim(); }

}  // extern "C"
