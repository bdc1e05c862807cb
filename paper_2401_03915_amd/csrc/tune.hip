// Autotuned launch shapes, each picked at setup by timing the candidates
// (autotune = 1) and kept in a text cache keyed by the problem's shape
// (tune_cache): a cached pick is reused without timing.
//
// 1. Persistent triangular solves: workgroup count, task order and block
//    rows per task (1 to 4 in FP32, 1 or 2 in FP64).
// 2. Symmetric product with the explicit local inverses: block side of
//    4, 6 or 8 tiles (partial sums per block against workgroups in flight).
// 3. Batched factorization: panel width of 4, 8 or 16 tile columns (the
//    trailing update's K = 64 x width against the number of launches).
//
// Triangular solves:
// The solves are bound by HBM bandwidth and by how many tiles are in flight,
// which depends on how many workgroups are resident, and, for uneven
// subdomains, by the dependency chain of the largest one, which depends on
// when its block rows are handed out. The default is a fixed number of
// workgroups per compute unit for each precision (LDS and register use allow
// about 7 FP32 or 3 FP64 workgroups per CU) and rows handed out by the
// fraction of their subdomain already done, with a lead for the largest
// subdomains (order 4).
// With autotune = 1 the setup times the local forward + backward solves for
// each order and a handful of workgroup counts and keeps the fastest; picks
// are appended to a text cache keyed by the problem's shape and reused
// without timing when the key is present.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <fstream>
#include <sstream>

#include "kernels.hpp"

namespace tls {

namespace {

std::string tune_key(const tls_ctx* c) {
  std::ostringstream k;
  k << "trsv:v7 prec=" << (c->fp32 ? 32 : 64) << " kind=" << c->kind << " N=" << c->N << " n=" << c->n
    << " sumM=" << c->sum_M << " maxnt=" << c->max_nt;
  return k.str();
}

int cu_count() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus > 0 ? cus : 256;
}

// the last line of the cache whose key matches, as `count` integers
bool cache_lookup_ints(const char* path, const std::string& key, int* v, int count) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    auto tab = line.rfind('\t');
    if (tab == std::string::npos || line.substr(0, tab) != key) continue;
    std::istringstream in(line.substr(tab + 1));
    std::vector<int> got(count);
    bool ok = true;
    for (int k = 0; k < count && ok; k++) ok = static_cast<bool>(in >> got[k]);
    if (ok) {
      std::copy(got.begin(), got.end(), v);
      found = true;
    }
  }
  return found;
}

void cache_store_ints(const char* path, const std::string& key, const int* v, int count) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  if (!f) return;
  f << key << '\t';
  for (int k = 0; k < count; k++) f << (k ? " " : "") << v[k];
  f << '\n';
}

std::string shape_key(const tls_ctx* c, const char* what) {
  std::ostringstream k;
  k << what << " prec=" << (c->fp32 ? 32 : 64) << " kind=" << c->kind << " N=" << c->N << " n=" << c->n
    << " sumM=" << c->sum_M << " maxnt=" << c->max_nt;
  return k.str();
}

// Mean forward and backward times (ms) of reps local solves.
void time_local_dirs(tls_ctx* c, int grid, int reps, double* tf, double* tb) {
  const int keep = c->solve_grid;
  c->solve_grid = grid;
  hipEvent_t e0, e1, e2;
  TLS_HIP(hipEventCreate(&e0));
  TLS_HIP(hipEventCreate(&e1));
  TLS_HIP(hipEventCreate(&e2));
  local_solve(c, c->zero_int.p);  // warm-up
  double f = 0.0, b = 0.0;
  for (int k = 0; k < reps; k++) {
    local_solve(c, c->zero_int.p, e0, e1, e2);
    TLS_HIP(hipEventSynchronize(e2));
    float m1 = 0.f, m2 = 0.f;
    TLS_HIP(hipEventElapsedTime(&m1, e0, e1));
    TLS_HIP(hipEventElapsedTime(&m2, e1, e2));
    f += m1;
    b += m2;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);
  c->solve_grid = keep;
  *tf = f / reps;
  *tb = b / reps;
}

double time_local_solves(tls_ctx* c, int grid, int reps) {
  const int keep = c->solve_grid;
  c->solve_grid = grid;
  hipEvent_t e0, e1;
  TLS_HIP(hipEventCreate(&e0));
  TLS_HIP(hipEventCreate(&e1));
  local_solve(c, c->zero_int.p);  // warm-up
  TLS_HIP(hipEventRecord(e0, c->stream));
  for (int k = 0; k < reps; k++) local_solve(c, c->zero_int.p);
  TLS_HIP(hipEventRecord(e1, c->stream));
  TLS_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  TLS_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->solve_grid = keep;
  return ms / reps;
}

double time_symv(tls_ctx* c, int reps) {
  hipEvent_t e0, e1;
  TLS_HIP(hipEventCreate(&e0));
  TLS_HIP(hipEventCreate(&e1));
  local_solve(c, c->zero_int.p);  // warm-up
  TLS_HIP(hipEventRecord(e0, c->stream));
  for (int k = 0; k < reps; k++) local_solve(c, c->zero_int.p);
  TLS_HIP(hipEventRecord(e1, c->stream));
  TLS_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  TLS_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

}  // namespace

void choose_symv_block(tls_ctx* c) {
  if (!c->opt.autotune || !c->inv_formed) return;
  const std::string key = shape_key(c, "symv:v1");
  int b = 0;
  if (cache_lookup_ints(c->opt.tune_cache, key, &b, 1) && (b == 4 || b == 6 || b == 8)) {
    if (b != c->symv_block) {
      c->symv_block = b;
      build_symv_work(c->inv_work, c->stream, c->N, c->h_nt, c->h_foff, c->h_voff, c->fp32, b);
    }
    c->tuned = std::max(c->tuned, 2);
    return;
  }
  double best = 1e300;
  int best_b = c->symv_block;
  for (int cand : {4, 6, 8}) {
    c->symv_block = cand;
    build_symv_work(c->inv_work, c->stream, c->N, c->h_nt, c->h_foff, c->h_voff, c->fp32, cand);
    const double t = time_symv(c, 5);
    if (t < best) {
      best = t;
      best_b = cand;
    }
  }
  if (best_b != c->symv_block) {
    c->symv_block = best_b;
    build_symv_work(c->inv_work, c->stream, c->N, c->h_nt, c->h_foff, c->h_voff, c->fp32, best_b);
  }
  c->tuned = 1;
  cache_store_ints(c->opt.tune_cache, key, &best_b, 1);
}

void factor_local_tuned(tls_ctx* c) {
  if (!c->opt.autotune) {
    factor_local(c);
    return;
  }
  const std::string key = shape_key(c, "factor:v1");
  int pw = 0;
  if (cache_lookup_ints(c->opt.tune_cache, key, &pw, 1) && (pw == 4 || pw == 8 || pw == 16)) {
    c->factor_panel = pw;
    factor_local(c);
    return;
  }
  // the factorization works in place: the local matrices are gathered again
  // before each candidate (the default, 8, goes last and is kept if best)
  double best = 1e300;
  int best_pw = 8;
  const int cands[3] = {4, 16, 8};
  for (int q = 0; q < 3; q++) {
    if (q > 0) gather_local(c);
    c->factor_panel = cands[q];
    const auto t0 = std::chrono::steady_clock::now();
    factor_local(c);
    const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (t < best) {
      best = t;
      best_pw = cands[q];
    }
  }
  if (best_pw != cands[2]) {
    gather_local(c);
    c->factor_panel = best_pw;
    factor_local(c);
  }
  cache_store_ints(c->opt.tune_cache, key, &best_pw, 1);
}

void choose_solve_grid(tls_ctx* c) {
  const int cus = cu_count();
  const int per_cu = c->fp32 ? 4 : 3;
  c->solve_grid = cus * per_cu;
  c->tuned = 0;
  const int rows0 = c->opt.solve_rows > 0 ? c->opt.solve_rows : 1;
  const int order0 = c->opt.solve_order > 0 ? c->opt.solve_order : c->solve_order;
  if (order0 != c->solve_order || order0 != c->solve_order_b || rows0 != c->solve_rows)
    build_local_plans(c, order0, rows0);
  if (c->opt.solve_wgs > 0 || c->opt.solve_order > 0) {
    if (c->opt.solve_wgs > 0) c->solve_grid = c->opt.solve_wgs;
    return;
  }
  if (!c->opt.autotune || c->inv_formed) return;  // the symmetric product has no launch shape to tune
  // a solve_rows option fixes the rows per task; the rest is still tuned
  const std::string key = tune_key(c) + (c->opt.solve_rows > 0 ? " rows=" + std::to_string(c->opt.solve_rows) : "");
  int v[4] = {0, 0, 0, 0};
  if (cache_lookup_ints(c->opt.tune_cache, key, v, 4) && v[0] > 0 && v[1] >= 1 && v[1] <= 5 && v[2] >= 1 &&
      v[2] <= (c->fp32 ? 4 : 2) && v[3] >= 1 && v[3] <= 5) {
    c->solve_grid = v[0];
    if (v[1] != c->solve_order || v[3] != c->solve_order_b || v[2] != c->solve_rows)
      build_local_plans(c, v[1], v[2], v[3]);
    c->tuned = 2;
    return;
  }
  // rows per task and workgroups are shared by both directions; each
  // direction takes the task order that is fastest for it
  const int maxper = c->fp32 ? 7 : 3;
  constexpr int NORD = 5;
  double best = 1e300;
  int best_g = c->solve_grid, best_f = c->solve_order, best_b = c->solve_order_b, best_rows = c->solve_rows;
  for (int rows : {1, 2, 3, 4}) {
    if (c->opt.solve_rows > 0 && rows != c->opt.solve_rows) continue;
    if (!c->fp32 && rows > 2) continue;  // FP64 tasks hold at most two rows
    std::vector<int> grids;
    for (int p = 2; p <= maxper; p += 2) grids.push_back(cus * std::min(p, maxper));
    std::vector<double> tf(grids.size() * NORD, 1e300), tb(grids.size() * NORD, 1e300);
    for (int order = 1; order <= NORD; order++) {
      build_local_plans(c, order, rows);
      for (size_t g = 0; g < grids.size(); g++)
        time_local_dirs(c, grids[g], 3, &tf[g * NORD + order - 1], &tb[g * NORD + order - 1]);
    }
    for (size_t g = 0; g < grids.size(); g++) {
      int of = 1, ob = 1;
      for (int o = 2; o <= NORD; o++) {
        if (tf[g * NORD + o - 1] < tf[g * NORD + of - 1]) of = o;
        if (tb[g * NORD + o - 1] < tb[g * NORD + ob - 1]) ob = o;
      }
      const double t = tf[g * NORD + of - 1] + tb[g * NORD + ob - 1];
      if (t < best) {
        best = t;
        best_g = grids[g];
        best_f = of;
        best_b = ob;
        best_rows = rows;
      }
    }
  }
  if (best_f != c->solve_order || best_b != c->solve_order_b || best_rows != c->solve_rows)
    build_local_plans(c, best_f, best_rows, best_b);
  c->solve_grid = best_g;
  c->tuned = 1;
  const int pick[4] = {best_g, best_f, best_rows, best_b};
  cache_store_ints(c->opt.tune_cache, key, pick, 4);
}

}  // namespace tls
