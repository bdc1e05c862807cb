// Launch shape of the persistent triangular solves: workgroup count and
// task order.
//
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
#include <cstdio>
#include <fstream>
#include <sstream>

#include "kernels.hpp"

namespace tls {

namespace {

std::string tune_key(const tls_ctx* c) {
  std::ostringstream k;
  k << "trsv:v5 prec=" << (c->fp32 ? 32 : 64) << " kind=" << c->kind << " N=" << c->N << " n=" << c->n
    << " sumM=" << c->sum_M << " maxnt=" << c->max_nt;
  return k.str();
}

int cu_count() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus > 0 ? cus : 256;
}

bool cache_lookup(const char* path, const std::string& key, int* grid, int* order) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    auto tab = line.rfind('\t');
    if (tab == std::string::npos) continue;
    if (line.substr(0, tab) == key) {
      int g = 0, ch = 0;
      if (std::sscanf(line.c_str() + tab + 1, "%d %d", &g, &ch) == 2 && g > 0 && ch >= 1 && ch <= 5) {
        *grid = g;
        *order = ch;
        found = true;
      }
    }
  }
  return found;
}

void cache_store(const char* path, const std::string& key, int grid, int order) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  if (f) f << key << '\t' << grid << ' ' << order << '\n';
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

}  // namespace

void choose_solve_grid(tls_ctx* c) {
  const int cus = cu_count();
  const int per_cu = c->fp32 ? 4 : 3;
  c->solve_grid = cus * per_cu;
  c->tuned = 0;
  if (c->opt.solve_order > 0 && c->opt.solve_order != c->solve_order) build_local_plans(c, c->opt.solve_order);
  if (c->opt.solve_wgs > 0 || c->opt.solve_order > 0) {
    if (c->opt.solve_wgs > 0) c->solve_grid = c->opt.solve_wgs;
    return;
  }
  if (!c->opt.autotune || c->inv_formed) return;  // the symmetric product has no launch shape to tune
  const std::string key = tune_key(c);
  int g = 0, ch = 0;
  if (cache_lookup(c->opt.tune_cache, key, &g, &ch)) {
    c->solve_grid = g;
    if (ch != c->solve_order) build_local_plans(c, ch);
    c->tuned = 2;
    return;
  }
  const int maxper = c->fp32 ? 7 : 3;
  double best = 1e300;
  int best_g = c->solve_grid, best_ch = c->solve_order;
  for (int order : {1, 2, 3, 4, 5}) {
    build_local_plans(c, order);
    for (int p = 2; p <= maxper; p += 2) {
      const int cg = cus * std::min(p, maxper);
      double t = time_local_solves(c, cg, 3);
      if (t < best) {
        best = t;
        best_g = cg;
        best_ch = order;
      }
    }
  }
  if (best_ch != c->solve_order) build_local_plans(c, best_ch);
  c->solve_grid = best_g;
  c->tuned = 1;
  cache_store(c->opt.tune_cache, key, best_g, best_ch);
}

}  // namespace tls
