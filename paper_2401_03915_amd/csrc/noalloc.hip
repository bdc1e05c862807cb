// tls_solve_noalloc: the Krylov solve of tls_solve with no device
// allocation, for callers that cannot allocate.
//
// tls_solve keeps its Krylov vectors, reduction partials, flags and residual
// history in buffers that the context allocates on first use (and FGMRES its
// Hessenberg state). Here the same solver runs with that work in `scratch`,
// a file-scope device array of TLS_NOALLOC_SCRATCH_BYTES: every GPU that the
// library runs on holds its own copy until the process ends. Host code never
// takes the array's name as an address; at the first call on a device, with
// that device current, the array's device address is looked up with
// hipGetSymbolAddress and kept per device, and only that address reaches the
// kernels and the copies. Everything the solver needs at zero (reduction
// counter, stop flags, FGMRES state) is cleared by each call; the rest of the
// array keeps the previous call's contents. Calls on one GPU share the array,
// so calls that overlap on one GPU (several threads, or several streams
// without ordering) race.
#include <mutex>

#include "kernels.hpp"

namespace {

constexpr size_t kScratchBytes = TLS_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// device address of this device's copy of the array (looked up once)
unsigned char* scratch_address(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    TLS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) tls::fail(TLS_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch[dev] = static_cast<unsigned char*>(p);
  }
  return g_scratch[dev];
}

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// Carves the solver's work out of the scratch array; returns the bytes used.
size_t carve(const tls::KrylovNeeds& k, unsigned char* base, tls::KWork* w) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base ? base + o : nullptr;
    o += up256(bytes);
    return p;
  };
  w->done = reinterpret_cast<int*>(take(4 * sizeof(int)));
  w->gi = reinterpret_cast<int*>(take(4 * sizeof(int)));
  w->redctr = reinterpret_cast<unsigned*>(take(sizeof(unsigned)));
  w->scal = reinterpret_cast<double*>(take(16 * sizeof(double)));
  w->partial = reinterpret_cast<double*>(take(k.partial * sizeof(double)));
  w->hist = reinterpret_cast<double*>(take((size_t)k.hist * sizeof(double)));
  w->gm = reinterpret_cast<double*>(take(std::max<size_t>(k.gm, 1) * sizeof(double)));
  w->kr = reinterpret_cast<double*>(take(k.kr * sizeof(double)));
  w->context_bufs = false;
  return o;
}

}  // namespace

extern "C" tls_status tls_solve_noalloc(tls_ctx* c, const double* b, double* x, double tol, int32_t* iters,
                                        double* relres) {
  if (!c) return TLS_E_STATE;
  if (!b || !x || b == x || !(tol > 0.0)) {
    c->err = "b and x must be distinct non-NULL device vectors and tol > 0";
    return TLS_E_ARG;
  }
  bool conv = false;
  try {
    int dev = -1;
    TLS_HIP(hipGetDevice(&dev));
    if (dev != c->device) tls::fail(TLS_E_STATE, "the context's device must be current");
    if (dev < 0 || dev >= kMaxDevices) tls::fail(TLS_E_STATE, "device index beyond the scratch table");
    const tls::KrylovNeeds need = tls::krylov_needs(c);
    tls::KWork w;
    const size_t bytes = carve(need, nullptr, &w);
    if (bytes > kScratchBytes)
      tls::fail(TLS_E_ARG, "tls_solve_noalloc: the solver needs " + std::to_string(bytes) +
                               " bytes of work, more than the scratch array's " + std::to_string(kScratchBytes) +
                               " (n too large for this solver; use tls_solve)");
    carve(need, scratch_address(dev), &w);
    int it = 0;
    double rr = 0.0;
    tls::krylov_run(c, w, b, x, tol, &it, &rr, &conv);
    c->last_iters = it;
    c->last_relres = rr;
  } catch (const tls::TlsError& e) {
    c->err = e.msg;
    if (iters) *iters = c->last_iters;
    if (relres) *relres = c->last_relres;
    return e.code;
  } catch (const std::exception& e) {
    c->err = e.what();
    return TLS_E_HIP;
  }
  if (iters) *iters = c->last_iters;
  if (relres) *relres = c->last_relres;
  if (!conv) {
    c->err = "maximum number of iterations reached";
    return TLS_E_NOCONV;
  }
  return TLS_OK;
}
