// Device exclusive prefix sums (three passes: block scan, scan of block
// totals, add-back). Deterministic; used for CSR-like offset arrays.
#pragma once

#include "common.hpp"

namespace tls {

// out[0..count] = exclusive scan of in[0..count), out[count] = total.
// in and out may alias only if they are the same pointer.
void scan_exclusive_i32(const int* in, int* out, int count, hipStream_t s);
void scan_exclusive_i64(const int64_t* in, int64_t* out, int count, hipStream_t s);

}  // namespace tls
