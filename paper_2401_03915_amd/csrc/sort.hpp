// Device sort of 64-bit keys (stable LSD radix, 8-bit digits). Used by the
// overlap construction, whose keys pack (subdomain, global row).
#pragma once

#include "common.hpp"

namespace tls {

// Sorts keys[0..count) ascending on bits [lo_bit, hi_bit); bits at or above
// hi_bit must be zero, and keys equal on the sorted bits keep their input
// order (so keys already ascending on bits below lo_bit end up fully
// sorted). `a` holds the input and `b` is scratch of the same size; the
// result is in the returned buffer (a or b). Synchronizes the stream.
uint64_t* radix_sort_u64(uint64_t* a, uint64_t* b, int count, int lo_bit, int hi_bit, hipStream_t s);

}  // namespace tls
