// XCD-aware workgroup order for gfx950 (8 XCDs, one L2 each).
#pragma once
#include <hip/hip_runtime.h>

namespace pfft {

// The dispatcher sends workgroup b to XCD b % 8, and each XCD has its own
// L2; this bijection gives XCD x the contiguous range of logical blocks
// [x*(nb/8) + min(x, nb%8), ...), so logical neighbours, which read
// overlapping data, share one L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned x = b & 7u, k = b >> 3, q = nb >> 3, rem = nb & 7u;
  return x * q + (x < rem ? x : rem) + k;
}

}  // namespace pfft
