// Device helpers shared by the graph aggregations (compatible matching, classical smoothed
// aggregation): the SplitMix64 output function used to break ties at random, a lookup of
// a_{row, c} in a CSR row with ascending columns, and a scoped device buffer for setup.
#pragma once

#include <algorithm>

#include "internal.h"

namespace amgp {
namespace graph {

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__device__ __forceinline__ unsigned long long edge_hash(int lo, int hi) {
  return splitmix64(((unsigned long long)(unsigned)lo << 32) | (unsigned)hi);
}

// a_{row, c} from a row with ascending columns, or nothing
__device__ __forceinline__ bool find_entry(const int32_t* ptr, const int32_t* col, const double* val, int row, int c,
                                           double* out) {
  int lo = ptr[row], hi = ptr[row + 1] - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int cm = col[mid];
    if (cm == c) {
      *out = val[mid];
      return true;
    }
    if (cm < c) lo = mid + 1; else hi = mid - 1;
  }
  return false;
}

template <typename T>
struct DevBuf {
  T* p = nullptr;
  ~DevBuf() { hipFree(p); }
  int alloc(int64_t count) {
    return hipMalloc(&p, sizeof(T) * (size_t)std::max<int64_t>(count, 1)) == hipSuccess ? AMG_OK : AMG_ENOMEM;
  }
};

}  // namespace graph
}  // namespace amgp
