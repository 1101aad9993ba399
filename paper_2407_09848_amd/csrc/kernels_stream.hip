// Bandwidth ceiling of the HBM on this GPU, measured with kernels of known
// byte counts: a plain read (a sum) and a plain copy of a float64 array.
//
// Both use 16-byte nontemporal loads (and stores) and a grid-stride loop over a
// fixed grid of AMG_HBM_PARTIALS blocks of 256 threads (64 per CU), with eight
// (read) or two (copy) independent loads in flight per thread: the shape that
// measured fastest among grids of 1024..16384 blocks and unrolls of 2..8
// (read 6.7 TB/s, copy 5.2 TB/s on 4 GiB arrays).  They are the
// reference the smoother kernels are compared with: the smoother steps read
// and write their vectors once per step, so no kernel on the path can move
// more bytes per second than these.
#include "internal.h"

namespace amgp {

namespace {

typedef double f64x2 __attribute__((ext_vector_type(2)));

constexpr int kReadUnroll = 8;
constexpr int kCopyUnroll = 2;

__device__ __forceinline__ f64x2 ld_nt(const f64x2* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_nt(f64x2* p, f64x2 v) { __builtin_nontemporal_store(v, p); }

// part[block] = sum of the pairs the block visits (pairs i = block * 256 + t + m * stride),
// and block 0 adds the odd last element.
__global__ __launch_bounds__(kBlock) void k_hbm_read(int64_t n, const double* __restrict__ x,
                                                     double* __restrict__ part) {
  const int64_t n2 = n >> 1;
  const f64x2* x2 = reinterpret_cast<const f64x2*>(x);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  f64x2 acc[kReadUnroll];
#pragma unroll
  for (int u = 0; u < kReadUnroll; ++u) acc[u] = f64x2{0.0, 0.0};
  for (; i + (kReadUnroll - 1) * stride < n2; i += kReadUnroll * stride) {
    f64x2 v[kReadUnroll];
#pragma unroll
    for (int u = 0; u < kReadUnroll; ++u) v[u] = ld_nt(x2 + i + u * stride);
#pragma unroll
    for (int u = 0; u < kReadUnroll; ++u) acc[u] += v[u];
  }
  for (; i < n2; i += stride) acc[0] += ld_nt(x2 + i);
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < kReadUnroll; ++u) s += acc[u].x + acc[u].y;
  if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) s += x[n - 1];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
  __shared__ double sm[kBlock / kWave];
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) t += sm[w];
    part[blockIdx.x] = t;
  }
}

// y = x, pairs as in k_hbm_read
__global__ __launch_bounds__(kBlock) void k_hbm_copy(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t n2 = n >> 1;
  const f64x2* x2 = reinterpret_cast<const f64x2*>(x);
  f64x2* y2 = reinterpret_cast<f64x2*>(y);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  for (; i + (kCopyUnroll - 1) * stride < n2; i += kCopyUnroll * stride) {
    f64x2 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) v[u] = ld_nt(x2 + i + u * stride);
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) st_nt(y2 + i + u * stride, v[u]);
  }
  for (; i < n2; i += stride) st_nt(y2 + i, ld_nt(x2 + i));
  if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) y[n - 1] = x[n - 1];
}

}  // namespace

int launch_hbm_read(hipStream_t s, int64_t n, const double* x, double* part) {
  hipLaunchKernelGGL(k_hbm_read, dim3(AMG_HBM_PARTIALS), dim3(kBlock), 0, s, n, x, part);
  return hipGetLastError() == hipSuccess ? AMG_OK : AMG_EHIP;
}

int launch_hbm_copy(hipStream_t s, int64_t n, const double* x, double* y) {
  hipLaunchKernelGGL(k_hbm_copy, dim3(AMG_HBM_PARTIALS), dim3(kBlock), 0, s, n, x, y);
  return hipGetLastError() == hipSuccess ? AMG_OK : AMG_EHIP;
}

}  // namespace amgp
