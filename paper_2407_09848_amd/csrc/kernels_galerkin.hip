// General sparse products for the hierarchies whose prolongator is not the
// plain 2x2x2 box indicator: the smoothed prolongator of Section 4,
// P = (I - omega D^{-1} A) P_hat, and box aggregates of any edge.  Setup only.
//
// * spgemm: C = X Y for CSR X (m x k) and Y (k x n), one wavefront per row of
//   C.  The distinct columns of the row are collected in an LDS hash table,
//   compacted and sorted; the values are then accumulated in X-row order
//   (the lanes of a wavefront take distinct entries of one Y row, so no two
//   lanes add to the same slot), which makes C bitwise reproducible.
// * drop_small: removes the entries whose magnitude is at most tau times the
//   largest of their row (tau = 2^-46): the Galerkin product and the smoothed
//   prolongator create exact cancellations that rounding turns into +-1e-17.
// * transpose: column counts, a scan, scatter, then each row of the
//   transpose sorted by column (unique keys), so the result is deterministic.
#include <algorithm>

#include "internal.h"

namespace amgp {

namespace {

constexpr int kMaxHash = 4096;  // distinct columns per product row (LDS table size)

__device__ __forceinline__ unsigned hslot(int key, int cap) {
  return ((unsigned)key * 2654435761u) & (unsigned)(cap - 1);
}

// Insert key into the table; returns 1 if it was new, 0 if present, -1 if the table is full.
template <int CAP>
__device__ __forceinline__ int hinsert(int32_t* keys, int key) {
  unsigned h = hslot(key, CAP);
  for (int probe = 0; probe < CAP; ++probe) {
    const int old = atomicCAS(&keys[h], -1, key);
    if (old == -1) return 1;
    if (old == key) return 0;
    h = (h + 1) & (CAP - 1);
  }
  return -1;
}

// Upper bound of the row lengths of X Y: sum over the X row of the Y row lengths.
__global__ void k_prod_bound(int64_t m, const int32_t* __restrict__ xp, const int32_t* __restrict__ xc,
                             const int32_t* __restrict__ yp, int32_t* __restrict__ bound) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  int64_t s = 0;
  for (int p = xp[i]; p < xp[i + 1]; ++p) s += yp[xc[p] + 1] - yp[xc[p]];
  bound[i] = (int32_t)std::min<int64_t>(s, INT32_MAX);
}

// Symbolic pass: cnt[i] = number of distinct columns of row i of X Y.
template <int CAP>
__global__ __launch_bounds__(kWave) void k_spgemm_count(int64_t m, const int32_t* __restrict__ xp,
                                                        const int32_t* __restrict__ xc,
                                                        const int32_t* __restrict__ yp,
                                                        const int32_t* __restrict__ yc, int32_t* __restrict__ cnt,
                                                        int* flag) {
  __shared__ int32_t keys[CAP];
  __shared__ int nk;
  __shared__ int full;
  const int64_t i = blockIdx.x;
  if (i >= m) return;
  for (int t = threadIdx.x; t < CAP; t += kWave) keys[t] = -1;
  if (threadIdx.x == 0) {
    nk = 0;
    full = 0;
  }
  __syncthreads();
  for (int p = xp[i]; p < xp[i + 1]; ++p) {
    const int j = xc[p];
    for (int q = yp[j] + threadIdx.x; q < yp[j + 1]; q += kWave) {
      const int r = hinsert<CAP>(keys, yc[q]);
      if (r == 1) atomicAdd(&nk, 1);
      if (r < 0) full = 1;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cnt[i] = nk;
    if (full || nk > CAP * 3 / 4) atomicOr(&flag[F_CAPACITY], 1);
  }
}

// Numeric pass: row i of X Y in columns cols[cptr[i] ...] (ascending) and values.
template <int CAP>
__global__ __launch_bounds__(kWave) void k_spgemm_fill(int64_t m, const int32_t* __restrict__ xp,
                                                       const int32_t* __restrict__ xc, const double* __restrict__ xv,
                                                       const int32_t* __restrict__ yp, const int32_t* __restrict__ yc,
                                                       const double* __restrict__ yv, const int32_t* __restrict__ cptr,
                                                       int32_t* __restrict__ ccol, double* __restrict__ cval) {
  __shared__ int32_t keys[CAP];
  __shared__ int32_t list[CAP];
  __shared__ double acc[CAP];
  __shared__ int nk;
  const int64_t i = blockIdx.x;
  if (i >= m) return;
  const int lane = threadIdx.x;
  for (int t = lane; t < CAP; t += kWave) keys[t] = -1;
  if (lane == 0) nk = 0;
  __syncthreads();
  for (int p = xp[i]; p < xp[i + 1]; ++p) {
    const int j = xc[p];
    for (int q = yp[j] + lane; q < yp[j + 1]; q += kWave) hinsert<CAP>(keys, yc[q]);
    __syncthreads();
  }
  // compact the occupied slots (their order is fixed by the table, not by timing)
  for (int t0 = 0; t0 < CAP; t0 += kWave) {
    const int key = keys[t0 + lane];
    const unsigned long long m_ = __ballot(key >= 0);
    const int before = __popcll(m_ & ((1ull << lane) - 1ull));
    const int base = nk;
    if (key >= 0) list[base + before] = key;
    __syncthreads();
    if (lane == 0) nk = base + __popcll(m_);
    __syncthreads();
  }
  const int len = nk;
  int pw = 1;
  while (pw < len) pw <<= 1;
  for (int t = len + lane; t < pw; t += kWave) list[t] = INT32_MAX;
  __syncthreads();
  // bitonic sort of list[0, pw)
  for (int size = 2; size <= pw; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = lane; t < pw; t += kWave) {
        const int u = t ^ stride;
        if (u > t) {
          const bool up = (t & size) == 0;
          const int a = list[t], b = list[u];
          if ((a > b) == up) {
            list[t] = b;
            list[u] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int t = lane; t < len; t += kWave) acc[t] = 0.0;
  __syncthreads();
  for (int p = xp[i]; p < xp[i + 1]; ++p) {
    const int j = xc[p];
    const double a = xv[p];
    for (int q = yp[j] + lane; q < yp[j + 1]; q += kWave) {
      const int key = yc[q];
      int lo = 0, hi = len - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (list[mid] < key) lo = mid + 1; else hi = mid;
      }
      acc[lo] += a * yv[q];
    }
    __syncthreads();
  }
  const int base = cptr[i];
  for (int t = lane; t < len; t += kWave) {
    ccol[base + t] = list[t];
    cval[base + t] = acc[t];
  }
}

__global__ void k_keep_count(int64_t m, const int32_t* __restrict__ ptr, const double* __restrict__ val, double tau,
                             int32_t* __restrict__ kept) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double mx = 0.0;
  for (int p = ptr[i]; p < ptr[i + 1]; ++p) mx = fmax(mx, fabs(val[p]));
  int c = 0;
  for (int p = ptr[i]; p < ptr[i + 1]; ++p) c += fabs(val[p]) > tau * mx;
  kept[i] = c;
}

__global__ void k_keep_copy(int64_t m, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                            const double* __restrict__ val, double tau, const int32_t* __restrict__ optr,
                            int32_t* __restrict__ ocol, double* __restrict__ oval) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double mx = 0.0;
  for (int p = ptr[i]; p < ptr[i + 1]; ++p) mx = fmax(mx, fabs(val[p]));
  int o = optr[i];
  for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
    if (fabs(val[p]) > tau * mx) {
      ocol[o] = col[p];
      oval[o] = val[p];
      ++o;
    }
  }
}

__global__ void k_col_count(int64_t nnz, const int32_t* __restrict__ col, int32_t* __restrict__ cnt) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nnz) atomicAdd(&cnt[col[q]], 1);
}

__global__ void k_transpose_scatter(int64_t m, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                    const double* __restrict__ val, const int32_t* __restrict__ tptr,
                                    int32_t* __restrict__ fill, int32_t* __restrict__ tcol,
                                    double* __restrict__ tval) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
    const int c = col[p];
    const int o = tptr[c] + atomicAdd(&fill[c], 1);
    tcol[o] = (int32_t)i;
    tval[o] = val[p];
  }
}

// Sorting the rows of the transpose by column (the keys of a row are distinct, so the result
// is unique): rows of up to kShortRow entries by one thread each (insertion sort), longer ones
// by one wavefront each (bitonic network in LDS, up to kSortCap entries).
constexpr int kShortRow = 64;
constexpr int kSortCap = 4096;

__device__ void insertion_sort_row(int32_t* __restrict__ col, double* __restrict__ val, int len) {
  for (int p = 1; p < len; ++p) {
    const int c = col[p];
    const double v = val[p];
    int q = p - 1;
    while (q >= 0 && col[q] > c) {
      col[q + 1] = col[q];
      val[q + 1] = val[q];
      --q;
    }
    col[q + 1] = c;
    val[q + 1] = v;
  }
}

__global__ void k_row_sort(int64_t m, const int32_t* __restrict__ ptr, int32_t* __restrict__ col,
                           double* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int b = ptr[i], len = ptr[i + 1] - b;
  if (len <= kShortRow) insertion_sort_row(col + b, val + b, len);
}

// One wavefront per listed row longer than kShortRow.
__global__ __launch_bounds__(kWave) void k_row_sort_long(const int32_t* __restrict__ rows,
                                                         const int32_t* __restrict__ ptr, int32_t* __restrict__ col,
                                                         double* __restrict__ val) {
  __shared__ int32_t key[kSortCap];
  __shared__ double v[kSortCap];
  const int i = rows[blockIdx.x];
  const int b = ptr[i], len = ptr[i + 1] - b;
  const int lane = threadIdx.x;
  if (len > kSortCap) {
    if (lane == 0) insertion_sort_row(col + b, val + b, len);
    return;
  }
  int pw = 1;
  while (pw < len) pw <<= 1;
  for (int t = lane; t < pw; t += kWave) {
    key[t] = t < len ? col[b + t] : INT_MAX;
    v[t] = t < len ? val[b + t] : 0.0;
  }
  __syncthreads();
  for (int size = 2; size <= pw; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = lane; t < pw; t += kWave) {
        const int u = t ^ stride;
        if (u > t) {
          const bool up = (t & size) == 0;
          const int ka = key[t], kb = key[u];
          if ((ka > kb) == up) {
            key[t] = kb;
            key[u] = ka;
            const double va = v[t];
            v[t] = v[u];
            v[u] = va;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int t = lane; t < len; t += kWave) {
    col[b + t] = key[t];
    val[b + t] = v[t];
  }
}

// Diagonal and ||row of D^{-1} A||_1 of every row; the largest ratio of each stacked problem is
// accumulated into lam[p] (non-negative doubles order like their bit patterns).
__global__ void k_diag_ratio(int64_t n, int64_t rpp, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                             const double* __restrict__ val, double* __restrict__ diag,
                             unsigned long long* __restrict__ lam, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 0.0, s = 0.0;
  for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
    if (col[p] == i) d = val[p];
    s += fabs(val[p]);
  }
  if (!(d > 0.0)) {
    atomicOr(&flag[F_NOTSPD], 1);
    d = 1.0;
  }
  diag[i] = d;
  atomicMax(&lam[i / rpp], (unsigned long long)__double_as_longlong(s / d));
}

// P = P_hat - omega_p D^{-1} (A P_hat), in place on the pattern of A P_hat, which holds the
// single entry (hcol[i], hval[i]) of row i of P_hat.
__global__ void k_smooth_prol(int64_t n, int64_t rpp, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                              double* __restrict__ val, const int32_t* __restrict__ hcol,
                              const double* __restrict__ hval, const double* __restrict__ diag,
                              const double* __restrict__ omega) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = omega[i / rpp] / diag[i];
  const int a = hcol[i];
  const double h = hval[i];
  for (int p = ptr[i]; p < ptr[i + 1]; ++p) val[p] = (col[p] == a ? h : 0.0) - s * val[p];
}

__global__ void k_identity_rows(int64_t n, const int32_t* __restrict__ agg, int32_t* __restrict__ ptr,
                                int32_t* __restrict__ col, double* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  ptr[i] = (int32_t)i;
  if (i < n) {
    col[i] = agg[i];
    val[i] = 1.0;
  }
}

template <int CAP>
void go_spgemm(bool fill, hipStream_t s, int64_t m, const Csr& X, const Csr& Y, int32_t* cnt, const int32_t* cptr,
               int32_t* ccol, double* cval, int* flag) {
  if (!fill)
    hipLaunchKernelGGL(k_spgemm_count<CAP>, dim3((unsigned)m), dim3(kWave), 0, s, m, X.ptr, X.col, Y.ptr, Y.col,
                       cnt, flag);
  else
    hipLaunchKernelGGL(k_spgemm_fill<CAP>, dim3((unsigned)m), dim3(kWave), 0, s, m, X.ptr, X.col, X.val, Y.ptr,
                       Y.col, Y.val, cptr, ccol, cval);
}

int run_spgemm(int cap, bool fill, hipStream_t s, int64_t m, const Csr& X, const Csr& Y, int32_t* cnt,
               const int32_t* cptr, int32_t* ccol, double* cval, int* flag) {
  switch (cap) {
    case 64: go_spgemm<64>(fill, s, m, X, Y, cnt, cptr, ccol, cval, flag); break;
    case 128: go_spgemm<128>(fill, s, m, X, Y, cnt, cptr, ccol, cval, flag); break;
    case 256: go_spgemm<256>(fill, s, m, X, Y, cnt, cptr, ccol, cval, flag); break;
    case 512: go_spgemm<512>(fill, s, m, X, Y, cnt, cptr, ccol, cval, flag); break;
    case 1024: go_spgemm<1024>(fill, s, m, X, Y, cnt, cptr, ccol, cval, flag); break;
    case 2048: go_spgemm<2048>(fill, s, m, X, Y, cnt, cptr, ccol, cval, flag); break;
    default: go_spgemm<4096>(fill, s, m, X, Y, cnt, cptr, ccol, cval, flag); break;
  }
  return hipGetLastError() == hipSuccess ? AMG_OK : AMG_EHIP;
}

int read_flag(hipStream_t s, const int* flag, int which) {
  int h[F_NFLAG];
  if (hipMemcpyAsync(h, flag, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  return h[which];
}

}  // namespace

// Host exclusive scan of cnt[0, m) into ptr[0, m]; returns the total or -1 beyond int32.
int64_t scan_ptr(hipStream_t s, int64_t m, const int32_t* cnt, int32_t* ptr, int* rc) {
  std::vector<int32_t> h(m);
  *rc = AMG_OK;
  if (m > 0 && hipMemcpyAsync(h.data(), cnt, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s) != hipSuccess) {
    *rc = AMG_EHIP;
    return -1;
  }
  if (hipStreamSynchronize(s) != hipSuccess) {
    *rc = AMG_EHIP;
    return -1;
  }
  std::vector<int32_t> p(m + 1);
  int64_t acc = 0;
  for (int64_t i = 0; i < m; ++i) {
    p[i] = (int32_t)acc;
    acc += h[i];
    if (acc >= (int64_t)INT32_MAX) {
      *rc = AMG_ECAPACITY;
      return -1;
    }
  }
  p[m] = (int32_t)acc;
  if (hipMemcpyAsync(ptr, p.data(), sizeof(int32_t) * (m + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    *rc = AMG_EHIP;
    return -1;
  }
  return acc;
}

void free_csr(Csr& a) {
  hipFree(a.ptr);
  hipFree(a.col);
  hipFree(a.val);
  a = Csr();
}

int spgemm(hipStream_t s, const Csr& X, const Csr& Y, Csr* C, int* flag) {
  const int64_t m = X.m;
  *C = Csr();
  if (m <= 0 || m > (int64_t)UINT32_MAX) return AMG_EINVAL;
  int32_t* cnt = nullptr;
  if (hipMalloc(&cnt, sizeof(int32_t) * (m + 1)) != hipSuccess) return AMG_ENOMEM;
  // table size: the smallest power of two of at least twice the longest row bound
  hipLaunchKernelGGL(k_prod_bound, dim3(grid_for(m)), dim3(kBlock), 0, s, m, X.ptr, X.col, Y.ptr, cnt);
  std::vector<int32_t> hb(m);
  int rc = AMG_OK;
  if (hipMemcpyAsync(hb.data(), cnt, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    hipFree(cnt);
    return AMG_EHIP;
  }
  const int64_t bound = *std::max_element(hb.begin(), hb.end());
  int cap = 64;
  while (cap < 2 * bound && cap < kMaxHash) cap <<= 1;
  rc = run_spgemm(cap, false, s, m, X, Y, cnt, nullptr, nullptr, nullptr, flag);
  if (rc != AMG_OK) {
    hipFree(cnt);
    return rc;
  }
  const int full = read_flag(s, flag, F_CAPACITY);
  if (full != 0) {
    hipFree(cnt);
    return full < 0 ? AMG_EHIP : AMG_ECAPACITY;
  }
  Csr c;
  c.m = m;
  c.ncols = Y.ncols;
  if (hipMalloc(&c.ptr, sizeof(int32_t) * (m + 1)) != hipSuccess) {
    hipFree(cnt);
    return AMG_ENOMEM;
  }
  const int64_t nnz = scan_ptr(s, m, cnt, c.ptr, &rc);
  hipFree(cnt);
  if (rc != AMG_OK) {
    free_csr(c);
    return rc;
  }
  c.nnz = nnz;
  if (hipMalloc(&c.col, sizeof(int32_t) * std::max<int64_t>(nnz, 1)) != hipSuccess ||
      hipMalloc(&c.val, sizeof(double) * std::max<int64_t>(nnz, 1)) != hipSuccess) {
    free_csr(c);
    return AMG_ENOMEM;
  }
  rc = run_spgemm(cap, true, s, m, X, Y, nullptr, c.ptr, c.col, c.val, flag);
  if (rc == AMG_OK && hipStreamSynchronize(s) != hipSuccess) rc = AMG_EHIP;
  if (rc != AMG_OK) {
    free_csr(c);
    return rc;
  }
  *C = c;
  return AMG_OK;
}

int drop_small(hipStream_t s, Csr* a, double tau) {
  Csr o;
  o.m = a->m;
  o.ncols = a->ncols;
  int32_t* kept = nullptr;
  if (hipMalloc(&kept, sizeof(int32_t) * (a->m + 1)) != hipSuccess) return AMG_ENOMEM;
  hipLaunchKernelGGL(k_keep_count, dim3(grid_for(a->m)), dim3(kBlock), 0, s, a->m, a->ptr, a->val, tau, kept);
  if (hipMalloc(&o.ptr, sizeof(int32_t) * (a->m + 1)) != hipSuccess) {
    hipFree(kept);
    return AMG_ENOMEM;
  }
  int rc = AMG_OK;
  o.nnz = scan_ptr(s, a->m, kept, o.ptr, &rc);
  hipFree(kept);
  if (rc != AMG_OK) {
    free_csr(o);
    return rc;
  }
  if (hipMalloc(&o.col, sizeof(int32_t) * std::max<int64_t>(o.nnz, 1)) != hipSuccess ||
      hipMalloc(&o.val, sizeof(double) * std::max<int64_t>(o.nnz, 1)) != hipSuccess) {
    free_csr(o);
    return AMG_ENOMEM;
  }
  hipLaunchKernelGGL(k_keep_copy, dim3(grid_for(a->m)), dim3(kBlock), 0, s, a->m, a->ptr, a->col, a->val, tau,
                     o.ptr, o.col, o.val);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    free_csr(o);
    return AMG_EHIP;
  }
  free_csr(*a);
  *a = o;
  return AMG_OK;
}

int transpose(hipStream_t s, const Csr& a, Csr* t) {
  Csr o;
  o.m = a.ncols;
  o.ncols = a.m;
  o.nnz = a.nnz;
  int32_t* cnt = nullptr;
  if (hipMalloc(&cnt, sizeof(int32_t) * (o.m + 1)) != hipSuccess) return AMG_ENOMEM;
  int rc = AMG_OK;
  if (hipMemsetAsync(cnt, 0, sizeof(int32_t) * (o.m + 1), s) != hipSuccess) rc = AMG_EHIP;
  if (rc == AMG_OK) {
    hipLaunchKernelGGL(k_col_count, dim3(grid_for(a.nnz)), dim3(kBlock), 0, s, a.nnz, a.col, cnt);
    if (hipMalloc(&o.ptr, sizeof(int32_t) * (o.m + 1)) != hipSuccess) rc = AMG_ENOMEM;
  }
  if (rc == AMG_OK) scan_ptr(s, o.m, cnt, o.ptr, &rc);
  if (rc == AMG_OK && (hipMalloc(&o.col, sizeof(int32_t) * std::max<int64_t>(o.nnz, 1)) != hipSuccess ||
                       hipMalloc(&o.val, sizeof(double) * std::max<int64_t>(o.nnz, 1)) != hipSuccess))
    rc = AMG_ENOMEM;
  if (rc == AMG_OK && hipMemsetAsync(cnt, 0, sizeof(int32_t) * (o.m + 1), s) != hipSuccess) rc = AMG_EHIP;
  if (rc == AMG_OK) {
    hipLaunchKernelGGL(k_transpose_scatter, dim3(grid_for(a.m)), dim3(kBlock), 0, s, a.m, a.ptr, a.col, a.val,
                       o.ptr, cnt, o.col, o.val);
    hipLaunchKernelGGL(k_row_sort, dim3(grid_for(o.m)), dim3(kBlock), 0, s, o.m, o.ptr, o.col, o.val);
    if (hipGetLastError() != hipSuccess) rc = AMG_EHIP;
  }
  if (rc == AMG_OK) {
    // the rows longer than kShortRow, listed on the host from the row pointers
    std::vector<int32_t> hp(o.m + 1);
    std::vector<int32_t> longrows;
    if (hipMemcpyAsync(hp.data(), o.ptr, sizeof(int32_t) * (o.m + 1), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = AMG_EHIP;
    } else {
      for (int64_t i = 0; i < o.m; ++i)
        if (hp[i + 1] - hp[i] > kShortRow) longrows.push_back((int32_t)i);
    }
    if (rc == AMG_OK && !longrows.empty()) {
      int32_t* drows = nullptr;
      if (hipMalloc(&drows, sizeof(int32_t) * longrows.size()) != hipSuccess) {
        rc = AMG_ENOMEM;
      } else {
        if (hipMemcpyAsync(drows, longrows.data(), sizeof(int32_t) * longrows.size(), hipMemcpyHostToDevice, s) !=
            hipSuccess)
          rc = AMG_EHIP;
        if (rc == AMG_OK)
          hipLaunchKernelGGL(k_row_sort_long, dim3((unsigned)longrows.size()), dim3(kWave), 0, s, drows, o.ptr, o.col,
                             o.val);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) rc = AMG_EHIP;
        hipFree(drows);
      }
    }
  }
  hipFree(cnt);
  if (rc != AMG_OK) {
    free_csr(o);
    return rc;
  }
  *t = o;
  return AMG_OK;
}

int tentative_prolongator(hipStream_t s, int64_t n, int64_t nc, const int32_t* agg, Csr* P) {
  Csr o;
  o.m = n;
  o.ncols = nc;
  o.nnz = n;
  if (hipMalloc(&o.ptr, sizeof(int32_t) * (n + 1)) != hipSuccess ||
      hipMalloc(&o.col, sizeof(int32_t) * n) != hipSuccess || hipMalloc(&o.val, sizeof(double) * n) != hipSuccess) {
    free_csr(o);
    return AMG_ENOMEM;
  }
  hipLaunchKernelGGL(k_identity_rows, dim3(grid_for(n + 1)), dim3(kBlock), 0, s, n, agg, o.ptr, o.col, o.val);
  if (hipGetLastError() != hipSuccess) {
    free_csr(o);
    return AMG_EHIP;
  }
  *P = o;
  return AMG_OK;
}

int smoothed_prolongator(hipStream_t s, const Csr& A, int nbatch, const Csr& Ph, Csr* P, int* flag) {
  const int64_t n = A.m, rpp = n / nbatch;
  Csr AP;
  int rc = spgemm(s, A, Ph, &AP, flag);
  if (rc != AMG_OK) return rc;
  double* diag = nullptr;
  unsigned long long* lam = nullptr;
  double* om = nullptr;
  if (hipMalloc(&diag, sizeof(double) * n) != hipSuccess || hipMalloc(&lam, sizeof(unsigned long long) * nbatch) !=
      hipSuccess || hipMalloc(&om, sizeof(double) * nbatch) != hipSuccess)
    rc = AMG_ENOMEM;
  std::vector<double> hl(nbatch), ho(nbatch);
  if (rc == AMG_OK && hipMemsetAsync(lam, 0, sizeof(unsigned long long) * nbatch, s) != hipSuccess) rc = AMG_EHIP;
  if (rc == AMG_OK) {
    hipLaunchKernelGGL(k_diag_ratio, dim3(grid_for(n)), dim3(kBlock), 0, s, n, rpp, A.ptr, A.col, A.val, diag, lam,
                       flag);
    if (hipMemcpyAsync(hl.data(), lam, sizeof(double) * nbatch, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      rc = AMG_EHIP;
  }
  if (rc == AMG_OK) {
    // omega = 4 / (3 lambda), lambda = ||D^{-1} A||_inf per stacked problem
    for (int p = 0; p < nbatch; ++p) ho[p] = 4.0 / (3.0 * hl[p]);
    if (hipMemcpyAsync(om, ho.data(), sizeof(double) * nbatch, hipMemcpyHostToDevice, s) != hipSuccess) rc = AMG_EHIP;
  }
  if (rc == AMG_OK) {
    hipLaunchKernelGGL(k_smooth_prol, dim3(grid_for(n)), dim3(kBlock), 0, s, n, rpp, AP.ptr, AP.col, AP.val, Ph.col,
                       Ph.val, diag, om);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) rc = AMG_EHIP;
  }
  hipFree(diag);
  hipFree(lam);
  hipFree(om);
  if (rc == AMG_OK) rc = drop_small(s, &AP, kDropTau);
  if (rc != AMG_OK) {
    free_csr(AP);
    return rc;
  }
  *P = AP;
  return AMG_OK;
}

int galerkin_general(hipStream_t s, const Csr& A, const Csr& P, const Csr& PT, Csr* Ac, int* flag) {
  Csr AP;
  AMGP_TRY(spgemm(s, A, P, &AP, flag));
  const int rc = spgemm(s, PT, AP, Ac, flag);
  free_csr(AP);
  if (rc != AMG_OK) return rc;
  return drop_small(s, Ac, kDropTau);
}

}  // namespace amgp
