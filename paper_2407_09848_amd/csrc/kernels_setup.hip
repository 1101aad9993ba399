// Setup kernels: l1-Jacobi diagonal, CSR -> sliced ELL, box aggregation and the
// Galerkin product A_c = P^T A P for a piecewise-constant P.
#include <algorithm>
#include <vector>

#include <climits>

#include "internal.h"

namespace amgp {

namespace {

// CSR validation, in two passes so that nothing is read through an
// unchecked index: first row_ptr alone, then the column indices.
__global__ void k_check_ptr(int64_t n, int64_t nnz, const int32_t* __restrict__ ptr, int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  const int32_t v = ptr[i];
  if (i == 0 && v != 0) flag[F_BADCSR] = 1;
  if (i == n && v != nnz) flag[F_BADCSR] = 1;
  if (i < n && (ptr[i + 1] < v || v < 0 || v > nnz)) flag[F_BADCSR] = 1;
}

__global__ void k_check_col(int64_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                            int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t prev = -1;
  for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
    const int32_t c = col[p];
    if (c <= prev || c >= n) flag[F_BADCSR] = 1;
    prev = c;
  }
}

// M_i = a_ii + sum_{j != i} |a_ij| (eq. l1smooth); minv = 1/M.  Flags a
// non-positive or non-finite diagonal or l1 sum as "not SPD".
__global__ void k_l1_diag(int64_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                          const double* __restrict__ val, double* __restrict__ minv, int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 0.0, off = 0.0;
  bool has_diag = false;
  for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
    const double v = val[p];
    if (col[p] == i) {
      d += v;
      has_diag = true;
    } else {
      off += fabs(v);
    }
  }
  const double m = d + off;
  if (!has_diag || !(d > 0.0) || !(m > 0.0) || m > 1.0e308) flag[F_NOTSPD] = 1;
  minv[i] = 1.0 / m;
}

// width of every slice of R rows = longest row in it
__global__ void k_slice_width(int64_t n, int64_t nslices, int R, const int32_t* __restrict__ ptr,
                              int32_t* __restrict__ w) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslices) return;
  int m = 0;
  for (int l = 0; l < R; ++l) {
    const int64_t i = s * R + l;
    if (i >= n) break;
    m = max(m, ptr[i + 1] - ptr[i]);
  }
  w[s] = m;
}

// one thread per (slice, lane): lane l of slice s serves row s R + l / G, entries j = l % G + G t
__global__ void k_ell_fill(int64_t n, int64_t ncols, int64_t nslices, int G, const int32_t* __restrict__ ptr,
                           const int32_t* __restrict__ col, const double* __restrict__ val,
                           const int32_t* __restrict__ sptr, int32_t* __restrict__ ecol, double* __restrict__ eval) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslices * kSlice) return;
  const int64_t s = t / kSlice;
  const int lane = (int)(t % kSlice);
  const int64_t i = s * (kSlice / G) + lane / G;
  const int g = lane % G;
  const int base = sptr[s];
  const int steps = (sptr[s + 1] - base) / kSlice;
  int len = 0, p0 = 0;
  if (i < n) {
    p0 = ptr[i];
    len = ptr[i + 1] - p0;
  }
  const int32_t padcol = (i < n && i < ncols) ? (int32_t)i : 0;
  for (int st = 0; st < steps; ++st) {
    const int j = st * G + g;
    const int64_t q = base + (int64_t)st * kSlice + lane;
    if (j < len) {
      ecol[q] = col[p0 + j];
      eval[q] = val[p0 + j];
    } else {
      ecol[q] = padcol;
      eval[q] = 0.0;
    }
  }
}

// Distinct column offsets (col - row, or col - anchor[row * astride]) of every 64-row slice,
// sorted: offs[s * 64 + t], count width[s] (-1 when there are more than 64).  One wavefront per
// slice, an LDS hash set.
constexpr int kOffHash = 256;
constexpr int kOffEmpty = INT_MIN;

__global__ __launch_bounds__(kWave) void k_slice_offsets(int64_t n, const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ col, const int32_t* anchor,
                                                         int astride, int32_t* __restrict__ offs,
                                                         int32_t* __restrict__ width) {
  __shared__ int set[kOffHash];
  __shared__ int list[kOffHash];
  __shared__ int cnt;
  const int64_t s = blockIdx.x;
  const int lane = threadIdx.x;
  for (int t = lane; t < kOffHash; t += kWave) set[t] = kOffEmpty;
  if (lane == 0) cnt = 0;
  __syncthreads();
  const int64_t r = s * kSlice + lane;
  if (r < n) {
    const int base = anchor ? anchor[r * astride] : (int)r;
    for (int p = ptr[r]; p < ptr[r + 1]; ++p) {
      const int o = col[p] - base;
      unsigned h = ((unsigned)o * 2654435761u) & (kOffHash - 1);
      for (int probe = 0; probe < kOffHash; ++probe) {
        const int old = atomicCAS(&set[h], kOffEmpty, o);
        if (old == kOffEmpty) {
          atomicAdd(&cnt, 1);
          break;
        }
        if (old == o) break;
        h = (h + 1) & (kOffHash - 1);
      }
    }
  }
  __syncthreads();
  const int c = cnt;
  if (c > kSlice) {
    if (lane == 0) width[s] = -1;
    return;
  }
  // compact (slot order), then an odd-even transposition sort of at most 64 values by the wavefront
  __shared__ int k;
  if (lane == 0) k = 0;
  __syncthreads();
  for (int t = lane; t < kOffHash; t += kWave) {
    const int v = set[t];
    if (v != kOffEmpty) list[atomicAdd(&k, 1)] = v;
  }
  __syncthreads();
  for (int phase = 0; phase < c; ++phase) {
    const int i = 2 * lane + (phase & 1);
    if (i + 1 < c && list[i] > list[i + 1]) {
      const int a = list[i];
      list[i] = list[i + 1];
      list[i + 1] = a;
    }
    __syncthreads();
  }
  if (lane < c) offs[s * kSlice + lane] = list[lane];
  if (lane == 0) width[s] = c;
}

// Offset-aligned fill: lane l of slice s (row r, anchor a = r or anchor[r * astride]) puts, at
// step t, its entry of column a + offs[t] (0 when the row has none), with the steps of a lane in
// pairs: step t at 64 (t - t % 2) + 2 l + t % 2 while t has a partner, an odd last step at 64 t + l.
__global__ void k_ell_fill_aligned(int64_t n, int64_t nslices, const int32_t* __restrict__ ptr,
                                   const int32_t* __restrict__ col, const double* __restrict__ val,
                                   const int32_t* anchor, int astride, const int32_t* __restrict__ offs,
                                   const int32_t* __restrict__ sptr, double* __restrict__ eval,
                                   int32_t* __restrict__ doff) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslices * kSlice) return;
  const int64_t s = t / kSlice;
  const int lane = (int)(t % kSlice);
  const int64_t r = s * kSlice + lane;
  const int base = sptr[s];
  const int steps = (sptr[s + 1] - base) / kSlice;
  int p = 0, pe = 0;
  int64_t a = r;
  if (r < n) {
    p = ptr[r];
    pe = ptr[r + 1];
    if (anchor) a = anchor[r * astride];
  }
  const int paired = steps & ~1;
  for (int st = 0; st < steps; ++st) {
    const int o = offs[s * kSlice + st];
    const int64_t c = a + o;
    double v = 0.0;
    while (p < pe && col[p] < c) ++p;
    if (p < pe && col[p] == c) v = val[p++];
    const int dst = st < paired ? kSlice * (st & ~1) + 2 * lane + (st & 1) : kSlice * st + lane;
    eval[base + dst] = v;
    if (lane == 0) doff[(base >> 6) + st] = o;
  }
}

__global__ void k_round_f32(int64_t m, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) b[i] = (float)a[i];
}

// FP32 copy of offset-aligned slices: slices of at least kQuadMinSteps steps put each lane's steps in
// quads (step t of lane l at 64 (t - t % 4) + 4 l + t % 4 for t below w - w % 4, then a pair at
// 64 (t - t % 2) + 2 l + t % 2, then a single step at 64 t + l), narrower ones keep the FP64 pairs.
__global__ void k_round_f32_aligned(int64_t nslices, const int32_t* __restrict__ sptr, const double* __restrict__ a,
                                    float* __restrict__ b) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t s = g >> 6;
  const int lane = (int)(g & 63);
  if (s >= nslices) return;
  const int beg = sptr[s];
  const int w = (sptr[s + 1] - beg) >> 6;
  const int w2 = w & ~1, w4 = w >= kQuadMinSteps ? (w & ~3) : 0;
  for (int t = 0; t < w; ++t) {
    const int pair = t < w2 ? 64 * (t & ~1) + 2 * lane + (t & 1) : 64 * t + lane;
    const int dst = t < w4 ? 64 * (t & ~3) + 4 * lane + (t & 3) : pair;
    b[beg + dst] = (float)a[beg + pair];
  }
}


// Box aggregates of edge e: row (i, j, k) of problem p -> coarse (i/e, j/e, k/e) of
// problem p; an axis of extent 1 is not coarsened.  For e = 2, children[I*8 + c]
// lists the rows of aggregate I in ascending order (z, then y, then x), -1 padded.
__global__ void k_agg(int64_t n, int nx, int ny, int nz, int e, int cx, int cy, int cz, int32_t* __restrict__ agg) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t per = (int64_t)nx * ny * nz;
  const int64_t p = r / per, q = r % per;
  const int i = (int)(q % nx), j = (int)((q / nx) % ny), k = (int)(q / ((int64_t)nx * ny));
  const int ci = nx == 1 ? i : i / e, cj = ny == 1 ? j : j / e, ck = nz == 1 ? k : k / e;
  agg[r] = (int32_t)(p * (int64_t)cx * cy * cz + ci + (int64_t)cx * cj + (int64_t)cx * cy * ck);
}

__global__ void k_children(int64_t nc, int nx, int ny, int nz, int cx, int cy, int cz, int32_t* __restrict__ ch) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int64_t cper = (int64_t)cx * cy * cz, per = (int64_t)nx * ny * nz;
  const int64_t p = I / cper, q = I % cper;
  const int ci = (int)(q % cx), cj = (int)((q / cx) % cy), ck = (int)(q / ((int64_t)cx * cy));
  const int sx = nx == 1 ? 1 : 2, sy = ny == 1 ? 1 : 2, sz = nz == 1 ? 1 : 2;
  int c = 0;
  for (int dz = 0; dz < sz; ++dz) {
    const int k = ck * sz + dz;
    if (k >= nz) continue;
    for (int dy = 0; dy < sy; ++dy) {
      const int j = cj * sy + dy;
      if (j >= ny) continue;
      for (int dx = 0; dx < sx; ++dx) {
        const int i = ci * sx + dx;
        if (i >= nx) continue;
        ch[I * kMaxChildren + c++] = (int32_t)(p * per + i + (int64_t)nx * j + (int64_t)nx * ny * k);
      }
    }
  }
  for (; c < kMaxChildren; ++c) ch[I * kMaxChildren + c] = -1;
}

// Galerkin row I of P^T A P: sum the entries of the aggregate's rows, mapping
// column j to agg[j].  Columns kept sorted in a small per-thread list
// (insertion), duplicates merged.  Pass 0 counts, pass 1 writes.
constexpr int kRapCap = 64;

template <bool FILL>
__global__ __launch_bounds__(64) void k_rap(int64_t nc, const int32_t* __restrict__ ptr,
                                            const int32_t* __restrict__ col, const double* __restrict__ val,
                                            const int32_t* __restrict__ agg, const int32_t* __restrict__ ch,
                                            int32_t* __restrict__ cnt_or_ptr, int32_t* __restrict__ ccol,
                                            double* __restrict__ cval, int* __restrict__ flag) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  int32_t cols[kRapCap];
  double vals[kRapCap];
  int m = 0;
  bool over = false;
  for (int c = 0; c < kMaxChildren; ++c) {
    const int i = ch[I * kMaxChildren + c];
    if (i < 0) break;
    for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
      const int32_t J = agg[col[p]];
      const double v = val[p];
      int pos = m;
      while (pos > 0 && cols[pos - 1] > J) --pos;
      if (pos > 0 && cols[pos - 1] == J) {
        vals[pos - 1] += v;
      } else if (m < kRapCap) {
        for (int t = m; t > pos; --t) {
          cols[t] = cols[t - 1];
          vals[t] = vals[t - 1];
        }
        cols[pos] = J;
        vals[pos] = v;
        ++m;
      } else {
        over = true;
      }
    }
  }
  if (over) flag[F_CAPACITY] = 1;
  if (!FILL) {
    cnt_or_ptr[I] = m;
  } else {
    const int base = cnt_or_ptr[I];
    for (int t = 0; t < m; ++t) {
      ccol[base + t] = cols[t];
      cval[base + t] = vals[t];
    }
  }
}

__global__ void k_to_dense(int64_t total_rows, int64_t nl, int64_t np, const int32_t* __restrict__ ptr,
                           const int32_t* __restrict__ col, const double* __restrict__ val,
                           double* __restrict__ dense, int* __restrict__ flag) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= total_rows) return;
  const int64_t p = r / np, lr = r % np;
  double* row = dense + p * np * np + lr * np;
  for (int64_t j = 0; j < np; ++j) row[j] = 0.0;
  if (lr >= nl) {
    row[lr] = 1.0;  // padding: identity
    return;
  }
  const int64_t g = p * nl + lr;
  for (int q = ptr[g]; q < ptr[g + 1]; ++q) {
    const int64_t c = col[q] - p * nl;
    if (c >= 0 && c < nl) {
      row[c] = val[q];
    } else {
      flag[F_NOTSPD] = 1;  // coupling between stacked problems: not block diagonal
    }
  }
}

}  // namespace

int validate_csr(hipStream_t s, int64_t n, int64_t nnz, const int32_t* ptr, const int32_t* col, int* flag) {
  int h[F_NFLAG];
  hipLaunchKernelGGL(k_check_ptr, dim3(grid_for(n + 1)), dim3(kBlock), 0, s, n, nnz, ptr, flag);
  AMGP_HIP(hipGetLastError());
  AMGP_HIP(hipMemcpyAsync(h, flag, sizeof(h), hipMemcpyDeviceToHost, s));
  AMGP_HIP(hipStreamSynchronize(s));
  if (h[F_BADCSR]) return AMG_EINVAL;
  hipLaunchKernelGGL(k_check_col, dim3(grid_for(n)), dim3(kBlock), 0, s, n, ptr, col, flag);
  AMGP_HIP(hipGetLastError());
  AMGP_HIP(hipMemcpyAsync(h, flag, sizeof(h), hipMemcpyDeviceToHost, s));
  AMGP_HIP(hipStreamSynchronize(s));
  return h[F_BADCSR] ? AMG_EINVAL : AMG_OK;
}

int launch_l1_diag(hipStream_t s, int64_t n, const int32_t* ptr, const int32_t* col, const double* val,
                   double* minv, int* flag) {
  hipLaunchKernelGGL(k_l1_diag, dim3(grid_for(n)), dim3(kBlock), 0, s, n, ptr, col, val, minv, flag);
  return hipGetLastError() == hipSuccess ? AMG_OK : AMG_EHIP;
}

// Offset-aligned sliced ELL (one row per lane) when every slice has at most 64 distinct column
// offsets and the layout is at most 10% larger than the packed one; AMG_EINVAL otherwise.
int build_ell_aligned(hipStream_t s, int64_t n, const int32_t* ptr, const int32_t* col, const double* val,
                      Ell<double>* out, const int32_t* anchor, int astride, int64_t ncols, bool any_size) {
  const int64_t nslices = (n + kSlice - 1) / kSlice;
  int32_t *offs = nullptr, *wd = nullptr, *lw = nullptr;
  auto cleanup = [&]() {
    hipFree(offs);
    hipFree(wd);
    hipFree(lw);
  };
  if (hipMalloc(&offs, sizeof(int32_t) * nslices * kSlice) != hipSuccess ||
      hipMalloc(&wd, sizeof(int32_t) * nslices) != hipSuccess ||
      hipMalloc(&lw, sizeof(int32_t) * nslices) != hipSuccess) {
    cleanup();
    return AMG_ENOMEM;
  }
  hipLaunchKernelGGL(k_slice_offsets, dim3((unsigned)nslices), dim3(kWave), 0, s, n, ptr, col, anchor, astride, offs,
                     wd);
  hipLaunchKernelGGL(k_slice_width, dim3(grid_for(nslices)), dim3(kBlock), 0, s, n, nslices, kSlice, ptr, lw);
  std::vector<int32_t> w(nslices), lwh(nslices);
  if (hipMemcpyAsync(w.data(), wd, sizeof(int32_t) * nslices, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(lwh.data(), lw, sizeof(int32_t) * nslices, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    cleanup();
    return AMG_EHIP;
  }
  int64_t aligned = 0, packed = 0;
  for (int64_t i = 0; i < nslices; ++i) {
    if (w[i] < 0) {
      cleanup();
      return AMG_EINVAL;
    }
    aligned += (int64_t)w[i] * kSlice;
    packed += (int64_t)lwh[i] * kSlice;
  }
  if ((!any_size && aligned > packed + packed / 10) || aligned >= (int64_t)INT32_MAX) {
    cleanup();
    return AMG_EINVAL;
  }
  std::vector<int32_t> sp(nslices + 1);
  int64_t acc = 0;
  for (int64_t i = 0; i < nslices; ++i) {
    sp[i] = (int32_t)acc;
    acc += (int64_t)w[i] * kSlice;
  }
  sp[nslices] = (int32_t)acc;
  Ell<double> e;
  e.n = n;
  e.ncols = ncols < 0 ? n : ncols;
  e.anchor = anchor;
  e.astride = astride;
  e.group = 1;
  e.nslices = nslices;
  e.padded = acc;
  if (hipMalloc(&e.sptr, sizeof(int32_t) * (nslices + 1)) != hipSuccess ||
      hipMalloc(&e.val, sizeof(double) * std::max<int64_t>(acc, 1)) != hipSuccess ||
      hipMalloc(&e.doff, sizeof(int32_t) * std::max<int64_t>(acc / kSlice, 1)) != hipSuccess) {
    free_ell(e);
    cleanup();
    return AMG_ENOMEM;
  }
  int rc = AMG_OK;
  if (hipMemcpyAsync(e.sptr, sp.data(), sizeof(int32_t) * (nslices + 1), hipMemcpyHostToDevice, s) != hipSuccess)
    rc = AMG_EHIP;
  if (rc == AMG_OK) {
    hipLaunchKernelGGL(k_ell_fill_aligned, dim3(grid_for(nslices * kSlice)), dim3(kBlock), 0, s, n, nslices, ptr,
                       col, val, anchor, astride, offs, e.sptr, e.val, e.doff);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) rc = AMG_EHIP;
  }
  cleanup();
  if (rc != AMG_OK) {
    free_ell(e);
    return rc;
  }
  *out = e;
  return AMG_OK;
}

int build_ell64(hipStream_t s, int64_t n, const int32_t* ptr, const int32_t* col, const double* val,
                Ell<double>* out, int64_t ncols, int group) {
  if (ncols < 0) ncols = n;
  if (group == 0) {
    // lanes per row from the mean row length: about four entries or more per lane
    int32_t last = 0;
    AMGP_HIP(hipMemcpyAsync(&last, ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    AMGP_HIP(hipStreamSynchronize(s));
    const double mean = (double)last / (double)n;
    group = mean >= 256 ? 64 : mean >= 64 ? 16 : mean >= 16 ? 4 : 1;
    if (group == 4 && n >= kAlignedWideMinRows && ncols == n) {
      // a coarse stencil (27 points on Q1 boxes) on a large level: one row per lane without
      // column indices moves 4 bytes less per entry than four lanes per row with them
      const int rc = build_ell_aligned(s, n, ptr, col, val, out);
      if (rc != AMG_EINVAL) return rc;
    }
  }
  if (group != 1 && group != 4 && group != 16 && group != 64) return AMG_EINVAL;
  if (group == 1 && ncols == n) {
    const int rc = build_ell_aligned(s, n, ptr, col, val, out);
    if (rc != AMG_EINVAL) return rc;  // EINVAL: the slices are not offset-aligned; use the packed layout
  }
  const int R = kSlice / group;
  Ell<double> e;
  e.n = n;
  e.group = group;
  e.nslices = (n + R - 1) / R;
  int32_t* dw = nullptr;
  AMGP_HIP(hipMalloc(&dw, sizeof(int32_t) * e.nslices));
  hipLaunchKernelGGL(k_slice_width, dim3(grid_for(e.nslices)), dim3(kBlock), 0, s, n, e.nslices, R, ptr, dw);
  std::vector<int32_t> w(e.nslices);
  AMGP_HIP(hipMemcpyAsync(w.data(), dw, sizeof(int32_t) * e.nslices, hipMemcpyDeviceToHost, s));
  AMGP_HIP(hipStreamSynchronize(s));
  hipFree(dw);
  std::vector<int32_t> sp(e.nslices + 1);
  int64_t acc = 0;
  for (int64_t i = 0; i < e.nslices; ++i) {
    sp[i] = (int32_t)acc;
    acc += (int64_t)((w[i] + group - 1) / group) * kSlice;
    if (acc >= (int64_t)INT32_MAX) return AMG_ECAPACITY;
  }
  sp[e.nslices] = (int32_t)acc;
  e.padded = acc;
  if (hipMalloc(&e.sptr, sizeof(int32_t) * (e.nslices + 1)) != hipSuccess) return AMG_ENOMEM;
  if (hipMalloc(&e.col, sizeof(int32_t) * std::max<int64_t>(acc, 1)) != hipSuccess) return AMG_ENOMEM;
  if (hipMalloc(&e.val, sizeof(double) * std::max<int64_t>(acc, 1)) != hipSuccess) return AMG_ENOMEM;
  AMGP_HIP(hipMemcpyAsync(e.sptr, sp.data(), sizeof(int32_t) * (e.nslices + 1), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_ell_fill, dim3(grid_for(e.nslices * kSlice)), dim3(kBlock), 0, s, n, ncols, e.nslices, group,
                     ptr, col, val, e.sptr, e.col, e.val);
  AMGP_HIP(hipGetLastError());
  AMGP_HIP(hipStreamSynchronize(s));
  *out = e;
  return AMG_OK;
}

int build_ell32(hipStream_t s, const Ell<double>& a, Ell<float>* out) {
  Ell<float> e;
  e.n = a.n;
  e.ncols = a.ncols;
  e.anchor = a.anchor;
  e.astride = a.astride;
  e.nslices = a.nslices;
  e.padded = a.padded;
  e.group = a.group;
  if (hipMalloc(&e.sptr, sizeof(int32_t) * (e.nslices + 1)) != hipSuccess) return AMG_ENOMEM;
  if (hipMalloc(&e.val, sizeof(float) * std::max<int64_t>(e.padded, 1)) != hipSuccess) return AMG_ENOMEM;
  AMGP_HIP(hipMemcpyAsync(e.sptr, a.sptr, sizeof(int32_t) * (e.nslices + 1), hipMemcpyDeviceToDevice, s));
  if (a.col) {
    if (hipMalloc(&e.col, sizeof(int32_t) * std::max<int64_t>(e.padded, 1)) != hipSuccess) return AMG_ENOMEM;
    AMGP_HIP(hipMemcpyAsync(e.col, a.col, sizeof(int32_t) * e.padded, hipMemcpyDeviceToDevice, s));
  }
  if (a.doff) {
    if (hipMalloc(&e.doff, sizeof(int32_t) * std::max<int64_t>(e.padded / kSlice, 1)) != hipSuccess) return AMG_ENOMEM;
    AMGP_HIP(hipMemcpyAsync(e.doff, a.doff, sizeof(int32_t) * (e.padded / kSlice), hipMemcpyDeviceToDevice, s));
  }
  if (a.doff)
    hipLaunchKernelGGL(k_round_f32_aligned, dim3(grid_for(e.nslices * kSlice)), dim3(kBlock), 0, s, e.nslices, e.sptr,
                       a.val, e.val);
  else
    hipLaunchKernelGGL(k_round_f32, dim3(grid_for(e.padded)), dim3(kBlock), 0, s, e.padded, a.val, e.val);
  AMGP_HIP(hipGetLastError());
  *out = e;
  return AMG_OK;
}

void free_ell(Ell<double>& e) {
  hipFree(e.sptr);
  hipFree(e.col);
  hipFree(e.val);
  hipFree(e.doff);
  e = Ell<double>();
}

void free_ell(Ell<float>& e) {
  hipFree(e.sptr);
  hipFree(e.col);
  hipFree(e.val);
  hipFree(e.doff);
  e = Ell<float>();
}

int launch_aggregates(hipStream_t s, int nx, int ny, int nz, int nbatch, int e, int32_t* agg, int32_t* children,
                      int* cnx, int* cny, int* cnz) {
  if (e < 2 || (children && e != 2)) return AMG_EINVAL;
  const int cx = nx == 1 ? 1 : (nx + e - 1) / e, cy = ny == 1 ? 1 : (ny + e - 1) / e,
            cz = nz == 1 ? 1 : (nz + e - 1) / e;
  const int64_t n = (int64_t)nx * ny * nz * nbatch, nc = (int64_t)cx * cy * cz * nbatch;
  hipLaunchKernelGGL(k_agg, dim3(grid_for(n)), dim3(kBlock), 0, s, n, nx, ny, nz, e, cx, cy, cz, agg);
  if (children)
    hipLaunchKernelGGL(k_children, dim3(grid_for(nc)), dim3(kBlock), 0, s, nc, nx, ny, nz, cx, cy, cz, children);
  *cnx = cx;
  *cny = cy;
  *cnz = cz;
  return hipGetLastError() == hipSuccess ? AMG_OK : AMG_EHIP;
}

int galerkin(hipStream_t s, int64_t n, const int32_t* ptr, const int32_t* col, const double* val,
             const int32_t* agg, int64_t nc, const int32_t* children, int32_t** cptr, int32_t** ccol,
             double** cval, int64_t* cnnz, int* flag) {
  (void)n;
  // the arrays belong to the caller as soon as they exist, also when a later step fails
  int32_t* cnt = nullptr;
  if (hipMalloc(&cnt, sizeof(int32_t) * (nc + 1)) != hipSuccess) return AMG_ENOMEM;
  *cptr = cnt;
  hipLaunchKernelGGL((k_rap<false>), dim3((unsigned)((nc + 63) / 64)), dim3(64), 0, s, nc, ptr, col, val, agg,
                     children, cnt, (int32_t*)nullptr, (double*)nullptr, flag);
  AMGP_HIP(hipGetLastError());
  std::vector<int32_t> h(nc + 1);
  AMGP_HIP(hipMemcpyAsync(h.data(), cnt, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
  int hflag[F_NFLAG];
  AMGP_HIP(hipMemcpyAsync(hflag, flag, sizeof(hflag), hipMemcpyDeviceToHost, s));
  AMGP_HIP(hipStreamSynchronize(s));
  if (hflag[F_CAPACITY]) return AMG_ECAPACITY;
  int64_t acc = 0;
  for (int64_t I = 0; I < nc; ++I) {
    const int32_t c = h[I];
    h[I] = (int32_t)acc;
    acc += c;
    if (acc >= (int64_t)INT32_MAX) return AMG_ECAPACITY;
  }
  h[nc] = (int32_t)acc;
  AMGP_HIP(hipMemcpyAsync(cnt, h.data(), sizeof(int32_t) * (nc + 1), hipMemcpyHostToDevice, s));
  if (hipMalloc(ccol, sizeof(int32_t) * std::max<int64_t>(acc, 1)) != hipSuccess) return AMG_ENOMEM;
  if (hipMalloc(cval, sizeof(double) * std::max<int64_t>(acc, 1)) != hipSuccess) return AMG_ENOMEM;
  hipLaunchKernelGGL((k_rap<true>), dim3((unsigned)((nc + 63) / 64)), dim3(64), 0, s, nc, ptr, col, val, agg,
                     children, cnt, *ccol, *cval, flag);
  AMGP_HIP(hipGetLastError());
  AMGP_HIP(hipStreamSynchronize(s));
  *cnnz = acc;
  return AMG_OK;
}

int launch_to_dense(hipStream_t s, int nbatch, int64_t nl, int64_t np, const int32_t* ptr, const int32_t* col,
                    const double* val, double* dense, int* flag) {
  const int64_t rows = (int64_t)nbatch * np;
  hipLaunchKernelGGL(k_to_dense, dim3(grid_for(rows)), dim3(kBlock), 0, s, rows, nl, np, ptr, col, val, dense,
                     flag);
  return hipGetLastError() == hipSuccess ? AMG_OK : AMG_EHIP;
}

}  // namespace amgp
