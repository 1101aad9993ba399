// Row-parallel sparse and vector kernels for gfx950: SpMV, the fused smoother
// recurrence steps, grid transfers and the CG vector updates with
// deterministic two-stage reductions.
//
// Layout and launch shape: one row per lane, 256-thread blocks (4 waves), the
// matrix in sliced ELL with 64-row slices so that every load of val/col by a
// wavefront is one contiguous 512 B (float64) segment.  On levels of up to
// 3.1M rows, blocks are remapped so that each of the 8 XCDs (which receive
// workgroups round-robin) walks one contiguous range of rows: the neighbours
// gathered by a row (the previous and next grid lines and planes) were then
// recently touched by the same XCD and are served from its L2 instead of HBM.
#include <type_traits>

#include "internal.h"

namespace amgp {

namespace {

// BEGIN fused-step (the launch helpers and the fused step; bench.py hashes this region to tie
// stored counters to the code)

constexpr int kXcd = 8;

inline unsigned xcd_grid(int64_t n) {
  unsigned g = grid_for(n);
  return (g + kXcd - 1) / kXcd * kXcd;
}

// Logical block index.  Block b runs on XCD b % 8.  For levels up to
// kRemapMaxBlocks blocks (3.1M rows, a working set near the 256 MB MALL) each
// XCD is given the contiguous blocks [x * G/8, (x+1) * G/8), so the
// neighbouring planes a row gathers were recently touched by the same XCD and
// hit its L2 (measured: 40.9 vs 44.8 us per fused step at 128^3).  Larger
// levels stream from HBM: there each XCD takes runs of kXcdChunk consecutive
// blocks in turn (blocks past the last whole round of 8 runs keep the launch
// order), so that a block's neighbouring grid lines (the adjacent blocks) are
// mostly on its own XCD and each XCD streams long contiguous stretches of the
// matrix.  Measured on the fused step with runs of 8, 16, ..., 400 blocks:
// 128 is the fastest on the 27-point level at 320^3 (1.63 ms; 8: 1.71,
// 64: 1.67, 400: 1.73) and within 1.5% of the fastest on the 7-point level at
// 256^3; whole contiguous ranges per XCD are slower on both (1.79 ms; a
// plane's reuse is then too far away in time).  G is a multiple of 8 (xcd_grid).
// The threshold sits between the 128^3 fine level (8192 blocks, 235 MB per fused step, which
// the hints below make 15-20% slower) and level 1 of the 27-point 320^3 problem (16000 blocks,
// 1.1 GB per step: streaming it took the solve from 0.496 to 0.493 s).
constexpr unsigned kRemapMaxBlocks = 12288;
constexpr unsigned kXcdChunk = 128;

__device__ __forceinline__ int64_t logical_block() {
  if (gridDim.x > kRemapMaxBlocks) {
    constexpr unsigned span = kXcd * kXcdChunk;
    if (blockIdx.x >= gridDim.x - gridDim.x % span) return blockIdx.x;
    const unsigned x = blockIdx.x % kXcd, q = blockIdx.x / kXcd;
    return (int64_t)(q / kXcdChunk) * span + x * kXcdChunk + q % kXcdChunk;
  }
  const unsigned per = gridDim.x / kXcd;
  return (int64_t)(blockIdx.x % kXcd) * per + blockIdx.x / kXcd;
}

__device__ __forceinline__ int64_t row_index() { return logical_block() * kBlock + threadIdx.x; }

template <typename T>
__device__ __forceinline__ T wsel(const Wt& w, T scalar, int64_t i) {
  return w.v ? (T)w.v[(int)i / w.rpp * w.stride] : scalar;
}

// Levels larger than kRemapMaxBlocks blocks stream from HBM: there the matrix
// and the row-local vectors are read and written with nontemporal hints (NT),
// which keeps them from displacing the gathered vector in the caches
// (measured at 256^3: 380 vs 424 us per fused step; on 128^3, whose working
// set is close to the MALL, the hints cost 15-20%, so smaller levels keep the
// default policy).  Gathered vectors always use ordinary loads and stores.
template <bool NT, typename T>
__device__ __forceinline__ T ld(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p); else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p); else *p = v;
}

// The row's l1 inverse diagonal, read by every step of a level: an ordinary load on wide
// (27-point) FP64 levels and on FP32 levels, a nontemporal one on the other streaming FP64
// levels.  Measured: 320^3 27-point solve 482.5 -> 480.5 ms, the 256^3 diffusion solve with the
// FP32 hierarchy 61.2 -> 60.7 ms; on the 7-point FP64 level ordinary loads cost 5% (294 -> 310 us).
template <bool NT, bool W, typename T>
__device__ __forceinline__ T ld_minv(const T* p) {
  if constexpr (W || std::is_same_v<T, float>) return *p; else return ld<NT>(p);
}

// Offset-aligned slices keep each lane's steps in pairs: steps 2q and 2q + 1 of lane l sit at
// 128 q + 2 l and 128 q + 2 l + 1 of the slice (an odd last step t at 64 t + l), so one load per
// lane serves two steps: 16 bytes in FP64 (a wavefront load is 1 KB contiguous), 8 in FP32.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ f64x2 ld2(const double* p) {
  const f64x2* q = reinterpret_cast<const f64x2*>(p);
  if constexpr (NT) return __builtin_nontemporal_load(q); else return *q;
}
template <bool NT>
__device__ __forceinline__ f32x2 ld2(const float* p) {
  const f32x2* q = reinterpret_cast<const f32x2*>(p);
  if constexpr (NT) return __builtin_nontemporal_load(q); else return *q;
}

// FP32 slices of at least kQuadMinSteps steps keep each lane's steps in quads instead: steps 4q ..
// 4q + 3 of lane l at 256 q + 4 l of the slice, then (w mod 4 >= 2) a pair at 64 t + 2 l, then (w odd)
// a single step at 64 t + l, so that one 16-byte load serves four steps; narrower slices keep
// the pairs.  Measured on the FP32 fused step: 27-point level at 320^3 776 us in quads (batches of
// 12 steps) against 812 us in pairs one at a time; 7-point level at 256^3 150 us in pairs
// (batches of 6) against 159 us one pair at a time and 157 us in quads.
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ __forceinline__ f32x4 ld4(const float* p) {
  const f32x4* q = reinterpret_cast<const f32x4*>(p);
  if constexpr (NT) return __builtin_nontemporal_load(q); else return *q;
}

// Sum over the steps t of an FP32 offset-aligned slice [beg, end) of val_t * g(column_t), in
// ascending t (the order of the FP64 loops), for the row r served by this lane, with the requests
// issued in batches as in the FP64 form below.  Batched = false: one load per iteration.
template <bool NT, typename Gf, bool Batched = true>
__device__ __forceinline__ float aligned_sum_f32(const float* __restrict__ val, int beg, int end, int lane,
                                                 const int32_t* __restrict__ off, int r, int last, Gf g) {
  const int w = (end - beg) >> 6;
  const float* v = val + beg;
  auto col = [&](int t) { return min(max(r + off[t], 0), last); };
  float acc = 0.0f;
  int t = 0;
  if (w >= kQuadMinSteps) {
    constexpr int B = 12, H = B / 4;
    const int w4 = w & ~3;
    const int nb = Batched ? w4 / B : 0;
    const float* vq = v + 4 * lane;  // quad u of batch q at vq + 64 (q B) + 256 u
    f32x4 nxt[H];
    if (nb > 0) {
#pragma unroll
      for (int u = 0; u < H; ++u) nxt[u] = ld4<NT>(vq + 256 * u);
    }
    for (int q = 0; q < nb; ++q, t += B) {
      f32x4 cur[H];
      float gv[B];
#pragma unroll
      for (int u = 0; u < H; ++u) cur[u] = nxt[u];
#pragma unroll
      for (int u = 0; u < B; ++u) gv[u] = g(col(t + u));
      if (q + 1 < nb) {
#pragma unroll
        for (int u = 0; u < H; ++u) nxt[u] = ld4<NT>(vq + 64 * (t + B) + 256 * u);
      }
#pragma unroll
      for (int u = 0; u < H; ++u) {
        acc += cur[u].x * gv[4 * u];
        acc += cur[u].y * gv[4 * u + 1];
        acc += cur[u].z * gv[4 * u + 2];
        acc += cur[u].w * gv[4 * u + 3];
      }
    }
    for (; t < w4; t += 4) {
      const f32x4 p = ld4<NT>(vq + 64 * t);
      acc += p.x * g(col(t));
      acc += p.y * g(col(t + 1));
      acc += p.z * g(col(t + 2));
      acc += p.w * g(col(t + 3));
    }
    if (t + 1 < w) {
      const f32x2 p = ld2<NT>(v + 64 * t + 2 * lane);
      acc += p.x * g(col(t));
      acc += p.y * g(col(t + 1));
      t += 2;
    }
  } else {
    constexpr int B = 6, H = B / 2;
    const int wp = w & ~1;
    const int nb = Batched ? wp / B : 0;
    const float* vp = v + 2 * lane;  // pair u of batch q at vp + 64 (q B) + 128 u
    f32x2 nxt[H];
    if (nb > 0) {
#pragma unroll
      for (int u = 0; u < H; ++u) nxt[u] = ld2<NT>(vp + 128 * u);
    }
    for (int q = 0; q < nb; ++q, t += B) {
      f32x2 cur[H];
      float gv[B];
#pragma unroll
      for (int u = 0; u < H; ++u) cur[u] = nxt[u];
#pragma unroll
      for (int u = 0; u < B; ++u) gv[u] = g(col(t + u));
      if (q + 1 < nb) {
#pragma unroll
        for (int u = 0; u < H; ++u) nxt[u] = ld2<NT>(vp + 64 * (t + B) + 128 * u);
      }
#pragma unroll
      for (int u = 0; u < H; ++u) {
        acc += cur[u].x * gv[2 * u];
        acc += cur[u].y * gv[2 * u + 1];
      }
    }
    for (; t < wp; t += 2) {
      const f32x2 p = ld2<NT>(vp + 64 * t);
      acc += p.x * g(col(t));
      acc += p.y * g(col(t + 1));
    }
  }
  if (t < w) acc += ld<NT>(v + 64 * t + lane) * g(col(t));
  return acc;
}

// The FP64 form: the same sum in ascending t, with the requests issued in batches of
// kAlignedBatch steps (three 16-byte loads per lane) and the next batch's values requested
// before this batch's products are added, so that each wavefront keeps a batch of matrix loads
// in flight while it waits for its gathers.  Measured on the fused step: 27-point level at 320^3
// 1.63 ms (one pair per iteration: 1.71; one unpaired step per iteration, unrolled by 2: 1.85),
// 7-point level at 256^3 0.296 ms (batches of 8: 0.305; unpaired: 0.319).
constexpr int kAlignedBatch = 6;

// Wide slices (levels averaging at least kWideMinSteps steps per row: the 27-point ones) take
// batches of kWideBatch steps, six 16-byte loads per lane, and their kernels request the row's
// own vectors before the product.  Measured on the fused step of a synthetic 27-point level of
// 32.8M rows (three runs each): 1620-1621 us against 1651-1652 us for batches of 6 with the row
// vectors after the product; batches of 12 alone: 1631 us.  Seven-step slices never fill a
// batch of 12 (299 against 320-336 us), so narrower levels keep batches of 6.
constexpr int kWideBatch = 12;
constexpr int kWideMinSteps = 2 * kWideBatch;

// Batched = false: one pair per iteration (rows of a wavefront in different slices, where the
// batches would diverge).
template <bool NT, typename Gf, bool Batched = true, int B = kAlignedBatch>
__device__ __forceinline__ double aligned_sum_f64(const double* __restrict__ val, int beg, int end, int lane,
                                                  const int32_t* __restrict__ off, int r, int last, Gf g) {
  constexpr int H = B / 2;
  const int w = (end - beg) >> 6;
  const int wp = w & ~1;
  const int nb = Batched ? wp / B : 0;
  const double* v = val + beg + 2 * lane;  // pair u of batch q at v + 64 (q B) + 128 u
  double acc = 0.0;
  int t = 0;
  f64x2 nxt[H];
  if (nb > 0) {
#pragma unroll
    for (int u = 0; u < H; ++u) nxt[u] = ld2<NT>(v + 128 * u);
  }
  for (int q = 0; q < nb; ++q, t += B) {
    f64x2 cur[H];
    double gv[B];
#pragma unroll
    for (int u = 0; u < H; ++u) cur[u] = nxt[u];
#pragma unroll
    for (int u = 0; u < B; ++u) gv[u] = g(min(max(r + off[t + u], 0), last));
    if (q + 1 < nb) {
#pragma unroll
      for (int u = 0; u < H; ++u) nxt[u] = ld2<NT>(v + 64 * (t + B) + 128 * u);
    }
#pragma unroll
    for (int u = 0; u < H; ++u) {
      acc += cur[u].x * gv[2 * u];
      acc += cur[u].y * gv[2 * u + 1];
    }
  }
  for (; t < wp; t += 2) {
    const f64x2 p = ld2<NT>(v + 64 * t);
    acc += p.x * g(min(max(r + off[t], 0), last));
    acc += p.y * g(min(max(r + off[t + 1], 0), last));
  }
  if (t < w) acc += ld<NT>(val + beg + 64 * t + lane) * g(min(max(r + off[t], 0), last));
  return acc;
}

// Rows with G lanes each (Ell::group): thread t of the grid serves row t / G, and a
// wavefront covers exactly one slice of 64 / G rows.
template <int G>
__device__ __forceinline__ int64_t row_of_thread() {
  return (logical_block() * kBlock + threadIdx.x) / G;
}

// True when every row of this wavefront is past n (a uniform exit).  With G > 1 a
// wavefront whose first row is below n runs whole: its rows past n lie in the padded
// tail of the last slice (values 0), and every lane takes part in the row sums.
template <int G>
__device__ __forceinline__ bool exit_rows(int64_t i, int64_t n) {
  if constexpr (G == 1) return i >= n;
  return (logical_block() * kBlock + (threadIdx.x & ~(kWave - 1))) / G >= n;
}

// (A x)_row; with G > 1 every lane of the row's group returns the sum.  AB: the batch of the
// FP64 offset-aligned sum.
template <bool NT, int G, int AB = kAlignedBatch, typename T>
__device__ __forceinline__ T ell_dot(EllView<T> A, int64_t row, const T* __restrict__ x) {
  constexpr int R = kSlice / G;
  // every lane of the wavefront is in the same slice: read its bounds once, as scalars
  const int s = __builtin_amdgcn_readfirstlane((int)(row / R));
  const int beg = __builtin_amdgcn_readfirstlane(A.sptr[s]);
  const int end = __builtin_amdgcn_readfirstlane(A.sptr[s + 1]);
  const int lane = G == 1 ? (int)(row & 63) : (int)(threadIdx.x & 63);
  T acc = T(0);
  if (G == 1 && A.doff) {
    // offset-aligned slice: the column is the row plus the step's (uniform) offset
    const int32_t* off = A.doff + (beg >> 6);
    const int r = (int)row;
    if constexpr (std::is_same_v<T, float>) {
      return aligned_sum_f32<NT>(A.val, beg, end, lane, off, r, A.last, [&](int c) { return x[c]; });
    } else {
      auto g = [&](int c) { return x[c]; };
      return aligned_sum_f64<NT, decltype(g), true, AB>(A.val, beg, end, lane, off, r, A.last, g);
    }
  }
#pragma unroll 4
  for (int p = beg + lane; p < end; p += kSlice) {
    acc += ld<NT>(A.val + p) * x[ld<NT>(A.col + p)];
  }
  if constexpr (G > 1) {
    for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
  }
  return acc;
}

// lane 0 of a row's group, on a row below n, does the row's updates
template <int G>
__device__ __forceinline__ bool row_owner(int64_t i, int64_t n) {
  return i < n && (G == 1 || (threadIdx.x & (G - 1)) == 0);
}

// Wave-level sum with cross-lane shuffles, then across the block's 4 waves via LDS.
// Fixed association order: bitwise reproducible for a fixed launch shape.
__device__ __forceinline__ double block_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  __shared__ double part[kBlock / kWave];
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & 63) == 0) part[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < kBlock / kWave; ++i) s += part[i];
  }
  return s;
}

// ---------------------------------------------------------------------------
// SpMV and residual
// ---------------------------------------------------------------------------
template <typename T, bool NT, int G>
__global__ __launch_bounds__(kBlock) void k_spmv(int64_t n, EllView<T> A, const T* __restrict__ x,
                                                 T* __restrict__ y) {
  const int64_t i = row_of_thread<G>();
  if (exit_rows<G>(i, n)) return;
  const T v = ell_dot<NT, G>(A, i, x);
  if (row_owner<G>(i, n)) st<NT>(y + i, v);
}

template <typename T, bool NT, int G>
__global__ __launch_bounds__(kBlock) void k_residual(int64_t n, EllView<T> A, const T* __restrict__ b,
                                                     const T* __restrict__ x, T* __restrict__ r) {
  const int64_t i = row_of_thread<G>();
  if (exit_rows<G>(i, n)) return;
  const T v = ell_dot<NT, G>(A, i, x);
  if (row_owner<G>(i, n)) r[i] = ld<NT>(b + i) - v;
}

// ---------------------------------------------------------------------------
// Smoother recurrence steps.
//
// MODE 0 (4th kind, optimal 4th kind; eqs. polsmoother / polsmootheropt):
//   r   = r_in - A g_old                      (residual of the previous step)
//   g   = alpha g_old + c M^{-1} r            (z^(j))
//   x  += wprev g_old + w g                   (beta_j-weighted update)
// MODE 1 (1st kind; Algorithm 1, the loop body):
//   r   = r_in - M^{-1} A g_old               (r^(j) = r^(j-1) - s^(j))
//   g   = alpha g_old + c r                   (d^(j) = rho_j rho_{j-1} d + (2 rho_j / delta) r)
//   x  += wprev g_old + g
// g_old is gathered by neighbouring rows, so g is written to the other buffer
// of a ping-pong pair; r and x are row-local and updated in place.  wprev
// carries an x update deferred by the previous step (a first step that gathered
// x itself, or a k_fused_keep_x step, which leaves x alone: the next step adds
// both directions, which it reads anyway, in the same order).
// STORE = false on the last step of an application: only x is needed.
// Returns the x it stores (0 on rows that store none).
// ---------------------------------------------------------------------------
// W: wide slices (one row per lane): the row's vectors are requested before the product, whose
// steps go in batches of kWideBatch.
template <typename T, int MODE, bool STORE, bool NT, int G, bool XUPD, bool W>
__device__ __forceinline__ T fused_step(int64_t n, EllView<T> A, const T* __restrict__ minv,
                                          const T* __restrict__ gold, T* __restrict__ gnew, const T* rin, T* rout,
                                          T* __restrict__ x, T alpha, T c, T w, T wprev, Wt wv, Wt wpv, Prol<T> pr) {
  const int64_t i = row_of_thread<G>();
  if (exit_rows<G>(i, n)) return T(0);
  T mi, go, ri, xi = T(0);
  if constexpr (W) {
    mi = ld_minv<NT, W>(minv + i);
    go = gold[i];
    ri = ld<NT>(rin + i);
    if constexpr (XUPD) xi = ld<NT>(x + i);
  }
  const T ag = ell_dot<NT, G, W ? kWideBatch : kAlignedBatch>(A, i, gold);
  if (!row_owner<G>(i, n)) return T(0);
  if constexpr (!W) {
    mi = ld_minv<NT, W>(minv + i);
    go = gold[i];
    ri = ld<NT>(rin + i);
  }
  const T r = (MODE == 0) ? ri - ag : ri - mi * ag;
  const T g = (MODE == 0) ? alpha * go + c * (mi * r) : alpha * go + c * r;
  T xn = T(0);
  if constexpr (XUPD) {
    w = wsel(wv, w, i);
    wprev = wsel(wpv, wprev, i);
    if constexpr (!W) xi = ld<NT>(x + i);
    if (pr.agg) xi = xi + pr.xc[pr.agg[i]];
    xn = xi + wprev * go + w * g;
    st<NT>(x + i, xn);
  }
  if (STORE) {
    st<NT>(rout + i, r);
    gnew[i] = g;
  }
  return xn;
}

template <typename T, int MODE, bool STORE, bool NT, int G, bool W = false>
__global__ __launch_bounds__(kBlock) void k_fused(int64_t n, EllView<T> A, const T* __restrict__ minv,
                                                  const T* __restrict__ gold, T* __restrict__ gnew,
                                                  const T* rin, T* rout, T* __restrict__ x, T alpha, T c, T w,
                                                  T wprev, Wt wv, Wt wpv, Prol<T> pr) {
  fused_step<T, MODE, STORE, NT, G, true, W>(n, A, minv, gold, gnew, rin, rout, x, alpha, c, w, wprev, wv, wpv, pr);
}

// A stored step that leaves x alone: the next step adds this step's weighted direction (which it
// reads anyway as its own old direction) together with its own.
template <typename T, int MODE, bool NT, int G, bool W = false>
__global__ __launch_bounds__(kBlock) void k_fused_keep_x(int64_t n, EllView<T> A, const T* __restrict__ minv,
                                                         const T* __restrict__ gold, T* __restrict__ gnew,
                                                         const T* rin, T* rout, T alpha, T c) {
  fused_step<T, MODE, true, NT, G, false, W>(n, A, minv, gold, gnew, rin, rout, nullptr, alpha, c, T(0), T(0), Wt(),
                                             Wt(), Prol<T>());
}

// END fused-step

// The last step of an application with the CG's dot products of its result fused in: block
// partials of (dr, x) and, with drold, of (drold, x), over the x this step stores (an FP32 x is
// converted exactly).  The products, the block order and the sums are those of k_dot2 on the
// same grid, so the partials are the same numbers.
template <typename T, int MODE, bool NT, bool W>
__global__ __launch_bounds__(kBlock) void k_fused_dot(int64_t n, EllView<T> A, const T* __restrict__ minv,
                                                      const T* __restrict__ gold, const T* rin, T* __restrict__ x,
                                                      T alpha, T c, T w, T wprev, Wt wv, Wt wpv, Prol<T> pr,
                                                      const double* __restrict__ dr, const double* __restrict__ drold,
                                                      double* __restrict__ partial) {
  const double xn = (double)fused_step<T, MODE, false, NT, 1, true, W>(n, A, minv, gold, nullptr, rin, nullptr, x,
                                                                        alpha, c, w, wprev, wv, wpv, pr);
  const int64_t i = row_index();
  double v = 0.0, u = 0.0;
  if (i < n) {
    v = ld<NT>(dr + i) * xn;
    if (drold) u = ld<NT>(drold + i) * xn;
  }
  const double sv = block_sum(v);
  __syncthreads();
  const double su = drold ? block_sum(u) : 0.0;
  if (threadIdx.x == 0) {
    partial[logical_block()] = sv;
    partial[gridDim.x + logical_block()] = su;
  }
}

// First step from x = 0 (r^(0) = b, no SpMV).
// MODE 0: g = c M^{-1} b, x = w g.   MODE 1: r = M^{-1} b, g = r / c (c = theta), x = g.
template <typename T, int MODE, bool STORE, bool NT>
__global__ __launch_bounds__(kBlock) void k_first_zero(int64_t n, const T* __restrict__ minv,
                                                       const T* __restrict__ b, T* __restrict__ g,
                                                       T* __restrict__ r, T* __restrict__ x, T c, T w, Wt wv) {
  const int64_t i = row_index();
  if (i >= n) return;
  w = wsel(wv, w, i);
  const T mi = ld<NT>(minv + i);
  const T bi = ld<NT>(b + i);
  if (MODE == 0) {
    const T gi = c * (mi * bi);
    st<NT>(x + i, w * gi);
    if (STORE) g[i] = gi;
  } else {
    const T ri = mi * bi;
    const T gi = ri / c;
    st<NT>(x + i, gi);
    if (STORE) {
      st<NT>(r + i, ri);
      g[i] = gi;
    }
  }
}

// Steps 1 and 2 of an application from x = 0, merged (degree >= 2).  The
// step-1 direction of a neighbour j is recomputed from b_j and M^{-1}_j
// (exactly the value step 1 would have stored), so the step-1 pass over the
// vectors disappears.
// MODE 0: g1 = c1 M^{-1} b, r1 = b - A g1, g2 = alpha g1 + c M^{-1} r1, x = w1 g1 + w2 g2.
// MODE 1: r0 = M^{-1} b, d0 = r0 / theta, r1 = r0 - M^{-1} A d0, d1 = alpha d0 + c r1, x = d0 + d1.
// U: u = M^{-1} b (the same products) was written beforehand by the kernel that produced b (the
// CG's residual update), so the neighbours' step-1 directions gather one vector instead of two.
template <typename T, int MODE, bool STORE, bool NT, int G, bool W = false, bool U = false>
__global__ __launch_bounds__(kBlock) void k_first2_zero(int64_t n, EllView<T> A, const T* __restrict__ minv,
                                                        const T* __restrict__ b, T* __restrict__ gnew,
                                                        T* __restrict__ r, T* __restrict__ x, T c1, T alpha, T c,
                                                        T w1, T w2, Wt w1v, Wt w2v, const T* __restrict__ u) {
  const int64_t i = row_of_thread<G>();
  if (exit_rows<G>(i, n)) return;
  constexpr int R = kSlice / G;
  const int s = __builtin_amdgcn_readfirstlane((int)(i / R));
  const int beg = __builtin_amdgcn_readfirstlane(A.sptr[s]);
  const int end = __builtin_amdgcn_readfirstlane(A.sptr[s + 1]);
  const int lane = G == 1 ? (int)(i & 63) : (int)(threadIdx.x & 63);
  T mi = T(0), bi = T(0);
  if constexpr (W) {  // wide slices: the row's own entries first (see kWideBatch)
    mi = minv[i];
    bi = b[i];
  }
  T ag = T(0);
  auto g1of = [&](int j) {
    const T mb = U ? u[j] : minv[j] * b[j];
    return (MODE == 0) ? c1 * mb : mb / c1;
  };
  if (G == 1 && A.doff) {
    const int32_t* off = A.doff + (beg >> 6);
    if constexpr (std::is_same_v<T, float>) {
      ag = aligned_sum_f32<NT>(A.val, beg, end, lane, off, (int)i, A.last, g1of);
    } else {
      ag = aligned_sum_f64<NT, decltype(g1of), true, W ? kWideBatch : kAlignedBatch>(A.val, beg, end, lane, off, (int)i,
                                                                                    A.last, g1of);
    }
  } else {
#pragma unroll 4
    for (int p = beg + lane; p < end; p += kSlice) {
      const int j = ld<NT>(A.col + p);
      ag += ld<NT>(A.val + p) * g1of(j);
    }
  }
  if constexpr (G > 1) {
    for (int off = G / 2; off > 0; off >>= 1) ag += __shfl_xor(ag, off, kWave);
  }
  if (!row_owner<G>(i, n)) return;
  w1 = wsel(w1v, w1, i);
  w2 = wsel(w2v, w2, i);
  if constexpr (!W) {
    mi = minv[i];
    bi = b[i];
  }
  T g1, r1, g2;
  if (MODE == 0) {
    g1 = c1 * (mi * bi);
    r1 = bi - ag;
    g2 = alpha * g1 + c * (mi * r1);
    st<NT>(x + i, w1 * g1 + w2 * g2);
  } else {
    const T r0 = mi * bi;
    g1 = r0 / c1;
    r1 = r0 - mi * ag;
    g2 = alpha * g1 + c * r1;
    st<NT>(x + i, g1 + g2);
  }
  if (STORE) {
    st<NT>(r + i, r1);
    gnew[i] = g2;
  }
}

// First step from a nonzero x: r^(0) from b - A x.  x is gathered here, so its
// update is deferred to the next step (or a separate axpy when k = 1).
// MODE 0: r = b - A x, g = c M^{-1} r.   MODE 1: r = M^{-1}(b - A x), g = r / c (c = theta).
template <typename T, int MODE, bool NT, int G, bool W = false>
__global__ __launch_bounds__(kBlock) void k_first_res(int64_t n, EllView<T> A, const T* __restrict__ minv,
                                                      const T* __restrict__ b, const T* __restrict__ x,
                                                      T* __restrict__ r, T* __restrict__ g, T c) {
  const int64_t i = row_of_thread<G>();
  if (exit_rows<G>(i, n)) return;
  T bi = T(0), mi = T(0);
  if constexpr (W) {  // wide slices: the row's own entries first (see kWideBatch)
    bi = ld<NT>(b + i);
    mi = ld_minv<NT, W>(minv + i);
  }
  const T ax = ell_dot<NT, G, W ? kWideBatch : kAlignedBatch>(A, i, x);
  if (!row_owner<G>(i, n)) return;
  if constexpr (!W) {
    bi = ld<NT>(b + i);
    mi = ld_minv<NT, W>(minv + i);
  }
  const T res = bi - ax;
  if (MODE == 0) {
    st<NT>(r + i, res);
    g[i] = c * (mi * res);
  } else {
    const T ri = mi * res;
    st<NT>(r + i, ri);
    g[i] = ri / c;
  }
}

// (A (x + P x_c))_row for one row per lane (wave-uniform slice, as ell_dot<NT, 1>): the
// box prolongation x_j + x_c[agg_j] of every gathered entry, in the arithmetic of k_prolong.
template <bool NT, typename T>
__device__ __forceinline__ T ell_dot_prol(EllView<T> A, int64_t row, const T* __restrict__ x, Prol<T> pr) {
  const int s = __builtin_amdgcn_readfirstlane((int)(row / kSlice));
  const int beg = __builtin_amdgcn_readfirstlane(A.sptr[s]);
  const int end = __builtin_amdgcn_readfirstlane(A.sptr[s + 1]);
  const int lane = (int)(row & 63);
  T acc = T(0);
  if (A.doff) {
    const int32_t* off = A.doff + (beg >> 6);
    const int r = (int)row;
    if constexpr (std::is_same_v<T, float>) {
      return aligned_sum_f32<NT>(A.val, beg, end, lane, off, r, A.last,
                                 [&](int c) { return x[c] + pr.xc[pr.agg[c]]; });
    } else {
      return aligned_sum_f64<NT>(A.val, beg, end, lane, off, r, A.last,
                                 [&](int c) { return x[c] + pr.xc[pr.agg[c]]; });
    }
  }
#pragma unroll 4
  for (int p = beg + lane; p < end; p += kSlice) {
    const int c = ld<NT>(A.col + p);
    acc += ld<NT>(A.val + p) * (x[c] + pr.xc[pr.agg[c]]);
  }
  return acc;
}

// k_first_res on x + P x_c (the post-smoothing's first step takes over the prolongation;
// x itself is left for the next kernel, which adds the row's own x_c term).
template <typename T, int MODE, bool NT>
__global__ __launch_bounds__(kBlock) void k_first_res_prol(int64_t n, EllView<T> A, const T* __restrict__ minv,
                                                           const T* __restrict__ b, const T* __restrict__ x,
                                                           Prol<T> pr, T* __restrict__ r, T* __restrict__ g, T c) {
  const int64_t i = row_index();
  if (i >= n) return;
  const T res = ld<NT>(b + i) - ell_dot_prol<NT>(A, i, x, pr);
  const T mi = ld<NT>(minv + i);
  if (MODE == 0) {
    st<NT>(r + i, res);
    g[i] = c * (mi * res);
  } else {
    const T ri = mi * res;
    st<NT>(r + i, ri);
    g[i] = ri / c;
  }
}

// One l1-Jacobi sweep x_new = x_old + M^{-1}(b - A x_old) (eq. l1smooth).
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_jacobi(int64_t n, EllView<T> A, const T* __restrict__ minv,
                                                   const T* __restrict__ b, const T* __restrict__ xold,
                                                   T* __restrict__ xnew) {
  const int64_t i = row_of_thread<G>();
  if (exit_rows<G>(i, n)) return;
  const T ax = ell_dot<false, G>(A, i, xold);
  if (row_owner<G>(i, n)) xnew[i] = xold[i] + minv[i] * (b[i] - ax);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_jacobi_zero(int64_t n, const T* __restrict__ minv,
                                                        const T* __restrict__ b, T* __restrict__ x) {
  const int64_t i = row_index();
  if (i >= n) return;
  x[i] = minv[i] * b[i];
}

// ---------------------------------------------------------------------------
// Grid transfers (piecewise-constant P from box aggregates)
// ---------------------------------------------------------------------------
// b_c[I] = sum over the rows i of aggregate I (ascending) of r_i, r = b - A x
// computed beforehand by k_residual (one row per lane, coalesced).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(int64_t nc, const int32_t* __restrict__ ch,
                                                     const T* __restrict__ r, T* __restrict__ bc) {
  const int64_t I = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (I >= nc) return;
  const int4 c0 = reinterpret_cast<const int4*>(ch)[2 * I];
  const int4 c1 = reinterpret_cast<const int4*>(ch)[2 * I + 1];
  const int c[kMaxChildren] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
  T s = T(0);
#pragma unroll
  for (int k = 0; k < kMaxChildren; ++k) {
    if (c[k] >= 0) s += r[c[k]];
  }
  bc[I] = s;
}

// b_c = P^T b - R x for the 2x2x2 box P, with the restriction product R = P^T A stored in
// offset-aligned slices whose offsets are taken against the aggregate's first row (one coarse row
// per lane): the coarse right-hand side comes without forming the fine residual b - A x.  A
// 27-point fine level has 64 entries per aggregate in R (8 per fine row, against 27 in A), a
// 7-point one 32; R is the same matrix as P^T A, summed in another order, so b_c equals
// P^T (b - A x) up to rounding.
template <typename T, bool NT>
__global__ __launch_bounds__(kBlock) void k_restrict_product(int64_t nc, EllView<T> R, const int32_t* __restrict__ ch,
                                                             const T* __restrict__ b, const T* __restrict__ x,
                                                             T* __restrict__ bc) {
  const int64_t I = row_index();
  if (I >= nc) return;
  const int4 c0 = reinterpret_cast<const int4*>(ch)[2 * I];
  const int4 c1 = reinterpret_cast<const int4*>(ch)[2 * I + 1];
  const int s = __builtin_amdgcn_readfirstlane((int)(I >> 6));
  const int beg = __builtin_amdgcn_readfirstlane(R.sptr[s]);
  const int end = __builtin_amdgcn_readfirstlane(R.sptr[s + 1]);
  const int32_t* off = R.doff + (beg >> 6);
  const int lane = (int)(I & 63);
  auto gx = [&](int j) { return x[j]; };
  T rx;
  if constexpr (std::is_same_v<T, float>)
    rx = aligned_sum_f32<NT>(R.val, beg, end, lane, off, c0.x, R.last, gx);
  else
    rx = aligned_sum_f64<NT>(R.val, beg, end, lane, off, c0.x, R.last, gx);
  const int c[kMaxChildren] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
  T sb = T(0);
#pragma unroll
  for (int k = 0; k < kMaxChildren; ++k) {
    if (c[k] >= 0) sb += ld<NT>(b + c[k]);
  }
  bc[I] = sb - rx;
}

// (A x)_row for a row of any slice: the rows of a wavefront may lie in different slices,
// so the bounds and offsets are per-lane loads.  Same products in the same order as
// ell_dot<NT, 1>.
template <bool NT, typename T>
__device__ __forceinline__ T ell_dot_any(EllView<T> A, int row, const T* __restrict__ x) {
  const int s = row >> 6;
  const int beg = A.sptr[s], end = A.sptr[s + 1];
  T acc = T(0);
  if (A.doff) {
    const int32_t* off = A.doff + (beg >> 6);
    if constexpr (std::is_same_v<T, float>) {
      auto g = [&](int c) { return x[c]; };
      return aligned_sum_f32<NT, decltype(g), false>(A.val, beg, end, row & 63, off, row, A.last, g);
    } else {
      auto g = [&](int c) { return x[c]; };
      return aligned_sum_f64<NT, decltype(g), false>(A.val, beg, end, row & 63, off, row, A.last, g);
    }
  }
#pragma unroll 4
  for (int p = beg + (row & 63); p < end; p += kSlice) acc += ld<NT>(A.val + p) * x[ld<NT>(A.col + p)];
  return acc;
}

// b_c = P^T (b - A x) for the box P in one pass (one row per lane levels): eight lanes per
// aggregate, one per child (ascending, -1 padded), each forming its child's residual; the
// first lane of the eight adds them in ascending order (the absent ones as +0, which
// leaves the sum unchanged), the order of k_residual followed by k_restrict.  A wavefront's
// children form four runs of 16 rows, so its loads are less coalesced than the residual's:
// on large levels the two-kernel path is faster (measured at 128^3: 36.2 vs 26.0 + 6.8 us
// on the fine level; one launch saved on 262144 rows, 6.5 vs 5.0 + 4.8 us).
constexpr int64_t kFusedRestrictMaxRows = 1 << 20;

template <typename T, bool NT>
__global__ __launch_bounds__(kBlock) void k_res_restrict(int64_t nc, EllView<T> A, const int32_t* __restrict__ ch,
                                                         const T* __restrict__ b, const T* __restrict__ x,
                                                         T* __restrict__ bc) {
  const int64_t t = row_index();
  const int64_t I = t / kMaxChildren;
  T res = T(0);
  if (I < nc) {
    const int c = ld<NT>(ch + t);
    if (c >= 0) res = ld<NT>(b + c) - ell_dot_any<NT>(A, c, x);
  }
  const int base = (int)(threadIdx.x & (kWave - 1)) & ~(kMaxChildren - 1);
  T sum = T(0);
#pragma unroll
  for (int k = 0; k < kMaxChildren; ++k) sum += __shfl(res, base + k, kWave);
  if (I < nc && (t & (kMaxChildren - 1)) == 0) bc[I] = sum;
}

template <typename T, bool NT>
__global__ __launch_bounds__(kBlock) void k_prolong(int64_t n, const int32_t* __restrict__ agg,
                                                    const T* __restrict__ xc, T* __restrict__ x) {
  const int64_t i = row_index();
  if (i >= n) return;
  x[i] = ld<NT>(x + i) + xc[ld<NT>(agg + i)];
}

// y += A x for an explicit (smoothed) prolongator in sliced ELL
template <typename T, bool NT, int G>
__global__ __launch_bounds__(kBlock) void k_spmv_add(int64_t n, EllView<T> A, const T* __restrict__ x,
                                                     T* __restrict__ y) {
  const int64_t i = row_of_thread<G>();
  if (exit_rows<G>(i, n)) return;
  const T v = ell_dot<NT, G>(A, i, x);
  if (row_owner<G>(i, n)) y[i] = ld<NT>(y + i) + v;
}

// ---------------------------------------------------------------------------
// Vector kernels
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpy(int64_t n, T a, const T* __restrict__ x, T* __restrict__ y, Wt av,
                                                 Prol<T> pr) {
  const int64_t i = row_index();
  if (i >= n) return;
  T yi = y[i];
  if (pr.agg) yi = yi + pr.xc[pr.agg[i]];
  y[i] = yi + wsel(av, a, i) * x[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(int64_t n, const T* __restrict__ x, T* __restrict__ y) {
  const int64_t i = row_index();
  if (i >= n) return;
  y[i] = x[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, T v, T* __restrict__ y) {
  const int64_t i = row_index();
  if (i >= n) return;
  y[i] = v;
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kBlock) void k_cast(int64_t n, const Tin* __restrict__ x, Tout* __restrict__ y) {
  const int64_t i = row_index();
  if (i >= n) return;
  y[i] = (Tout)x[i];
}

// b = (float) r and u = M^{-1} b, the products the merged first two steps form for their gathered
// neighbours (an FP32 hierarchy's fine level, read by k_first2_zero<..., U>)
template <bool NT>
__global__ __launch_bounds__(kBlock) void k_cast_u(int64_t n, const double* __restrict__ r,
                                                   const float* __restrict__ minv, float* __restrict__ b,
                                                   float* __restrict__ u) {
  const int64_t i = row_index();
  if (i >= n) return;
  const float bi = (float)ld<NT>(r + i);
  b[i] = bi;
  u[i] = minv[i] * bi;
}

// ---------------------------------------------------------------------------
// CG kernels (float64): fused SpMV + dot, update + dot, and a single-block
// second-stage reduction that also forms the CG scalars on the device.
// ---------------------------------------------------------------------------
// b and d may be float (the FP32 hierarchy's preconditioned vector): the conversion to
// double is exact, so the products are those of a converted copy.
template <bool NT, typename TZ>
__global__ __launch_bounds__(kBlock) void k_dot2(int64_t n, const double* __restrict__ a,
                                                 const TZ* __restrict__ b, const double* __restrict__ c,
                                                 const TZ* __restrict__ d, double* __restrict__ partial) {
  const int64_t i = row_index();
  double v = 0.0, u = 0.0;
  if (i < n) {
    v = ld<NT>(a + i) * (double)ld<NT>(b + i);
    if (c) u = ld<NT>(c + i) * (double)ld<NT>(d + i);
  }
  const double sv = block_sum(v);
  __syncthreads();
  const double su = c ? block_sum(u) : 0.0;
  if (threadIdx.x == 0) {
    partial[logical_block()] = sv;
    partial[gridDim.x + logical_block()] = su;
  }
}

// The CG direction update fused into the next SpMV: p_new = z + beta p_old and
// q = A p_new, with (p_new, q) partials.  p_new of a neighbour is formed on the
// fly from z and p_old (exactly the value stored for it), so p_new is written
// to the other buffer of a pair.  z may be float (exactly converted, as in k_dot2).
// x (optional): the previous iteration's x += alpha p_old (alpha still in the device scalars),
// done here because the pass reads p_old anyway; the update kernel then leaves x alone.
// PRE: p_new was formed beforehand by k_form_p (streaming levels): the product gathers one vector
// instead of two (measured on a 27-point level of 32.8M rows: 1.36 ms + 0.13 ms for the separate
// pass, against 1.77 ms with z and p_old both gathered; 7-point 256^3: 0.191 + 0.071 against
// 0.284 ms).  The values and the products are the same either way.
template <bool NT, typename TZ, bool PRE, bool W = false>
__global__ __launch_bounds__(kBlock) void k_spmv_dot_p(int64_t n, EllView<double> A, const double* __restrict__ scal,
                                                       const TZ* __restrict__ z, const double* __restrict__ pold,
                                                       double* pnew, double* __restrict__ q,
                                                       double* __restrict__ partial, double* __restrict__ x) {
  // with an FP32 hierarchy (float z) this product is the only reader of the FP64 matrix, once
  // per iteration: its values are streamed so that they do not displace the FP32 smoother's
  // matrix and vectors from the caches (128^3: FP32-hierarchy solve 6.63 to 6.36 ms)
  constexpr bool kStreamVal = NT || std::is_same_v<TZ, float>;
  const int64_t i = row_index();
  const double beta = scal[S_BETA];
  auto pj = [&](int j) {
    if constexpr (PRE) return pnew[j]; else return (double)z[j] + beta * pold[j];
  };
  double v = 0.0;
  if (i < n) {
    const int s = __builtin_amdgcn_readfirstlane((int)(i >> 6));
    const int beg = __builtin_amdgcn_readfirstlane(A.sptr[s]);
    const int end = __builtin_amdgcn_readfirstlane(A.sptr[s + 1]);
    double pw = 0.0;
    if constexpr (PRE && W) pw = pnew[i];  // wide slices: the row's own entry first (see kWideBatch)
    double acc = 0.0;
    if (A.doff) {
      const int32_t* off = A.doff + (beg >> 6);
      acc = aligned_sum_f64<kStreamVal, decltype(pj), true, W ? kWideBatch : kAlignedBatch>(
          A.val, beg, end, (int)(i & 63), off, (int)i, A.last, pj);
    } else {
#pragma unroll 4
      for (int p = beg + (int)(i & 63); p < end; p += kSlice) {
        const int j = ld<NT>(A.col + p);
        acc += ld<kStreamVal>(A.val + p) * pj(j);
      }
    }
    double pi;
    if constexpr (PRE) {
      pi = W ? pw : pnew[i];
    } else {
      const double po = pold[i];
      pi = z[i] + beta * po;
      st<NT>(pnew + i, pi);
      if (x) st<NT>(x + i, ld<NT>(x + i) + scal[S_ALPHA] * po);
    }
    st<NT>(q + i, acc);
    v = pi * acc;
  }
  const double sum = block_sum(v);
  if (threadIdx.x == 0) partial[logical_block()] = sum;
}

// p_new = z + beta p_old (beta from the device scalars), the expression of k_spmv_dot_p, and
// (x given) the previous iteration's x += alpha p_old, as there
template <bool NT, typename TZ>
__global__ __launch_bounds__(kBlock) void k_form_p(int64_t n, const double* __restrict__ scal,
                                                   const TZ* __restrict__ z, const double* __restrict__ pold,
                                                   double* __restrict__ pnew, double* __restrict__ x) {
  const int64_t i = row_index();
  if (i >= n) return;
  const double po = ld<NT>(pold + i);
  pnew[i] = (double)ld<NT>(z + i) + scal[S_BETA] * po;
  if (x) st<NT>(x + i, ld<NT>(x + i) + scal[S_ALPHA] * po);
}

// x += alpha p (alpha from the device scalars): the last iteration's update of x, which the
// iterations before leave to the next direction pass
template <bool NT>
__global__ __launch_bounds__(kBlock) void k_cg_x(int64_t n, const double* __restrict__ scal,
                                                 const double* __restrict__ p, double* __restrict__ x) {
  const int64_t i = row_index();
  if (i >= n) return;
  st<NT>(x + i, ld<NT>(x + i) + scal[S_ALPHA] * ld<NT>(p + i));
}

// r -= alpha q (alpha from the device scalars), partial (r, r); rold (flexible CG) receives the
// previous r.  x is updated by the next direction pass (k_form_p, k_spmv_dot_p) or k_cg_x.
// u (optional) receives M^{-1} r for the preconditioner's first kernel (k_first2_zero, U).
template <bool NT>
__global__ __launch_bounds__(kBlock) void k_cg_update(int64_t n, const double* __restrict__ scal,
                                                      const double* __restrict__ q, double* __restrict__ r,
                                                      double* __restrict__ rold, double* __restrict__ partial,
                                                      const double* __restrict__ minv, double* __restrict__ u) {
  const int64_t i = row_index();
  const double alpha = scal[S_ALPHA];
  double v = 0.0;
  if (i < n) {
    const double ro = ld<NT>(r + i);
    if (rold) st<NT>(rold + i, ro);
    const double rn = ro - alpha * ld<NT>(q + i);
    r[i] = rn;
    if (u) st<NT>(u + i, minv[i] * rn);
    v = rn * rn;
  }
  const double s = block_sum(v);
  if (threadIdx.x == 0) partial[logical_block()] = s;
}

// Optional middle stage for long partial lists: block b sums the contiguous chunk b of both
// arrays into out[b] and out[gridDim.x + b].
__global__ __launch_bounds__(1024) void k_reduce_chunks(unsigned nb, int two, const double* __restrict__ partial,
                                                        double* __restrict__ out) {
  __shared__ double sm[2][1024 / kWave];
  const unsigned chunk = (nb + gridDim.x - 1) / gridDim.x;
  const unsigned lo = blockIdx.x * chunk, hi = min(nb, lo + chunk);
  double v = 0.0, u = 0.0;
  for (unsigned j = lo + threadIdx.x; j < hi; j += 1024) {
    v += partial[j];
    if (two) u += partial[nb + j];
  }
  for (int off = 32; off > 0; off >>= 1) {
    v += __shfl_xor(v, off, kWave);
    u += __shfl_xor(u, off, kWave);
  }
  if ((threadIdx.x & 63) == 0) {
    sm[0][threadIdx.x / kWave] = v;
    sm[1][threadIdx.x / kWave] = u;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double s = 0.0, t = 0.0;
  for (int w = 0; w < 1024 / kWave; ++w) {
    s += sm[0][w];
    t += sm[1][w];
  }
  out[blockIdx.x] = s;
  out[gridDim.x + blockIdx.x] = t;
}

__global__ __launch_bounds__(1024) void k_reduce(int mode, unsigned nb, const double* __restrict__ partial,
                                                 double* __restrict__ scal, int* __restrict__ flag,
                                                 double* __restrict__ pub) {
  __shared__ double sm[2][1024 / kWave];
  const bool two = (mode == RED_BETA_FLEX);
  double v = 0.0, u = 0.0;
  for (unsigned j = threadIdx.x; j < nb; j += 1024) {
    v += partial[j];
    if (two) u += partial[nb + j];
  }
  for (int off = 32; off > 0; off >>= 1) {
    v += __shfl_xor(v, off, kWave);
    u += __shfl_xor(u, off, kWave);
  }
  if ((threadIdx.x & 63) == 0) {
    sm[0][threadIdx.x / kWave] = v;
    sm[1][threadIdx.x / kWave] = u;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double s = 0.0, t = 0.0;
  for (int w = 0; w < 1024 / kWave; ++w) {
    s += sm[0][w];
    t += sm[1][w];
  }
  switch (mode) {
    case RED_BB:
      scal[S_BB] = s;
      break;
    case RED_RZ0:
      scal[S_RZ] = s;
      scal[S_BETA] = 0.0;
      break;
    case RED_ALPHA:
      scal[S_PQ] = s;
      if (s > 0.0) {
        scal[S_ALPHA] = scal[S_RZ] / s;
      } else {  // breakdown: the update that follows leaves x and r as they are
        flag[F_BREAKDOWN] = 1;
        scal[S_ALPHA] = 0.0;
      }
      break;
    case RED_RR:
      scal[S_RR] = s;
      if (!(s == s) || s > 1.0e300) flag[F_NAN] = 1;
      if (pub) {
        pub[0] = s;
        pub[1] = (double)flag[F_BREAKDOWN];
        pub[2] = (double)flag[F_NAN];
      }
      break;
    case RED_BETA:
      scal[S_BETA] = s / scal[S_RZ];
      scal[S_RZ] = s;
      break;
    case RED_BETA_FLEX:  // s = (r_new, z_new), t = (r_old, z_new)
      scal[S_BETA] = (s - t) / scal[S_RZ];
      scal[S_RZ] = s;
      break;
  }
}

__global__ __launch_bounds__(kBlock) void k_check_finite(int64_t n, const double* __restrict__ x,
                                                         int* __restrict__ flag) {
  const int64_t i = row_index();
  if (i >= n) return;
  const double v = x[i];
  if (!(v == v) || v > 1.0e308 || v < -1.0e308) flag[F_NAN] = 1;
}

}  // namespace

#define LAUNCH_OK() (hipGetLastError() == hipSuccess ? AMG_OK : AMG_EHIP)

// Levels above kRemapMaxBlocks blocks take the streaming (NT) kernels (one row per lane).
inline bool streamed(unsigned grid) { return grid > kRemapMaxBlocks; }

// FP64 offset-aligned levels of one row per lane averaging at least kWideMinSteps stored steps
// per row take the wide-batch kernels (W = true); FP32 levels keep theirs (quads in batches of
// 12 steps already).
inline bool wide(const Ell<double>& A) {
  return A.doff && A.group == 1 && A.padded >= (int64_t)kWideMinSteps * A.n;
}

// The levels whose merged first two steps can read u = M^{-1} b instead of gathering M^{-1} and b
bool first2_takes_u(const Ell<double>& A) { return streamed(xcd_grid(A.n)) && wide(A); }
bool first2_takes_u(const Ell<float>& A) {
  return streamed(xcd_grid(A.n)) && A.doff && A.group == 1 && A.padded >= (int64_t)kWideMinSteps * A.n;
}

// Runs f(std::integral_constant<int, G>) for the matrix's lanes per row G.
template <typename F>
int with_group(int group, F&& f) {
  switch (group) {
    case 1: f(std::integral_constant<int, 1>()); break;
    case 4: f(std::integral_constant<int, 4>()); break;
    case 16: f(std::integral_constant<int, 16>()); break;
    case 64: f(std::integral_constant<int, 64>()); break;
    default: return AMG_EINVAL;
  }
  return LAUNCH_OK();
}

template <typename T>
int launch_spmv(hipStream_t s, const Ell<T>& A, const T* x, T* y) {
  return with_group(A.group, [&](auto gc) {
    constexpr int G = decltype(gc)::value;
    const unsigned g = xcd_grid(A.n * G);
    if constexpr (G == 1) {
      if (streamed(g)) {
        hipLaunchKernelGGL((k_spmv<T, true, 1>), dim3(g), dim3(kBlock), 0, s, A.n, view(A), x, y);
        return;
      }
    }
    hipLaunchKernelGGL((k_spmv<T, false, G>), dim3(g), dim3(kBlock), 0, s, A.n, view(A), x, y);
  });
}

template <typename T>
int launch_residual(hipStream_t s, const Ell<T>& A, const T* b, const T* x, T* r) {
  return with_group(A.group, [&](auto gc) {
    constexpr int G = decltype(gc)::value;
    const unsigned g = xcd_grid(A.n * G);
    if constexpr (G == 1) {
      if (streamed(g)) {
        hipLaunchKernelGGL((k_residual<T, true, 1>), dim3(g), dim3(kBlock), 0, s, A.n, view(A), b, x, r);
        return;
      }
    }
    hipLaunchKernelGGL((k_residual<T, false, G>), dim3(g), dim3(kBlock), 0, s, A.n, view(A), b, x, r);
  });
}

template <typename T, bool NT>
void go_first_zero(dim3 gr, hipStream_t s, int mode, bool store, int64_t n, const T* minv, const T* b, T* g, T* r,
                   T* x, T c, T w, Wt wv) {
  dim3 bl(kBlock);
  if (mode == 0 && store)
    hipLaunchKernelGGL((k_first_zero<T, 0, true, NT>), gr, bl, 0, s, n, minv, b, g, r, x, c, w, wv);
  else if (mode == 0)
    hipLaunchKernelGGL((k_first_zero<T, 0, false, NT>), gr, bl, 0, s, n, minv, b, g, r, x, c, w, wv);
  else if (store)
    hipLaunchKernelGGL((k_first_zero<T, 1, true, NT>), gr, bl, 0, s, n, minv, b, g, r, x, c, w, wv);
  else
    hipLaunchKernelGGL((k_first_zero<T, 1, false, NT>), gr, bl, 0, s, n, minv, b, g, r, x, c, w, wv);
}

template <typename T>
int launch_first_zero(hipStream_t s, int mode, bool store, int64_t n, const T* minv, const T* b, T* g, T* r,
                      T* x, double c, double w, Wt wv) {
  const dim3 gr(xcd_grid(n));
  if (streamed(gr.x))
    go_first_zero<T, true>(gr, s, mode, store, n, minv, b, g, r, x, (T)c, (T)w, wv);
  else
    go_first_zero<T, false>(gr, s, mode, store, n, minv, b, g, r, x, (T)c, (T)w, wv);
  return LAUNCH_OK();
}

template <typename T, bool NT, int G, bool W = false, bool U = false>
void go_first2_zero(dim3 gr, hipStream_t s, int mode, bool store, EllView<T> A, int64_t n, const T* minv,
                    const T* b, T* gnew, T* r, T* x, T a1, T a2, T a3, T a4, T a5, Wt w1v, Wt w2v,
                    const T* u = nullptr) {
  dim3 bl(kBlock);
  if (mode == 0 && store)
    hipLaunchKernelGGL((k_first2_zero<T, 0, true, NT, G, W, U>), gr, bl, 0, s, n, A, minv, b, gnew, r, x, a1, a2,
                       a3, a4, a5, w1v, w2v, u);
  else if (mode == 0)
    hipLaunchKernelGGL((k_first2_zero<T, 0, false, NT, G, W, U>), gr, bl, 0, s, n, A, minv, b, gnew, r, x, a1, a2,
                       a3, a4, a5, w1v, w2v, u);
  else if (store)
    hipLaunchKernelGGL((k_first2_zero<T, 1, true, NT, G, W, U>), gr, bl, 0, s, n, A, minv, b, gnew, r, x, a1, a2,
                       a3, a4, a5, w1v, w2v, u);
  else
    hipLaunchKernelGGL((k_first2_zero<T, 1, false, NT, G, W, U>), gr, bl, 0, s, n, A, minv, b, gnew, r, x, a1, a2,
                       a3, a4, a5, w1v, w2v, u);
}

template <typename T>
int launch_first2_zero(hipStream_t s, int mode, bool store, const Ell<T>& A, const T* minv, const T* b, T* gnew,
                       T* r, T* x, double c1, double alpha, double c, double w1, double w2, Wt w1v, Wt w2v,
                       const T* u) {
  return with_group(A.group, [&](auto gc) {
    constexpr int G = decltype(gc)::value;
    const dim3 gr(xcd_grid(A.n * G));
    if constexpr (G == 1) {
      if (streamed(gr.x)) {
        if constexpr (std::is_same_v<T, double>) {
          if (wide(A)) {
            if (u)
              go_first2_zero<T, true, 1, true, true>(gr, s, mode, store, view(A), A.n, minv, b, gnew, r, x, (T)c1,
                                                     (T)alpha, (T)c, (T)w1, (T)w2, w1v, w2v, u);
            else
              go_first2_zero<T, true, 1, true>(gr, s, mode, store, view(A), A.n, minv, b, gnew, r, x, (T)c1,
                                               (T)alpha, (T)c, (T)w1, (T)w2, w1v, w2v);
            return;
          }
        } else if (u) {
          go_first2_zero<T, true, 1, false, true>(gr, s, mode, store, view(A), A.n, minv, b, gnew, r, x, (T)c1,
                                                  (T)alpha, (T)c, (T)w1, (T)w2, w1v, w2v, u);
          return;
        }
        go_first2_zero<T, true, 1>(gr, s, mode, store, view(A), A.n, minv, b, gnew, r, x, (T)c1, (T)alpha, (T)c,
                                   (T)w1, (T)w2, w1v, w2v);
        return;
      }
    }
    go_first2_zero<T, false, G>(gr, s, mode, store, view(A), A.n, minv, b, gnew, r, x, (T)c1, (T)alpha, (T)c,
                                (T)w1, (T)w2, w1v, w2v);
  });
}

template <typename T, bool NT, int G, bool W = false>
void go_first_res(dim3 gr, hipStream_t s, int mode, EllView<T> A, int64_t n, const T* minv, const T* b, const T* x,
                  T* r, T* g, T c) {
  if (mode == 0)
    hipLaunchKernelGGL((k_first_res<T, 0, NT, G, W>), gr, dim3(kBlock), 0, s, n, A, minv, b, x, r, g, c);
  else
    hipLaunchKernelGGL((k_first_res<T, 1, NT, G, W>), gr, dim3(kBlock), 0, s, n, A, minv, b, x, r, g, c);
}

template <typename T>
int launch_first_res(hipStream_t s, int mode, const Ell<T>& A, const T* minv, const T* b, const T* x, T* r,
                     T* g, double c, Prol<T> pr) {
  if (pr.agg) {
    if (A.group != 1) return AMG_EINVAL;
    const dim3 gr(xcd_grid(A.n));
    const T cc = (T)c;
    const EllView<T> av = view(A);
    const dim3 bl(kBlock);
    if (streamed(gr.x)) {
      if (mode == 0)
        hipLaunchKernelGGL((k_first_res_prol<T, 0, true>), gr, bl, 0, s, A.n, av, minv, b, x, pr, r, g, cc);
      else
        hipLaunchKernelGGL((k_first_res_prol<T, 1, true>), gr, bl, 0, s, A.n, av, minv, b, x, pr, r, g, cc);
    } else {
      if (mode == 0)
        hipLaunchKernelGGL((k_first_res_prol<T, 0, false>), gr, bl, 0, s, A.n, av, minv, b, x, pr, r, g, cc);
      else
        hipLaunchKernelGGL((k_first_res_prol<T, 1, false>), gr, bl, 0, s, A.n, av, minv, b, x, pr, r, g, cc);
    }
    return LAUNCH_OK();
  }
  return with_group(A.group, [&](auto gc) {
    constexpr int G = decltype(gc)::value;
    const dim3 gr(xcd_grid(A.n * G));
    if constexpr (G == 1) {
      if (streamed(gr.x)) {
        if constexpr (std::is_same_v<T, double>) {
          if (wide(A)) {
            go_first_res<T, true, 1, true>(gr, s, mode, view(A), A.n, minv, b, x, r, g, (T)c);
            return;
          }
        }
        go_first_res<T, true, 1>(gr, s, mode, view(A), A.n, minv, b, x, r, g, (T)c);
        return;
      }
    }
    go_first_res<T, false, G>(gr, s, mode, view(A), A.n, minv, b, x, r, g, (T)c);
  });
}

template <typename T, bool NT, int G, bool W = false>
void go_fused(dim3 gr, hipStream_t s, int mode, bool store, EllView<T> A, int64_t n, const T* minv, const T* gold,
              T* gnew, const T* rin, T* rout, T* x, T a_, T c_, T w_, T wp_, Wt wv, Wt wpv, Prol<T> pr) {
  dim3 bl(kBlock);
  if (!x) {  // a stored step that leaves x alone (the caller only passes null x with store set)
    if (mode == 0)
      hipLaunchKernelGGL((k_fused_keep_x<T, 0, NT, G, W>), gr, bl, 0, s, n, A, minv, gold, gnew, rin, rout, a_, c_);
    else
      hipLaunchKernelGGL((k_fused_keep_x<T, 1, NT, G, W>), gr, bl, 0, s, n, A, minv, gold, gnew, rin, rout, a_, c_);
    return;
  }
  if (mode == 0 && store)
    hipLaunchKernelGGL((k_fused<T, 0, true, NT, G, W>), gr, bl, 0, s, n, A, minv, gold, gnew, rin, rout, x, a_, c_,
                       w_, wp_, wv, wpv, pr);
  else if (mode == 0)
    hipLaunchKernelGGL((k_fused<T, 0, false, NT, G, W>), gr, bl, 0, s, n, A, minv, gold, gnew, rin, rout, x, a_, c_,
                       w_, wp_, wv, wpv, pr);
  else if (store)
    hipLaunchKernelGGL((k_fused<T, 1, true, NT, G, W>), gr, bl, 0, s, n, A, minv, gold, gnew, rin, rout, x, a_, c_,
                       w_, wp_, wv, wpv, pr);
  else
    hipLaunchKernelGGL((k_fused<T, 1, false, NT, G, W>), gr, bl, 0, s, n, A, minv, gold, gnew, rin, rout, x, a_, c_,
                       w_, wp_, wv, wpv, pr);
}

template <typename T>
int launch_fused(hipStream_t s, int mode, bool store, const Ell<T>& A, const T* minv, const T* gold, T* gnew,
                 const T* rin, T* rout, T* x, double alpha, double c, double w, double wprev, Wt wv, Wt wpv,
                 Prol<T> pr) {
  return with_group(A.group, [&](auto gc) {
    constexpr int G = decltype(gc)::value;
    const dim3 gr(xcd_grid(A.n * G));
    if constexpr (G == 1) {
      if (streamed(gr.x)) {
        if constexpr (std::is_same_v<T, double>) {
          if (wide(A)) {
            go_fused<T, true, 1, true>(gr, s, mode, store, view(A), A.n, minv, gold, gnew, rin, rout, x, (T)alpha,
                                       (T)c, (T)w, (T)wprev, wv, wpv, pr);
            return;
          }
        }
        go_fused<T, true, 1>(gr, s, mode, store, view(A), A.n, minv, gold, gnew, rin, rout, x, (T)alpha, (T)c, (T)w,
                             (T)wprev, wv, wpv, pr);
        return;
      }
    }
    go_fused<T, false, G>(gr, s, mode, store, view(A), A.n, minv, gold, gnew, rin, rout, x, (T)alpha, (T)c, (T)w,
                          (T)wprev, wv, wpv, pr);
  });
}

template <typename T>
int launch_fused_dot(hipStream_t s, int mode, const Ell<T>& A, const T* minv, const T* gold, const T* rin, T* x,
                     double alpha, double c, double w, double wprev, Wt wv, Wt wpv, Prol<T> pr, const double* dr,
                     const double* drold, double* partial, unsigned* nblocks) {
  if (A.group != 1) return AMG_EINVAL;
  const dim3 gr(xcd_grid(A.n)), bl(kBlock);
  auto go = [&](auto nt, auto wd) {
    constexpr bool NT = decltype(nt)::value, W = decltype(wd)::value;
    if (mode == 0)
      hipLaunchKernelGGL((k_fused_dot<T, 0, NT, W>), gr, bl, 0, s, A.n, view(A), minv, gold, rin, x, (T)alpha, (T)c,
                         (T)w, (T)wprev, wv, wpv, pr, dr, drold, partial);
    else
      hipLaunchKernelGGL((k_fused_dot<T, 1, NT, W>), gr, bl, 0, s, A.n, view(A), minv, gold, rin, x, (T)alpha, (T)c,
                         (T)w, (T)wprev, wv, wpv, pr, dr, drold, partial);
  };
  using T_ = std::true_type;
  using F_ = std::false_type;
  bool wd = false;
  if constexpr (std::is_same_v<T, double>) wd = wide(A);  // the wide batches are FP64 only, as in launch_fused
  if (!streamed(gr.x))
    go(F_(), F_());
  else if (wd)
    go(T_(), std::integral_constant<bool, std::is_same_v<T, double>>());
  else
    go(T_(), F_());
  *nblocks = gr.x;
  return LAUNCH_OK();
}
template int launch_fused_dot<double>(hipStream_t, int, const Ell<double>&, const double*, const double*,
                                      const double*, double*, double, double, double, double, Wt, Wt, Prol<double>,
                                      const double*, const double*, double*, unsigned*);
template int launch_fused_dot<float>(hipStream_t, int, const Ell<float>&, const float*, const float*, const float*,
                                     float*, double, double, double, double, Wt, Wt, Prol<float>, const double*,
                                     const double*, double*, unsigned*);

template <typename T>
int launch_jacobi(hipStream_t s, const Ell<T>& A, const T* minv, const T* b, const T* xold, T* xnew) {
  return with_group(A.group, [&](auto gc) {
    constexpr int G = decltype(gc)::value;
    hipLaunchKernelGGL((k_jacobi<T, G>), dim3(xcd_grid(A.n * G)), dim3(kBlock), 0, s, A.n, view(A), minv, b, xold,
                       xnew);
  });
}

template <typename T>
int launch_jacobi_zero(hipStream_t s, int64_t n, const T* minv, const T* b, T* x) {
  hipLaunchKernelGGL(k_jacobi_zero<T>, dim3(xcd_grid(n)), dim3(kBlock), 0, s, n, minv, b, x);
  return LAUNCH_OK();
}

template <typename T>
int launch_restrict(hipStream_t s, const Ell<T>& A, int64_t nc, const int32_t* children, const T* b,
                    const T* x, T* tmp, T* bc) {
  static_assert(kMaxChildren == 8 && kWave % kMaxChildren == 0, "eight lanes per aggregate");
  if (A.group == 1 && A.n <= kFusedRestrictMaxRows) {
    const unsigned g = xcd_grid(nc * kMaxChildren);
    if (streamed(g))
      hipLaunchKernelGGL((k_res_restrict<T, true>), dim3(g), dim3(kBlock), 0, s, nc, view(A), children, b, x, bc);
    else
      hipLaunchKernelGGL((k_res_restrict<T, false>), dim3(g), dim3(kBlock), 0, s, nc, view(A), children, b, x, bc);
    return LAUNCH_OK();
  }
  AMGP_TRY(launch_residual<T>(s, A, b, x, tmp));
  hipLaunchKernelGGL(k_restrict<T>, dim3(grid_for(nc)), dim3(kBlock), 0, s, nc, children, (const T*)tmp, bc);
  return LAUNCH_OK();
}

template <typename T>
int launch_restrict_product(hipStream_t s, const Ell<T>& R, const int32_t* children, const T* b, const T* x,
                            T* bc) {
  // streaming loads when the fine level streams
  const unsigned g = xcd_grid(R.n);
  if (streamed(xcd_grid(R.ncols)))
    hipLaunchKernelGGL((k_restrict_product<T, true>), dim3(g), dim3(kBlock), 0, s, R.n, view(R), children, b, x, bc);
  else
    hipLaunchKernelGGL((k_restrict_product<T, false>), dim3(g), dim3(kBlock), 0, s, R.n, view(R), children, b, x, bc);
  return LAUNCH_OK();
}

template <typename T>
int launch_prolong(hipStream_t s, int64_t n, const int32_t* agg, const T* xc, T* x) {
  const unsigned g = xcd_grid(n);
  if (streamed(g))
    hipLaunchKernelGGL((k_prolong<T, true>), dim3(g), dim3(kBlock), 0, s, n, agg, xc, x);
  else
    hipLaunchKernelGGL((k_prolong<T, false>), dim3(g), dim3(kBlock), 0, s, n, agg, xc, x);
  return LAUNCH_OK();
}

template <typename T>
int launch_spmv_add(hipStream_t s, const Ell<T>& A, const T* x, T* y) {
  return with_group(A.group, [&](auto gc) {
    constexpr int G = decltype(gc)::value;
    const unsigned g = xcd_grid(A.n * G);
    if constexpr (G == 1) {
      if (streamed(g)) {
        hipLaunchKernelGGL((k_spmv_add<T, true, 1>), dim3(g), dim3(kBlock), 0, s, A.n, view(A), x, y);
        return;
      }
    }
    hipLaunchKernelGGL((k_spmv_add<T, false, G>), dim3(g), dim3(kBlock), 0, s, A.n, view(A), x, y);
  });
}

template <typename T>
int launch_axpy(hipStream_t s, int64_t n, double a, const T* x, T* y, Wt av, Prol<T> pr) {
  hipLaunchKernelGGL(k_axpy<T>, dim3(xcd_grid(n)), dim3(kBlock), 0, s, n, (T)a, x, y, av, pr);
  return LAUNCH_OK();
}

template <typename T>
int launch_copy(hipStream_t s, int64_t n, const T* x, T* y) {
  hipLaunchKernelGGL(k_copy<T>, dim3(xcd_grid(n)), dim3(kBlock), 0, s, n, x, y);
  return LAUNCH_OK();
}

template <typename T>
int launch_fill(hipStream_t s, int64_t n, T v, T* y) {
  hipLaunchKernelGGL(k_fill<T>, dim3(xcd_grid(n)), dim3(kBlock), 0, s, n, v, y);
  return LAUNCH_OK();
}

template <typename Tin, typename Tout>
int launch_cast(hipStream_t s, int64_t n, const Tin* x, Tout* y) {
  hipLaunchKernelGGL((k_cast<Tin, Tout>), dim3(xcd_grid(n)), dim3(kBlock), 0, s, n, x, y);
  return LAUNCH_OK();
}

int launch_cast_u(hipStream_t s, int64_t n, const double* r, const float* minv, float* b, float* u) {
  const unsigned g = xcd_grid(n);
  if (streamed(g))
    hipLaunchKernelGGL(k_cast_u<true>, dim3(g), dim3(kBlock), 0, s, n, r, minv, b, u);
  else
    hipLaunchKernelGGL(k_cast_u<false>, dim3(g), dim3(kBlock), 0, s, n, r, minv, b, u);
  return LAUNCH_OK();
}

template <typename TZ>
int launch_dot2(hipStream_t s, int64_t n, const double* a, const TZ* b, const double* c, const TZ* d,
                double* partial, unsigned* nblocks) {
  const unsigned g = xcd_grid(n);
  if (streamed(g))
    hipLaunchKernelGGL((k_dot2<true, TZ>), dim3(g), dim3(kBlock), 0, s, n, a, b, c, d, partial);
  else
    hipLaunchKernelGGL((k_dot2<false, TZ>), dim3(g), dim3(kBlock), 0, s, n, a, b, c, d, partial);
  *nblocks = g;
  return LAUNCH_OK();
}
template int launch_dot2<double>(hipStream_t, int64_t, const double*, const double*, const double*, const double*,
                                 double*, unsigned*);
template int launch_dot2<float>(hipStream_t, int64_t, const double*, const float*, const double*, const float*,
                                double*, unsigned*);

template <typename TZ>
int launch_spmv_dot_p(hipStream_t s, const Ell<double>& A, const double* scal, const TZ* z, const double* pold,
                      double* pnew, double* q, double* partial, double* x, unsigned* nblocks) {
  const unsigned g = xcd_grid(A.n);
  if (streamed(g)) {
    hipLaunchKernelGGL((k_form_p<true, TZ>), dim3(g), dim3(kBlock), 0, s, A.n, scal, z, pold, pnew, x);
    if (wide(A))
      hipLaunchKernelGGL((k_spmv_dot_p<true, TZ, true, true>), dim3(g), dim3(kBlock), 0, s, A.n, view(A), scal, z,
                         pold, pnew, q, partial, nullptr);
    else
      hipLaunchKernelGGL((k_spmv_dot_p<true, TZ, true>), dim3(g), dim3(kBlock), 0, s, A.n, view(A), scal, z, pold,
                         pnew, q, partial, nullptr);
  } else {
    hipLaunchKernelGGL((k_spmv_dot_p<false, TZ, false>), dim3(g), dim3(kBlock), 0, s, A.n, view(A), scal, z, pold,
                       pnew, q, partial, x);
  }
  *nblocks = g;
  return LAUNCH_OK();
}
template int launch_spmv_dot_p<double>(hipStream_t, const Ell<double>&, const double*, const double*, const double*,
                                       double*, double*, double*, double*, unsigned*);
template int launch_spmv_dot_p<float>(hipStream_t, const Ell<double>&, const double*, const float*, const double*,
                                      double*, double*, double*, double*, unsigned*);

int launch_cg_update(hipStream_t s, int64_t n, const double* scal, const double* q, double* r, double* rold,
                     double* partial, unsigned* nblocks, const double* minv, double* u) {
  const unsigned g = xcd_grid(n);
  if (streamed(g))
    hipLaunchKernelGGL(k_cg_update<true>, dim3(g), dim3(kBlock), 0, s, n, scal, q, r, rold, partial, minv, u);
  else
    hipLaunchKernelGGL(k_cg_update<false>, dim3(g), dim3(kBlock), 0, s, n, scal, q, r, rold, partial, minv, u);
  *nblocks = g;
  return LAUNCH_OK();
}

int launch_cg_x(hipStream_t s, int64_t n, const double* scal, const double* p, double* x) {
  const unsigned g = xcd_grid(n);
  if (streamed(g))
    hipLaunchKernelGGL(k_cg_x<true>, dim3(g), dim3(kBlock), 0, s, n, scal, p, x);
  else
    hipLaunchKernelGGL(k_cg_x<false>, dim3(g), dim3(kBlock), 0, s, n, scal, p, x);
  return LAUNCH_OK();
}

int launch_reduce(hipStream_t s, int mode, unsigned nblocks, const double* partial, double* scal, int* flag,
                  double* pub) {
  constexpr unsigned kChunks = 64;
  if (nblocks > 16 * 1024) {
    // long lists: 64 blocks sum contiguous chunks into the tail of the partial buffer, then one block
    double* mid = const_cast<double*>(partial) + 2 * (size_t)nblocks;
    hipLaunchKernelGGL(k_reduce_chunks, dim3(kChunks), dim3(1024), 0, s, nblocks, mode == RED_BETA_FLEX ? 1 : 0,
                       partial, mid);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, s, mode, kChunks, (const double*)mid, scal, flag, pub);
  } else {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, s, mode, nblocks, partial, scal, flag, pub);
  }
  return LAUNCH_OK();
}

int launch_check_finite(hipStream_t s, int64_t n, const double* x, int* flag) {
  hipLaunchKernelGGL(k_check_finite, dim3(xcd_grid(n)), dim3(kBlock), 0, s, n, x, flag);
  return LAUNCH_OK();
}

#define INST(T)                                                                                               \
  template int launch_spmv<T>(hipStream_t, const Ell<T>&, const T*, T*);                                      \
  template int launch_residual<T>(hipStream_t, const Ell<T>&, const T*, const T*, T*);                        \
  template int launch_first_zero<T>(hipStream_t, int, bool, int64_t, const T*, const T*, T*, T*, T*, double,   \
                                    double, Wt);                                                              \
  template int launch_first2_zero<T>(hipStream_t, int, bool, const Ell<T>&, const T*, const T*, T*, T*, T*,    \
                                     double, double, double, double, double, Wt, Wt, const T*);               \
  template int launch_first_res<T>(hipStream_t, int, const Ell<T>&, const T*, const T*, const T*, T*, T*,      \
                                   double, Prol<T>);                                                          \
  template int launch_fused<T>(hipStream_t, int, bool, const Ell<T>&, const T*, const T*, T*, const T*, T*, T*,  \
                               double, double, double, double, Wt, Wt, Prol<T>);                              \
  template int launch_jacobi<T>(hipStream_t, const Ell<T>&, const T*, const T*, const T*, T*);                \
  template int launch_jacobi_zero<T>(hipStream_t, int64_t, const T*, const T*, T*);                           \
  template int launch_restrict<T>(hipStream_t, const Ell<T>&, int64_t, const int32_t*, const T*, const T*, T*, T*); \
  template int launch_restrict_product<T>(hipStream_t, const Ell<T>&, const int32_t*, const T*, const T*, T*); \
  template int launch_prolong<T>(hipStream_t, int64_t, const int32_t*, const T*, T*);                         \
  template int launch_spmv_add<T>(hipStream_t, const Ell<T>&, const T*, T*);                                 \
  template int launch_axpy<T>(hipStream_t, int64_t, double, const T*, T*, Wt, Prol<T>);                                \
  template int launch_copy<T>(hipStream_t, int64_t, const T*, T*);                                           \
  template int launch_fill<T>(hipStream_t, int64_t, T, T*);


INST(double)
INST(float)
template int launch_cast<double, float>(hipStream_t, int64_t, const double*, float*);
template int launch_cast<float, double>(hipStream_t, int64_t, const float*, double*);
template int launch_cast<double, double>(hipStream_t, int64_t, const double*, double*);

}  // namespace amgp
