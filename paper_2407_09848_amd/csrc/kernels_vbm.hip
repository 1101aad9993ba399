// Classical smoothed-aggregation aggregates of Vanek, Mandel and Brezina (Section 4, "VBM"),
// determined on all rows of the level (one device holds every row, so the decoupled and the
// coupled variants coincide).  Setup only.
//
// * Strength: the coupling of the edge {i, j}, i != j, is q_ij = rint(2^30 a_ij^2 / |a_ii a_jj|)
//   (explicitly rounded operations, a_ij read from the row of the smaller index, so both ends
//   see one value; the 2^-30 grid makes couplings that are equal in exact arithmetic compare
//   equal whatever the rounding of the Galerkin products).  The edge is strong when a_ij != 0
//   and q_ij >= rint(2^30 theta^2).  N_i is i with its strong neighbours.
// * Phase 1: roots are the greedy maximal independent set of the square of the strength graph
//   in decreasing SplitMix64 order of the vertex index, found by rounds: an undecided vertex
//   whose hash is the largest among the undecided vertices within two strong edges becomes a
//   root, then the undecided vertices within two edges of a root drop out.  Each round fixes at
//   least the undecided vertex of largest hash, and the result is the greedy one whatever the
//   timing.  The aggregate of a root r is N_r (disjoint for distinct roots).
// * Phase 2: a vertex outside every N_r joins the phase-1 aggregate of its strong neighbour j
//   with the largest q_ij (ties: the smallest j); a vertex with none (unreachable when phase 1
//   is maximal) forms a singleton.
// * Aggregates are numbered in increasing order of their root.
#include <cmath>

#include "graph.h"

namespace amgp {

namespace {

using graph::DevBuf;
using graph::find_entry;
using graph::splitmix64;

__global__ void k_vbm_diag(int64_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                           const double* __restrict__ val, double* __restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = 0.0;
  find_entry(ptr, col, val, (int)i, (int)i, &v);
  d[i] = v;
}

// mag[p] = q_ij for a strong stored entry p, else -1 (not an edge); qt = rint(2^30 theta^2)
__global__ void k_vbm_strength(int64_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                               const double* __restrict__ val, const double* __restrict__ d, double qt,
                               double* __restrict__ mag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
    const int j = col[p];
    double m = -1.0;
    if (j != (int)i) {
      const int lo = min((int)i, j), hi = max((int)i, j);
      double a = val[p];
      bool ok = true;
      if (lo != (int)i) ok = find_entry(ptr, col, val, lo, hi, &a);
      if (ok && a != 0.0) {
        const double q = rint(__dmul_rn(__ddiv_rn(__dmul_rn(a, a), fabs(__dmul_rn(d[lo], d[hi]))), 1073741824.0));
        if (q >= qt) m = q;
      }
    }
    mag[p] = m;
  }
}

enum : int8_t { kUndecided = 0, kRoot = 1, kOut = 2 };

// the one of vertices a, b (either may be -1) with the larger hash
__device__ __forceinline__ int first_of(int a, int b) {
  if (a < 0) return b;
  if (b < 0) return a;
  return splitmix64((unsigned)a) > splitmix64((unsigned)b) ? a : b;
}

// m1[j]: the undecided vertex of largest hash in the closed strong neighbourhood of j, or -1
__global__ void k_vbm_m1(int64_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                         const double* __restrict__ mag, const int8_t* __restrict__ st, int32_t* __restrict__ m1) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int best = st[j] == kUndecided ? (int)j : -1;
  for (int p = ptr[j]; p < ptr[j + 1]; ++p) {
    const int u = col[p];
    if (mag[p] >= 0.0 && st[u] == kUndecided) best = first_of(best, u);
  }
  m1[j] = best;
}

// an undecided vertex that is first among the undecided within two strong edges becomes a root
__global__ void k_vbm_join(int64_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                           const double* __restrict__ mag, const int32_t* __restrict__ m1, int8_t* __restrict__ st) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || st[i] != kUndecided) return;
  int best = m1[i];
  for (int p = ptr[i]; p < ptr[i + 1]; ++p)
    if (mag[p] >= 0.0) best = first_of(best, m1[col[p]]);
  if (best == (int)i) st[i] = kRoot;
}

// near[j] = 1 when the closed strong neighbourhood of j holds a root
__global__ void k_vbm_near(int64_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                           const double* __restrict__ mag, const int8_t* __restrict__ st, int8_t* __restrict__ near) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int8_t f = st[j] == kRoot;
  for (int p = ptr[j]; p < ptr[j + 1] && !f; ++p)
    if (mag[p] >= 0.0 && st[col[p]] == kRoot) f = 1;
  near[j] = f;
}

// undecided vertices within two strong edges of a root drop out; count the rest
__global__ void k_vbm_out(int64_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                          const double* __restrict__ mag, const int8_t* __restrict__ near, int8_t* __restrict__ st,
                          int* __restrict__ left) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || st[i] != kUndecided) return;
  bool f = near[i];
  for (int p = ptr[i]; p < ptr[i + 1] && !f; ++p)
    if (mag[p] >= 0.0 && near[col[p]]) f = true;
  if (f)
    st[i] = kOut;
  else
    atomicAdd(left, 1);
}

// phase 1: owner[i] = the root whose neighbourhood holds i, or -1
__global__ void k_vbm_owner(int64_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                            const double* __restrict__ mag, const int8_t* __restrict__ st,
                            int32_t* __restrict__ owner) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int o = st[i] == kRoot ? (int)i : -1;
  for (int p = ptr[i]; p < ptr[i + 1] && o < 0; ++p)
    if (mag[p] >= 0.0 && st[col[p]] == kRoot) o = col[p];
  owner[i] = o;
}

// phase 2 (and the singleton remainder): root[i] of the final aggregate; lead[i] = 1 for the
// vertices that name an aggregate
__global__ void k_vbm_attach(int64_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                             const double* __restrict__ mag, const int32_t* __restrict__ owner,
                             int32_t* __restrict__ root, int32_t* __restrict__ lead) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int r = owner[i];
  if (r < 0) {
    int bj = -1;
    double bm = 0.0;
    for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
      const int j = col[p];
      const double m = mag[p];
      if (m < 0.0 || owner[j] < 0) continue;
      if (bj < 0 || m > bm || (m == bm && j < bj)) {
        bj = j;
        bm = m;
      }
    }
    r = bj >= 0 ? owner[bj] : (int)i;
  }
  root[i] = r;
  lead[i] = r == (int)i;
}

__global__ void k_vbm_number(int64_t n, const int32_t* __restrict__ root, const int32_t* __restrict__ rank,
                             int32_t* __restrict__ agg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) agg[i] = rank[root[i]];
}

}  // namespace

int vbm_aggregates(hipStream_t s, const Csr& A, double theta, int32_t* agg, int64_t* nc) {
  const int64_t n = A.m;
  DevBuf<double> d, mag;
  DevBuf<int8_t> st, near;
  DevBuf<int32_t> m1, owner, root, lead, rank;
  DevBuf<int> left;
  AMGP_TRY(d.alloc(n));
  AMGP_TRY(mag.alloc(A.nnz));
  AMGP_TRY(st.alloc(n));
  AMGP_TRY(near.alloc(n));
  AMGP_TRY(m1.alloc(n));
  AMGP_TRY(owner.alloc(n));
  AMGP_TRY(root.alloc(n));
  AMGP_TRY(lead.alloc(n));
  AMGP_TRY(rank.alloc(n + 1));
  AMGP_TRY(left.alloc(1));
  const dim3 g(grid_for(n)), b(kBlock);
  hipLaunchKernelGGL(k_vbm_diag, g, b, 0, s, n, A.ptr, A.col, A.val, d.p);
  const double qt = std::rint(theta * theta * 1073741824.0);
  hipLaunchKernelGGL(k_vbm_strength, g, b, 0, s, n, A.ptr, A.col, A.val, d.p, qt, mag.p);
  AMGP_HIP(hipMemsetAsync(st.p, kUndecided, n, s));
  // every round fixes at least the undecided vertex of largest hash
  for (int64_t round = 0;; ++round) {
    if (round > n) return AMG_ECAPACITY;
    AMGP_HIP(hipMemsetAsync(left.p, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_vbm_m1, g, b, 0, s, n, A.ptr, A.col, mag.p, st.p, m1.p);
    hipLaunchKernelGGL(k_vbm_join, g, b, 0, s, n, A.ptr, A.col, mag.p, m1.p, st.p);
    hipLaunchKernelGGL(k_vbm_near, g, b, 0, s, n, A.ptr, A.col, mag.p, st.p, near.p);
    hipLaunchKernelGGL(k_vbm_out, g, b, 0, s, n, A.ptr, A.col, mag.p, near.p, st.p, left.p);
    AMGP_HIP(hipGetLastError());
    int hl = 0;
    AMGP_HIP(hipMemcpyAsync(&hl, left.p, sizeof(int), hipMemcpyDeviceToHost, s));
    AMGP_HIP(hipStreamSynchronize(s));
    if (hl == 0) break;
  }
  hipLaunchKernelGGL(k_vbm_owner, g, b, 0, s, n, A.ptr, A.col, mag.p, st.p, owner.p);
  hipLaunchKernelGGL(k_vbm_attach, g, b, 0, s, n, A.ptr, A.col, mag.p, owner.p, root.p, lead.p);
  AMGP_HIP(hipGetLastError());
  int rc = AMG_OK;
  const int64_t count = scan_ptr(s, n, lead.p, rank.p, &rc);
  if (rc != AMG_OK) return rc;
  hipLaunchKernelGGL(k_vbm_number, g, b, 0, s, n, root.p, rank.p, agg);
  AMGP_HIP(hipGetLastError());
  AMGP_HIP(hipStreamSynchronize(s));
  *nc = count;
  return AMG_OK;
}

}  // namespace amgp
