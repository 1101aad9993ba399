// Compatible weighted-matching aggregation (Section 4, "Compatible Matching"): aggregates
// of up to 2^steps vertices from repeated approximate maximum-weight matchings of the graph
// of A, and the tentative prolongator they define.  Setup only.
//
// * Edge weight for the smooth vector w: w_ij = 1 - 2 a_ij w_i w_j / (a_ii w_i^2 + a_jj w_j^2),
//   with a_ij read from the row of the smaller index, evaluated with explicitly rounded
//   operations (no contraction) and rounded to a 2^-30 grid; the resulting integer keys are
//   compared exactly.
// * Matching: rounds of locally dominant edges.  Every free vertex points at its best free
//   neighbour under the strict order (key, SplitMix64 hash of the edge, -min, -max); mutual
//   pointers are matched.  Each round matches at least the best remaining free-free edge,
//   and the result is the greedy matching in decreasing edge order (independent of timing).
//   The hash breaks the ties of constant-coefficient stencils at random, so few rounds suffice.
// * A pair forms an aggregate, an unmatched vertex a singleton; aggregates are numbered by
//   their smallest vertex; the column of aggregate J holds w_i / nu_J, nu_J = ||w|_J||.
#include <climits>

#include "graph.h"

namespace amgp {

namespace {

using graph::DevBuf;
using graph::edge_hash;
using graph::find_entry;

__global__ void k_diag(int64_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                       const double* __restrict__ val, double* __restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = 0.0;
  find_entry(ptr, col, val, (int)i, (int)i, &v);
  d[i] = v;
}

constexpr long long kNoEdge = LLONG_MIN;

__global__ void k_edge_keys(int64_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                            const double* __restrict__ val, const double* __restrict__ d,
                            const double* __restrict__ w, long long* __restrict__ key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
    const int j = col[p];
    long long k = kNoEdge;
    if (j != (int)i) {
      const int lo = min((int)i, j), hi = max((int)i, j);
      double a = val[p];
      bool ok = true;
      if (lo != (int)i) ok = find_entry(ptr, col, val, lo, hi, &a);
      if (ok) {
        const double num = __dmul_rn(__dmul_rn(2.0, a), __dmul_rn(w[lo], w[hi]));
        const double den = __dadd_rn(__dmul_rn(__dmul_rn(d[lo], w[lo]), w[lo]), __dmul_rn(__dmul_rn(d[hi], w[hi]), w[hi]));
        const double wij = __dsub_rn(1.0, __ddiv_rn(num, den));
        k = (long long)rint(__dmul_rn(wij, 1073741824.0));
      }
    }
    key[p] = k;
  }
}

// true when edge (key a, lo a, hi a) precedes edge b in the matching order
__device__ __forceinline__ bool better(long long ka, int loa, int hia, long long kb, int lob, int hib) {
  if (ka != kb) return ka > kb;
  const unsigned long long ha = edge_hash(loa, hia), hb = edge_hash(lob, hib);
  if (ha != hb) return ha > hb;
  if (loa != lob) return loa < lob;
  return hia < hib;
}

__global__ void k_match_pick(int64_t n, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                             const long long* __restrict__ key, const int32_t* __restrict__ mate,
                             int32_t* __restrict__ cand) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int best = -1;
  long long bk = 0;
  int blo = 0, bhi = 0;
  if (mate[i] < 0) {
    for (int p = ptr[i]; p < ptr[i + 1]; ++p) {
      const int j = col[p];
      const long long k = key[p];
      if (k == kNoEdge || mate[j] >= 0) continue;
      const int lo = min((int)i, j), hi = max((int)i, j);
      if (best < 0 || better(k, lo, hi, bk, blo, bhi)) {
        best = j;
        bk = k;
        blo = lo;
        bhi = hi;
      }
    }
  }
  cand[i] = best;
}

__global__ void k_match_commit(int64_t n, const int32_t* __restrict__ cand, int32_t* __restrict__ mate,
                               int* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (mate[i] >= 0) return;
  const int c = cand[i];
  if (c >= 0 && cand[c] == (int)i) {
    mate[i] = c;
    atomicAdd(count, 1);
  }
}

__global__ void k_match_leaders(int64_t n, const int32_t* __restrict__ mate, int32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = (mate[i] < 0 || (int)i < mate[i]) ? 1 : 0;
}

// Tentative prolongator rows (one entry each) and the coarse smooth vector.
__global__ void k_match_prol(int64_t n, const int32_t* __restrict__ mate, const int32_t* __restrict__ rank,
                             const double* __restrict__ w, int32_t* __restrict__ pptr, int32_t* __restrict__ pcol,
                             double* __restrict__ pval, double* __restrict__ wc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  pptr[i] = (int32_t)i;
  if (i == n) return;
  const int m = mate[i];
  const int lo = m < 0 ? (int)i : min((int)i, m), hi = m < 0 ? (int)i : max((int)i, m);
  const double nu = m < 0 ? fabs(w[i]) : __dsqrt_rn(__dadd_rn(__dmul_rn(w[lo], w[lo]), __dmul_rn(w[hi], w[hi])));
  const int J = rank[lo];
  pcol[i] = J;
  pval[i] = __ddiv_rn(w[i], nu);
  if ((int)i == lo) wc[J] = nu;
}

__global__ void k_ones(int64_t n, double* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = 1.0;
}

struct Hold {
  Csr c;
  ~Hold() { free_csr(c); }
};


// One matching step on A (CSR, ascending columns, structurally symmetric) with smooth vector w.
int matching_step(hipStream_t s, const Csr& A, const double* w, Csr* P, double** wc, int* flag) {
  (void)flag;
  const int64_t n = A.m;
  DevBuf<double> d;
  DevBuf<long long> key;
  DevBuf<int32_t> mate, cand, flagv, rank;
  DevBuf<int> count;
  AMGP_TRY(d.alloc(n));
  AMGP_TRY(key.alloc(A.nnz));
  AMGP_TRY(mate.alloc(n));
  AMGP_TRY(cand.alloc(n));
  AMGP_TRY(flagv.alloc(n));
  AMGP_TRY(rank.alloc(n + 1));
  AMGP_TRY(count.alloc(1));
  hipLaunchKernelGGL(k_diag, dim3(grid_for(n)), dim3(kBlock), 0, s, n, A.ptr, A.col, A.val, d.p);
  hipLaunchKernelGGL(k_edge_keys, dim3(grid_for(n)), dim3(kBlock), 0, s, n, A.ptr, A.col, A.val, d.p, w, key.p);
  AMGP_HIP(hipMemsetAsync(mate.p, 0xff, sizeof(int32_t) * n, s));  // -1
  // at most n/2 + 1 rounds can match something; the hashed order needs far fewer
  const int64_t max_rounds = n / 2 + 2;
  for (int64_t round = 0;; ++round) {
    if (round > max_rounds) return AMG_ECAPACITY;
    AMGP_HIP(hipMemsetAsync(count.p, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_match_pick, dim3(grid_for(n)), dim3(kBlock), 0, s, n, A.ptr, A.col, key.p, mate.p, cand.p);
    hipLaunchKernelGGL(k_match_commit, dim3(grid_for(n)), dim3(kBlock), 0, s, n, cand.p, mate.p, count.p);
    AMGP_HIP(hipGetLastError());
    int hc = 0;
    AMGP_HIP(hipMemcpyAsync(&hc, count.p, sizeof(int), hipMemcpyDeviceToHost, s));
    AMGP_HIP(hipStreamSynchronize(s));
    if (hc == 0) break;
  }
  hipLaunchKernelGGL(k_match_leaders, dim3(grid_for(n)), dim3(kBlock), 0, s, n, mate.p, flagv.p);
  int rc = AMG_OK;
  const int64_t nc = scan_ptr(s, n, flagv.p, rank.p, &rc);
  if (rc != AMG_OK) return rc;
  Csr o;
  o.m = n;
  o.ncols = nc;
  o.nnz = n;
  double* wcn = nullptr;
  if (hipMalloc(&o.ptr, sizeof(int32_t) * (n + 1)) != hipSuccess || hipMalloc(&o.col, sizeof(int32_t) * n) !=
      hipSuccess || hipMalloc(&o.val, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&wcn, sizeof(double) * std::max<int64_t>(nc, 1)) != hipSuccess) {
    free_csr(o);
    hipFree(wcn);
    return AMG_ENOMEM;
  }
  hipLaunchKernelGGL(k_match_prol, dim3(grid_for(n + 1)), dim3(kBlock), 0, s, n, mate.p, rank.p, w, o.ptr, o.col,
                     o.val, wcn);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    free_csr(o);
    hipFree(wcn);
    return AMG_EHIP;
  }
  *P = o;
  *wc = wcn;
  return AMG_OK;
}

}  // namespace

int matching_prolongator(hipStream_t s, const Csr& A, const double* w0, int steps, Csr* Phat, double** wnext,
                         int* flag) {
  const int64_t n = A.m;
  double* w = nullptr;
  if (hipMalloc(&w, sizeof(double) * n) != hipSuccess) return AMG_ENOMEM;
  if (w0)
    AMGP_HIP(hipMemcpyAsync(w, w0, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  else
    hipLaunchKernelGGL(k_ones, dim3(grid_for(n)), dim3(kBlock), 0, s, n, w);
  Hold P, Acur;  // composite prolongator, current step's operator (owned from step 2 on)
  const Csr* Aview = &A;
  int rc = AMG_OK;
  for (int st = 0; st < steps && rc == AMG_OK; ++st) {
    Hold Ps, PsT, Ac;
    double* wc = nullptr;
    rc = matching_step(s, *Aview, w, &Ps.c, &wc, flag);
    if (rc != AMG_OK) break;
    hipFree(w);
    w = wc;
    if (P.c.ptr == nullptr) {
      P.c = Ps.c;
      Ps.c = Csr();
    } else {
      Hold C;
      rc = spgemm(s, P.c, Ps.c, &C.c, flag);
      if (rc != AMG_OK) break;
      std::swap(P.c, C.c);
    }
    if (st + 1 == steps) break;
    // operator of the next step
    const Csr& Pst = Ps.c.ptr ? Ps.c : P.c;  // the step's own prolongator (first step: already moved)
    rc = transpose(s, Pst, &PsT.c);
    if (rc == AMG_OK) rc = galerkin_general(s, *Aview, Pst, PsT.c, &Ac.c, flag);
    if (rc != AMG_OK) break;
    std::swap(Acur.c, Ac.c);
    Aview = &Acur.c;
    if (Acur.c.m <= 1) break;
  }
  if (rc != AMG_OK) {
    hipFree(w);
    return rc;
  }
  *Phat = P.c;
  P.c = Csr();
  *wnext = w;
  return AMG_OK;
}

}  // namespace amgp
