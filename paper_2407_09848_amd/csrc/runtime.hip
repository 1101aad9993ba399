// Host runtime and C ABI: hierarchy setup, smoother dispatch, V-cycle and PCG.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "coeffs.inc"
#include "internal.h"

static_assert(AMGP_KMAX == AMG_MAX_DEGREE, "coefficient table and public degree limit disagree");

namespace amgp {

namespace {

template <typename T>
struct Prec;
template <>
struct Prec<double> {
  static const Ell<double>& A(const Level& l) { return l.A64; }
  static const Ell<double>& P(const Level& l) { return l.P64; }
  static const Ell<double>& PT(const Level& l) { return l.PT64; }
  static const Ell<double>& R(const Level& l) { return l.R64; }
  static Vecs<double>& v(Level& l) { return l.v64; }
};
template <>
struct Prec<float> {
  static const Ell<float>& A(const Level& l) { return l.A32; }
  static const Ell<float>& P(const Level& l) { return l.P32; }
  static const Ell<float>& PT(const Level& l) { return l.PT32; }
  static const Ell<float>& R(const Level& l) { return l.R32; }
  static Vecs<float>& v(Level& l) { return l.v32; }
};

template <typename T>
int dalloc(T** p, int64_t count) {
  if (count < 1) count = 1;
  if (hipMalloc((void**)p, sizeof(T) * (size_t)count) != hipSuccess) {
    *p = nullptr;
    return AMG_ENOMEM;
  }
  return AMG_OK;
}

template <typename T>
void free_vecs(Vecs<T>& v, bool own_bx) {
  if (own_bx) {
    hipFree(v.b);
    hipFree(v.x);
  }
  hipFree(v.r);
  hipFree(v.g0);
  hipFree(v.g1);
  hipFree(v.minv);
  v = Vecs<T>();
}

template <typename T>
void free_adj(std::vector<AdjVecs<T>>& adj);

void drop_graphs(Handle* h) {
  if (h->graphs.empty()) return;
  hipDeviceSynchronize();  // no cached graph may still be executing when it is destroyed
  for (auto& g : h->graphs) hipGraphExecDestroy(g.exec);
  h->graphs.clear();
}

// Free everything the handle owns (the Handle object itself stays).
void release(Handle* h) {
  drop_graphs(h);
  if (h->cap) hipStreamDestroy(h->cap);
  for (size_t l = 0; l < h->lv.size(); ++l) {
    Level& L = h->lv[l];
    if (!L.csr_borrowed) {
      hipFree(L.csr_ptr);
      hipFree(L.csr_col);
      hipFree(L.csr_val);
    }
    free_ell(L.A64);
    free_ell(L.A32);
    free_vecs(L.v64, l > 0);
    free_vecs(L.v32, true);
    hipFree(L.agg);
    hipFree(L.children);
    hipFree(L.wsmooth);
    free_ell(L.P64);
    free_ell(L.PT64);
    free_ell(L.P32);
    free_ell(L.PT32);
    free_ell(L.R64);
    free_ell(L.R32);
  }
  hipFree(h->ainv);
  hipFree(h->cpart);
  hipFree(h->partial);
  hipFree(h->scal);
  hipFree(h->dflag);
  if (h->hscal) hipHostFree(h->hscal);
  if (h->hpub) hipHostFree(h->hpub);
  if (h->ev) hipEventDestroy(h->ev);
  hipFree(h->cg_r);
  hipFree(h->cg_z);
  hipFree(h->cg_p);
  hipFree(h->cg_p2);
  hipFree(h->cg_q);
  hipFree(h->cg_rold);
  hipFree(h->cg_u);
  free_adj(h->adj64);
  free_adj(h->adj32);
  hipFree(h->tr_buf);
  hipFree(h->tr_sq);
  hipFree(h->tr_loss);
  hipFree(h->tr_partial);
  *h = Handle();
}

int read_flags(Handle* h, hipStream_t s, int* out) {
  AMGP_HIP(hipMemcpyAsync(out, h->dflag, sizeof(int) * F_NFLAG, hipMemcpyDeviceToHost, s));
  AMGP_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

// ---------------------------------------------------------------------------
// Smoother application on level l in precision T (Sections 2.1-2.2, Algorithm 1).
// ---------------------------------------------------------------------------
// Weight descriptor of step j on level l: the per-problem device table when a
// differentiable V-cycle is running, else none (the launch scalar is used).
inline Wt step_weight(const Handle* h, int l, int kind, int k, int j) {
  Wt w;
  if (kind == AMG_OPTCHEB4 && h->dbeta) {
    w.v = h->dbeta + (size_t)l * k + (j - 1);
    w.rpp = (int)(h->lv[l].n / h->nbatch);
    w.stride = h->nlevels * k;
  }
  return w;
}

// The CG's dot products of a preconditioner result with r (and, flexible, r_old), taken by the
// preconditioner's last kernel when that kernel is a recurrence step (done is then set).
struct DotOut {
  const double* r = nullptr;
  const double* rold = nullptr;
  double* partial = nullptr;
  unsigned nb = 0;
  bool done = false;
};

// r0_copy (optional, x_in != 0 only): receives r^(0) = b - A x_in, the input of the recurrence.
// pr (optional, x_in != 0, Chebyshev kinds, one row per lane): the smoother runs on
// x_in + P x_c, the box prolongation being applied inside its first two kernels.
// u (optional, x = 0): M^{-1} b, written by the kernel that produced b, for the merged first
// two steps.  dot (optional): the dot products of the result, see DotOut.
template <typename T>
int smooth(Handle* h, int l, int kind, int k, const T* b, T* x, bool xz, hipStream_t s, T* r0_copy = nullptr,
           Prol<T> pr = Prol<T>(), const T* u = nullptr, DotOut* dot = nullptr) {
  Level& L = h->lv[l];
  const Ell<T>& A = Prec<T>::A(L);
  Vecs<T>& v = Prec<T>::v(L);
  const T* minv = v.minv;
  const int64_t n = L.n;
  if (kind == AMG_L1JAC) {
    if (xz) {
      // sweep sw writes bufs[(k - sw) % 2], so the last one lands in x
      T* bufs[2] = {x, v.g0};
      AMGP_TRY(launch_jacobi_zero<T>(s, n, minv, b, bufs[(k - 1) % 2]));
      for (int sw = 2; sw <= k; ++sw)
        AMGP_TRY(launch_jacobi<T>(s, A, minv, b, bufs[(k - sw + 1) % 2], bufs[(k - sw) % 2]));
    } else {
      T* cur = x;
      T* oth = v.g0;
      for (int sw = 1; sw <= k; ++sw) {
        AMGP_TRY(launch_jacobi<T>(s, A, minv, b, cur, oth));
        T* t = cur;
        cur = oth;
        oth = t;
      }
      if (cur != x) AMGP_TRY(launch_copy<T>(s, n, cur, x));
    }
    return AMG_OK;
  }
  T* g[2] = {v.g0, v.g1};
  int cur = 0;
  double pending = 0.0;
  if (kind == AMG_CHEB4 || kind == AMG_OPTCHEB4) {
    auto w = [&](int j) { return kind == AMG_OPTCHEB4 ? h->beta_at(l, k, j - 1) : 1.0; };
    const double c1 = (8.0 * 1 - 4.0) / (2.0 * 1 + 1.0);
    const T* rsrc;
    int j0 = 2;
    Wt wpend;
    if (xz && k >= 2) {
      // steps 1 and 2 in one pass
      const double alpha2 = (2.0 * 2 - 3.0) / (2.0 * 2 + 1.0), c2 = (8.0 * 2 - 4.0) / (2.0 * 2 + 1.0);
      AMGP_TRY(launch_first2_zero<T>(s, 0, k > 2, A, minv, b, g[1 - cur], v.r, x, c1, alpha2, c2, w(1), w(2),
                                     step_weight(h, l, kind, k, 1), step_weight(h, l, kind, k, 2), u));
      rsrc = v.r;
      cur = 1 - cur;
      j0 = 3;
    } else if (xz) {
      AMGP_TRY(launch_first_zero<T>(s, 0, k > 1, n, minv, b, g[cur], nullptr, x, c1, w(1),
                                    step_weight(h, l, kind, k, 1)));
      rsrc = b;
    } else {
      AMGP_TRY(launch_first_res<T>(s, 0, A, minv, b, x, v.r, g[cur], c1, pr));
      if (r0_copy) AMGP_TRY(launch_copy<T>(s, n, v.r, r0_copy));
      rsrc = v.r;
      pending = w(1);
      wpend = step_weight(h, l, kind, k, 1);
      if (k == 1) return launch_axpy<T>(s, n, pending, g[cur], x, wpend, pr);
    }
    for (int j = j0; j <= k; ++j) {
      const double alpha = (2.0 * j - 3.0) / (2.0 * j + 1.0);
      const double c = (8.0 * j - 4.0) / (2.0 * j + 1.0);
      // x is brought up to date on every other step (and on the last): a step that finds no
      // update pending leaves x alone and hands its own to the next step (16 bytes per row less)
      const bool defer = j < k && pending == 0.0 && !wpend.v && !pr.agg;
      if (dot && j == k && A.group == 1) {
        AMGP_TRY(launch_fused_dot<T>(s, 0, A, minv, g[cur], rsrc, x, alpha, c, w(j), pending,
                                     step_weight(h, l, kind, k, j), wpend, pr, dot->r, dot->rold, dot->partial,
                                     &dot->nb));
        dot->done = true;
        return AMG_OK;
      }
      AMGP_TRY(launch_fused<T>(s, 0, j < k, A, minv, g[cur], g[1 - cur], rsrc, v.r, defer ? nullptr : x, alpha, c,
                               w(j), pending, step_weight(h, l, kind, k, j), wpend, pr));
      rsrc = v.r;
      pending = defer ? w(j) : 0.0;
      wpend = defer ? step_weight(h, l, kind, k, j) : Wt();
      pr = Prol<T>();
      cur = 1 - cur;
    }
    return AMG_OK;
  }
  // AMG_OPTCHEB1: interval [a*_k, 1]
  const double a = kAStar[k];
  const double theta = (1.0 + a) / 2.0, delta = (1.0 - a) / 2.0;
  const double sigma1 = theta / delta;
  double rho_prev = 1.0 / sigma1;
  int j0 = 1;
  if (xz && k >= 2) {
    // steps 0 and 1 of Algorithm 1 in one pass
    const double rho = 1.0 / (2.0 * sigma1 - rho_prev);
    AMGP_TRY(launch_first2_zero<T>(s, 1, k > 2, A, minv, b, g[1 - cur], v.r, x, theta, rho * rho_prev,
                                   2.0 * rho / delta, 1.0, 1.0, Wt(), Wt(), u));
    rho_prev = rho;
    cur = 1 - cur;
    j0 = 2;
  } else if (xz) {
    AMGP_TRY(launch_first_zero<T>(s, 1, k > 1, n, minv, b, g[cur], v.r, x, theta, 1.0));
  } else {
    AMGP_TRY(launch_first_res<T>(s, 1, A, minv, b, x, v.r, g[cur], theta, pr));
    pending = 1.0;
    if (k == 1) return launch_axpy<T>(s, n, pending, g[cur], x, Wt(), pr);
  }
  for (int j = j0; j <= k - 1; ++j) {
    const double rho = 1.0 / (2.0 * sigma1 - rho_prev);
    const bool defer = j < k - 1 && pending == 0.0 && !pr.agg;  // as in the 4th kinds
    if (dot && j == k - 1 && A.group == 1) {
      AMGP_TRY(launch_fused_dot<T>(s, 1, A, minv, g[cur], v.r, x, rho * rho_prev, 2.0 * rho / delta, 1.0, pending,
                                   Wt(), Wt(), pr, dot->r, dot->rold, dot->partial, &dot->nb));
      dot->done = true;
      return AMG_OK;
    }
    AMGP_TRY(launch_fused<T>(s, 1, j < k - 1, A, minv, g[cur], g[1 - cur], v.r, v.r, defer ? nullptr : x,
                             rho * rho_prev, 2.0 * rho / delta, 1.0, pending, Wt(), Wt(), pr));
    pending = defer ? 1.0 : 0.0;
    pr = Prol<T>();
    rho_prev = rho;
    cur = 1 - cur;
  }
  return AMG_OK;
}

template <typename T>
int coarse(Handle* h, const T* b, T* x, hipStream_t s) {
  if (h->coarse_sweeps > 0) return smooth<T>(h, h->nlevels - 1, AMG_L1JAC, h->coarse_sweeps, b, x, true, s);
  return launch_coarse_symv<T>(s, h->nbatch, h->ncl, h->ncp, h->ainv, b, x, h->cpart);
}

// Transfers between level l and l + 1 (Section 2): b_c = P^T (b - A x) (tmp receives
// b - A x), x += P x_c, and the plain products y_c = P^T y and y = P y_c used by the
// adjoint.  P is the 2x2x2 box indicator (children / aggregate gathers) or explicit.
template <typename T>
int restrict_res(Handle* h, int l, const T* b, const T* x, T* tmp, T* bc, hipStream_t s) {
  Level& L = h->lv[l];
  if (!L.general && Prec<T>::R(L).val) return launch_restrict_product<T>(s, Prec<T>::R(L), L.children, b, x, bc);
  if (!L.general) return launch_restrict<T>(s, Prec<T>::A(L), L.nc, L.children, b, x, tmp, bc);
  AMGP_TRY(launch_residual<T>(s, Prec<T>::A(L), b, x, tmp));
  return launch_spmv<T>(s, Prec<T>::PT(L), tmp, bc);
}

template <typename T>
int prolong_add(Handle* h, int l, const T* xc, T* x, hipStream_t s) {
  Level& L = h->lv[l];
  if (!L.general) return launch_prolong<T>(s, L.n, L.agg, xc, x);
  return launch_spmv_add<T>(s, Prec<T>::P(L), xc, x);
}

template <typename T>
int restrict_apply(Handle* h, int l, const T* y, T* yc, hipStream_t s) {
  Level& L = h->lv[l];
  if (!L.general) return launch_restrict_sum<T>(s, L.nc, L.children, y, yc);
  return launch_spmv<T>(s, Prec<T>::PT(L), y, yc);
}

template <typename T>
int prolong_set(Handle* h, int l, const T* yc, T* y, hipStream_t s) {
  Level& L = h->lv[l];
  if (!L.general) return launch_prolong_set<T>(s, L.n, L.agg, yc, y);
  return launch_spmv<T>(s, Prec<T>::P(L), yc, y);
}

constexpr int64_t kFusedTransferMaxRows = 1 << 20;

// V-cycle of eq. (amg) from level l: x = B_l b.  u (optional): M^{-1} b for the pre-smoothing;
// dot (optional): the CG's dot products of x, taken by the post-smoothing's last kernel.
template <typename T>
int vcycle(Handle* h, int l, int kind, int k, const T* b, T* x, hipStream_t s, const T* u = nullptr,
           DotOut* dot = nullptr) {
  if (l == h->nlevels - 1) return coarse<T>(h, b, x, s);
  Level& L = h->lv[l];
  Vecs<T>& vc = Prec<T>::v(h->lv[l + 1]);
  AMGP_TRY(smooth<T>(h, l, kind, k, b, x, true, s, nullptr, Prol<T>(), u));
  AMGP_TRY(restrict_res<T>(h, l, b, x, Prec<T>::v(L).r, vc.b, s));
  AMGP_TRY(vcycle<T>(h, l + 1, kind, k, vc.b, vc.x, s));
  // small box levels with one row per lane: the prolongation rides on the post-smoothing's
  // kernels, saving a launch (measured at 128^3: 9.7 vs 7.3 + 4.6 us on 262144 rows, 6.2 vs
  // 4.7 + 4.7 us on 32768).  On large levels the dependent aggregate / coarse-value gather of
  // every neighbour costs more than the pass it saves (43.4 vs 34.1 + 9.8 us on 2097152 rows,
  // 361 vs 284 + 59 us on 16777216), so they keep the separate prolongation.
  if (!L.general && kind != AMG_L1JAC && Prec<T>::A(L).group == 1 && L.n <= kFusedTransferMaxRows)
    return smooth<T>(h, l, kind, k, b, x, false, s, nullptr, Prol<T>{L.agg, vc.x}, nullptr, dot);
  AMGP_TRY(prolong_add<T>(h, l, vc.x, x, s));
  return smooth<T>(h, l, kind, k, b, x, false, s, nullptr, Prol<T>(), nullptr, dot);
}

// keep32 (FP32 hierarchy): leave the result in the level-0 float vector v32.x instead of
// converting it into z (the CG kernels read it there).
int vcycle_top(Handle* h, int kind, int k, const double* r, double* z, hipStream_t s, bool keep32 = false,
               const double* u = nullptr, DotOut* dot = nullptr) {
  if (h->precision == AMG_FP32) {
    Vecs<float>& v = h->lv[0].v32;
    // on large 27-point levels the conversion of r also writes u = M^{-1} b for the merged first
    // two steps (the handle's FP64 u vector is free with an FP32 hierarchy)
    float* u32 = kind != AMG_L1JAC && k >= 2 && h->nlevels > 1 && first2_takes_u(h->lv[0].A32)
                     ? reinterpret_cast<float*>(h->cg_u)
                     : nullptr;
    if (u32)
      AMGP_TRY(launch_cast_u(s, h->lv[0].n, r, v.minv, v.b, u32));
    else
      AMGP_TRY((launch_cast<double, float>(s, h->lv[0].n, r, v.b)));
    AMGP_TRY(vcycle<float>(h, 0, kind, k, v.b, v.x, s, u32, dot));
    if (keep32) return AMG_OK;
    return launch_cast<float, double>(s, h->lv[0].n, v.x, z);
  }
  return vcycle<double>(h, 0, kind, k, r, z, s, u, dot);
}

// The V-cycle as one HIP graph: captured on the handle's own stream the first
// time a (kind, degree, r, z) combination is seen, then replayed on the
// caller's stream.  The coarse levels are launch-latency bound; a graph
// removes the per-launch host overhead.  The kernel arguments (including the
// beta weights) are baked in, so changing beta drops the cached graphs.
// Runs body(stream) as a HIP graph cached under `key`: captured on the handle's own
// stream the first time, replayed on the caller's stream afterwards.
template <typename F>
int run_graph(Handle* h, const GraphEntry& key, hipStream_t s, F&& body) {
  if (!h->use_graphs) return body(s);
  for (auto& g : h->graphs)
    if (g.kind == key.kind && g.k == key.k && g.mode == key.mode && g.poly == key.poly && g.r == key.r &&
        g.z == key.z && g.aux == key.aux) {
      AMGP_HIP(hipGraphLaunch(g.exec, s));
      return AMG_OK;
    }
  if (h->graphs.size() >= 32) drop_graphs(h);
  if (!h->cap) AMGP_HIP(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  AMGP_HIP(hipStreamBeginCapture(h->cap, hipStreamCaptureModeRelaxed));
  const int rc = body(h->cap);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(h->cap, &graph);
  if (rc != AMG_OK || e != hipSuccess) {
    if (graph) hipGraphDestroy(graph);
    return rc != AMG_OK ? rc : AMG_EHIP;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (ei != hipSuccess) return AMG_EHIP;
  GraphEntry g = key;
  g.exec = exec;
  h->graphs.push_back(g);
  AMGP_HIP(hipGraphLaunch(exec, s));
  return AMG_OK;
}

int vcycle_run(Handle* h, int kind, int k, const double* r, double* z, hipStream_t s) {
  const GraphEntry key{kind, k, -1, false, r, z, nullptr, nullptr};
  return run_graph(h, key, s, [&](hipStream_t cs) { return vcycle_top(h, kind, k, r, z, cs); });
}

// ---------------------------------------------------------------------------
// Differentiable V-cycle (optimal 4th kind, per-problem per-level weights).
//
// Forward: the V-cycle of eq. (amg), saving for every level the input of each
// smoother recurrence: the level right-hand side b_l (pre-smoothing from 0)
// and r^(0) = b_l - A_l x_mid (post-smoothing).
//
// Backward: every smoother correction Q = sum_j beta_j h_j(M^{-1}A) M^{-1}
// is symmetric (M diagonal, A symmetric), so the smoother is its own
// adjoint: for x_out = x_in + Q (b - A x_in),
//   b_bar += Q x_out_bar,  x_in_bar = x_out_bar - A Q x_out_bar,
//   d/d beta_j = < z_j(x_out_bar), r^(0) >
// where z_j(v) is the j-th direction of the recurrence run from zero on v.
// The transfers are adjoint to each other (P and P^T) and the coarsest solve
// is symmetric.  A = A^T, so the backward pass reuses the forward SpMV.
// ---------------------------------------------------------------------------
template <typename T>
struct TrainPrec;
template <>
struct TrainPrec<double> {
  static AdjVecs<double>& a(Handle* h, int l) { return h->adj64[l]; }
};
template <>
struct TrainPrec<float> {
  static AdjVecs<float>& a(Handle* h, int l) { return h->adj32[l]; }
};

template <typename T>
int alloc_adj(Handle* h, std::vector<AdjVecs<T>>& adj) {
  adj.resize(h->nlevels);
  for (int l = 0; l < h->nlevels; ++l) {
    const int64_t n = h->lv[l].n;
    AMGP_TRY(dalloc(&adj[l].u, n));
    AMGP_TRY(dalloc(&adj[l].xmid, n));
    AMGP_TRY(dalloc(&adj[l].xpre, n));
    AMGP_TRY(dalloc(&adj[l].res, n));
    AMGP_TRY(dalloc(&adj[l].xin, n));
    AMGP_TRY(dalloc(&adj[l].bout, n));
  }
  return AMG_OK;
}

template <typename T>
void free_adj(std::vector<AdjVecs<T>>& adj) {
  for (auto& a : adj) {
    hipFree(a.u);
    hipFree(a.xmid);
    hipFree(a.xpre);
    hipFree(a.res);
    hipFree(a.xin);
    hipFree(a.bout);
  }
  adj.clear();
}

void train_release(Handle* h) {
  free_adj(h->adj64);
  free_adj(h->adj32);
  hipFree(h->tr_buf);
  hipFree(h->tr_sq);
  hipFree(h->tr_loss);
  hipFree(h->tr_partial);
  h->tr_buf = nullptr;
  h->tr_sq = nullptr;
  h->tr_loss = nullptr;
  h->tr_partial = nullptr;
}

int train_prepare(Handle* h) {
  if (h->train_ready) return AMG_OK;
  h->ck_off.assign(h->nlevels, 0);
  int64_t off = 0;
  for (int l = 0; l < h->nlevels - 1; ++l) {
    h->ck_off[l] = off;
    off += 2 * h->lv[l].n;
  }
  h->ck_count = off;
  const size_t w = h->precision == AMG_FP32 ? sizeof(float) : sizeof(double);
  const int64_t n0 = h->lv[0].n;
  int rc = h->precision == AMG_FP32 ? alloc_adj<float>(h, h->adj32) : alloc_adj<double>(h, h->adj64);
  // driver: r0, z, r1, r2, g, t (6 x n0) + two checkpoints
  if (rc == AMG_OK &&
      hipMalloc(&h->tr_buf, w * (size_t)(6 * n0 + 2 * std::max<int64_t>(h->ck_count, 1))) != hipSuccess) {
    h->tr_buf = nullptr;
    rc = AMG_ENOMEM;
  }
  if (rc == AMG_OK) rc = dalloc(&h->tr_sq, 2 * h->nbatch);
  if (rc == AMG_OK) rc = dalloc(&h->tr_loss, 1 + h->nbatch);
  if (rc == AMG_OK) rc = dalloc(&h->tr_partial, 64 * (int64_t)std::max(2 * h->nbatch, 8));
  if (rc != AMG_OK) {  // nothing half-allocated is kept: a later call starts over
    train_release(h);
    return rc;
  }
  h->train_ready = true;
  return AMG_OK;
}

template <typename T>
int vcycle_fwd_ck(Handle* h, int l, int k, const T* b, T* x, T* ck, hipStream_t s) {
  if (l == h->nlevels - 1) return coarse<T>(h, b, x, s);
  Level& L = h->lv[l];
  Vecs<T>& vc = Prec<T>::v(h->lv[l + 1]);
  T* ck_pre = ck + h->ck_off[l];
  T* ck_post = ck_pre + L.n;
  AMGP_TRY(launch_copy<T>(s, L.n, b, ck_pre));
  AMGP_TRY(smooth<T>(h, l, AMG_OPTCHEB4, k, b, x, true, s));
  AMGP_TRY(restrict_res<T>(h, l, b, x, Prec<T>::v(L).r, vc.b, s));
  AMGP_TRY(vcycle_fwd_ck<T>(h, l + 1, k, vc.b, vc.x, ck, s));
  AMGP_TRY(prolong_add<T>(h, l, vc.x, x, s));
  return smooth<T>(h, l, AMG_OPTCHEB4, k, b, x, false, s, ck_post);
}

// u = Q v (smoother from zero on v, every direction z_j kept) and
// gbeta[p][l][j-1] += < z_j, r0 >_p for every problem p.
template <typename T>
int smooth_adjoint(Handle* h, int l, int k, const T* v, T* u, const T* r0, double* gbeta, hipStream_t s) {
  Level& L = h->lv[l];
  const Ell<T>& A = Prec<T>::A(L);
  Vecs<T>& vv = Prec<T>::v(L);
  const int64_t n = L.n, rpp = n / h->nbatch;
  const int stride = h->nlevels * k;
  T* g[2] = {vv.g0, vv.g1};
  int cur = 0;
  // gbeta[.][l][j-1] += <z_j, r0>: each dot's per-problem sums are done by the next dot's first
  // block (the same sums in the same order), its partials alternating between the two halves
  // of the partial buffer; the last ones by a kernel of their own
  const bool chain = h->nbatch <= kBlock;
  SegFin pending;
  int half = 0;
  auto seg_dot = [&](const T* z, double* out) -> int {
    if (!chain) return launch_seg_dot<T>(s, h->nbatch, rpp, z, r0, h->tr_partial, out, stride, true);
    double* part = h->tr_partial + (size_t)half * kSegBlocks * h->nbatch;
    AMGP_TRY(launch_seg_dot_chain<T>(s, h->nbatch, rpp, z, r0, part, pending));
    pending.partial = part;
    pending.out = out;
    pending.nseg = h->nbatch;
    pending.ostride = stride;
    pending.acc = 1;
    half = 1 - half;
    return AMG_OK;
  };
  const double c1 = (8.0 * 1 - 4.0) / (2.0 * 1 + 1.0);
  AMGP_TRY(launch_first_zero<T>(s, 0, true, n, vv.minv, v, g[cur], nullptr, u, c1, h->beta_at(l, k, 0),
                                step_weight(h, l, AMG_OPTCHEB4, k, 1)));
  AMGP_TRY(seg_dot(g[cur], gbeta + (size_t)l * k));
  const T* rsrc = v;
  for (int j = 2; j <= k; ++j) {
    const double alpha = (2.0 * j - 3.0) / (2.0 * j + 1.0);
    const double c = (8.0 * j - 4.0) / (2.0 * j + 1.0);
    AMGP_TRY(launch_fused<T>(s, 0, true, A, vv.minv, g[cur], g[1 - cur], rsrc, vv.r, u, alpha, c,
                             h->beta_at(l, k, j - 1), 0.0, step_weight(h, l, AMG_OPTCHEB4, k, j), Wt()));
    rsrc = vv.r;
    cur = 1 - cur;
    AMGP_TRY(seg_dot(g[cur], gbeta + (size_t)l * k + (j - 1)));
  }
  return launch_seg_finish(s, pending);
}

template <typename T>
int vcycle_bwd_rec(Handle* h, int l, int k, const T* xo_bar, T* b_bar, const T* ck, double* gbeta, hipStream_t s) {
  if (l == h->nlevels - 1) return coarse<T>(h, xo_bar, b_bar, s);
  Level& L = h->lv[l];
  const Ell<T>& A = Prec<T>::A(L);
  AdjVecs<T>& a = TrainPrec<T>::a(h, l);
  AdjVecs<T>& ac = TrainPrec<T>::a(h, l + 1);
  const T* ck_pre = ck + h->ck_off[l];
  const T* ck_post = ck_pre + L.n;
  // post-smoothing: x_out = x_mid + Q (b - A x_mid)
  AMGP_TRY(smooth_adjoint<T>(h, l, k, xo_bar, a.u, ck_post, gbeta, s));
  AMGP_TRY(launch_residual<T>(s, A, xo_bar, a.u, a.xmid));  // x_mid_bar = x_out_bar - A u
  // x_mid = x_pre + P x_c
  AMGP_TRY(restrict_apply<T>(h, l, a.xmid, ac.xin, s));
  AMGP_TRY(vcycle_bwd_rec<T>(h, l + 1, k, ac.xin, ac.bout, ck, gbeta, s));
  // b_c = P^T (b - A x_pre)
  AMGP_TRY(prolong_set<T>(h, l, ac.bout, a.res, s));
  AMGP_TRY(launch_residual<T>(s, A, a.xmid, a.res, a.xpre));  // x_pre_bar = x_mid_bar - A res_bar
  // pre-smoothing from zero: x_pre = Q b
  AMGP_TRY(smooth_adjoint<T>(h, l, k, a.xpre, b_bar, ck_pre, gbeta, s));
  AMGP_TRY(launch_axpy<T>(s, L.n, 1.0, a.u, b_bar));
  return launch_axpy<T>(s, L.n, 1.0, a.res, b_bar);
}

template <typename T>
int train_loss_grad(Handle* h, int k, const double* b, double* hloss, double* gbeta, hipStream_t s) {
  const int64_t n = h->lv[0].n, rpp = n / h->nbatch;
  const int P = h->nbatch;
  const Ell<T>& A = Prec<T>::A(h->lv[0]);
  T* base = static_cast<T*>(h->tr_buf);
  T *r0 = base, *z = base + n, *r1 = base + 2 * n, *r2 = base + 3 * n, *g = base + 4 * n, *t = base + 5 * n;
  T* ckA = base + 6 * n;
  T* ckB = ckA + h->ck_count;
  AMGP_TRY((launch_cast<double, T>(s, n, b, r0)));
  AMGP_TRY(vcycle_fwd_ck<T>(h, 0, k, r0, z, ckA, s));
  AMGP_TRY(launch_residual<T>(s, A, r0, z, r1));
  AMGP_TRY(vcycle_fwd_ck<T>(h, 0, k, r1, z, ckB, s));
  AMGP_TRY(launch_residual<T>(s, A, r1, z, r2));
  AMGP_TRY(launch_seg_dot<T>(s, P, rpp, r0, nullptr, h->tr_partial, h->tr_sq, 1, false));
  AMGP_TRY(launch_seg_dot<T>(s, P, rpp, r2, nullptr, h->tr_partial, h->tr_sq + P, 1, false));
  AMGP_TRY(launch_loss_value(s, P, h->tr_sq, h->tr_loss));
  AMGP_TRY(launch_loss_seed<T>(s, n, rpp, P, h->tr_sq, r2, g));  // g = dL/dr2
  AMGP_TRY(launch_fill<double>(s, (int64_t)P * h->nlevels * k, 0.0, gbeta));
  // r2 = r1 - A z2
  AMGP_TRY(launch_spmv<T>(s, A, g, t));
  AMGP_TRY(launch_neg<T>(s, n, t, z));  // z2_bar
  AMGP_TRY(vcycle_bwd_rec<T>(h, 0, k, z, t, ckB, gbeta, s));  // t = r1_bar through z2
  AMGP_TRY(launch_axpy<T>(s, n, 1.0, g, t));                 // r1_bar = r2_bar + ...
  // r1 = r0 - A z1
  AMGP_TRY(launch_spmv<T>(s, A, t, g));
  AMGP_TRY(launch_neg<T>(s, n, g, z));  // z1_bar
  AMGP_TRY(vcycle_bwd_rec<T>(h, 0, k, z, t, ckA, gbeta, s));
  AMGP_HIP(hipMemcpyAsync(hloss, h->tr_loss, sizeof(double) * (1 + P), hipMemcpyDeviceToHost, s));
  AMGP_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

int check_kind_degree(int kind, int degree) {
  if (kind < AMG_L1JAC || kind > AMG_OPTCHEB1) return AMG_EINVAL;
  if (degree < 1 || degree > AMG_MAX_DEGREE) return AMG_EINVAL;
  return AMG_OK;
}

template <typename T>
int alloc_vecs(Vecs<T>& v, int64_t n, bool bx) {
  if (bx) {
    AMGP_TRY(dalloc(&v.b, n));
    AMGP_TRY(dalloc(&v.x, n));
  }
  AMGP_TRY(dalloc(&v.r, n));
  AMGP_TRY(dalloc(&v.g0, n));
  AMGP_TRY(dalloc(&v.g1, n));
  return AMG_OK;
}

__global__ void k_round_vec(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// Transfer operators and Galerkin product of level L with an explicit prolongator:
// P = P_hat or (I - omega D^{-1} A) P_hat, P^T, A_c = P^T (A P), and the sliced-ELL copies of P, P^T.
struct CsrHold {
  Csr c;
  ~CsrHold() { free_csr(c); }
};

Csr level_csr(const Level& L) {
  Csr A;
  A.m = L.n;
  A.ncols = L.n;
  A.nnz = L.nnz;
  A.ptr = L.csr_ptr;
  A.col = L.csr_col;
  A.val = L.csr_val;
  return A;
}

// Phat: the tentative prolongator (taken over); box aggregates when null (from L.agg)
int general_level(Handle* h, hipStream_t s, Level& L, Level* C, Csr* Phat) {
  const Csr A = level_csr(L);
  CsrHold Ph, P, PT, Ac;
  if (Phat) {
    Ph.c = *Phat;
    *Phat = Csr();
  } else {
    AMGP_TRY(tentative_prolongator(s, L.n, L.nc, L.agg, &Ph.c));
  }
  if (h->smoothed) {
    AMGP_TRY(smoothed_prolongator(s, A, h->nbatch, Ph.c, &P.c, h->dflag));
  } else {
    P.c = Ph.c;
    Ph.c = Csr();
  }
  AMGP_TRY(transpose(s, P.c, &PT.c));
  AMGP_TRY(galerkin_general(s, A, P.c, PT.c, &Ac.c, h->dflag));
  AMGP_TRY(build_ell64(s, P.c.m, P.c.ptr, P.c.col, P.c.val, &L.P64, P.c.ncols, 0));
  AMGP_TRY(build_ell64(s, PT.c.m, PT.c.ptr, PT.c.col, PT.c.val, &L.PT64, PT.c.ncols, 0));
  C->csr_ptr = Ac.c.ptr;
  C->csr_col = Ac.c.col;
  C->csr_val = Ac.c.val;
  C->nnz = Ac.c.nnz;
  Ac.c = Csr();  // now owned by the level
  return AMG_OK;
}

// R = P^T A for the 2x2x2 box P of level L (the restriction of k_restrict_product), in slices
// aligned on each aggregate's first row, whatever their padding (small ragged levels pad more
// than 10%, but one pass over R still costs less than the residual's pass over A).  Left empty
// (the residual and the sum over children are used instead) when a slice has more than 64
// offsets.
int restriction_product(Handle* h, hipStream_t s, Level& L) {
  CsrHold Ph, PhT, R;
  AMGP_TRY(tentative_prolongator(s, L.n, L.nc, L.agg, &Ph.c));
  AMGP_TRY(transpose(s, Ph.c, &PhT.c));
  AMGP_TRY(spgemm(s, PhT.c, level_csr(L), &R.c, h->dflag));
  const int rc =
      build_ell_aligned(s, L.nc, R.c.ptr, R.c.col, R.c.val, &L.R64, L.children, kMaxChildren, L.n, true);
  return rc == AMG_EINVAL ? AMG_OK : rc;
}

int setup(Handle* h, int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, const double* val,
          const amg_opts* o, hipStream_t s) {
  h->nbatch = o->nbatch > 0 ? o->nbatch : 1;
  h->max_coarse = o->max_coarse > 0 ? o->max_coarse : 4096;
  h->precision = o->precision;
  h->agg_edge = o->agg_edge > 0 ? o->agg_edge : 2;
  h->smoothed = o->smoothed != 0;
  h->coarse_sweeps = o->coarse_sweeps;
  h->aggregation = o->aggregation;
  h->match_steps = o->match_steps > 0 ? o->match_steps : 3;
  h->vbm_theta = o->vbm_theta;
  {
    const char* e = std::getenv("AMGP_NO_GRAPH");
    h->use_graphs = !(e && e[0] == '1');
  }
  AMGP_TRY(dalloc(&h->dflag, F_NFLAG));
  AMGP_HIP(hipMemsetAsync(h->dflag, 0, sizeof(int) * F_NFLAG, s));
  // level 0: a library-owned copy of the CSR matrix, or with drop_fine_csr the caller's arrays,
  // read (never written) until setup returns
  h->lv.emplace_back();
  {
    Level& L = h->lv.back();
    L.n = n;
    L.nnz = nnz;
    L.nx = o->nx;
    L.ny = o->ny;
    L.nz = o->nz;
    if (o->drop_fine_csr) {
      L.csr_ptr = const_cast<int32_t*>(row_ptr);
      L.csr_col = const_cast<int32_t*>(col);
      L.csr_val = const_cast<double*>(val);
      L.csr_borrowed = true;
    } else {
      AMGP_TRY(dalloc(&L.csr_ptr, n + 1));
      AMGP_TRY(dalloc(&L.csr_col, nnz));
      AMGP_TRY(dalloc(&L.csr_val, nnz));
      AMGP_HIP(hipMemcpyAsync(L.csr_ptr, row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
      AMGP_HIP(hipMemcpyAsync(L.csr_col, col, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, s));
      AMGP_HIP(hipMemcpyAsync(L.csr_val, val, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s));
    }
    AMGP_TRY(validate_csr(s, n, nnz, L.csr_ptr, L.csr_col, h->dflag));
  }
  for (;;) {
    Level& L = h->lv.back();
    AMGP_TRY(dalloc(&L.v64.minv, L.n));
    AMGP_TRY(launch_l1_diag(s, L.n, L.csr_ptr, L.csr_col, L.csr_val, L.v64.minv, h->dflag));
    int fl[F_NFLAG];
    AMGP_TRY(read_flags(h, s, fl));
    if (fl[F_NOTSPD]) return AMG_ENOTSPD;
    // the fine level keeps one row per lane (the CG kernels read it); coarse levels choose
    AMGP_TRY(build_ell64(s, L.n, L.csr_ptr, L.csr_col, L.csr_val, &L.A64, -1, h->lv.size() == 1 ? 1 : 0));
    const int64_t per = L.n / h->nbatch;
    if (per <= h->max_coarse) break;
    if (h->aggregation == AMG_AGG_MATCHING) {
      // compatible weighted matching: aggregates of up to 2^match_steps rows (Section 4)
      CsrHold Ph;
      double* wnext = nullptr;
      AMGP_TRY(matching_prolongator(s, level_csr(L), L.wsmooth, h->match_steps, &Ph.c, &wnext, h->dflag));
      const int64_t nc = Ph.c.ncols;
      if (nc >= L.n) {
        hipFree(wnext);
        break;
      }
      // the composite tentative prolongator has one entry per row: its column is the row's aggregate
      if (Ph.c.nnz == L.n) {
        AMGP_TRY(dalloc(&L.agg, L.n));
        AMGP_HIP(hipMemcpyAsync(L.agg, Ph.c.col, sizeof(int32_t) * L.n, hipMemcpyDeviceToDevice, s));
      }
      L.nc = nc;
      L.general = true;
      Level C;
      C.n = nc;
      C.nx = (int)nc;
      C.wsmooth = wnext;
      const int rc = general_level(h, s, L, &C, &Ph.c);
      h->lv.push_back(C);  // owned by the handle from here on, also on error
      if (rc != AMG_OK) return rc;
      continue;
    }
    if (h->aggregation == AMG_AGG_VBM) {
      // classical smoothed aggregation; the threshold is halved on each coarser level (Section 4)
      const double th = std::ldexp(h->vbm_theta, -(int)(h->lv.size() - 1));
      int64_t nc = 0;
      AMGP_TRY(dalloc(&L.agg, L.n));
      AMGP_TRY(vbm_aggregates(s, level_csr(L), th, L.agg, &nc));
      if (nc >= L.n) break;
      L.nc = nc;
      L.general = true;
      Level C;
      C.n = nc;
      C.nx = (int)nc;
      const int rc = general_level(h, s, L, &C, nullptr);
      h->lv.push_back(C);  // owned by the handle from here on, also on error
      if (rc != AMG_OK) return rc;
      continue;
    }
    int cx, cy, cz;
    const int e = h->agg_edge;
    auto cdim = [e](int v) { return v == 1 ? 1 : (v + e - 1) / e; };
    const int64_t nc = (int64_t)cdim(L.nx) * cdim(L.ny) * cdim(L.nz) * h->nbatch;
    if (nc >= L.n) break;
    L.nc = nc;
    L.general = h->smoothed || e != 2;
    AMGP_TRY(dalloc(&L.agg, L.n));
    if (!L.general) AMGP_TRY(dalloc(&L.children, nc * kMaxChildren));
    AMGP_TRY(launch_aggregates(s, L.nx, L.ny, L.nz, h->nbatch, e, L.agg, L.children, &cx, &cy, &cz));
    Level C;
    C.n = nc;
    C.nx = cx;
    C.ny = cy;
    C.nz = cz;
    if (!L.general) {
      int rc = galerkin(s, L.n, L.csr_ptr, L.csr_col, L.csr_val, L.agg, nc, L.children, &C.csr_ptr, &C.csr_col,
                        &C.csr_val, &C.nnz, h->dflag);
      // entries of the product that are exactly zero are not stored, as in a general sparse
      // product: couplings carried only by zero stencil entries (the Q1 face entries between
      // aggregates one cell wide in two directions)
      Csr cc;
      cc.m = nc;
      cc.ncols = nc;
      cc.nnz = C.nnz;
      cc.ptr = C.csr_ptr;
      cc.col = C.csr_col;
      cc.val = C.csr_val;
      if (rc == AMG_OK) rc = drop_small(s, &cc, 0.0);
      C.csr_ptr = cc.ptr;
      C.csr_col = cc.col;
      C.csr_val = cc.val;
      C.nnz = cc.nnz;
      if (rc == AMG_OK) rc = restriction_product(h, s, L);
      if (rc != AMG_OK) {
        h->lv.push_back(C);  // owned by the handle from here on, also on error
        return rc;
      }
    } else {
      AMGP_TRY(general_level(h, s, L, &C, nullptr));
    }
    h->lv.push_back(C);
  }
  h->nlevels = (int)h->lv.size();
  // coarsest level: dense inverse through the Cholesky factor (unless it is smoothed instead)
  if (h->coarse_sweeps <= 0) {
    Level& L = h->lv.back();
    h->ncl = L.n / h->nbatch;
    h->ncp = (h->ncl + kDenseTile - 1) / kDenseTile * kDenseTile;
    AMGP_TRY(dalloc(&h->cpart, (int64_t)h->nbatch * (h->ncp / kDenseTile) * (h->ncp / kDenseTile) * kDenseTile));
    double* dense = nullptr;
    AMGP_TRY(dalloc(&dense, (int64_t)h->nbatch * h->ncp * h->ncp));
    int rc = launch_to_dense(s, h->nbatch, h->ncl, h->ncp, L.csr_ptr, L.csr_col, L.csr_val, dense, h->dflag);
    if (rc == AMG_OK) rc = dense_spd_inverse(s, h->nbatch, h->ncp, dense, h->dflag);
    if (rc == AMG_OK) rc = pack_lower_tiles(s, h->nbatch, h->ncp, dense, &h->ainv);
    if (rc == AMG_OK && hipStreamSynchronize(s) != hipSuccess) rc = AMG_EHIP;
    hipFree(dense);
    if (rc != AMG_OK) return rc;
    int fl[F_NFLAG];
    AMGP_TRY(read_flags(h, s, fl));
    if (fl[F_NOTSPD]) return AMG_ENOTSPD;
  }
  // work vectors and the float32 copies
  for (int l = 0; l < h->nlevels; ++l) {
    Level& L = h->lv[l];
    AMGP_TRY(alloc_vecs(L.v64, L.n, l > 0));
    if (h->precision == AMG_FP32) {
      AMGP_TRY(build_ell32(s, L.A64, &L.A32));
      if (L.R64.val) AMGP_TRY(build_ell32(s, L.R64, &L.R32));
      if (L.general) {
        AMGP_TRY(build_ell32(s, L.P64, &L.P32));
        AMGP_TRY(build_ell32(s, L.PT64, &L.PT32));
      }
      AMGP_TRY(alloc_vecs(L.v32, L.n, true));
      AMGP_TRY(dalloc(&L.v32.minv, L.n));
      hipLaunchKernelGGL(k_round_vec, dim3(grid_for(L.n)), dim3(kBlock), 0, s, L.n, L.v64.minv, L.v32.minv);
      AMGP_HIP(hipGetLastError());
    }
  }
  // CG and reduction workspace
  const int64_t n0 = h->lv[0].n;
  const int64_t maxblocks = ((n0 + kBlock - 1) / kBlock + 7) / 8 * 8 + 8;
  AMGP_TRY(dalloc(&h->partial, 2 * maxblocks + 2 * 64));  // + the middle-stage sums of long lists
  AMGP_TRY(dalloc(&h->scal, S_NSCAL));
  if (hipHostMalloc((void**)&h->hscal, sizeof(double) * (S_NSCAL + F_NFLAG)) != hipSuccess) return AMG_ENOMEM;
  if (hipHostMalloc((void**)&h->hpub, sizeof(double) * 4, hipHostMallocMapped | hipHostMallocCoherent) !=
      hipSuccess)
    return AMG_ENOMEM;
  AMGP_HIP(hipHostGetDevicePointer((void**)&h->dpub, h->hpub, 0));
  AMGP_HIP(hipEventCreateWithFlags(&h->ev, hipEventDisableTiming));
  AMGP_TRY(dalloc(&h->cg_r, n0));
  AMGP_TRY(dalloc(&h->cg_z, n0));
  AMGP_TRY(dalloc(&h->cg_p, n0));
  AMGP_TRY(dalloc(&h->cg_p2, n0));
  AMGP_TRY(dalloc(&h->cg_q, n0));
  AMGP_TRY(dalloc(&h->cg_rold, n0));
  AMGP_TRY(dalloc(&h->cg_u, n0));
  // default coefficients
  h->beta.assign((size_t)h->nlevels * (AMG_MAX_DEGREE + 1) * AMG_MAX_DEGREE, 0.0);
  for (int l = 0; l < h->nlevels; ++l)
    for (int k = 1; k <= AMG_MAX_DEGREE; ++k)
      for (int j = 0; j < k; ++j) h->beta_at(l, k, j) = kOptBeta[k][j];
  AMGP_HIP(hipStreamSynchronize(s));
  // Without export or features of level 0 no CSR form of it is needed once the hierarchy is
  // built (the kernels read the sliced-ELL form): forget the caller's arrays.
  if (h->lv[0].csr_borrowed) {
    Level& L0 = h->lv[0];
    L0.csr_ptr = nullptr;
    L0.csr_col = nullptr;
    L0.csr_val = nullptr;
    L0.csr_borrowed = false;
  }
  return AMG_OK;
}

template <typename TZ>
int sum_dot(Handle* h, hipStream_t s, int mode, const double* a, const TZ* b, const double* c, const TZ* d,
            int64_t n) {
  unsigned nb = 0;
  AMGP_TRY(launch_dot2<TZ>(s, n, a, b, c, d, h->partial, &nb));
  return launch_reduce(s, mode, nb, h->partial, h->scal, h->dflag);
}

// The preconditioned vector the CG kernels read: the FP32 hierarchy's own float output
// (exactly converted inside them), else the float64 z.
const float* cg_z32(const Handle* h, bool poly) {
  return h->precision == AMG_FP32 && !poly ? h->lv[0].v32.x : nullptr;
}

int fetch_scalars(Handle* h, hipStream_t s) {
  AMGP_HIP(hipMemcpyAsync(h->hscal, h->scal, sizeof(double) * S_NSCAL, hipMemcpyDeviceToHost, s));
  AMGP_HIP(hipMemcpyAsync(h->hscal + S_NSCAL, h->dflag, sizeof(int) * F_NFLAG, hipMemcpyDeviceToHost, s));
  AMGP_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

// z = B r followed by the reduction `mode` of (r, z) (and (r_old, z) for the flexible beta),
// captured together as one graph.  B is the V-cycle, or with poly the level-0 smoother
// alone from z = 0 (the polynomial preconditioning of the remark after Fig. boundcomparison).
int precond_dot(Handle* h, int kind, int k, bool poly, int mode, const double* r, double* z, const double* rold,
                hipStream_t s, const double* u = nullptr) {
  const int64_t n = h->lv[0].n;
  const GraphEntry key{kind, k, mode, poly, r, z, rold, nullptr};  // u is fixed by (h, kind, k, mode)
  const float* z32 = cg_z32(h, poly);
  DotOut d;
  d.r = r;
  d.rold = mode == RED_BETA_FLEX ? rold : nullptr;
  d.partial = h->partial;
  return run_graph(h, key, s, [&](hipStream_t cs) {
    AMGP_TRY(poly ? smooth<double>(h, 0, kind, k, r, z, true, cs, nullptr, Prol<double>(), u, &d)
                  : vcycle_top(h, kind, k, r, z, cs, z32 != nullptr, u, &d));
    if (d.done) return launch_reduce(cs, mode, d.nb, h->partial, h->scal, h->dflag);
    if (z32) return sum_dot<float>(h, cs, mode, r, z32, mode == RED_BETA_FLEX ? rold : nullptr,
                                   mode == RED_BETA_FLEX ? z32 : nullptr, n);
    if (mode == RED_BETA_FLEX) return sum_dot<double>(h, cs, mode, r, z, rold, z, n);
    return sum_dot<double>(h, cs, mode, r, z, nullptr, nullptr, n);
  });
}

// Preconditioned CG.  Each iteration's update publishes (r, r) and the error flags to mapped
// host memory; while the host waits for them, the next preconditioner application is
// already enqueued (it reads r and writes only the handle's workspace), so the GPU does not
// idle across the convergence test.  When the iteration is predicted to converge (from the
// last residual reduction rate) the next application is not started ahead.
int pcg(Handle* h, int kind, int k, const double* b, double* x, bool xz, double rtol, int maxit, bool flex,
        bool poly_only, int* iters, double* relres, double* hist, hipStream_t s) {
  const int64_t n = h->lv[0].n;
  const Ell<double>& A = h->lv[0].A64;
  double *r = h->cg_r, *z = h->cg_z, *p = h->cg_p, *q = h->cg_q, *rold = flex ? h->cg_rold : nullptr;
  const float* z32 = cg_z32(h, poly_only);
  const int* hflag = reinterpret_cast<const int*>(h->hscal + S_NSCAL);
  AMGP_HIP(hipMemsetAsync(h->dflag, 0, sizeof(int) * F_NFLAG, s));
  AMGP_TRY(launch_check_finite(s, n, b, h->dflag));
  AMGP_TRY(sum_dot<double>(h, s, RED_BB, b, b, nullptr, nullptr, n));
  AMGP_TRY(fetch_scalars(h, s));
  if (hflag[F_NAN]) return AMG_ENAN;
  const double bnorm = std::sqrt(h->hscal[S_BB]);
  *iters = 0;
  if (bnorm == 0.0) {
    AMGP_TRY(launch_fill<double>(s, n, 0.0, x));
    AMGP_HIP(hipStreamSynchronize(s));
    *relres = 0.0;
    if (hist) hist[0] = 0.0;
    return AMG_OK;
  }
  double rel0 = 1.0;
  if (xz) {
    AMGP_TRY(launch_fill<double>(s, n, 0.0, x));
    AMGP_TRY(launch_copy<double>(s, n, b, r));
  } else {
    AMGP_TRY(launch_residual<double>(s, A, b, x, r));
    AMGP_TRY(sum_dot<double>(h, s, RED_RR, r, r, nullptr, nullptr, n));
    AMGP_TRY(fetch_scalars(h, s));
    rel0 = std::sqrt(h->hscal[S_RR]) / bnorm;
  }
  if (hist) hist[0] = rel0;
  *relres = rel0;
  if (rel0 <= rtol) return AMG_OK;
  AMGP_TRY(precond_dot(h, kind, k, poly_only, RED_RZ0, r, z, nullptr, s));  // also beta = 0: p_1 = z_0
  double* pold = h->cg_p2;
  AMGP_TRY(launch_fill<double>(s, n, 0.0, pold));
  // on large 27-point FP64 levels the residual update also writes u = M^{-1} r, so that the
  // preconditioner's merged first two steps gather u alone instead of M^{-1} and r
  double* u = h->precision == AMG_FP64 && kind != AMG_L1JAC && k >= 2 && first2_takes_u(A) ? h->cg_u : nullptr;
  const double* minv0 = h->lv[0].v64.minv;
  const int next_mode = flex ? RED_BETA_FLEX : RED_BETA;
  double rel_prev = rel0, rate = 1.0;
  for (int it = 1; it <= maxit; ++it) {
    unsigned nb = 0;
    // x += alpha p of the previous iteration rides on the pass that forms the new direction
    double* xprev = it > 1 ? x : nullptr;
    if (z32)
      AMGP_TRY(launch_spmv_dot_p<float>(s, A, h->scal, z32, pold, p, q, h->partial, xprev, &nb));
    else
      AMGP_TRY(launch_spmv_dot_p<double>(s, A, h->scal, z, pold, p, q, h->partial, xprev, &nb));
    AMGP_TRY(launch_reduce(s, RED_ALPHA, nb, h->partial, h->scal, h->dflag));
    AMGP_TRY(launch_cg_update(s, n, h->scal, q, r, rold, h->partial, &nb, minv0, u));
    AMGP_TRY(launch_reduce(s, RED_RR, nb, h->partial, h->scal, h->dflag, h->dpub));
    AMGP_HIP(hipEventRecord(h->ev, s));
    const bool ahead = it < maxit && rel_prev * rate > 2.0 * rtol;
    if (ahead) AMGP_TRY(precond_dot(h, kind, k, poly_only, next_mode, r, z, rold, s, u));
    AMGP_HIP(hipEventSynchronize(h->ev));
    *iters = it;
    const double rr = h->hpub[0];
    const bool breakdown = h->hpub[1] != 0.0, nan = h->hpub[2] != 0.0;
    const double rel = std::sqrt(rr) / bnorm;
    *relres = rel;
    if (hist) hist[it] = rel;
    if (breakdown || nan || rel <= rtol || it == maxit) {
      AMGP_TRY(launch_cg_x(s, n, h->scal, p, x));  // this iteration's x += alpha p (alpha = 0 on breakdown)
      AMGP_HIP(hipStreamSynchronize(s));
      if (breakdown) return AMG_EBREAKDOWN;
      if (nan) return AMG_ENAN;
      return rel <= rtol ? AMG_OK : AMG_NOT_CONVERGED;
    }
    if (!ahead) AMGP_TRY(precond_dot(h, kind, k, poly_only, next_mode, r, z, rold, s, u));
    rate = rel / rel_prev;
    rel_prev = rel;
    std::swap(p, pold);  // the next iteration forms p = z + beta pold inside its SpMV
  }
  return AMG_NOT_CONVERGED;
}

}  // namespace

}  // namespace amgp

using amgp::Handle;

struct amg_handle {
  Handle impl;
};

extern "C" {

int amg_setup(int64_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col, const double* d_val,
              const amg_opts* h_opts, void* stream, amg_handle** out) {
  if (!out) return AMG_EINVAL;
  *out = nullptr;
  if (!d_row_ptr || !d_col || !d_val || !h_opts) return AMG_EINVAL;
  if (n < 1 || nnz < n || nnz >= (int64_t)INT32_MAX || n >= (int64_t)INT32_MAX) return AMG_EINVAL;
  const amg_opts& o = *h_opts;
  const int64_t nb = o.nbatch > 0 ? o.nbatch : 1;
  if (o.nx < 1 || o.ny < 1 || o.nz < 1 || o.max_coarse < 0) return AMG_EINVAL;
  if ((int64_t)o.nx * o.ny * o.nz * nb != n) return AMG_EINVAL;
  if (o.precision != AMG_FP64 && o.precision != AMG_FP32) return AMG_EINVAL;
  if (o.agg_edge < 0 || o.agg_edge == 1 || o.agg_edge > 4) return AMG_EINVAL;
  if (o.smoothed != 0 && o.smoothed != 1) return AMG_EINVAL;
  if (o.coarse_sweeps < 0 || o.coarse_sweeps > 1000) return AMG_EINVAL;
  if (o.aggregation != AMG_AGG_BOX && o.aggregation != AMG_AGG_MATCHING && o.aggregation != AMG_AGG_VBM)
    return AMG_EINVAL;
  if (o.aggregation != AMG_AGG_BOX && nb != 1) return AMG_EINVAL;
  if (!(o.vbm_theta >= 0.0) || !std::isfinite(o.vbm_theta)) return AMG_EINVAL;
  if (o.match_steps < 0 || o.match_steps > 3) return AMG_EINVAL;
  if (o.drop_fine_csr != 0 && o.drop_fine_csr != 1) return AMG_EINVAL;
  amg_handle* h = new (std::nothrow) amg_handle;
  if (!h) return AMG_ENOMEM;
  const int rc = amgp::setup(&h->impl, n, nnz, d_row_ptr, d_col, d_val, &o, (hipStream_t)stream);
  if (rc != AMG_OK) {
    hipStreamSynchronize((hipStream_t)stream);
    amgp::release(&h->impl);
    delete h;
    return rc;
  }
  *out = h;
  return AMG_OK;
}

int amg_destroy(amg_handle* h) {
  if (!h) return AMG_OK;
  hipDeviceSynchronize();
  amgp::release(&h->impl);
  delete h;
  return AMG_OK;
}

int amg_num_levels(const amg_handle* h, int* h_nlevels) {
  if (!h || !h_nlevels) return AMG_EINVAL;
  *h_nlevels = h->impl.nlevels;
  return AMG_OK;
}

int amg_level_info(const amg_handle* h, int level, int64_t* h_n, int64_t* h_nnz) {
  if (!h || level < 0 || level >= h->impl.nlevels) return AMG_EINVAL;
  if (h_n) *h_n = h->impl.lv[level].n;
  if (h_nnz) *h_nnz = h->impl.lv[level].nnz;
  return AMG_OK;
}

int amg_level_layout(const amg_handle* h, int level, int64_t* h_padded, int* h_lanes, int* h_aligned) {
  if (!h || level < 0 || level >= h->impl.nlevels) return AMG_EINVAL;
  const amgp::Ell<double>& A = h->impl.lv[level].A64;
  if (h_padded) *h_padded = A.padded;
  if (h_lanes) *h_lanes = A.group;
  if (h_aligned) *h_aligned = A.doff != nullptr;
  return AMG_OK;
}

int amg_level_transfer(const amg_handle* h, int level, int* h_form, int64_t* h_stored) {
  if (!h || level < 0 || level >= h->impl.nlevels - 1) return AMG_EINVAL;
  const amgp::Level& L = h->impl.lv[level];
  const int form = L.general ? AMG_TRANSFER_EXPLICIT : (L.R64.val ? AMG_TRANSFER_PRODUCT : AMG_TRANSFER_RESIDUAL);
  if (h_form) *h_form = form;
  if (h_stored) *h_stored = form == AMG_TRANSFER_EXPLICIT ? L.PT64.padded : (form == AMG_TRANSFER_PRODUCT ? L.R64.padded : 0);
  return AMG_OK;
}

int amg_level_export(const amg_handle* h, int level, int32_t* d_row_ptr, int32_t* d_col, double* d_val,
                     double* d_minv, void* stream) {
  if (!h || level < 0 || level >= h->impl.nlevels) return AMG_EINVAL;
  const amgp::Level& L = h->impl.lv[level];
  if (!L.csr_ptr && (d_row_ptr || d_col || d_val)) return AMG_EINVAL;  // dropped after setup
  hipStream_t s = (hipStream_t)stream;
  if (d_row_ptr) AMGP_HIP(hipMemcpyAsync(d_row_ptr, L.csr_ptr, sizeof(int32_t) * (L.n + 1), hipMemcpyDeviceToDevice, s));
  if (d_col) AMGP_HIP(hipMemcpyAsync(d_col, L.csr_col, sizeof(int32_t) * L.nnz, hipMemcpyDeviceToDevice, s));
  if (d_val) AMGP_HIP(hipMemcpyAsync(d_val, L.csr_val, sizeof(double) * L.nnz, hipMemcpyDeviceToDevice, s));
  if (d_minv) AMGP_HIP(hipMemcpyAsync(d_minv, L.v64.minv, sizeof(double) * L.n, hipMemcpyDeviceToDevice, s));
  return AMG_OK;
}

int amg_level_aggregates(const amg_handle* h, int level, int32_t* d_agg, void* stream) {
  if (!h || !d_agg || level < 0 || level >= h->impl.nlevels - 1) return AMG_EINVAL;
  const amgp::Level& L = h->impl.lv[level];
  if (!L.agg) return AMG_EINVAL;
  AMGP_HIP(hipMemcpyAsync(d_agg, L.agg, sizeof(int32_t) * L.n, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return AMG_OK;
}

int amg_default_beta(int degree, double* h_beta) {
  if (!h_beta || degree < 1 || degree > AMG_MAX_DEGREE) return AMG_EINVAL;
  for (int j = 0; j < degree; ++j) h_beta[j] = kOptBeta[degree][j];
  return AMG_OK;
}

int amg_default_astar(int degree, double* h_a) {
  if (!h_a || degree < 1 || degree > AMG_MAX_DEGREE) return AMG_EINVAL;
  *h_a = kAStar[degree];
  return AMG_OK;
}

int amg_set_beta(amg_handle* h, int degree, int level, const double* h_beta) {
  if (!h || !h_beta || degree < 1 || degree > AMG_MAX_DEGREE) return AMG_EINVAL;
  Handle& H = h->impl;
  if (level < -1 || level >= H.nlevels) return AMG_EINVAL;
  for (int j = 0; j < degree; ++j)
    if (!std::isfinite(h_beta[j])) return AMG_EINVAL;
  amgp::drop_graphs(&H);
  for (int l = 0; l < H.nlevels; ++l) {
    if (level != -1 && l != level) continue;
    for (int j = 0; j < degree; ++j) H.beta_at(l, degree, j) = h_beta[j];
  }
  return AMG_OK;
}

int amg_reset_beta(amg_handle* h) {
  if (!h) return AMG_EINVAL;
  Handle& H = h->impl;
  amgp::drop_graphs(&H);
  for (int l = 0; l < H.nlevels; ++l)
    for (int k = 1; k <= AMG_MAX_DEGREE; ++k)
      for (int j = 0; j < k; ++j) H.beta_at(l, k, j) = kOptBeta[k][j];
  return AMG_OK;
}

int amg_spmv(amg_handle* h, int level, const double* d_x, double* d_y, void* stream) {
  if (!h || !d_x || !d_y || level < 0 || level >= h->impl.nlevels) return AMG_EINVAL;
  return amgp::launch_spmv<double>((hipStream_t)stream, h->impl.lv[level].A64, d_x, d_y);
}

int smoother_apply(amg_handle* h, int level, int kind, int degree, const double* d_b, double* d_x, int x_is_zero,
                   void* stream) {
  if (!h || !d_b || !d_x || level < 0 || level >= h->impl.nlevels) return AMG_EINVAL;
  AMGP_TRY(amgp::check_kind_degree(kind, degree));
  return amgp::smooth<double>(&h->impl, level, kind, degree, d_b, d_x, x_is_zero != 0, (hipStream_t)stream);
}

int smoother_apply_f32(amg_handle* h, int level, int kind, int degree, const float* d_b, float* d_x, int x_is_zero,
                       void* stream) {
  if (!h || !d_b || !d_x || level < 0 || level >= h->impl.nlevels) return AMG_EINVAL;
  if (h->impl.precision != AMG_FP32) return AMG_EINVAL;
  AMGP_TRY(amgp::check_kind_degree(kind, degree));
  return amgp::smooth<float>(&h->impl, level, kind, degree, d_b, d_x, x_is_zero != 0, (hipStream_t)stream);
}

int amg_restrict_residual(amg_handle* h, int level, const double* d_b, const double* d_x, double* d_bc,
                          void* stream) {
  if (!h || !d_b || !d_x || !d_bc || level < 0 || level >= h->impl.nlevels - 1) return AMG_EINVAL;
  amgp::Level& L = h->impl.lv[level];
  return amgp::restrict_res<double>(&h->impl, level, d_b, d_x, L.v64.r, d_bc, (hipStream_t)stream);
}

int amg_prolong_add(amg_handle* h, int level, const double* d_xc, double* d_x, void* stream) {
  if (!h || !d_xc || !d_x || level < 0 || level >= h->impl.nlevels - 1) return AMG_EINVAL;
  return amgp::prolong_add<double>(&h->impl, level, d_xc, d_x, (hipStream_t)stream);
}

int amg_coarse_solve(amg_handle* h, const double* d_b, double* d_x, void* stream) {
  if (!h || !d_b || !d_x) return AMG_EINVAL;
  return amgp::coarse<double>(&h->impl, d_b, d_x, (hipStream_t)stream);
}

int vcycle_apply(amg_handle* h, int kind, int degree, const double* d_r, double* d_z, void* stream) {
  if (!h || !d_r || !d_z) return AMG_EINVAL;
  AMGP_TRY(amgp::check_kind_degree(kind, degree));
  return amgp::vcycle_run(&h->impl, kind, degree, d_r, d_z, (hipStream_t)stream);
}

int pcg_solve(amg_handle* h, int kind, int degree, const double* d_b, double* d_x, int x_is_zero, double rtol,
              int maxit, int flexible, int* h_iters, double* h_relres, double* h_hist, void* stream) {
  if (!h || !d_b || !d_x || !h_iters || !h_relres || maxit < 1 || !(rtol >= 0.0)) return AMG_EINVAL;
  AMGP_TRY(amgp::check_kind_degree(kind, degree));
  return amgp::pcg(&h->impl, kind, degree, d_b, d_x, x_is_zero != 0, rtol, maxit, flexible != 0, false, h_iters,
                   h_relres, h_hist, (hipStream_t)stream);
}

int pcg_solve_smoother(amg_handle* h, int kind, int degree, const double* d_b, double* d_x, int x_is_zero,
                       double rtol, int maxit, int flexible, int* h_iters, double* h_relres, double* h_hist,
                       void* stream) {
  if (!h || !d_b || !d_x || !h_iters || !h_relres || maxit < 1 || !(rtol >= 0.0)) return AMG_EINVAL;
  AMGP_TRY(amgp::check_kind_degree(kind, degree));
  return amgp::pcg(&h->impl, kind, degree, d_b, d_x, x_is_zero != 0, rtol, maxit, flexible != 0, true, h_iters,
                   h_relres, h_hist, (hipStream_t)stream);
}

int amg_ckpt_bytes(const amg_handle* h, int64_t* h_bytes) {
  if (!h || !h_bytes) return AMG_EINVAL;
  Handle* H = const_cast<Handle*>(&h->impl);
  AMGP_TRY(amgp::train_prepare(H));
  *h_bytes = H->ck_count * (int64_t)(H->precision == AMG_FP32 ? sizeof(float) : sizeof(double));
  return AMG_OK;
}

namespace {
struct DbetaScope {  // installs the per-problem weight table for the duration of one call
  Handle* h;
  DbetaScope(Handle* hh, const double* b, int k) : h(hh) {
    h->dbeta = b;
    h->dbeta_k = k;
  }
  ~DbetaScope() {
    h->dbeta = nullptr;
    h->dbeta_k = 0;
  }
};
}  // namespace

int vcycle_fwd_ckpt(amg_handle* h, int degree, const double* d_beta, const double* d_r, double* d_z, void* d_ckpt,
                    void* stream) {
  if (!h || !d_beta || !d_r || !d_z || !d_ckpt || degree < 1 || degree > AMG_MAX_DEGREE) return AMG_EINVAL;
  Handle* H = &h->impl;
  hipStream_t s = (hipStream_t)stream;
  AMGP_TRY(amgp::train_prepare(H));
  DbetaScope scope(H, d_beta, degree);
  if (H->precision == AMG_FP32) {
    amgp::Vecs<float>& v = H->lv[0].v32;
    AMGP_TRY((amgp::launch_cast<double, float>(s, H->lv[0].n, d_r, v.b)));
    AMGP_TRY(amgp::vcycle_fwd_ck<float>(H, 0, degree, v.b, v.x, static_cast<float*>(d_ckpt), s));
    return amgp::launch_cast<float, double>(s, H->lv[0].n, v.x, d_z);
  }
  return amgp::vcycle_fwd_ck<double>(H, 0, degree, d_r, d_z, static_cast<double*>(d_ckpt), s);
}

int vcycle_bwd(amg_handle* h, int degree, const double* d_beta, const void* d_ckpt, const double* d_gz,
               double* d_gr, double* d_gbeta, void* stream) {
  if (!h || !d_beta || !d_ckpt || !d_gz || !d_gr || !d_gbeta || degree < 1 || degree > AMG_MAX_DEGREE)
    return AMG_EINVAL;
  Handle* H = &h->impl;
  hipStream_t s = (hipStream_t)stream;
  AMGP_TRY(amgp::train_prepare(H));
  DbetaScope scope(H, d_beta, degree);
  if (H->precision == AMG_FP32) {
    amgp::AdjVecs<float>& a = H->adj32[0];
    AMGP_TRY((amgp::launch_cast<double, float>(s, H->lv[0].n, d_gz, a.xin)));
    AMGP_TRY(amgp::vcycle_bwd_rec<float>(H, 0, degree, a.xin, a.bout, static_cast<const float*>(d_ckpt), d_gbeta, s));
    return amgp::launch_cast<float, double>(s, H->lv[0].n, a.bout, d_gr);
  }
  return amgp::vcycle_bwd_rec<double>(H, 0, degree, d_gz, d_gr, static_cast<const double*>(d_ckpt), d_gbeta, s);
}

int amg_train_loss_grad(amg_handle* h, int degree, const double* d_beta, const double* d_b, double* h_loss,
                        double* d_gbeta, void* stream) {
  if (!h || !d_beta || !d_b || !h_loss || !d_gbeta || degree < 1 || degree > AMG_MAX_DEGREE) return AMG_EINVAL;
  Handle* H = &h->impl;
  if (H->nlevels < 2) return AMG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  AMGP_TRY(amgp::train_prepare(H));
  DbetaScope scope(H, d_beta, degree);
  if (H->precision == AMG_FP32) return amgp::train_loss_grad<float>(H, degree, d_b, h_loss, d_gbeta, s);
  return amgp::train_loss_grad<double>(H, degree, d_b, h_loss, d_gbeta, s);
}

int amg_level_features(amg_handle* h, int degree, const double* h_sigma, float* d_feat, void* stream) {
  if (!h || !h_sigma || !d_feat || degree < 1 || degree > AMG_MAX_DEGREE) return AMG_EINVAL;
  Handle* H = &h->impl;
  if (H->nlevels < 2) return AMG_EINVAL;
  for (int l = 0; l < H->nlevels - 1; ++l)
    if (!H->lv[l].csr_ptr) return AMG_EINVAL;  // the level-0 CSR copy was dropped after setup
  hipStream_t s = (hipStream_t)stream;
  const int P = H->nbatch, NL = H->nlevels - 1;
  std::vector<float> feat((size_t)P * NL * 8);
  double* buf = nullptr;
  double* red = nullptr;
  double* part = nullptr;
  const int64_t n0 = H->lv[0].n;
  if (hipMalloc(&buf, sizeof(double) * 3 * n0) != hipSuccess || hipMalloc(&red, sizeof(double) * 3 * P) != hipSuccess ||
      hipMalloc(&part, sizeof(double) * 64 * P) != hipSuccess) {
    hipFree(buf);
    hipFree(red);
    hipFree(part);
    return AMG_ENOMEM;
  }
  int rc = AMG_OK;
  std::vector<double> hr(3 * P);
  for (int l = 0; l < NL && rc == AMG_OK; ++l) {
    amgp::Level& L = H->lv[l];
    const int64_t n = L.n, rpp = n / P;
    double *v = buf, *w = buf + n, *t = buf + 2 * n;
    // 20 power iterations on M^{-1} A from the all-ones vector: lambda ~ ||v_20|| / ||v_19|| per problem
    rc = amgp::launch_fill<double>(s, n, 1.0, v);
    for (int it = 0; it < 20 && rc == AMG_OK; ++it) {
      rc = amgp::launch_spmv<double>(s, L.A64, v, t);
      if (rc == AMG_OK) rc = amgp::launch_mul(s, n, L.v64.minv, t, w);
      std::swap(v, w);
    }
    if (rc == AMG_OK) rc = amgp::launch_seg_dot<double>(s, P, rpp, v, nullptr, part, red, 1, false);
    if (rc == AMG_OK) rc = amgp::launch_seg_dot<double>(s, P, rpp, w, nullptr, part, red + P, 1, false);
    // mean off-diagonal l1 ratio: plain per-problem sum = dot with a vector of ones
    if (rc == AMG_OK) rc = amgp::launch_offdiag_ratio(s, n, L.csr_ptr, L.csr_col, L.csr_val, L.v64.minv, t);
    if (rc == AMG_OK) rc = amgp::launch_fill<double>(s, n, 1.0, w);
    if (rc == AMG_OK) rc = amgp::launch_seg_dot<double>(s, P, rpp, t, w, part, red + 2 * P, 1, false);
    if (rc != AMG_OK) break;
    if (hipMemcpyAsync(hr.data(), red, sizeof(double) * 3 * P, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = AMG_EHIP;
      break;
    }
    const double nnz_per_row = (double)L.nnz / (double)n;
    const double ratio_next = (double)H->lv[l + 1].n / (double)n;
    for (int p = 0; p < P; ++p) {
      const double lam = hr[P + p] > 0.0 ? std::sqrt(hr[p] / hr[P + p]) : 0.0;
      float* f = &feat[((size_t)p * NL + l) * 8];
      f[0] = (float)(degree / 6.0);
      f[1] = (float)((double)l / (double)(H->nlevels - 1));
      f[2] = (float)(1.0 - lam);
      f[3] = (float)(nnz_per_row / 27.0);
      f[4] = (float)(std::log2((double)rpp) / 24.0);
      f[5] = (float)h_sigma[p];
      f[6] = (float)ratio_next;
      f[7] = (float)(hr[2 * P + p] / (double)rpp);
    }
  }
  if (rc == AMG_OK && hipMemcpyAsync(d_feat, feat.data(), sizeof(float) * feat.size(), hipMemcpyHostToDevice, s) != hipSuccess)
    rc = AMG_EHIP;
  hipStreamSynchronize(s);
  hipFree(buf);
  hipFree(red);
  hipFree(part);
  return rc;
}

int mlp_num_params(void) { return amgp::mlp_num_params(); }

int mlp_fwd(const float* d_params, const float* d_x, int batch, float* d_y, float* d_cache, void* stream) {
  if (!d_params || !d_x || !d_y || !d_cache || batch < 1 || batch > 256) return AMG_EINVAL;
  return amgp::launch_mlp_fwd((hipStream_t)stream, batch, d_params, d_x, d_y, d_cache);
}

int mlp_bwd(const float* d_params, const float* d_x, int batch, const float* d_cache, const float* d_gy,
            float* d_gparams, float* d_work, void* stream) {
  if (!d_params || !d_x || !d_cache || !d_gy || !d_gparams || !d_work || batch < 1 || batch > 256) return AMG_EINVAL;
  return amgp::launch_mlp_bwd((hipStream_t)stream, batch, d_params, d_x, d_cache, d_gy, d_gparams, d_work);
}

int mlp_bwd_noalloc(const float* d_params, const float* d_x, int batch, const float* d_cache, const float* d_gy,
                    float* d_gparams, void* stream) {
  if (!d_params || !d_x || !d_cache || !d_gy || !d_gparams || batch < 1) return AMG_EINVAL;
  return amgp::launch_mlp_bwd_noalloc((hipStream_t)stream, batch, d_params, d_x, d_cache, d_gy, d_gparams);
}

int mlp_adam(float* d_params, const float* d_g, float* d_m, float* d_v, int n, int step, float lr, float b1, float b2,
             float eps, void* stream) {
  if (!d_params || !d_g || !d_m || !d_v || n < 1 || step < 1) return AMG_EINVAL;
  const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
  return amgp::launch_adam((hipStream_t)stream, n, d_params, d_g, d_m, d_v, lr, b1, b2, eps, c1, c2);
}

int amg_learned_beta(const amg_handle* h, int degree, const float* d_y, int ngrid, double* d_beta, int* d_valid,
                     void* stream) {
  if (!h || !d_beta || !d_valid || degree < 1 || degree > 6 || ngrid < 1) return AMG_EINVAL;
  const Handle& H = h->impl;
  if (H.nlevels < 2) return AMG_EINVAL;
  amgp::BetaRow tab{};
  for (int j = 0; j < degree; ++j) tab.v[j] = kOptBeta[degree][j];
  return amgp::launch_learned_beta((hipStream_t)stream, H.nbatch, H.nlevels, degree, tab, d_y, ngrid, d_beta,
                                   d_valid);
}

int amg_learned_beta_grad(const amg_handle* h, int degree, const double* d_gbeta, const int* d_valid, float* d_gy,
                          void* stream) {
  if (!h || !d_gbeta || !d_valid || !d_gy || degree < 1 || degree > 6) return AMG_EINVAL;
  const Handle& H = h->impl;
  if (H.nlevels < 2) return AMG_EINVAL;
  return amgp::launch_learned_beta_grad((hipStream_t)stream, H.nbatch, H.nlevels, degree, d_gbeta, d_valid, d_gy);
}

int amg_hbm_read(const double* d_x, int64_t n, double* d_partial, void* stream) {
  // an empty array may come with a null pointer; the block sums are still written (zeros)
  if (!d_partial || n < 0 || (n > 0 && !d_x) || (reinterpret_cast<uintptr_t>(d_x) & 15) != 0) return AMG_EINVAL;
  return amgp::launch_hbm_read((hipStream_t)stream, n, d_x, d_partial);
}

int amg_hbm_copy(const double* d_x, double* d_y, int64_t n, void* stream) {
  if (n < 0 || (n > 0 && (!d_x || !d_y)) ||
      ((reinterpret_cast<uintptr_t>(d_x) | reinterpret_cast<uintptr_t>(d_y)) & 15) != 0)
    return AMG_EINVAL;
  if (n == 0) return AMG_OK;
  const uintptr_t a = reinterpret_cast<uintptr_t>(d_x), b = reinterpret_cast<uintptr_t>(d_y);
  const uintptr_t bytes = (uintptr_t)n * sizeof(double);
  if (n > 0 && a < b + bytes && b < a + bytes) return AMG_EINVAL;
  return amgp::launch_hbm_copy((hipStream_t)stream, n, d_x, d_y);
}

int amg_beta_valid(const double* d_beta, int count, int degree, int ngrid, int* d_valid, void* stream) {
  if (!d_beta || !d_valid || count < 1 || degree < 1 || degree > AMG_MAX_DEGREE || ngrid < 1) return AMG_EINVAL;
  return amgp::launch_beta_valid((hipStream_t)stream, count, degree, d_beta, ngrid, d_valid);
}

const char* amg_strerror(int code) {
  switch (code) {
    case AMG_OK: return "success";
    case AMG_NOT_CONVERGED: return "iteration limit reached before the tolerance";
    case AMG_EINVAL: return "invalid argument";
    case AMG_ENOTSPD: return "matrix is not SPD (non-positive diagonal, l1 row sum or Cholesky pivot)";
    case AMG_ENOMEM: return "device allocation failed";
    case AMG_EHIP: return "HIP runtime error";
    case AMG_EBREAKDOWN: return "CG breakdown: (p, A p) <= 0";
    case AMG_ENAN: return "non-finite value";
    case AMG_ECAPACITY: return "capacity exceeded (coarse row width or int32 index range)";
    default: return "unknown error";
  }
}

}  // extern "C"
