// Host runtime and C ABI: hierarchy setup, smoother dispatch, V-cycle and PCG.
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
  static Vecs<double>& v(Level& l) { return l.v64; }
};
template <>
struct Prec<float> {
  static const Ell<float>& A(const Level& l) { return l.A32; }
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
    hipFree(L.csr_ptr);
    hipFree(L.csr_col);
    hipFree(L.csr_val);
    free_ell(L.A64);
    free_ell(L.A32);
    free_vecs(L.v64, l > 0);
    free_vecs(L.v32, true);
    hipFree(L.agg);
    hipFree(L.children);
  }
  hipFree(h->ainv);
  hipFree(h->cb);
  hipFree(h->cx);
  hipFree(h->partial);
  hipFree(h->scal);
  hipFree(h->dflag);
  if (h->hscal) hipHostFree(h->hscal);
  hipFree(h->cg_r);
  hipFree(h->cg_z);
  hipFree(h->cg_p);
  hipFree(h->cg_q);
  hipFree(h->cg_rold);
  hipFree(h->tmp64);
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
template <typename T>
int smooth(Handle* h, int l, int kind, int k, const T* b, T* x, bool xz, hipStream_t s) {
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
    if (xz && k >= 2) {
      // steps 1 and 2 in one pass
      const double alpha2 = (2.0 * 2 - 3.0) / (2.0 * 2 + 1.0), c2 = (8.0 * 2 - 4.0) / (2.0 * 2 + 1.0);
      AMGP_TRY(launch_first2_zero<T>(s, 0, k > 2, A, minv, b, g[1 - cur], v.r, x, c1, alpha2, c2, w(1), w(2)));
      rsrc = v.r;
      cur = 1 - cur;
      j0 = 3;
    } else if (xz) {
      AMGP_TRY(launch_first_zero<T>(s, 0, k > 1, n, minv, b, g[cur], nullptr, x, c1, w(1)));
      rsrc = b;
    } else {
      AMGP_TRY(launch_first_res<T>(s, 0, A, minv, b, x, v.r, g[cur], c1));
      rsrc = v.r;
      pending = w(1);
      if (k == 1) return launch_axpy<T>(s, n, pending, g[cur], x);
    }
    for (int j = j0; j <= k; ++j) {
      const double alpha = (2.0 * j - 3.0) / (2.0 * j + 1.0);
      const double c = (8.0 * j - 4.0) / (2.0 * j + 1.0);
      AMGP_TRY(launch_fused<T>(s, 0, j < k, A, minv, g[cur], g[1 - cur], rsrc, v.r, x, alpha, c, w(j), pending));
      rsrc = v.r;
      pending = 0.0;
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
                                   2.0 * rho / delta, 1.0, 1.0));
    rho_prev = rho;
    cur = 1 - cur;
    j0 = 2;
  } else if (xz) {
    AMGP_TRY(launch_first_zero<T>(s, 1, k > 1, n, minv, b, g[cur], v.r, x, theta, 1.0));
  } else {
    AMGP_TRY(launch_first_res<T>(s, 1, A, minv, b, x, v.r, g[cur], theta));
    pending = 1.0;
    if (k == 1) return launch_axpy<T>(s, n, pending, g[cur], x);
  }
  for (int j = j0; j <= k - 1; ++j) {
    const double rho = 1.0 / (2.0 * sigma1 - rho_prev);
    AMGP_TRY(launch_fused<T>(s, 1, j < k - 1, A, minv, g[cur], g[1 - cur], v.r, v.r, x, rho * rho_prev,
                             2.0 * rho / delta, 1.0, pending));
    pending = 0.0;
    rho_prev = rho;
    cur = 1 - cur;
  }
  return AMG_OK;
}

template <typename T>
int coarse(Handle* h, const T* b, T* x, hipStream_t s) {
  AMGP_TRY(launch_pad_in<T>(s, h->nbatch, h->ncl, h->ncp, b, h->cb));
  AMGP_TRY(launch_coarse_gemv(s, h->nbatch, h->ncp, h->ainv, h->cb, h->cx));
  return launch_pad_out<T>(s, h->nbatch, h->ncl, h->ncp, h->cx, x);
}

// V-cycle of eq. (amg) from level l: x = B_l b.
template <typename T>
int vcycle(Handle* h, int l, int kind, int k, const T* b, T* x, hipStream_t s) {
  if (l == h->nlevels - 1) return coarse<T>(h, b, x, s);
  Level& L = h->lv[l];
  Vecs<T>& vc = Prec<T>::v(h->lv[l + 1]);
  AMGP_TRY(smooth<T>(h, l, kind, k, b, x, true, s));
  AMGP_TRY(launch_restrict<T>(s, Prec<T>::A(L), L.nc, L.children, b, x, Prec<T>::v(L).r, vc.b));
  AMGP_TRY(vcycle<T>(h, l + 1, kind, k, vc.b, vc.x, s));
  AMGP_TRY(launch_prolong<T>(s, L.n, L.agg, vc.x, x));
  return smooth<T>(h, l, kind, k, b, x, false, s);
}

int vcycle_top(Handle* h, int kind, int k, const double* r, double* z, hipStream_t s) {
  if (h->precision == AMG_FP32) {
    Vecs<float>& v = h->lv[0].v32;
    AMGP_TRY((launch_cast<double, float>(s, h->lv[0].n, r, v.b)));
    AMGP_TRY(vcycle<float>(h, 0, kind, k, v.b, v.x, s));
    return launch_cast<float, double>(s, h->lv[0].n, v.x, z);
  }
  return vcycle<double>(h, 0, kind, k, r, z, s);
}

// The V-cycle as one HIP graph: captured on the handle's own stream the first
// time a (kind, degree, r, z) combination is seen, then replayed on the
// caller's stream.  The coarse levels are launch-latency bound; a graph
// removes the per-launch host overhead.  The kernel arguments (including the
// beta weights) are baked in, so changing beta drops the cached graphs.
int vcycle_run(Handle* h, int kind, int k, const double* r, double* z, hipStream_t s) {
  if (!h->use_graphs) return vcycle_top(h, kind, k, r, z, s);
  for (auto& g : h->graphs)
    if (g.kind == kind && g.k == k && g.r == r && g.z == z) {
      AMGP_HIP(hipGraphLaunch(g.exec, s));
      return AMG_OK;
    }
  if (h->graphs.size() >= 32) drop_graphs(h);
  if (!h->cap) AMGP_HIP(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  AMGP_HIP(hipStreamBeginCapture(h->cap, hipStreamCaptureModeRelaxed));
  const int rc = vcycle_top(h, kind, k, r, z, h->cap);
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
  h->graphs.push_back(GraphEntry{kind, k, r, z, exec});
  AMGP_HIP(hipGraphLaunch(exec, s));
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

int setup(Handle* h, int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, const double* val,
          const amg_opts* o, hipStream_t s) {
  h->nbatch = o->nbatch > 0 ? o->nbatch : 1;
  h->max_coarse = o->max_coarse > 0 ? o->max_coarse : 4096;
  h->precision = o->precision;
  {
    const char* e = std::getenv("AMGP_NO_GRAPH");
    h->use_graphs = !(e && e[0] == '1');
  }
  AMGP_TRY(dalloc(&h->dflag, F_NFLAG));
  AMGP_HIP(hipMemsetAsync(h->dflag, 0, sizeof(int) * F_NFLAG, s));
  // level 0: library-owned copy of the CSR matrix
  h->lv.emplace_back();
  {
    Level& L = h->lv.back();
    L.n = n;
    L.nnz = nnz;
    L.nx = o->nx;
    L.ny = o->ny;
    L.nz = o->nz;
    AMGP_TRY(dalloc(&L.csr_ptr, n + 1));
    AMGP_TRY(dalloc(&L.csr_col, nnz));
    AMGP_TRY(dalloc(&L.csr_val, nnz));
    AMGP_HIP(hipMemcpyAsync(L.csr_ptr, row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
    AMGP_HIP(hipMemcpyAsync(L.csr_col, col, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, s));
    AMGP_HIP(hipMemcpyAsync(L.csr_val, val, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s));
    AMGP_TRY(validate_csr(s, n, nnz, L.csr_ptr, L.csr_col, h->dflag));
  }
  for (;;) {
    Level& L = h->lv.back();
    AMGP_TRY(dalloc(&L.v64.minv, L.n));
    AMGP_TRY(launch_l1_diag(s, L.n, L.csr_ptr, L.csr_col, L.csr_val, L.v64.minv, h->dflag));
    int fl[F_NFLAG];
    AMGP_TRY(read_flags(h, s, fl));
    if (fl[F_NOTSPD]) return AMG_ENOTSPD;
    AMGP_TRY(build_ell64(s, L.n, L.csr_ptr, L.csr_col, L.csr_val, &L.A64));
    const int64_t per = L.n / h->nbatch;
    if (per <= h->max_coarse) break;
    int cx, cy, cz;
    const int64_t nc = (int64_t)(L.nx == 1 ? 1 : (L.nx + 1) / 2) * (L.ny == 1 ? 1 : (L.ny + 1) / 2) *
                       (L.nz == 1 ? 1 : (L.nz + 1) / 2) * h->nbatch;
    if (nc >= L.n) break;
    L.nc = nc;
    AMGP_TRY(dalloc(&L.agg, L.n));
    AMGP_TRY(dalloc(&L.children, nc * kMaxChildren));
    AMGP_TRY(launch_aggregates(s, L.nx, L.ny, L.nz, h->nbatch, L.agg, L.children, &cx, &cy, &cz));
    Level C;
    C.n = nc;
    C.nx = cx;
    C.ny = cy;
    C.nz = cz;
    AMGP_TRY(galerkin(s, L.n, L.csr_ptr, L.csr_col, L.csr_val, L.agg, nc, L.children, &C.csr_ptr, &C.csr_col,
                      &C.csr_val, &C.nnz, h->dflag));
    h->lv.push_back(C);
  }
  h->nlevels = (int)h->lv.size();
  // coarsest level: dense inverse through the Cholesky factor
  {
    Level& L = h->lv.back();
    h->ncl = L.n / h->nbatch;
    h->ncp = (h->ncl + kDenseTile - 1) / kDenseTile * kDenseTile;
    AMGP_TRY(dalloc(&h->ainv, (int64_t)h->nbatch * h->ncp * h->ncp));
    AMGP_TRY(dalloc(&h->cb, (int64_t)h->nbatch * h->ncp));
    AMGP_TRY(dalloc(&h->cx, (int64_t)h->nbatch * h->ncp));
    AMGP_TRY(launch_to_dense(s, h->nbatch, h->ncl, h->ncp, L.csr_ptr, L.csr_col, L.csr_val, h->ainv, h->dflag));
    AMGP_TRY(dense_spd_inverse(s, h->nbatch, h->ncp, h->ainv, h->dflag));
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
      AMGP_TRY(alloc_vecs(L.v32, L.n, true));
      AMGP_TRY(dalloc(&L.v32.minv, L.n));
      hipLaunchKernelGGL(k_round_vec, dim3(grid_for(L.n)), dim3(kBlock), 0, s, L.n, L.v64.minv, L.v32.minv);
      AMGP_HIP(hipGetLastError());
    }
  }
  // CG and reduction workspace
  const int64_t n0 = h->lv[0].n;
  const int64_t maxblocks = ((n0 + kBlock - 1) / kBlock + 7) / 8 * 8 + 8;
  AMGP_TRY(dalloc(&h->partial, 2 * maxblocks));
  AMGP_TRY(dalloc(&h->scal, S_NSCAL));
  if (hipHostMalloc((void**)&h->hscal, sizeof(double) * (S_NSCAL + F_NFLAG)) != hipSuccess) return AMG_ENOMEM;
  AMGP_TRY(dalloc(&h->cg_r, n0));
  AMGP_TRY(dalloc(&h->cg_z, n0));
  AMGP_TRY(dalloc(&h->cg_p, n0));
  AMGP_TRY(dalloc(&h->cg_q, n0));
  AMGP_TRY(dalloc(&h->cg_rold, n0));
  AMGP_TRY(dalloc(&h->tmp64, n0));
  // default coefficients
  h->beta.assign((size_t)h->nlevels * (AMG_MAX_DEGREE + 1) * AMG_MAX_DEGREE, 0.0);
  for (int l = 0; l < h->nlevels; ++l)
    for (int k = 1; k <= AMG_MAX_DEGREE; ++k)
      for (int j = 0; j < k; ++j) h->beta_at(l, k, j) = kOptBeta[k][j];
  AMGP_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

int sum_dot(Handle* h, hipStream_t s, int mode, const double* a, const double* b, const double* c, const double* d,
            int64_t n) {
  unsigned nb = 0;
  AMGP_TRY(launch_dot2(s, n, a, b, c, d, h->partial, &nb));
  return launch_reduce(s, mode, nb, h->partial, h->scal, h->dflag);
}

int fetch_scalars(Handle* h, hipStream_t s) {
  AMGP_HIP(hipMemcpyAsync(h->hscal, h->scal, sizeof(double) * S_NSCAL, hipMemcpyDeviceToHost, s));
  AMGP_HIP(hipMemcpyAsync(h->hscal + S_NSCAL, h->dflag, sizeof(int) * F_NFLAG, hipMemcpyDeviceToHost, s));
  AMGP_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

int pcg(Handle* h, int kind, int k, const double* b, double* x, bool xz, double rtol, int maxit, bool flex,
        int* iters, double* relres, double* hist, hipStream_t s) {
  const int64_t n = h->lv[0].n;
  const Ell<double>& A = h->lv[0].A64;
  double *r = h->cg_r, *z = h->cg_z, *p = h->cg_p, *q = h->cg_q, *rold = flex ? h->cg_rold : nullptr;
  const int* hflag = reinterpret_cast<const int*>(h->hscal + S_NSCAL);
  AMGP_HIP(hipMemsetAsync(h->dflag, 0, sizeof(int) * F_NFLAG, s));
  AMGP_TRY(launch_check_finite(s, n, b, h->dflag));
  AMGP_TRY(sum_dot(h, s, RED_BB, b, b, nullptr, nullptr, n));
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
    AMGP_TRY(sum_dot(h, s, RED_RR, r, r, nullptr, nullptr, n));
    AMGP_TRY(fetch_scalars(h, s));
    rel0 = std::sqrt(h->hscal[S_RR]) / bnorm;
  }
  if (hist) hist[0] = rel0;
  *relres = rel0;
  if (rel0 <= rtol) return AMG_OK;
  AMGP_TRY(vcycle_run(h, kind, k, r, z, s));
  AMGP_TRY(sum_dot(h, s, RED_RZ0, r, z, nullptr, nullptr, n));
  AMGP_TRY(launch_copy<double>(s, n, z, p));
  for (int it = 1; it <= maxit; ++it) {
    unsigned nb = 0;
    AMGP_TRY(launch_spmv_dot(s, A, p, q, h->partial, &nb));
    AMGP_TRY(launch_reduce(s, RED_ALPHA, nb, h->partial, h->scal, h->dflag));
    AMGP_TRY(launch_cg_update(s, n, h->scal, p, q, x, r, rold, h->partial, &nb));
    AMGP_TRY(launch_reduce(s, RED_RR, nb, h->partial, h->scal, h->dflag));
    AMGP_TRY(fetch_scalars(h, s));
    *iters = it;
    if (hflag[F_BREAKDOWN]) return AMG_EBREAKDOWN;
    if (hflag[F_NAN]) return AMG_ENAN;
    const double rel = std::sqrt(h->hscal[S_RR]) / bnorm;
    *relres = rel;
    if (hist) hist[it] = rel;
    if (rel <= rtol) return AMG_OK;
    if (it == maxit) break;
    AMGP_TRY(vcycle_run(h, kind, k, r, z, s));
    if (flex)
      AMGP_TRY(sum_dot(h, s, RED_BETA_FLEX, r, z, rold, z, n));
    else
      AMGP_TRY(sum_dot(h, s, RED_BETA, r, z, nullptr, nullptr, n));
    AMGP_TRY(launch_cg_pupdate(s, n, h->scal, z, p));
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

int amg_level_export(const amg_handle* h, int level, int32_t* d_row_ptr, int32_t* d_col, double* d_val,
                     double* d_minv, void* stream) {
  if (!h || level < 0 || level >= h->impl.nlevels) return AMG_EINVAL;
  const amgp::Level& L = h->impl.lv[level];
  hipStream_t s = (hipStream_t)stream;
  if (d_row_ptr) AMGP_HIP(hipMemcpyAsync(d_row_ptr, L.csr_ptr, sizeof(int32_t) * (L.n + 1), hipMemcpyDeviceToDevice, s));
  if (d_col) AMGP_HIP(hipMemcpyAsync(d_col, L.csr_col, sizeof(int32_t) * L.nnz, hipMemcpyDeviceToDevice, s));
  if (d_val) AMGP_HIP(hipMemcpyAsync(d_val, L.csr_val, sizeof(double) * L.nnz, hipMemcpyDeviceToDevice, s));
  if (d_minv) AMGP_HIP(hipMemcpyAsync(d_minv, L.v64.minv, sizeof(double) * L.n, hipMemcpyDeviceToDevice, s));
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

int amg_restrict_residual(amg_handle* h, int level, const double* d_b, const double* d_x, double* d_bc,
                          void* stream) {
  if (!h || !d_b || !d_x || !d_bc || level < 0 || level >= h->impl.nlevels - 1) return AMG_EINVAL;
  amgp::Level& L = h->impl.lv[level];
  return amgp::launch_restrict<double>((hipStream_t)stream, L.A64, L.nc, L.children, d_b, d_x, L.v64.r, d_bc);
}

int amg_prolong_add(amg_handle* h, int level, const double* d_xc, double* d_x, void* stream) {
  if (!h || !d_xc || !d_x || level < 0 || level >= h->impl.nlevels - 1) return AMG_EINVAL;
  const amgp::Level& L = h->impl.lv[level];
  return amgp::launch_prolong<double>((hipStream_t)stream, L.n, L.agg, d_xc, d_x);
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
  return amgp::pcg(&h->impl, kind, degree, d_b, d_x, x_is_zero != 0, rtol, maxit, flexible != 0, h_iters, h_relres,
                   h_hist, (hipStream_t)stream);
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
