// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "amgpoly.h"

namespace amgp {

constexpr int kWave = 64;     // CDNA wavefront width
constexpr int kSlice = 64;    // sliced-ELL slice height = one wavefront, one row per lane
constexpr int kBlock = 256;   // threads per block for row-parallel kernels (4 waves)
constexpr int kMaxChildren = 8;  // 2x2x2 box aggregates
constexpr int kDenseTile = 64;   // dense coarsest level padded to a multiple of this
// coarse levels of 16..63 entries per row and at least this many rows take the offset-aligned
// layout (one row per lane, no column indices) when their slices allow it
constexpr int64_t kAlignedWideMinRows = int64_t(1) << 18;
// FP32 offset-aligned slices of at least this many steps store each lane's steps in quads
constexpr int kQuadMinSteps = 16;

// Sliced ELLPACK matrix with G = `group` lanes per row (G in {1, 4, 16, 64}): a
// slice holds 64 / G rows, one wavefront's worth.  Entry j of row r of slice s
// sits at sptr[s] + 64 * (j / G) + G * (r % (64 / G)) + j % G, so at every step
// the 64 lanes of a wavefront load consecutive addresses, and the G lanes of a
// row then sum their partial products.  G = 1 (one row per lane) suits short
// rows; long rows (wide coarse stencils) take more lanes.  Rows shorter than
// the slice width are padded with (col = row, or 0 past the column count; val = 0).
//
// Offset-aligned slices (square matrices with one row per lane): when every
// slice's rows share few distinct column offsets col - row (stencil matrices),
// step t of slice s holds the entries of offset doff[sptr[s] / 64 + t] for all
// its rows (0 where a row has none), so the kernels form the column as
// row + offset, clamped into [0, n), and read no column indices: 8 instead of
// 12 bytes per stored FP64 entry (`col` is null).  Each lane's steps are kept in
// pairs: steps 2q and 2q + 1 of lane l sit at 128 q + 2 l and 128 q + 2 l + 1 of
// the slice (an odd last step t at 64 t + l), so that one 16-byte (FP64) or
// 8-byte (FP32) load per lane serves two steps.  The FP32 copy of a slice of 16
// or more steps keeps them in quads instead (steps 4q .. 4q + 3 of lane l at
// 256 q + 4 l, then a pair, then a single step), one 16-byte load per four steps.
template <typename T>
struct Ell {
  int64_t n = 0;
  int64_t nslices = 0;
  int64_t padded = 0;
  int group = 1;
  int32_t* sptr = nullptr;  // [nslices + 1]
  int32_t* col = nullptr;   // [padded], null for offset-aligned slices
  T* val = nullptr;         // [padded]
  int32_t* doff = nullptr;  // [padded / 64] offsets of offset-aligned slices, or null
  int64_t ncols = 0;        // columns (0: square, n)
  // offset-aligned slices of a rectangular matrix are aligned on an anchor column per row
  // instead of the row itself: column = anchor[r * astride] + offset (null: the row)
  const int32_t* anchor = nullptr;
  int astride = 1;
};

// Per-problem smoother weights for stacked problems: the weight of row i is
// v[(i / rpp) * stride] when v is not null (otherwise the launch's scalar).
struct Wt {
  const double* v = nullptr;
  int rpp = 1;
  int stride = 0;
};

// The box prolongation x += P x_c (x_i += x_c[agg_i]) carried into the smoother kernels
// of the post-smoothing instead of a pass of its own: the first step gathers x + P x_c,
// the kernel after it adds the row's own term.  agg == nullptr: none.
template <typename T>
struct Prol {
  const int32_t* agg = nullptr;
  const T* xc = nullptr;
};

template <typename T>
struct EllView {
  const int32_t* __restrict__ sptr;
  const int32_t* __restrict__ col;
  const T* __restrict__ val;
  const int32_t* __restrict__ doff;
  int32_t last;  // columns - 1, the clamp of offset-aligned columns
};

template <typename T>
inline EllView<T> view(const Ell<T>& e) {
  return EllView<T>{e.sptr, e.col, e.val, e.doff, (int32_t)((e.ncols > 0 ? e.ncols : e.n) - 1)};
}

// Work vectors of one level in one precision.
template <typename T>
struct Vecs {
  T* b = nullptr;   // right-hand side of this level (levels > 0, or FP32 level 0)
  T* x = nullptr;   // solution/correction of this level
  T* r = nullptr;   // smoother recurrence residual
  T* g0 = nullptr;  // direction ping-pong (z / d), also l1-Jacobi ping-pong
  T* g1 = nullptr;
  T* minv = nullptr;
};

struct Level {
  int64_t n = 0, nnz = 0;
  int nx = 1, ny = 1, nz = 1;  // per-problem grid
  // Galerkin operator in CSR (float64), kept for export and the next Galerkin product.
  // csr_borrowed: level 0 reads the caller's arrays during setup (not freed by the handle).
  int32_t* csr_ptr = nullptr;
  int32_t* csr_col = nullptr;
  double* csr_val = nullptr;
  bool csr_borrowed = false;
  Ell<double> A64;
  Ell<float> A32;
  Vecs<double> v64;
  Vecs<float> v32;
  // transfer to level + 1
  int64_t nc = 0;                 // rows of level + 1
  int32_t* agg = nullptr;         // [n] aggregate of each row
  int32_t* children = nullptr;    // [nc * 8] rows of each aggregate, ascending, -1 padded (2x2x2 boxes)
  double* wsmooth = nullptr;      // smooth vector of the matching aggregation (device, n), null: ones
  // explicit prolongator (smoothed, or boxes of another edge): P (n x nc) and P^T (nc x n)
  bool general = false;
  Ell<double> P64, PT64;
  Ell<float> P32, PT32;
  // 2x2x2 boxes: the restriction product R = P^T A (nc x n) in slices aligned on each aggregate's
  // first row, so that b_c = P^T b - R x needs no fine residual (empty when it does not fit)
  Ell<double> R64;
  Ell<float> R32;
};

// Device CSR matrix (m x ncols) used by the setup's general sparse products.
struct Csr {
  int64_t m = 0, ncols = 0, nnz = 0;
  int32_t* ptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
};

// Entries of a computed product whose magnitude is at most kDropTau times the
// largest of their row are dropped (exact cancellations up to rounding).
constexpr double kDropTau = 1.4210854715202004e-14;  // 2^-46

// A captured V-cycle (one launch sequence for a given kind, degree and r/z buffers).
// mode: -1 for a bare V-cycle, else the reduction that follows the preconditioner
// (RED_RZ0 / RED_BETA / RED_BETA_FLEX); poly: the smoother alone instead of the V-cycle.
struct GraphEntry {
  int kind, k, mode;
  bool poly;
  const void* r;
  void* z;
  const void* aux;
  hipGraphExec_t exec;
};

// Workspace of the differentiable V-cycle (allocated on first use).
template <typename T>
struct AdjVecs {
  T *u = nullptr, *xmid = nullptr, *xpre = nullptr, *res = nullptr, *xin = nullptr, *bout = nullptr;
};

struct Handle {
  int nlevels = 0;
  // per-problem weights for AMG_OPTCHEB4 while a differentiable V-cycle runs:
  // dbeta[(p * nlevels + l) * dbeta_k + j - 1], else null (host table used)
  const double* dbeta = nullptr;
  int dbeta_k = 0;
  std::vector<int64_t> ck_off;  // checkpoint offset (elements) of level l: [pre n_l][post n_l]
  int64_t ck_count = 0;         // elements per V-cycle checkpoint
  bool train_ready = false;
  std::vector<AdjVecs<double>> adj64;
  std::vector<AdjVecs<float>> adj32;
  void* tr_buf = nullptr;       // training driver vectors and checkpoints
  double* tr_sq = nullptr;      // [2 * nbatch] squared norms
  double* tr_loss = nullptr;    // [1 + nbatch]
  double* tr_partial = nullptr; // segmented-reduction partials
  bool use_graphs = true;
  hipStream_t cap = nullptr;  // stream used only to capture V-cycles into graphs
  std::vector<GraphEntry> graphs;
  int nbatch = 1;
  int precision = AMG_FP64;
  int max_coarse = 4096;
  int agg_edge = 2;       // box aggregate edge
  bool smoothed = false;  // smoothed prolongator
  int coarse_sweeps = 0;  // > 0: l1-Jacobi sweeps instead of the dense coarsest solve
  int aggregation = AMG_AGG_BOX;
  int match_steps = 3;    // matching steps per level (aggregates of up to 2^steps rows)
  double vbm_theta = 0.0;  // strength threshold of the VBM aggregation on level 0
  std::vector<Level> lv;
  // coarsest level: dense inverse per problem, padded to ncp
  int64_t ncl = 0;   // rows per problem on the coarsest level
  int64_t ncp = 0;   // padded
  double* ainv = nullptr;  // [nbatch][nb(nb+1)/2][64][64]: lower 64x64 blocks of A_L^{-1}, packed (nb = ncp/64)
  double* cpart = nullptr; // [nbatch][ncp/64][ncp/64][64] partial products of the blocked symmetric solve
  // beta weights: [level][degree][j]
  std::vector<double> beta;  // size nlevels * (AMG_MAX_DEGREE+1) * AMG_MAX_DEGREE
  // reductions and CG workspace (fine level, float64)
  double* partial = nullptr;  // 2 * maxblocks
  double* scal = nullptr;     // device scalars
  double* hscal = nullptr;    // pinned host mirror
  double* hpub = nullptr;     // mapped host memory the (r, r) reduction publishes to: rr, breakdown, nan
  double* dpub = nullptr;     // its device address
  hipEvent_t ev = nullptr;    // end of a CG update (the host waits on it)
  int* dflag = nullptr;       // device error flags
  double *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_p2 = nullptr, *cg_q = nullptr, *cg_rold = nullptr;
  double* cg_u = nullptr;     // M^{-1} r of level 0, for the V-cycle's first kernel (n0)
  double& beta_at(int l, int k, int j) {
    return beta[((size_t)l * (AMG_MAX_DEGREE + 1) + k) * AMG_MAX_DEGREE + j];
  }
};

// Device scalar slots in Handle::scal.
enum Scal { S_RZ = 0, S_PQ, S_ALPHA, S_BETA, S_RR, S_BB, S_AUX, S_NSCAL };
// Device flag slots in Handle::dflag.
enum Flag { F_NOTSPD = 0, F_CAPACITY, F_BREAKDOWN, F_NAN, F_BADCSR, F_NFLAG };

// ---- error plumbing ----
#define AMGP_HIP(call)                          \
  do {                                          \
    hipError_t e_ = (call);                     \
    if (e_ != hipSuccess) return AMG_EHIP;      \
  } while (0)
#define AMGP_TRY(call)                          \
  do {                                          \
    int rc_ = (call);                           \
    if (rc_ != AMG_OK) return rc_;              \
  } while (0)

inline unsigned grid_for(int64_t n, int per_block = kBlock) {
  int64_t g = (n + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : g);
}

// ---- sparse / vector kernel launchers (kernels_sparse.hip) ----
template <typename T>
int launch_spmv(hipStream_t s, const Ell<T>& A, const T* x, T* y);
template <typename T>
int launch_residual(hipStream_t s, const Ell<T>& A, const T* b, const T* x, T* r);
// smoother steps
template <typename T>
int launch_first_zero(hipStream_t s, int mode, bool store, int64_t n, const T* minv, const T* b, T* g, T* r,
                      T* x, double c, double w, Wt wv = Wt());
template <typename T>
int launch_first2_zero(hipStream_t s, int mode, bool store, const Ell<T>& A, const T* minv, const T* b, T* gnew,
                       T* r, T* x, double c1, double alpha, double c, double w1, double w2, Wt w1v = Wt(),
                       Wt w2v = Wt(), const T* u = nullptr);
// u = M^{-1} b, given to launch_first2_zero, is read on these levels (and ignored on the others)
bool first2_takes_u(const Ell<double>& A);
bool first2_takes_u(const Ell<float>& A);
// b = (float) r and u = M^{-1} b for an FP32 fine level whose merged first two steps take u
int launch_cast_u(hipStream_t s, int64_t n, const double* r, const float* minv, float* b, float* u);
// The last step of an application (as launch_fused with store = false) on a level of one lane per
// row, with the block partials of (dr, x) and, with drold, of (drold, x) written as launch_dot2
// writes them; AMG_EINVAL on levels of several lanes per row.
template <typename T>
int launch_fused_dot(hipStream_t s, int mode, const Ell<T>& A, const T* minv, const T* gold, const T* rin, T* x,
                     double alpha, double c, double w, double wprev, Wt wv, Wt wpv, Prol<T> pr, const double* dr,
                     const double* drold, double* partial, unsigned* nblocks);
template <typename T>
int launch_first_res(hipStream_t s, int mode, const Ell<T>& A, const T* minv, const T* b, const T* x, T* r,
                     T* g, double c, Prol<T> pr = Prol<T>());  // pr: A.group must be 1
template <typename T>
int launch_fused(hipStream_t s, int mode, bool store, const Ell<T>& A, const T* minv, const T* gold, T* gnew,
                 const T* rin, T* rout, T* x, double alpha, double c, double w, double wprev, Wt wv = Wt(),
                 Wt wpv = Wt(), Prol<T> pr = Prol<T>());
template <typename T>
int launch_jacobi(hipStream_t s, const Ell<T>& A, const T* minv, const T* b, const T* xold, T* xnew);
template <typename T>
int launch_jacobi_zero(hipStream_t s, int64_t n, const T* minv, const T* b, T* x);
// transfers
// b_c = P^T (b - A x); tmp (n entries) is scratch (one row per lane matrices do not touch it)
// b_c = P^T b - R x with R = P^T A in anchor-aligned slices (2x2x2 boxes)
template <typename T>
int launch_restrict_product(hipStream_t s, const Ell<T>& R, const int32_t* children, const T* b, const T* x, T* bc);
template <typename T>
int launch_restrict(hipStream_t s, const Ell<T>& A, int64_t nc, const int32_t* children, const T* b,
                    const T* x, T* tmp, T* bc);
template <typename T>
int launch_prolong(hipStream_t s, int64_t n, const int32_t* agg, const T* xc, T* x);
template <typename T>
int launch_spmv_add(hipStream_t s, const Ell<T>& A, const T* x, T* y);  // y += A x
// vectors
template <typename T>
int launch_axpy(hipStream_t s, int64_t n, double a, const T* x, T* y, Wt av = Wt(),
                Prol<T> pr = Prol<T>());  // y += a x (after y += P x_c)
template <typename T>
int launch_copy(hipStream_t s, int64_t n, const T* x, T* y);
template <typename T>
int launch_fill(hipStream_t s, int64_t n, T v, T* y);
template <typename Tin, typename Tout>
int launch_cast(hipStream_t s, int64_t n, const Tin* x, Tout* y);
// CG (float64; the preconditioned vector b, d / z may be the FP32 hierarchy's float output)
template <typename TZ>
int launch_dot2(hipStream_t s, int64_t n, const double* a, const TZ* b, const double* c, const TZ* d,
                double* partial, unsigned* nblocks);  // (a,b) and optionally (c,d)
// p_new = z + beta p_old (beta from scal), q = A p_new, partials of (p_new, q); x (optional)
// receives the previous iteration's x += alpha p_old (alpha from scal)
template <typename TZ>
int launch_spmv_dot_p(hipStream_t s, const Ell<double>& A, const double* scal, const TZ* z, const double* pold,
                      double* pnew, double* q, double* partial, double* x, unsigned* nblocks);
// r -= alpha q, partials of (r, r); rold (optional) receives the old r, u (optional) M^{-1} r
int launch_cg_update(hipStream_t s, int64_t n, const double* scal, const double* q, double* r, double* rold,
                     double* partial, unsigned* nblocks, const double* minv = nullptr, double* u = nullptr);
// x += alpha p: the last iteration's update of x
int launch_cg_x(hipStream_t s, int64_t n, const double* scal, const double* p, double* x);
// pub (optional, RED_RR): receives (r, r) and the breakdown / NaN flags, for the host
int launch_reduce(hipStream_t s, int mode, unsigned nblocks, const double* partial, double* scal, int* flag,
                  double* pub = nullptr);
enum ReduceMode { RED_BB = 0, RED_RZ0, RED_ALPHA, RED_RR, RED_BETA, RED_BETA_FLEX };
int launch_check_finite(hipStream_t s, int64_t n, const double* x, int* flag);

// ---- differentiable V-cycle and learned-beta network (kernels_train.hip) ----
// out[p * ostride] (+)= (a_p, b_p) over segment p (b = nullptr: |a_p|^2); partial >= kSegBlocks * nseg
// doubles
constexpr int kSegBlocks = 64;  // blocks per problem segment in a segmented reduction
template <typename T>
int launch_seg_dot(hipStream_t s, int nseg, int64_t rpp, const T* a, const T* b, double* partial, double* out,
                   int ostride, bool acc);
// The per-problem sums of a segmented dot product's block partials, left to a later kernel.
struct SegFin {
  const double* partial = nullptr;
  double* out = nullptr;
  int nseg = 0, ostride = 0, acc = 0;
};
// The block partials of (a_p, b_p) into partial, with the pending sums prev (nseg <= 256) done
// first by the kernel's first block; the caller keeps {partial, out, nseg, ostride, acc} as the
// next pending sums and must not reuse partial before they are done.
template <typename T>
int launch_seg_dot_chain(hipStream_t s, int nseg, int64_t rpp, const T* a, const T* b, double* partial,
                         SegFin prev);
int launch_seg_finish(hipStream_t s, SegFin f);  // the pending sums alone (none: nothing)
template <typename T>
int launch_loss_seed(hipStream_t s, int64_t n, int64_t rpp, int P, const double* sq, const T* r2, T* g);
int launch_loss_value(hipStream_t s, int P, const double* sq, double* out);
template <typename T>
int launch_neg(hipStream_t s, int64_t n, const T* x, T* y);
template <typename T>
int launch_prolong_set(hipStream_t s, int64_t n, const int32_t* agg, const T* xc, T* x);
template <typename T>
int launch_restrict_sum(hipStream_t s, int64_t nc, const int32_t* children, const T* x, T* yc);
int launch_mlp_fwd(hipStream_t s, int B, const float* W, const float* X, float* Y, float* cache);
int launch_mlp_bwd(hipStream_t s, int B, const float* W, const float* X, const float* cache, const float* dY,
                   float* G, float* work);
// mlp_bwd with its scratch in the library's static per-device array (batch <= 256)
int launch_mlp_bwd_noalloc(hipStream_t s, int B, const float* W, const float* X, const float* cache,
                           const float* dY, float* G);
int launch_adam(hipStream_t s, int n, float* W, const float* G, float* m, float* v, float lr, float b1, float b2,
                float eps, float c1, float c2);
int launch_beta_valid(hipStream_t s, int count, int k, const double* beta, int ngrid, int* valid);
// learned weights: table + network output on the smoothing levels, |p| < 1 fallback (amg_learned_beta)
struct BetaRow {
  double v[AMG_MAX_DEGREE];
};
int launch_learned_beta(hipStream_t s, int P, int L, int k, const BetaRow& tab, const float* y, int ngrid,
                        double* beta, int* valid);
int launch_learned_beta_grad(hipStream_t s, int P, int L, int k, const double* gbeta, const int* valid, float* gy);
int mlp_num_params();
int launch_mul(hipStream_t s, int64_t n, const double* a, const double* x, double* y);
int launch_offdiag_ratio(hipStream_t s, int64_t n, const int32_t* ptr, const int32_t* col, const double* val,
                         const double* minv, double* out);

// ---- bandwidth ceiling (kernels_stream.hip) ----
int launch_hbm_read(hipStream_t s, int64_t n, const double* x, double* part);
int launch_hbm_copy(hipStream_t s, int64_t n, const double* x, double* y);

// ---- setup kernels (kernels_setup.hip) ----
// row_ptr monotone from 0 to nnz, columns strictly increasing within a row and in [0, n)
int validate_csr(hipStream_t s, int64_t n, int64_t nnz, const int32_t* ptr, const int32_t* col, int* flag);
int launch_l1_diag(hipStream_t s, int64_t n, const int32_t* ptr, const int32_t* col, const double* val,
                   double* minv, int* flag);
// ncols: number of columns (default n); padding entries use column i when i < ncols, else 0.
// group: lanes per row (1, 4, 16 or 64); 0 chooses from the mean row length
int build_ell64(hipStream_t s, int64_t n, const int32_t* ptr, const int32_t* col, const double* val,
                Ell<double>* out, int64_t ncols = -1, int group = 1);
int build_ell32(hipStream_t s, const Ell<double>& a, Ell<float>* out);
// offset-aligned slices (one row per lane) with the offsets taken against anchor[r * astride]
// (null: the row r) and columns clamped into [0, ncols) (-1: n); AMG_EINVAL when a slice has more
// than 64 offsets or (unless any_size) the layout is more than 10% larger than the packed one
int build_ell_aligned(hipStream_t s, int64_t n, const int32_t* ptr, const int32_t* col, const double* val,
                      Ell<double>* out, const int32_t* anchor = nullptr, int astride = 1, int64_t ncols = -1,
                      bool any_size = false);
// box aggregates of edge e; children (2x2x2 boxes only) may be null
int launch_aggregates(hipStream_t s, int nx, int ny, int nz, int nbatch, int e, int32_t* agg, int32_t* children,
                      int* cnx, int* cny, int* cnz);
// A_c = P^T A P for 2x2x2 boxes with unit prolongator entries (zero sums are kept); the three output
// arrays belong to the caller from their allocation on, also when the call fails
int galerkin(hipStream_t s, int64_t n, const int32_t* ptr, const int32_t* col, const double* val,
             const int32_t* agg, int64_t nc, const int32_t* children, int32_t** cptr, int32_t** ccol,
             double** cval, int64_t* cnnz, int* flag);
int launch_to_dense(hipStream_t s, int nbatch, int64_t nl, int64_t np, const int32_t* ptr, const int32_t* col,
                    const double* val, double* dense, int* flag);
void free_ell(Ell<double>& e);
// ---- general sparse products (kernels_galerkin.hip) ----
void free_csr(Csr& a);
int spgemm(hipStream_t s, const Csr& X, const Csr& Y, Csr* C, int* flag);  // C = X Y
int drop_small(hipStream_t s, Csr* a, double tau);
int transpose(hipStream_t s, const Csr& a, Csr* t);
int tentative_prolongator(hipStream_t s, int64_t n, int64_t nc, const int32_t* agg, Csr* P);
// P = (I - omega D^{-1} A) P_hat for a P_hat with one entry per row,
// omega = 4 / (3 ||D^{-1} A||_inf) per stacked problem
int smoothed_prolongator(hipStream_t s, const Csr& A, int nbatch, const Csr& Phat, Csr* P, int* flag);
// host exclusive scan of cnt[0, m) into ptr[0, m]; returns the total (rc = AMG_ECAPACITY beyond int32)
int64_t scan_ptr(hipStream_t s, int64_t m, const int32_t* cnt, int32_t* ptr, int* rc);
// ---- compatible weighted matching (kernels_match.hip) ----
// composite tentative prolongator of `steps` matching steps on A (structurally symmetric, ascending
// columns) from the smooth vector w0 (null: ones); *wnext (device, ncols entries) is the coarse one
int matching_prolongator(hipStream_t s, const Csr& A, const double* w0, int steps, Csr* Phat, double** wnext,
                         int* flag);
int galerkin_general(hipStream_t s, const Csr& A, const Csr& P, const Csr& PT, Csr* Ac, int* flag);
// ---- classical smoothed aggregation (kernels_vbm.hip) ----
// aggregate of every row of A (structurally symmetric, ascending columns) for the strength
// threshold theta, numbered by increasing root; *nc the number of aggregates
int vbm_aggregates(hipStream_t s, const Csr& A, double theta, int32_t* agg, int64_t* nc);
void free_ell(Ell<float>& e);

// ---- dense kernels (kernels_dense.hip) ----
// In place: dense[nbatch][np][np] (SPD, lower part used) -> inverse A^{-1}, full symmetric.
int dense_spd_inverse(hipStream_t s, int nbatch, int64_t np, double* dense, int* flag);
// copy the lower 64x64 blocks of each np x np matrix into contiguous tiles (tile J(J+1)/2 + I = block (J, I))
int pack_lower_tiles(hipStream_t s, int nbatch, int64_t np, const double* dense, double** packed);
// x = A^{-1} b from the lower blocks of the symmetric inverse; part holds nbatch * (np/64)^2 * 64 doubles
template <typename T>
int launch_coarse_symv(hipStream_t s, int nbatch, int64_t nl, int64_t np, const double* ainv, const T* b, T* x,
                       double* part);

}  // namespace amgp
