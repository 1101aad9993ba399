// Kernels of the differentiable V-cycle and the learned-beta network:
// per-problem (segmented) dot products and norms, residual-ratio loss seeds,
// the 8-64-64-6 tanh MLP forward / backward / Adam step, and the |p| <= 1
// validity check of a weighted 4th-kind polynomial.
//
// Every reduction has a fixed association order (one block per problem
// segment, then a fixed-order sum of the block partials), so results are
// bitwise reproducible.
#include <mutex>

#include "internal.h"

namespace amgp {

namespace {


template <typename T>
__device__ __forceinline__ double wave_block_sum(double v, double* sm) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & 63) == 0) sm[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / kWave; ++i) s += sm[i];
  return s;
}

// partial[p][bx] = sum over rows of segment p handled by block bx of a_i * b_i
// (b = nullptr: a_i^2).  grid = (kSegBlocks, nseg).
// out[p * ostride] (+)= sum_bx partial[p][bx]   (accumulate when acc != 0)
__device__ __forceinline__ void seg_finish_one(int p, const double* __restrict__ partial, double* __restrict__ out,
                                               int ostride, int acc) {
  double s = 0.0;
  for (int i = 0; i < kSegBlocks; ++i) s += partial[p * kSegBlocks + i];
  out[(int64_t)p * ostride] = acc ? out[(int64_t)p * ostride] + s : s;
}

// prev: the pending per-problem sums of an earlier call, done first by block (0, 0).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_seg_dot(int64_t rpp, const T* __restrict__ a, const T* __restrict__ b,
                                                    double* __restrict__ partial, SegFin prev) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && (int)threadIdx.x < prev.nseg)
    seg_finish_one(threadIdx.x, prev.partial, prev.out, prev.ostride, prev.acc);
  __shared__ double sm[kBlock / kWave];
  const int p = blockIdx.y;
  const T* ap = a + (int64_t)p * rpp;
  const T* bp = b ? b + (int64_t)p * rpp : nullptr;
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < rpp; i += (int64_t)kSegBlocks * kBlock) {
    const double x = (double)ap[i];
    v += bp ? x * (double)bp[i] : x * x;
  }
  const double s = wave_block_sum<T>(v, sm);
  if (threadIdx.x == 0) partial[p * kSegBlocks + blockIdx.x] = s;
}

__global__ void k_seg_finish(int nseg, const double* __restrict__ partial, double* __restrict__ out, int ostride,
                             int acc) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nseg) return;
  seg_finish_one(p, partial, out, ostride, acc);
}

// Loss seed: loss = mean_p ||r2_p|| / ||r0_p||; g = d loss / d r2 = r2_p / (P ||r2_p|| ||r0_p||).
// sq holds [P] squared norms of r0 then [P] of r2 (per problem).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_loss_seed(int64_t n, int64_t rpp, int P, const double* __restrict__ sq,
                                                      const T* __restrict__ r2, T* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int p = (int)(i / rpp);
  const double n0 = sqrt(sq[p]), n2 = sqrt(sq[P + p]);
  const double s = (n2 > 0.0 && n0 > 0.0) ? 1.0 / ((double)P * n2 * n0) : 0.0;
  g[i] = (T)((double)r2[i] * s);
}

__global__ void k_loss_value(int P, const double* __restrict__ sq, double* __restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double L = 0.0;
  for (int p = 0; p < P; ++p) {
    const double n0 = sqrt(sq[p]), n2 = sqrt(sq[P + p]);
    const double ratio = n0 > 0.0 ? n2 / n0 : 0.0;
    out[1 + p] = ratio;
    L += ratio;
  }
  out[0] = L / (double)P;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scale_neg(int64_t n, const T* __restrict__ x, T* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = -x[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_set(int64_t n, const int32_t* __restrict__ agg,
                                                        const T* __restrict__ xc, T* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = xc[agg[i]];
}

// plain restriction y_c[I] = sum of x over the rows of aggregate I (P^T x)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict_sum(int64_t nc, const int32_t* __restrict__ ch,
                                                         const T* __restrict__ x, T* __restrict__ yc) {
  const int64_t I = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (I >= nc) return;
  T s = T(0);
  for (int c = 0; c < kMaxChildren; ++c) {
    const int i = ch[I * kMaxChildren + c];
    if (i < 0) break;
    s += x[i];
  }
  yc[I] = s;
}

// ---------------------------------------------------------------------------
// MLP 8 -> 64 -> 64 -> 6, tanh hidden units, output scaled by kOutScale.
// Parameter vector (float32, 5126 entries):
//   W1[64][8], b1[64], W2[64][64], b2[64], W3[6][64], b3[6]
// cache per batch row: h1[64], h2[64].
// ---------------------------------------------------------------------------
constexpr int NI = 8, NH = 64, NO = 6;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NI, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NO * NH, NPARAM = OFF_B3 + NO;
static_assert(NPARAM == 5126, "parameter count");
constexpr float kOutScale = 0.1f;

// one block of 256 threads per 4 batch rows (one wavefront per row)
__global__ __launch_bounds__(256) void k_mlp_fwd(int B, const float* __restrict__ W, const float* __restrict__ X,
                                                 float* __restrict__ Y, float* __restrict__ cache) {
  __shared__ float h1s[4][NH];
  __shared__ float h2s[4][NH];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + w;
  const bool act = row < B;
  const float* x = X + (int64_t)(act ? row : 0) * NI;
  // layer 1: lane = hidden unit
  float z = W[OFF_B1 + lane];
  for (int i = 0; i < NI; ++i) z += W[OFF_W1 + lane * NI + i] * x[i];
  const float h1 = tanhf(z);
  h1s[w][lane] = h1;
  __syncthreads();
  z = W[OFF_B2 + lane];
  for (int i = 0; i < NH; ++i) z += W[OFF_W2 + lane * NH + i] * h1s[w][i];
  const float h2 = tanhf(z);
  h2s[w][lane] = h2;
  __syncthreads();
  if (act) {
    cache[(int64_t)row * 2 * NH + lane] = h1;
    cache[(int64_t)row * 2 * NH + NH + lane] = h2;
    if (lane < NO) {
      float y = W[OFF_B3 + lane];
      for (int i = 0; i < NH; ++i) y += W[OFF_W3 + lane * NH + i] * h2s[w][i];
      Y[(int64_t)row * NO + lane] = kOutScale * y;
    }
  }
}

// Backward, first part: dz2 and dz1 of every row into work (dz2[B][64], then dz1[B][64]).
// Rows are independent: each block takes four rows, one thread per (row, unit).
__global__ __launch_bounds__(256) void k_mlp_bwd(int B, const float* __restrict__ W,
                                                 const float* __restrict__ cache, const float* __restrict__ dY,
                                                 float* __restrict__ work) {
  float* dz2 = work;
  float* dz1 = work + (int64_t)B * NH;
  const int e = blockIdx.x * 4 * NH + threadIdx.x;  // row e / NH, unit e % NH
  const int r = e / NH, j = e % NH;
  // dz3 = kOutScale * dY; dh2 = dz3 W3; dz2 = dh2 (1 - h2^2)
  if (r < B) {
    float s = 0.f;
    for (int o = 0; o < NO; ++o) s += kOutScale * dY[r * NO + o] * W[OFF_W3 + o * NH + j];
    const float h2 = cache[(int64_t)r * 2 * NH + NH + j];
    dz2[e] = s * (1.f - h2 * h2);
  }
  __syncthreads();  // a row's dz1 reads the dz2 of its 64 units, all in this block
  if (r < B) {
    float s = 0.f;
    for (int i = 0; i < NH; ++i) s += dz2[r * NH + i] * W[OFF_W2 + i * NH + j];
    const float h1 = cache[(int64_t)r * 2 * NH + j];
    dz1[e] = s * (1.f - h1 * h1);
  }
}

// Backward, second part: the parameter gradients from the dz2, dz1 in work, one thread per
// parameter, each a sum over the batch in row order.  (Both parts in one block of 256 threads,
// as before, took 194 us on a batch of 64 rows.)
__global__ __launch_bounds__(256) void k_mlp_grad(int B, const float* __restrict__ X, const float* __restrict__ cache,
                                                  const float* __restrict__ dY, float* __restrict__ G,
                                                  const float* __restrict__ work) {
  const float* dz2 = work;
  const float* dz1 = work + (int64_t)B * NH;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < NPARAM) {
    float g = 0.f;
    if (e < OFF_B1) {
      const int j = e / NI, i = e % NI;
      for (int r = 0; r < B; ++r) g += dz1[r * NH + j] * X[r * NI + i];
    } else if (e < OFF_W2) {
      const int j = e - OFF_B1;
      for (int r = 0; r < B; ++r) g += dz1[r * NH + j];
    } else if (e < OFF_B2) {
      const int j = (e - OFF_W2) / NH, i = (e - OFF_W2) % NH;
      for (int r = 0; r < B; ++r) g += dz2[r * NH + j] * cache[(int64_t)r * 2 * NH + i];
    } else if (e < OFF_W3) {
      const int j = e - OFF_B2;
      for (int r = 0; r < B; ++r) g += dz2[r * NH + j];
    } else if (e < OFF_B3) {
      const int o = (e - OFF_W3) / NH, i = (e - OFF_W3) % NH;
      for (int r = 0; r < B; ++r) g += kOutScale * dY[r * NO + o] * cache[(int64_t)r * 2 * NH + NH + i];
    } else {
      const int o = e - OFF_B3;
      for (int r = 0; r < B; ++r) g += kOutScale * dY[r * NO + o];
    }
    G[e] = g;
  }
}

// Adam (bias-corrected), elementwise.
__global__ void k_adam(int n, float* __restrict__ W, const float* __restrict__ G, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = G[i];
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  W[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// True when p(x) = sum_j (beta_j - beta_{j+1})/(2j+1) W_j(1-2x) (beta_0 = 1, beta_{k+1} = 0,
// W_j the 4th-kind polynomials) has |p| < 1 at every x_m = m / ngrid, m = 1..ngrid (p(0) = 1 by
// construction).  Called by all threads of a block (uniformly); bq is the row's k weights.
__device__ bool row_inside_pik(const double* bq, int k, int ngrid) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int m = 1 + threadIdx.x; m <= ngrid; m += blockDim.x) {
    const double y = 1.0 - 2.0 * (double)m / ngrid;
    double wm = 1.0, w = 2.0 * y + 1.0;  // W_0, W_1
    double p = 1.0 - bq[0];              // (beta_0 - beta_1)/1 * W_0
    for (int j = 1; j <= k; ++j) {
      const double bj = bq[j - 1], bn = (j < k) ? bq[j] : 0.0;
      p += (bj - bn) / (2.0 * j + 1.0) * w;
      const double wn = 2.0 * y * w - wm;
      wm = w;
      w = wn;
    }
    if (!(fabs(p) < 1.0)) bad = 1;
  }
  __syncthreads();
  const bool ok = bad == 0;
  __syncthreads();
  return ok;
}

// valid[q] = 1 if the weight row q (k entries) keeps its polynomial inside Pi_k (eq. polspace).
__global__ __launch_bounds__(256) void k_beta_valid(int count, int k, const double* __restrict__ beta,
                                                    int ngrid, int* __restrict__ valid) {
  const int q = blockIdx.x;
  if (q >= count) return;
  const bool ok = row_inside_pik(beta + (int64_t)q * k, k, ngrid);
  if (threadIdx.x == 0) valid[q] = ok ? 1 : 0;
}

// Learned weights, one block per row (p, l) of the table [P][L][k]: on a smoothing level
// (l < L - 1) the tabulated optimal weights plus the network output y[p * (L - 1) + l][0..k),
// kept when the polynomial stays inside Pi_k, else the table (valid = 0); the coarsest row
// is the table.  y == nullptr: the table on every row.
__global__ __launch_bounds__(256) void k_learned_beta(int L, int k, BetaRow tab, const float* __restrict__ y,
                                                      int ngrid, double* __restrict__ beta, int* __restrict__ valid) {
  const int row = blockIdx.x;  // p * L + l
  const int p = row / L, l = row % L;
  double* out = beta + (int64_t)row * k;
  if (l == L - 1) {
    if (threadIdx.x < k) out[threadIdx.x] = tab.v[threadIdx.x];
    return;
  }
  const int q = p * (L - 1) + l;
  __shared__ double cand[AMG_MAX_DEGREE];
  if (threadIdx.x < k) cand[threadIdx.x] = tab.v[threadIdx.x] + (y ? (double)y[(int64_t)q * 6 + threadIdx.x] : 0.0);
  __syncthreads();
  const bool ok = y ? row_inside_pik(cand, k, ngrid) : true;
  if (threadIdx.x < k) out[threadIdx.x] = ok ? cand[threadIdx.x] : tab.v[threadIdx.x];
  if (threadIdx.x == 0) valid[q] = ok ? 1 : 0;
}

// gy[q][j] = valid[q] ? (float)gbeta[p][l][j] : 0 for j < k, 0 for k <= j < 6 (q = p * (L - 1) + l).
__global__ __launch_bounds__(256) void k_learned_beta_grad(int rows, int L, int k, const double* __restrict__ gbeta,
                                                           const int* __restrict__ valid, float* __restrict__ gy) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * 6) return;
  const int q = e / 6, j = e % 6;
  const int p = q / (L - 1), l = q % (L - 1);
  gy[e] = (j < k && valid[q]) ? (float)gbeta[((int64_t)p * L + l) * k + j] : 0.0f;
}

// y = M^{-1} x (elementwise)
__global__ __launch_bounds__(kBlock) void k_mul(int64_t n, const double* __restrict__ a, const double* __restrict__ x,
                                                double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = a[i] * x[i];
}

// out_i = (sum_{j != i} |a_ij|) / a_ii, from the l1 row sum M_i = 1/minv_i
__global__ __launch_bounds__(kBlock) void k_offdiag_ratio(int64_t n, const int32_t* __restrict__ ptr,
                                                          const int32_t* __restrict__ col,
                                                          const double* __restrict__ val,
                                                          const double* __restrict__ minv, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int p = ptr[i]; p < ptr[i + 1]; ++p)
    if (col[p] == i) d += val[p];
  out[i] = (1.0 / minv[i] - d) / d;
}

}  // namespace

#define LAUNCH_OK() (hipGetLastError() == hipSuccess ? AMG_OK : AMG_EHIP)

template <typename T>
int launch_seg_dot(hipStream_t s, int nseg, int64_t rpp, const T* a, const T* b, double* partial, double* out,
                   int ostride, bool acc) {
  hipLaunchKernelGGL(k_seg_dot<T>, dim3(kSegBlocks, nseg), dim3(kBlock), 0, s, rpp, a, b, partial, SegFin());
  hipLaunchKernelGGL(k_seg_finish, dim3((nseg + 63) / 64), dim3(64), 0, s, nseg, partial, out, ostride, acc ? 1 : 0);
  return LAUNCH_OK();
}

template <typename T>
int launch_seg_dot_chain(hipStream_t s, int nseg, int64_t rpp, const T* a, const T* b, double* partial,
                         SegFin prev) {
  if (prev.nseg > kBlock) return AMG_EINVAL;
  hipLaunchKernelGGL(k_seg_dot<T>, dim3(kSegBlocks, nseg), dim3(kBlock), 0, s, rpp, a, b, partial, prev);
  return LAUNCH_OK();
}

int launch_seg_finish(hipStream_t s, SegFin f) {
  if (f.nseg == 0) return AMG_OK;
  hipLaunchKernelGGL(k_seg_finish, dim3((f.nseg + 63) / 64), dim3(64), 0, s, f.nseg, f.partial, f.out, f.ostride,
                     f.acc);
  return LAUNCH_OK();
}

template <typename T>
int launch_loss_seed(hipStream_t s, int64_t n, int64_t rpp, int P, const double* sq, const T* r2, T* g) {
  hipLaunchKernelGGL(k_loss_seed<T>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, rpp, P, sq, r2, g);
  return LAUNCH_OK();
}

int launch_loss_value(hipStream_t s, int P, const double* sq, double* out) {
  hipLaunchKernelGGL(k_loss_value, dim3(1), dim3(64), 0, s, P, sq, out);
  return LAUNCH_OK();
}

template <typename T>
int launch_neg(hipStream_t s, int64_t n, const T* x, T* y) {
  hipLaunchKernelGGL(k_scale_neg<T>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, x, y);
  return LAUNCH_OK();
}

template <typename T>
int launch_prolong_set(hipStream_t s, int64_t n, const int32_t* agg, const T* xc, T* x) {
  hipLaunchKernelGGL(k_prolong_set<T>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, agg, xc, x);
  return LAUNCH_OK();
}

template <typename T>
int launch_restrict_sum(hipStream_t s, int64_t nc, const int32_t* children, const T* x, T* yc) {
  hipLaunchKernelGGL(k_restrict_sum<T>, dim3(grid_for(nc)), dim3(kBlock), 0, s, nc, children, x, yc);
  return LAUNCH_OK();
}

int launch_mlp_fwd(hipStream_t s, int B, const float* W, const float* X, float* Y, float* cache) {
  hipLaunchKernelGGL(k_mlp_fwd, dim3((B + 3) / 4), dim3(256), 0, s, B, W, X, Y, cache);
  return LAUNCH_OK();
}

int launch_mlp_bwd(hipStream_t s, int B, const float* W, const float* X, const float* cache, const float* dY,
                   float* G, float* work) {
  hipLaunchKernelGGL(k_mlp_bwd, dim3((B + 3) / 4), dim3(256), 0, s, B, W, cache, dY, work);
  hipLaunchKernelGGL(k_mlp_grad, dim3((NPARAM + 255) / 256), dim3(256), 0, s, B, X, cache, dY, G, work);
  return LAUNCH_OK();
}

// ---------------------------------------------------------------------------
// mlp_bwd without a caller-supplied workspace: the backward's scratch (dz2, dz1 of up to
// kMlpMaxBatch rows, 128 KB) is this file-scope device array, one copy per GPU, held until
// the process ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in for the symbol): each device's address comes from hipGetSymbolAddress,
// taken once per device with that device current, and is kept here.  Every call on a GPU
// shares that GPU's array, so calls that overlap on one GPU (different streams) race; the
// kernel writes every scratch entry it reads, so nothing needs clearing between calls.
// ---------------------------------------------------------------------------
constexpr int kMlpMaxBatch = 256;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) float scratch[2 * kMlpMaxBatch * NH];

static std::mutex g_scratch_mu;
static float* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (looked up on the first call on each device).
static int scratch_address(float** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return AMG_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return AMG_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return AMG_EHIP;
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return AMG_OK;
}

int launch_mlp_bwd_noalloc(hipStream_t s, int B, const float* W, const float* X, const float* cache,
                           const float* dY, float* G) {
  if (B > kMlpMaxBatch) return AMG_ECAPACITY;
  float* work = nullptr;
  const int rc = scratch_address(&work);
  if (rc != AMG_OK) return rc;
  return launch_mlp_bwd(s, B, W, X, cache, dY, G, work);
}

int launch_adam(hipStream_t s, int n, float* W, const float* G, float* m, float* v, float lr, float b1, float b2,
                float eps, float c1, float c2) {
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, n, W, G, m, v, lr, b1, b2, eps, c1, c2);
  return LAUNCH_OK();
}

int launch_beta_valid(hipStream_t s, int count, int k, const double* beta, int ngrid, int* valid) {
  hipLaunchKernelGGL(k_beta_valid, dim3(count), dim3(256), 0, s, count, k, beta, ngrid, valid);
  return LAUNCH_OK();
}

int launch_learned_beta(hipStream_t s, int P, int L, int k, const BetaRow& tab, const float* y, int ngrid,
                        double* beta, int* valid) {
  hipLaunchKernelGGL(k_learned_beta, dim3(P * L), dim3(256), 0, s, L, k, tab, y, ngrid, beta, valid);
  return LAUNCH_OK();
}

int launch_learned_beta_grad(hipStream_t s, int P, int L, int k, const double* gbeta, const int* valid, float* gy) {
  const int rows = P * (L - 1);
  hipLaunchKernelGGL(k_learned_beta_grad, dim3((rows * 6 + 255) / 256), dim3(256), 0, s, rows, L, k, gbeta, valid,
                     gy);
  return LAUNCH_OK();
}

int mlp_num_params() { return NPARAM; }

int launch_mul(hipStream_t s, int64_t n, const double* a, const double* x, double* y) {
  hipLaunchKernelGGL(k_mul, dim3(grid_for(n)), dim3(kBlock), 0, s, n, a, x, y);
  return LAUNCH_OK();
}

int launch_offdiag_ratio(hipStream_t s, int64_t n, const int32_t* ptr, const int32_t* col, const double* val,
                         const double* minv, double* out) {
  hipLaunchKernelGGL(k_offdiag_ratio, dim3(grid_for(n)), dim3(kBlock), 0, s, n, ptr, col, val, minv, out);
  return LAUNCH_OK();
}

#define INST_T(T)                                                                                          \
  template int launch_seg_dot<T>(hipStream_t, int, int64_t, const T*, const T*, double*, double*, int, bool); \
  template int launch_seg_dot_chain<T>(hipStream_t, int, int64_t, const T*, const T*, double*, SegFin);     \
  template int launch_loss_seed<T>(hipStream_t, int64_t, int64_t, int, const double*, const T*, T*);         \
  template int launch_neg<T>(hipStream_t, int64_t, const T*, T*);                                           \
  template int launch_prolong_set<T>(hipStream_t, int64_t, const int32_t*, const T*, T*);                   \
  template int launch_restrict_sum<T>(hipStream_t, int64_t, const int32_t*, const T*, T*);

INST_T(double)
INST_T(float)

}  // namespace amgp
