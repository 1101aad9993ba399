// Dense float64 kernels for the coarsest level.
//
// Setup (once): blocked right-looking Cholesky A = L L^T with 64x64 tiles, the
// block triangular inverse X = L^{-1}, and A^{-1} = X^T X.  The trailing
// updates, panel solves and products are matrix-matrix products on the FP64
// matrix cores (v_mfma_f64_16x16x4f64); the 64x64 diagonal tiles are factored
// and inverted inside one workgroup in LDS.
// Per cycle: x = A^{-1} b, one dense matrix-vector product per problem (the
// forward and back substitutions with L, applied through the inverse formed
// at setup: same bytes, no dependent sweep).
#include <vector>

#include "internal.h"

namespace amgp {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int TM = 64;  // output tile of a workgroup (TM x TM)
constexpr int TK = 16;  // k-chunk staged in LDS

// C = alpha op(A) op(B) + beta C for M, N, K multiples of 64 (row-major, leading dims, batch strides).
// 256 threads = 4 waves in a 2x2 arrangement, each wave a 32x32 sub-tile of four 16x16 MFMA accumulators.
// MFMA 16x16x4 f64 operand layout: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// accumulator element r of lane l is D[l / 16 + 4 r][l % 16] (checked on gfx950).
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, double alpha, const double* __restrict__ A,
                                              int lda, long long sA, const double* __restrict__ B, int ldb,
                                              long long sB, double beta, double* __restrict__ C, int ldc,
                                              long long sC) {
  __shared__ double As[TM][TK + 1];
  __shared__ double Bs[TK][TM + 1];
  const int bz = blockIdx.z;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TM;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  dbl4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += TK) {
    // stage A[m0:m0+64, k0:k0+16] and B[k0:k0+16, n0:n0+64]: 1024 elements each, 4 per thread
    for (int e = t; e < TM * TK; e += 256) {
      int mm, kk;
      if (TA) {  // A^T: consecutive threads walk m (contiguous in memory)
        mm = e % TM;
        kk = e / TM;
        As[mm][kk] = A[(long long)(k0 + kk) * lda + (m0 + mm)];
      } else {
        kk = e % TK;
        mm = e / TK;
        As[mm][kk] = A[(long long)(m0 + mm) * lda + (k0 + kk)];
      }
      int nn, kb;
      if (TB) {
        kb = e % TK;
        nn = e / TK;
        Bs[kb][nn] = B[(long long)(n0 + nn) * ldb + (k0 + kb)];
      } else {
        nn = e % TM;
        kb = e / TM;
        Bs[kb][nn] = B[(long long)(k0 + kb) * ldb + (n0 + nn)];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < TK; k4 += 4) {
      double av[2], bv[2];
      for (int a = 0; a < 2; ++a) av[a] = As[wr * 32 + a * 16 + (lane & 15)][k4 + (lane >> 4)];
      for (int b = 0; b < 2; ++b) bv[b] = Bs[k4 + (lane >> 4)][wc * 32 + b * 16 + (lane & 15)];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr * 32 + a * 16 + (lane >> 4) + 4 * r;
        const int col = n0 + wc * 32 + b * 16 + (lane & 15);
        double* c = C + (long long)row * ldc + col;
        const double v = alpha * acc[a][b][r];
        *c = (beta == 0.0) ? v : v + beta * (*c);
      }
}

// Factor the 64x64 diagonal tile at (k, k) of every batch matrix in place
// (lower triangle := L_kk, upper := 0) and write inv(L_kk) to dinv.
__global__ __launch_bounds__(256) void k_potrf_tile(double* __restrict__ Ab, long long sA, int ld, int k,
                                                    double* __restrict__ dinv, long long sD,
                                                    int* __restrict__ flag) {
  __shared__ double T[TM][TM + 1];
  __shared__ double X[TM][TM + 1];
  double* A = Ab + blockIdx.x * sA + (long long)k * TM * ld + (long long)k * TM;
  double* D = dinv + blockIdx.x * sD;
  const int t = threadIdx.x;
  for (int e = t; e < TM * TM; e += 256) T[e / TM][e % TM] = A[(long long)(e / TM) * ld + (e % TM)];
  __syncthreads();
  __shared__ int bad;
  if (t == 0) bad = 0;
  __syncthreads();
  for (int c = 0; c < TM; ++c) {
    if (t == 0) {
      const double d = T[c][c];
      if (!(d > 0.0)) bad = 1;
      T[c][c] = sqrt(d > 0.0 ? d : 1.0);
    }
    __syncthreads();
    const double piv = T[c][c];
    for (int i = c + 1 + t; i < TM; i += 256) T[i][c] /= piv;
    __syncthreads();
    // trailing update of the lower part: T[i][j] -= T[i][c] T[j][c], c < j <= i
    for (int e = t; e < TM * TM; e += 256) {
      const int i = e / TM, j = e % TM;
      if (j > c && i >= j) T[i][j] -= T[i][c] * T[j][c];
    }
    __syncthreads();
  }
  if (t == 0 && bad) flag[F_NOTSPD] = 1;
  // inverse of the lower-triangular tile, one column per thread: L X = I
  if (t < TM) {
    const int c = t;
    for (int i = 0; i < TM; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int m = c; m < i; ++m) s -= T[i][m] * X[m][c];
      X[i][c] = (i < c) ? 0.0 : s / T[i][i];
    }
  }
  __syncthreads();
  for (int e = t; e < TM * TM; e += 256) {
    const int i = e / TM, j = e % TM;
    A[(long long)i * ld + j] = (j <= i) ? T[i][j] : 0.0;
    D[(long long)i * TM + j] = X[i][j];
  }
}

// zero the strictly upper triangle (after the factorisation, whose updates also touch it)
__global__ void k_zero_upper(long long total, int np, double* __restrict__ A) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const long long q = e % ((long long)np * np);
  const int i = (int)(q / np), j = (int)(q % np);
  if (j > i) A[e] = 0.0;
}

// copy the 64x64 tile dinv into X at tile (i, i)
__global__ void k_put_tile(const double* __restrict__ D, long long sD, double* __restrict__ X, long long sX, int ld,
                           int i) {
  const int t = threadIdx.x;
  const double* d = D + blockIdx.x * sD;
  double* x = X + blockIdx.x * sX + (long long)i * TM * ld + (long long)i * TM;
  for (int e = t; e < TM * TM; e += 256) x[(long long)(e / TM) * ld + (e % TM)] = d[e];
}

// Tile q = J (J + 1) / 2 + I of the packed lower triangle holds block (J, I), J >= I.
__device__ __forceinline__ void tile_of(int q, int& J, int& I) {
  J = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
  while ((J + 1) * (J + 2) / 2 <= q) ++J;
  while (J * (J + 1) / 2 > q) --J;
  I = q - J * (J + 1) / 2;
}

// Copy the lower 64x64 blocks of each np x np matrix into contiguous 32 KB tiles.
__global__ __launch_bounds__(256) void k_pack_tiles(int64_t np, int ntiles, const double* __restrict__ dense,
                                                    double* __restrict__ packed) {
  const int q = blockIdx.x, p = blockIdx.y;
  int J, I;
  tile_of(q, J, I);
  const double* src = dense + (int64_t)p * np * np + (int64_t)J * TM * np + (int64_t)I * TM;
  double* dst = packed + ((int64_t)p * ntiles + q) * TM * TM;
  for (int e = threadIdx.x; e < TM * TM; e += 256) dst[e] = src[(int64_t)(e / TM) * np + e % TM];
}

// x = A^{-1} b for the symmetric dense inverse, reading only its lower 64x64
// blocks, each exactly once, from the packed contiguous tiles.  Tile (J, I) of
// problem p is handled by one wavefront that streams its 64 rows (one 512 B
// load each): it contributes A_JI b_I to rows of block J (row sums, through an
// LDS transpose) and, when J > I, A_JI^T b_J to rows of block I (column sums,
// in registers).  The 64-vectors land in part[p][row block][column block]; a
// second kernel sums them in a fixed order.  b and x are level vectors (nl rows
// per problem); padding rows read as 0.
// RB: rows of the tile transposed through LDS at a time (RB x (TM + 1) doubles of LDS per
// wavefront); every row sum still adds its 64 products in column order.
template <typename T, int RB = TM>
__global__ __launch_bounds__(TM) void k_symv_tiles(int nb, int ntiles, int64_t nl, const double* __restrict__ packed,
                                                   const T* __restrict__ b, double* __restrict__ part) {
  __shared__ double prod[RB][TM + 1];
  const int q = blockIdx.x, p = blockIdx.y, lane = threadIdx.x;
  int J, I;
  tile_of(q, J, I);
  const T* bp = b + (int64_t)p * nl;
  const int64_t ri = (int64_t)I * TM + lane, rj = (int64_t)J * TM + lane;
  const double bI = ri < nl ? (double)bp[ri] : 0.0;
  const double bJ = rj < nl ? (double)bp[rj] : 0.0;
  const double* src = packed + ((int64_t)p * ntiles + q) * TM * TM + lane;
  double col = 0.0, row = 0.0;
  // the tiles (67 MB at 4096 rows) are read once per cycle with streaming loads, so that they do
  // not displace the fine level's matrix and vectors from the caches (measured at 128^3: 18.3 to
  // 16.2 us here, and the whole PCG solve 9.20 to 9.00 ms)
  for (int a0 = 0; a0 < TM; a0 += RB) {
#pragma unroll 16
    for (int a = 0; a < RB; ++a) {
      const double v = __builtin_nontemporal_load(src + (a0 + a) * TM);
      col += v * __shfl(bJ, a0 + a, TM);
      prod[a][lane] = v * bI;
    }
    __syncthreads();
    if (lane >= a0 && lane < a0 + RB) {
#pragma unroll 8
      for (int c = 0; c < TM; ++c) row += prod[lane - a0][c];
    }
    __syncthreads();
  }
  double* out = part + (int64_t)p * nb * nb * TM;
  out[((int64_t)J * nb + I) * TM + lane] = row;
  if (J > I) out[((int64_t)I * nb + J) * TM + lane] = col;
}

// x_I = sum_J part[I][J]: four waves each sum a quarter of the J range, combined in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void k_symv_sum(int nb, int64_t nl, const double* __restrict__ part,
                                                  T* __restrict__ x) {
  __shared__ double sm[4][TM];
  const int p = blockIdx.y, I = blockIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double* in = part + (int64_t)p * nb * nb * TM + (int64_t)I * nb * TM;
  const int per = (nb + 3) / 4;
  double s = 0.0;
  for (int J = w * per; J < min(nb, (w + 1) * per); ++J) s += in[(int64_t)J * TM + lane];
  sm[w][lane] = s;
  __syncthreads();
  if (w == 0) {
    const double tot = ((sm[0][lane] + sm[1][lane]) + sm[2][lane]) + sm[3][lane];
    const int64_t row = (int64_t)I * TM + lane;
    if (row < nl) x[(int64_t)p * nl + row] = (T)tot;
  }
}

template <bool TA, bool TB>
int gemm(hipStream_t s, int batch, int M, int N, int K, double alpha, const double* A, int lda, long long sA,
         const double* B, int ldb, long long sB, double beta, double* C, int ldc, long long sC) {
  if (M <= 0 || N <= 0 || K <= 0) return AMG_OK;
  dim3 grid(N / TM, M / TM, batch);
  hipLaunchKernelGGL((k_gemm<TA, TB>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc,
                     sC);
  return hipGetLastError() == hipSuccess ? AMG_OK : AMG_EHIP;
}

}  // namespace

int dense_spd_inverse(hipStream_t s, int nbatch, int64_t np64, double* dense, int* flag) {
  const int np = (int)np64;
  const int nb = np / TM;
  const long long sA = (long long)np * np;
  double* dinv = nullptr;  // inverse diagonal tiles [batch][nb][64][64]
  double* X = nullptr;     // L^{-1}
  double* T = nullptr;     // scratch [batch][64 * np]: a 64 x np block row or an np x 64 panel
  if (hipMalloc(&dinv, sizeof(double) * nbatch * nb * TM * TM) != hipSuccess) return AMG_ENOMEM;
  if (hipMalloc(&X, sizeof(double) * nbatch * sA) != hipSuccess) return AMG_ENOMEM;
  if (hipMalloc(&T, sizeof(double) * nbatch * (long long)TM * np) != hipSuccess) return AMG_ENOMEM;
  const long long sD = (long long)nb * TM * TM;
  // 1. Cholesky, right looking
  for (int k = 0; k < nb; ++k) {
    hipLaunchKernelGGL(k_potrf_tile, dim3(nbatch), dim3(256), 0, s, dense, sA, np, k, dinv + (long long)k * TM * TM,
                       sD, flag);
    AMGP_HIP(hipGetLastError());
    const int rem = np - (k + 1) * TM;
    if (rem <= 0) break;
    double* panel = dense + (long long)(k + 1) * TM * np + (long long)k * TM;  // A[k+1:, k]
    // panel := panel inv(L_kk)^T, computed into the scratch T (rem x 64, ld 64) and copied back
    AMGP_TRY((gemm<false, true>(s, nbatch, rem, TM, TM, 1.0, panel, np, sA, dinv + (long long)k * TM * TM, TM, sD,
                                0.0, T, TM, (long long)TM * np)));
    for (int p = 0; p < nbatch; ++p)
      AMGP_HIP(hipMemcpy2DAsync(panel + p * sA, sizeof(double) * np, T + p * (long long)TM * np, sizeof(double) * TM,
                                sizeof(double) * TM, rem, hipMemcpyDeviceToDevice, s));
    // trailing update A[k+1:, k+1:] -= panel panel^T
    double* trail = dense + (long long)(k + 1) * TM * np + (long long)(k + 1) * TM;
    AMGP_TRY((gemm<false, true>(s, nbatch, rem, rem, TM, -1.0, panel, np, sA, panel, np, sA, 1.0, trail, np, sA)));
  }
  {
    const long long total = (long long)nbatch * sA;
    hipLaunchKernelGGL(k_zero_upper, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total, np, dense);
    AMGP_HIP(hipGetLastError());
  }
  // 2. X = L^{-1} by block rows: X[i, 0:i] = -inv(L_ii) (L[i, 0:i] X[0:i, 0:i]), X[i, i] = inv(L_ii)
  AMGP_HIP(hipMemsetAsync(X, 0, sizeof(double) * nbatch * sA, s));
  for (int i = 0; i < nb; ++i) {
    hipLaunchKernelGGL(k_put_tile, dim3(nbatch), dim3(256), 0, s, dinv + (long long)i * TM * TM, sD, X, sA, np, i);
    AMGP_HIP(hipGetLastError());
    if (i == 0) continue;
    const int w = i * TM;
    // T[0:64, 0:w] = L[i*64:(i+1)*64, 0:w] X[0:w, 0:w]
    AMGP_TRY((gemm<false, false>(s, nbatch, TM, w, w, 1.0, dense + (long long)i * TM * np, np, sA, X, np, sA, 0.0,
                                 T, np, (long long)TM * np)));
    // X[i rows, 0:w] = -inv(L_ii) T
    AMGP_TRY((gemm<false, false>(s, nbatch, TM, w, TM, -1.0, dinv + (long long)i * TM * TM, TM, sD, T, np,
                                 (long long)TM * np, 0.0, X + (long long)i * TM * np, np, sA)));
  }
  // 3. A^{-1} = X^T X (overwrites dense)
  AMGP_TRY((gemm<true, false>(s, nbatch, np, np, np, 1.0, X, np, sA, X, np, sA, 0.0, dense, np, sA)));
  AMGP_HIP(hipStreamSynchronize(s));
  hipFree(dinv);
  hipFree(X);
  hipFree(T);
  return AMG_OK;
}

// Half a tile through LDS at a time (16.6 KB per wavefront instead of 33 KB, so twice the
// wavefronts per CU): 4096 rows 21.8 -> 19.7 us, 32 stacked problems of 4096 rows (2.2 GB of
// tiles) 428 -> 391 us; a quarter (16 rows) is slower (30.6 and 565 us).
constexpr int kSymvRows = 32;

template <typename T>
int launch_coarse_symv(hipStream_t s, int nbatch, int64_t nl, int64_t np, const double* ainv, const T* b, T* x,
                       double* part) {
  const int nb = (int)(np / TM), ntiles = nb * (nb + 1) / 2;
  hipLaunchKernelGGL((k_symv_tiles<T, kSymvRows>), dim3(ntiles, nbatch), dim3(TM), 0, s, nb, ntiles, nl, ainv, b, part);
  hipLaunchKernelGGL(k_symv_sum<T>, dim3(nb, nbatch), dim3(256), 0, s, nb, nl, (const double*)part, x);
  return hipGetLastError() == hipSuccess ? AMG_OK : AMG_EHIP;
}
template int launch_coarse_symv<double>(hipStream_t, int, int64_t, int64_t, const double*, const double*, double*,
                                        double*);
template int launch_coarse_symv<float>(hipStream_t, int, int64_t, int64_t, const double*, const float*, float*,
                                       double*);

int pack_lower_tiles(hipStream_t s, int nbatch, int64_t np, const double* dense, double** packed) {
  const int nb = (int)(np / TM), ntiles = nb * (nb + 1) / 2;
  *packed = nullptr;
  if (hipMalloc(packed, sizeof(double) * (size_t)nbatch * ntiles * TM * TM) != hipSuccess) return AMG_ENOMEM;
  hipLaunchKernelGGL(k_pack_tiles, dim3(ntiles, nbatch), dim3(256), 0, s, np, ntiles, dense, *packed);
  return hipGetLastError() == hipSuccess ? AMG_OK : AMG_EHIP;
}

}  // namespace amgp
