/* A plain C caller of the library on the GPU, with no Python or torch in the process: reads a
 * CSR matrix and a right-hand side written by the test, moves them to the device with the HIP
 * runtime, and runs the hot path through the C ABI (setup, one smoother application, one
 * V-cycle, PCG), writing the results back as raw float64 files for the test to compare with the
 * oracle.
 *
 * usage: c_driver DIR NX NY NZ
 *   DIR/A.bin  int64 n, int64 nnz, int32 row_ptr[n + 1], int32 col[nnz], float64 val[nnz]
 *   DIR/b.bin  float64 b[n]
 * writes DIR/smooth.bin (optimal 4th kind, degree 4, from x = 0), DIR/vcycle.bin (optimal 1st
 * kind, degree 3), DIR/pcg.bin (optimal 4th kind, degree 4, rtol 1e-8), and prints
 * "levels L iters I relres R". */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "amgpoly.h"

#define HIP_OK(call)                                                          \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));      \
      exit(2);                                                                \
    }                                                                         \
  } while (0)

#define AMG_CALL(call)                                                        \
  do {                                                                        \
    int rc_ = (call);                                                         \
    if (rc_ != AMG_OK) {                                                      \
      fprintf(stderr, "%s failed: %s\n", #call, amg_strerror(rc_));          \
      exit(3);                                                                \
    }                                                                         \
  } while (0)

static void* read_exact(FILE* f, size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (!p || fread(p, 1, bytes, f) != bytes) {
    fprintf(stderr, "short read\n");
    exit(4);
  }
  return p;
}

static FILE* open_in(const char* dir, const char* name, const char* mode) {
  char path[4096];
  snprintf(path, sizeof(path), "%s/%s", dir, name);
  FILE* f = fopen(path, mode);
  if (!f) {
    fprintf(stderr, "cannot open %s\n", path);
    exit(4);
  }
  return f;
}

static void write_result(const char* dir, const char* name, const double* d_x, int64_t n) {
  double* h = (double*)malloc(sizeof(double) * (size_t)n);
  HIP_OK(hipMemcpy(h, d_x, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost));
  FILE* f = open_in(dir, name, "wb");
  if (fwrite(h, sizeof(double), (size_t)n, f) != (size_t)n) exit(4);
  fclose(f);
  free(h);
}

int main(int argc, char** argv) {
  if (argc != 5) {
    fprintf(stderr, "usage: %s DIR NX NY NZ\n", argv[0]);
    return 1;
  }
  const char* dir = argv[1];
  FILE* fa = open_in(dir, "A.bin", "rb");
  int64_t* head = (int64_t*)read_exact(fa, 2 * sizeof(int64_t));
  const int64_t n = head[0], nnz = head[1];
  int32_t* row_ptr = (int32_t*)read_exact(fa, sizeof(int32_t) * (size_t)(n + 1));
  int32_t* col = (int32_t*)read_exact(fa, sizeof(int32_t) * (size_t)nnz);
  double* val = (double*)read_exact(fa, sizeof(double) * (size_t)nnz);
  fclose(fa);
  FILE* fb = open_in(dir, "b.bin", "rb");
  double* b = (double*)read_exact(fb, sizeof(double) * (size_t)n);
  fclose(fb);

  int32_t *d_ptr, *d_col;
  double *d_val, *d_b, *d_x;
  HIP_OK(hipMalloc((void**)&d_ptr, sizeof(int32_t) * (size_t)(n + 1)));
  HIP_OK(hipMalloc((void**)&d_col, sizeof(int32_t) * (size_t)nnz));
  HIP_OK(hipMalloc((void**)&d_val, sizeof(double) * (size_t)nnz));
  HIP_OK(hipMalloc((void**)&d_b, sizeof(double) * (size_t)n));
  HIP_OK(hipMalloc((void**)&d_x, sizeof(double) * (size_t)n));
  HIP_OK(hipMemcpy(d_ptr, row_ptr, sizeof(int32_t) * (size_t)(n + 1), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_col, col, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_val, val, sizeof(double) * (size_t)nnz, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_b, b, sizeof(double) * (size_t)n, hipMemcpyHostToDevice));

  amg_opts o;
  memset(&o, 0, sizeof(o));
  o.nx = atoi(argv[2]);
  o.ny = atoi(argv[3]);
  o.nz = atoi(argv[4]);
  o.nbatch = 1;
  o.precision = AMG_FP64;
  amg_handle* h = NULL;
  AMG_CALL(amg_setup(n, nnz, d_ptr, d_col, d_val, &o, NULL, &h));
  /* the library keeps its own copy of A */
  HIP_OK(hipFree(d_ptr));
  HIP_OK(hipFree(d_col));
  HIP_OK(hipFree(d_val));
  int levels = 0;
  AMG_CALL(amg_num_levels(h, &levels));

  AMG_CALL(smoother_apply(h, 0, AMG_OPTCHEB4, 4, d_b, d_x, 1, NULL));
  HIP_OK(hipDeviceSynchronize());
  write_result(dir, "smooth.bin", d_x, n);

  AMG_CALL(vcycle_apply(h, AMG_OPTCHEB1, 3, d_b, d_x, NULL));
  HIP_OK(hipDeviceSynchronize());
  write_result(dir, "vcycle.bin", d_x, n);

  int iters = 0;
  double relres = 0.0;
  AMG_CALL(pcg_solve(h, AMG_OPTCHEB4, 4, d_b, d_x, 1, 1e-8, 1000, 0, &iters, &relres, NULL, NULL));
  write_result(dir, "pcg.bin", d_x, n);

  AMG_CALL(amg_destroy(h));
  HIP_OK(hipFree(d_b));
  HIP_OK(hipFree(d_x));
  printf("levels %d iters %d relres %.17g\n", levels, iters, relres);
  free(head);
  free(row_ptr);
  free(col);
  free(val);
  free(b);
  return 0;
}
