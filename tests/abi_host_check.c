/* Host-side check of the C ABI's argument validation, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host code (the device code is not instrumented).
 * Every call here returns before any HIP call, so no GPU is needed. */
#include <stdio.h>
#include <string.h>

#include "amgpoly.h"

#define EXPECT(cond)                                                  \
  do {                                                                \
    if (!(cond)) {                                                    \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      return 1;                                                       \
    }                                                                 \
  } while (0)

int main(void) {
  amg_handle* h = (amg_handle*)0x1;
  amg_opts o;
  memset(&o, 0, sizeof(o));
  o.nx = o.ny = o.nz = 4;
  EXPECT(amg_setup(64, 64, NULL, NULL, NULL, &o, NULL, &h) == AMG_EINVAL && h == NULL);
  EXPECT(amg_setup(64, 64, NULL, NULL, NULL, &o, NULL, NULL) == AMG_EINVAL);
  EXPECT(amg_destroy(NULL) == AMG_OK);
  EXPECT(amg_num_levels(NULL, NULL) == AMG_EINVAL);
  EXPECT(amg_level_info(NULL, 0, NULL, NULL) == AMG_EINVAL);
  double beta[AMG_MAX_DEGREE + 1];
  for (int k = 1; k <= AMG_MAX_DEGREE; ++k) {
    EXPECT(amg_default_beta(k, beta) == AMG_OK);
    double a = 0.0;
    EXPECT(amg_default_astar(k, &a) == AMG_OK && a > 0.0 && a < 1.0);
  }
  EXPECT(amg_default_beta(0, beta) == AMG_EINVAL);
  EXPECT(amg_default_beta(AMG_MAX_DEGREE + 1, beta) == AMG_EINVAL);
  EXPECT(amg_default_astar(AMG_MAX_DEGREE + 1, beta) == AMG_EINVAL);
  int it = 0;
  double rel = 0.0;
  EXPECT(pcg_solve(NULL, 2, 4, NULL, NULL, 1, 1e-8, 10, 0, &it, &rel, NULL, NULL) == AMG_EINVAL);
  EXPECT(pcg_solve_smoother(NULL, 2, 4, NULL, NULL, 1, 1e-8, 10, 0, &it, &rel, NULL, NULL) == AMG_EINVAL);
  EXPECT(smoother_apply(NULL, 0, 2, 4, NULL, NULL, 1, NULL) == AMG_EINVAL);
  EXPECT(vcycle_apply(NULL, 2, 4, NULL, NULL, NULL) == AMG_EINVAL);
  EXPECT(mlp_num_params() == 5126);
  for (int c = -8; c <= 1; ++c) EXPECT(amg_strerror(c) != NULL && strlen(amg_strerror(c)) > 0);
  printf("host ABI checks passed\n");
  return 0;
}
