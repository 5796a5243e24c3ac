/* A plain C99 user of the library's C ABI: host-side calls only (parameter
 * validation, buffer sizes, argument checks), so it runs without a GPU.
 * Exit status 0 when every result is as the header documents. */
#include <stdio.h>
#include <string.h>

#include "chromo_lbm.h"

static int fails = 0;
#define CHECK(cond)                                      \
  do {                                                   \
    if (!(cond)) {                                       \
      fprintf(stderr, "failed: %s (line %d)\n", #cond, __LINE__); \
      ++fails;                                           \
    }                                                    \
  } while (0)

int main(void) {
  lbm_params p;
  memset(&p, 0, sizeof p);
  p.nx = 128;
  p.ny = 96;
  p.storage = LBM_STORAGE_F32;
  for (int k = 0; k < 4; ++k) p.stencil[k] = 3;
  p.rho0_R = 1.0;
  p.rho0_B = 0.1;
  p.alpha_R = 0.95; /* (1 - alpha_B) = Lambda (1 - alpha_R), Lambda = 10 */
  p.alpha_B = 0.5;
  p.nu_R = p.nu_B = 1.0 / 6.0;
  p.lambda6 = 1.4;
  p.lambda7 = 1.2;
  p.eps_n = 1e-6;
  p.beta = 0.67;
  p.sigma = 0.01;
  CHECK(lbm_validate_params(&p) == LBM_OK);
  CHECK(lbm_pops_elems(&p) == (size_t)18 * 128 * 96);
  CHECK(lbm_pops_bytes(&p) == (size_t)4 * 18 * 128 * 96);
  CHECK(lbm_workspace_bytes(&p) > 0);
  CHECK(lbm_adjoint_workspace_bytes(&p) >= (size_t)39 * 4 * 128 * 96);
  p.storage = LBM_STORAGE_F16_OFS;
  CHECK(lbm_pops_bytes(&p) == (size_t)4 * 10 * 128 * 96);
  CHECK(lbm_adjoint_workspace_bytes(&p) == 0); /* no adjoint of the 16-bit formats */
  p.storage = LBM_STORAGE_F32;
  p.stencil[2] = 2; /* radius not in {1, 3} */
  CHECK(lbm_validate_params(&p) == LBM_EINVAL);
  CHECK(strlen(lbm_last_error()) > 0);
  p.stencil[2] = 3;
  p.alpha_B = 0.6; /* density-ratio relation violated */
  CHECK(lbm_validate_params(&p) == LBM_EINVAL);

  lbm_handle* h = NULL;
  CHECK(lbm_init(NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL, &h) == LBM_EINVAL);
  CHECK(lbm_step(NULL, 1, NULL, NULL) == LBM_EINVAL);
  CHECK(lbm_step_into(NULL, NULL, 0, NULL, NULL) == LBM_EINVAL);
  CHECK(lbm_adjoint_steps(NULL, 0, NULL, NULL, NULL, NULL, 0, NULL, NULL, NULL) == LBM_EINVAL);
  CHECK(lbm_set_cu_budget(NULL, 0, 0) == LBM_EINVAL);
  hipStream_t s = NULL;
  CHECK(lbm_partition_stream(4, 8, &s) == LBM_EINVAL);
  CHECK(s == NULL);
  CHECK(lbm_step_count(NULL) == -1);
  lbm_destroy(NULL);
  printf("c consumer: %d failed checks\n", fails);
  return fails != 0;
}
