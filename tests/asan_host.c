/* Host-side entry points of the C-ABI library under AddressSanitizer (built
 * with the sanitizer on the host pass only): structure sizes, tile counts,
 * workspace sizing over a spread of batch shapes and capacities, and the
 * context calls' error paths.  Exit status 0 when every call behaves. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "nsplat.h"

static int fails = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++fails;                                                    \
    }                                                             \
  } while (0)

int main(void) {
  CHECK(nsplat_abi_version() == NSPLAT_ABI_VERSION);
  int32_t hw[8] = {512, 512, 100, 37, 1, 1, 1024, 768};
  nsplat_scenes sc;
  memset(&sc, 0, sizeof sc);
  sc.n_scenes = 4;
  sc.hw_host = hw;
  const int64_t t16 = nsplat_num_tiles(&sc, 16);
  CHECK(t16 == 32 * 32 + 7 * 3 + 1 + 64 * 48);
  CHECK(nsplat_num_tiles(&sc, 8) > t16 && nsplat_num_tiles(&sc, 32) < t16);
  sc.n_scenes = 0;
  CHECK(nsplat_num_tiles(&sc, 16) == 0);
  sc.n_scenes = 4;
  /* workspace sizes grow with every capacity and with the batch shape */
  nsplat_curves cv;
  memset(&cv, 0, sizeof cv);
  nsplat_params pr;
  memset(&pr, 0, sizeof pr);
  pr.delta_c = 10.0f;
  pr.delta_b = 0.5f;
  pr.rho = 2.0f;
  pr.eta = 1.5f;
  pr.gamma = 5.0f;
  pr.nl_factor = 3.0f;
  pr.fill_pad = 0.1f;
  pr.h = 1.0f;
  pr.k_sigma = 6.0f;
  pr.alpha_max = 0.99f;
  pr.eps_T = 1e-6f;
  pr.delta_a = 0.25f;
  pr.kappa = 4;
  pr.tile = 16;
  pr.batch = 64;
  size_t prev = 0;
  for (int n = 0; n <= 4096; n = n ? 4 * n : 1) {
    cv.n_curves = n;
    cv.n_keys = 8 * n;
    cv.n_taus = 8 * n;
    cv.channels = 3;
    nsplat_caps caps = {(int64_t)1000 * n, (int64_t)3000 * n, (int64_t)200 * n};
    const size_t b = nsplat_workspace_size(&cv, &sc, &pr, &caps);
    CHECK(b >= prev);
    prev = b;
    nsplat_caps big = caps;
    big.pairs *= 2;
    CHECK(nsplat_workspace_size(&cv, &sc, &pr, &big) > b || n == 0);
  }
  /* contexts: a bad device index fails with a message, NULL is tolerated */
  nsplat_ctx* ctx = NULL;
  CHECK(nsplat_create(&ctx, -1) != NSPLAT_OK);
  CHECK(ctx != NULL && strlen(nsplat_last_error(ctx)) > 0);  /* the failed context carries the message */
  CHECK(nsplat_destroy(ctx) == NSPLAT_OK);
  ctx = NULL;
  CHECK(nsplat_create(NULL, 0) != NSPLAT_OK);
  CHECK(nsplat_last_error(NULL) != NULL);
  CHECK(nsplat_destroy(NULL) == NSPLAT_OK);
  /* device 0: succeeds only where a device exists; either way the context
     (with its message on failure) is the caller's to destroy */
  (void)nsplat_create(&ctx, 0);
  CHECK(ctx != NULL);
  CHECK(nsplat_destroy(ctx) == NSPLAT_OK);
  printf("asan host driver: %d failed checks\n", fails);
  return fails ? 1 : 0;
}
