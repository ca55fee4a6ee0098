/*
 * Host sanitizer run of the C-ABI's validation paths: every entry point with
 * arguments it must reject, the parameter rules of Lemma 1, Theorems 1-2 and
 * Lemma 5, and -- with no device -- the calls that need one (the Lemma 3
 * coefficients, the copy-in of host-resident matrices) failing cleanly.  Linked against a
 * build of the library whose host code carries AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  Exit status 0 means
 * every expectation held and no sanitizer report was raised.
 */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "entropy.h"

static int failures = 0;

#define EXPECT(cond)                                                          \
  do {                                                                        \
    if (!(cond)) {                                                            \
      fprintf(stderr, "line %d: expectation failed: %s (%s)\n", __LINE__,     \
              #cond, ent_last_error());                                       \
      ++failures;                                                             \
    }                                                                         \
  } while (0)

static ent_matrix dense(int64_t n, int32_t dtype, int64_t ld, const void *v) {
  ent_matrix M;
  memset(&M, 0, sizeof(M));
  M.n = n;
  M.layout = ENT_DENSE;
  M.dtype = dtype;
  M.ld = ld;
  M.values = v;
  return M;
}

int main(void) {
  ent_options o;
  ent_result res;
  memset(&res, 0, sizeof(res));
  ent_options_default(&o);
  EXPECT(o.power_iters == 20 && o.power_trials == 1 && o.u_factor == 6.0);
  EXPECT(ent_version() >= 100);

  /* parameter rules */
  EXPECT(ent_probes_for(0.1, 0.05) == 7378);
  EXPECT(ent_probes_for(0.0, 0.1) < 0);
  EXPECT(ent_degree_taylor(1.0, 0.01, 0.1) == 231);
  EXPECT(ent_degree_chebyshev(1.0, 0.01, 0.1) > 0);
  EXPECT(ent_power_trials_for(0.01) == (int32_t)ceil(4.82 * log(100.0)));
  EXPECT(ent_power_iters_for(5000) == (int32_t)ceil(log(sqrt(20000.0))));
  EXPECT(ent_power_iters_for((int64_t)1 << 40) > 0);

  /* Lemma 3 coefficients (computed on the device), and their argument checks */
  double alpha[65];
  ent_status cs = ent_chebyshev_coeffs(0.0, 1.0, 64, alpha);
  EXPECT(cs == ENT_OK || cs == ENT_EDEVICE);
  cs = ent_chebyshev_coeffs(1e-3, 1.0, 64, alpha);
  EXPECT(cs == ENT_OK || cs == ENT_EDEVICE);
  EXPECT(ent_chebyshev_coeffs(0.5, 0.4, 3, alpha) == ENT_EINVAL);
  EXPECT(ent_chebyshev_coeffs(0.0, 1.0, 0, alpha) == ENT_EINVAL);
  EXPECT(ent_chebyshev_coeffs(0.0, 1.0, 4, NULL) == ENT_EINVAL);

  /* descriptors and options that must be rejected before any device work */
  static double host[16 * 16];
  for (int i = 0; i < 16; ++i) host[i * 16 + i] = 1.0 / 16;
  ent_matrix M = dense(16, ENT_STORE_F64, 16, NULL);
  EXPECT(ent_entropy_estimate(NULL, ENT_CHEBYSHEV, 10, 4, 0, NULL, &res) == ENT_EINVAL);
  EXPECT(ent_entropy_estimate(&M, ENT_CHEBYSHEV, 10, 4, 0, NULL, NULL) == ENT_EINVAL);
  EXPECT(ent_entropy_estimate(&M, ENT_CHEBYSHEV, 10, 4, 0, NULL, &res) == ENT_EINVAL);
  M = dense(0, ENT_STORE_F64, 16, host);
  EXPECT(ent_entropy_estimate(&M, ENT_CHEBYSHEV, 10, 4, 0, NULL, &res) == ENT_EINVAL);
  M = dense(16, ENT_STORE_F64, 8, host);
  EXPECT(ent_entropy_estimate(&M, ENT_CHEBYSHEV, 10, 4, 0, NULL, &res) == ENT_EINVAL);
  M = dense(16, 9, 16, host);
  EXPECT(ent_entropy_estimate(&M, ENT_CHEBYSHEV, 10, 4, 0, NULL, &res) == ENT_EINVAL);
  M = dense(16, ENT_STORE_F64, 16, host);
  M.layout = 7;
  EXPECT(ent_entropy_estimate(&M, ENT_CHEBYSHEV, 10, 4, 0, NULL, &res) == ENT_EINVAL);
  M = dense(16, ENT_STORE_F64, 16, host);
  M.layout = ENT_CSR;
  M.nnz = 16;
  EXPECT(ent_entropy_estimate(&M, ENT_CHEBYSHEV, 10, 4, 0, NULL, &res) == ENT_EINVAL);
  M = dense(16, ENT_STORE_F64, 16, host);
  EXPECT(ent_entropy_estimate(&M, ENT_CHEBYSHEV, 0, 4, 0, NULL, &res) == ENT_EINVAL);
  EXPECT(ent_entropy_estimate(&M, ENT_CHEBYSHEV, 10, 0, 0, NULL, &res) == ENT_EINVAL);
  EXPECT(ent_entropy_estimate(&M, 9, 10, 4, 0, NULL, &res) == ENT_EINVAL);
  ent_options bad = o;
  bad.precision = 7;
  EXPECT(ent_entropy_estimate(&M, ENT_CHEBYSHEV, 10, 4, 0, &bad, &res) == ENT_EINVAL);
  bad = o;
  bad.probe_dist = 5;
  EXPECT(ent_entropy_estimate(&M, ENT_CHEBYSHEV, 10, 4, 0, &bad, &res) == ENT_EINVAL);
  bad = o;
  bad.u_fixed = 0.1;
  bad.cutoff = 0.2;
  EXPECT(ent_entropy_estimate(&M, ENT_CHEBYSHEV, 10, 4, 0, &bad, &res) == ENT_EINVAL);
  bad = o;
  bad.flags = ENT_FLAG_CLENSHAW;
  EXPECT(ent_entropy_estimate(&M, ENT_TAYLOR, 10, 4, 0, &bad, &res) == ENT_EINVAL);
  M = dense(16, ENT_STORE_C128, 16, host);
  M.layout = ENT_CSR;
  EXPECT(ent_entropy_estimate(&M, ENT_CHEBYSHEV, 10, 4, 0, NULL, &res) == ENT_EUNSUPPORTED);
  M = dense(16, ENT_STORE_C64, 16, host);
  EXPECT(ent_entropy_estimate(&M, ENT_RANDPROJ, 10, 4, 0, NULL, &res) == ENT_EUNSUPPORTED);

  /* host-resident R: copied in before use; with no device the copy fails
     and the result is left untouched */
  res.entropy = 123.0;
  M = dense(16, ENT_STORE_F64, 16, host);
  const ent_status st = ent_entropy_estimate(&M, ENT_CHEBYSHEV, 10, 4, 0, NULL, &res);
  EXPECT(st == ENT_OK || st == ENT_EDEVICE);
  if (st != ENT_OK) EXPECT(res.entropy == 123.0);
  double per[4], mom[11 * 4];
  (void)ent_entropy_estimate_detail(&M, ENT_CHEBYSHEV, 10, 4, 0, NULL, &res, per, mom);
  (void)ent_entropy_estimate_noalloc(&M, ENT_TAYLOR, 10, 4, 0, NULL, &res, per, NULL);
  double p1 = 7.0;
  (void)ent_power_method(&M, 5, 1, 0, NULL, &p1);
  EXPECT(ent_power_method(NULL, 5, 1, 0, NULL, &p1) == ENT_EINVAL);

  /* batches and graphs */
  ent_graph gr = NULL;
  EXPECT(ent_entropy_estimate_batched(NULL, 2, ENT_CHEBYSHEV, 10, 4, 0, NULL, &res) == ENT_EINVAL);
  ent_matrix two[2] = {dense(16, ENT_STORE_F64, 16, host), dense(16, ENT_STORE_F64, 16, host)};
  EXPECT(ent_graph_create(two, 0, ENT_CHEBYSHEV, 10, 4, 0, NULL, &gr) == ENT_EINVAL);
  EXPECT(ent_graph_create(two, 2, ENT_CHEBYSHEV, 10, 4, 0, NULL, NULL) == ENT_EINVAL);
  EXPECT(ent_graph_launch(NULL, &res) == ENT_EINVAL);
  EXPECT(ent_graph_tile_rows(NULL) <= 0);
  EXPECT(ent_graph_window_bytes(NULL) == 0);
  EXPECT(ent_graph_workspace_bytes(NULL) == 0);
  (void)ent_graph_destroy(NULL);

  /* MLP and selector arguments */
  EXPECT(ent_mlp_nparams() > 0);
  EXPECT(ent_mlp_forward(NULL, NULL, 4, NULL, NULL) == ENT_EINVAL);
  EXPECT(ent_selector_load(NULL, 3) == ENT_EINVAL);
  float feat[16], outp[2];
  M = dense(16, ENT_STORE_C128, 16, host);
  EXPECT(ent_selector_features(&M, 0, NULL, feat, outp) == ENT_EUNSUPPORTED);

  /* workspace and timing controls */
  EXPECT(ent_set_workspace_limit((size_t)1 << 30) == ENT_OK);
  EXPECT(ent_set_workspace_limit(0) == ENT_OK);
  (void)ent_workspace_bytes();
  (void)ent_release_workspace();
  EXPECT(ent_timing_enable(1) == ENT_OK);
  ent_timing tm;
  (void)ent_last_timing(&tm);
  EXPECT(ent_timing_enable(0) == ENT_OK);
  EXPECT(ent_last_error() != NULL);

  if (failures) {
    fprintf(stderr, "%d expectation(s) failed\n", failures);
    return 1;
  }
  printf("abi sanitizer run: ok\n");
  return 0;
}
