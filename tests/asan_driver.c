/* Host-side driver for the AddressSanitizer build of the library's host code
 * (tests/test_host_asan_cpu.py).  It runs on a machine without a GPU and
 * walks the paths that need no device: defaults, the lattice tables,
 * parameter validation of single lattices and ensembles, NULL arguments of
 * every entry point, the error strings, and the no-device error of
 * lb_create.  Exit status 0 when every expectation holds; the sanitizer
 * aborts the run on any invalid host memory access or leak. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "lb.h"

static int fails = 0;
#define EXPECT(cond)                                                      \
  do {                                                                    \
    if (!(cond)) {                                                        \
      fprintf(stderr, "FAIL line %d: %s (%s)\n", __LINE__, #cond,         \
              lb_last_error());                                           \
      ++fails;                                                            \
    }                                                                     \
  } while (0)

/* lb_create on a parameter set that validation rejects */
static void rejected(const lb_params* p, int n) {
  lb_handle* h = (lb_handle*)&fails; /* must come back NULL */
  EXPECT(lb_create(p, n, NULL, &h) == LB_EINVAL);
  EXPECT(h == NULL);
  EXPECT(strlen(lb_last_error()) > 0);
}

int main(void) {
  lb_params p;
  lb_params_default(&p);
  EXPECT(p.lattice == LB_D3Q27 && p.nx == 64 && p.tau == 1.0);

  /* lattice tables: weights sum to one, opposite directions pair up */
  const int lats[3] = {LB_D2Q9, LB_D3Q19, LB_D3Q27};
  const int qs[3] = {9, 19, 27};
  for (int k = 0; k < 3; ++k) {
    int q = 0, c[27 * 3], opp[27];
    double w[27], B[27];
    EXPECT(lb_lattice_table(lats[k], &q, c, w, opp, B) == LB_OK);
    EXPECT(q == qs[k]);
    double sw = 0.0;
    for (int i = 0; i < q; ++i) {
      sw += w[i];
      EXPECT(opp[i] >= 0 && opp[i] < q && opp[opp[i]] == i);
      for (int a = 0; a < 3; ++a) EXPECT(c[3 * opp[i] + a] == -c[3 * i + a]);
    }
    EXPECT(fabs(sw - 1.0) < 1e-15);
    EXPECT(lb_lattice_table(lats[k], &q, NULL, NULL, NULL, NULL) == LB_OK);
  }
  EXPECT(lb_lattice_table(7, NULL, NULL, NULL, NULL, NULL) == LB_EINVAL);

  /* validation: single lattices */
  lb_params b;
  b = p; b.nx = 0; rejected(&b, 1);
  b = p; b.tau = 0.5; rejected(&b, 1);
  b = p; b.tau_b = 0.25; rejected(&b, 1);
  b = p; b.storage = 1234; rejected(&b, 1);
  b = p; b.lattice = 9; rejected(&b, 1);
  b = p; b.nc_mode = 7; rejected(&b, 1);
  b = p; b.wall[1] = 2; rejected(&b, 1);
  b = p; b.rho0 = 0.0; rejected(&b, 1);
  b = p; b.phi_interface = 1.0; rejected(&b, 1);
  b = p; b.A = NAN; rejected(&b, 1);
  b = p; b.nc_mode = LB_NC_EXPLICIT; b.nz = 3; rejected(&b, 1);
  b = p; b.nc_mode = LB_NC_EXPLICIT; b.nc_hmax = 4.0; rejected(&b, 1);
  b = p; b.diag_every = -1; rejected(&b, 1);
  b = p; b.streaming = 5; rejected(&b, 1);
  b = p; b.rounding = LB_ROUND_STOCHASTIC; rejected(&b, 1); /* FP32 per colour */
  b = p; b.lattice = LB_D2Q9; rejected(&b, 1);                /* nz = 64 */
  b = p; b.nx = 2048; b.ny = 2048; b.nz = 1024; rejected(&b, 1); /* a pair beyond 4 GiB */
  rejected(NULL, 1);
  rejected(&p, 0);
  rejected(&p, 100000);

  /* validation: ensembles */
  lb_params e[3] = {p, p, p};
  e[1].lattice = LB_D3Q19;
  rejected(e, 3);
  e[1] = p;
  e[2].streaming = LB_STREAM_IN_PLACE;
  rejected(e, 3);
  e[2] = p;
  e[0].nc_mode = e[1].nc_mode = e[2].nc_mode = LB_NC_MLP;
  rejected(e, 3);

  /* a valid request on a machine without a device */
  lb_handle* h = NULL;
  const int rc = lb_create(&p, 1, NULL, &h);
  EXPECT(rc == LB_ENODEV || rc == LB_EHIP);
  EXPECT(h == NULL);
  e[0] = e[1] = e[2] = p;
  EXPECT(lb_create(e, 3, NULL, &h) == LB_ENODEV);
  EXPECT(h == NULL);

  /* NULL handles and arguments */
  double cen[3] = {1, 2, 3}, rad[1] = {2}, out8[8];
  size_t bytes = 0;
  long long t = 0;
  int n = 0;
  float buf[64];
  lb_tuning tune;
  memset(&tune, 0, sizeof tune);
  tune.z_per_block = 1;
  EXPECT(lb_init_droplets(NULL, 0, 1, cen, rad, 2.0, 1.0) == LB_EINVAL);
  EXPECT(lb_step(NULL, 1) == LB_EINVAL);
  EXPECT(lb_fields(NULL, 0, 1u, NULL, 0) == LB_EINVAL);
  EXPECT(lb_diagnostics(NULL, 0, out8) == LB_EINVAL);
  EXPECT(lb_state_bytes(NULL, &bytes) == LB_EINVAL);
  EXPECT(lb_get_state(NULL, buf, sizeof buf, 0) == LB_EINVAL);
  EXPECT(lb_set_state(NULL, buf, sizeof buf, 0) == LB_EINVAL);
  EXPECT(lb_step_count(NULL, &t) == LB_EINVAL);
  EXPECT(lb_profile_begin(NULL) == LB_EINVAL);
  EXPECT(lb_profile_end(NULL, NULL, NULL, NULL, NULL, NULL, NULL) == LB_EINVAL);
  EXPECT(lb_sync(NULL) == LB_EINVAL);
  EXPECT(lb_channel_count(NULL, &n) == LB_EINVAL);
  EXPECT(lb_get_tuning(NULL, &tune) == LB_EINVAL);
  EXPECT(lb_set_tuning(NULL, &tune) == LB_EINVAL);
  EXPECT(lb_autotune(NULL, 2, &tune, NULL, 0, &n) == LB_EINVAL);
  EXPECT(lb_nc_collect(NULL, 0, buf, buf, 1, &t, &t) == LB_EINVAL);
  EXPECT(lb_nc_collect_noalloc(NULL, 0, buf, buf, 1, &t, &t) == LB_EINVAL);
  EXPECT(lb_mlp_set_weights(NULL, buf, 1) == LB_EINVAL);
  EXPECT(lb_mlp_get_weights(NULL, buf, 1) == LB_EINVAL);
  EXPECT(lb_mlp_set_ranges(NULL, buf, buf, 0.0f) == LB_EINVAL);
  EXPECT(lb_mlp_get_ranges(NULL, buf, buf, buf) == LB_EINVAL);
  EXPECT(lb_mlp_train(NULL, buf, buf, 1, &n, 1, 1, 1e-3, NULL) == LB_EINVAL);
  EXPECT(lb_mlp_gradient(NULL, buf, buf, 1, buf, buf) == LB_EINVAL);
  EXPECT(lb_mlp_infer(NULL, buf, buf, 1) == LB_EINVAL);
  EXPECT(lb_destroy(NULL) == LB_OK);
  EXPECT(lb_create(&p, 1, NULL, NULL) == LB_EINVAL);

  /* error strings */
  for (int code = 0; code >= -6; --code) EXPECT(lb_error_string(code) != NULL && strlen(lb_error_string(code)) > 0);
  EXPECT(lb_error_string(-99) != NULL);
  EXPECT(lb_last_error() != NULL);

  printf("host driver: %d failed expectations\n", fails);
  return fails != 0;
}
