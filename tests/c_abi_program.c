/* A plain C client of the library (no Python, no torch): the library owns its
 * device arena (arena = NULL) and works on the null stream. Reads an initial
 * state of n particles (9 arrays of doubles in id order: x y ux uy qxx qxy rho
 * ax ay) and the number of steps, advances one box, and writes the state back
 * in the same layout followed by the FP64 diagnostics. Half way it saves a
 * checkpoint, destroys the simulation and continues in a new one loaded from
 * the checkpoint, so the output is also a test of resuming bit for bit.
 *
 *   c_abi_program <side> <steps> <state_in.bin> <state_out.bin>
 *
 * Exit status: 0 on success, 2 on bad arguments or I/O, 3 on a library error
 * (its code and message go to stderr). */
#include <stdio.h>
#include <stdlib.h>
#include "nematic_sph.h"

static int fail(nem_sim* s, int rc, const char* what) {
  fprintf(stderr, "%s: %d (%s) %s\n", what, rc, nem_strerror(rc), s ? nem_last_error(s) : "");
  if (s) nem_destroy(s);
  return 3;
}

int main(int argc, char** argv) {
  if (argc != 5) { fprintf(stderr, "usage: %s side steps in out\n", argv[0]); return 2; }
  const int side = atoi(argv[1]);
  const long steps = atol(argv[2]);
  if (side < 8 || steps < 0) { fprintf(stderr, "bad side or steps\n"); return 2; }
  const int64_t n = (int64_t)side * side;
  double* f = (double*)malloc(sizeof(double) * 9 * (size_t)n);
  if (!f) return 2;
  FILE* in = fopen(argv[3], "rb");
  if (!in || fread(f, sizeof(double), 9 * (size_t)n, in) != 9 * (size_t)n) { fprintf(stderr, "read failed\n"); return 2; }
  fclose(in);

  nem_params p = {0};
  p.L = side; p.dx = 1.0; p.h = 1.3; p.rho0 = 1.0; p.eta = 1.0; p.Gamma = 0.34; p.lam = 0.7;
  p.A = 0.0; p.B = 0.0; p.C = 0.5; p.K = 0.02; p.zeta = 0.02; p.dt = 1e-3; p.gamma_eos = 7.0;
  p.beta = 1.0; p.c0_factor = 10.0; p.skin = 0.1; p.form = 0; p.elastic = 0; p.apd = 1;

  nem_sim* s = NULL;
  int rc = nem_create(&p, &n, 1, NULL, 0, NULL, &s);
  if (rc) return fail(NULL, rc, "nem_create");
  double* a[9];
  for (int k = 0; k < 9; ++k) a[k] = f + (size_t)k * n;
  rc = nem_set_state(s, 0, a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7], a[8]);
  if (rc) return fail(s, rc, "nem_set_state");
  rc = nem_step(s, steps / 2);
  if (rc) return fail(s, rc, "nem_step");
  uint64_t cb = 0;
  rc = nem_raw_bytes(s, &cb);
  if (rc) return fail(s, rc, "nem_raw_bytes");
  void* ckpt = malloc((size_t)cb);
  if (!ckpt) return fail(s, NEM_E_NOMEM, "malloc");
  rc = nem_save_raw(s, ckpt, cb);
  if (rc) return fail(s, rc, "nem_save_raw");
  nem_destroy(s);
  s = NULL;
  rc = nem_create(&p, &n, 1, NULL, 0, NULL, &s);
  if (rc) return fail(NULL, rc, "nem_create (resume)");
  rc = nem_load_raw(s, ckpt, cb);
  free(ckpt);
  if (rc) return fail(s, rc, "nem_load_raw");
  rc = nem_step(s, steps - steps / 2);
  if (rc) return fail(s, rc, "nem_step");
  rc = nem_sync(s);
  if (rc) return fail(s, rc, "nem_sync");
  rc = nem_get_state(s, 0, a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7], a[8]);
  if (rc) return fail(s, rc, "nem_get_state");
  nem_diag d;
  rc = nem_diagnostics(s, 0, &d);
  if (rc) return fail(s, rc, "nem_diagnostics");
  nem_destroy(s);

  FILE* out = fopen(argv[4], "wb");
  if (!out) return 2;
  const double dg[8] = {d.px, d.py, d.ke, d.F, d.F_grad, d.umax, d.c0, d.qmax};
  if (fwrite(f, sizeof(double), 9 * (size_t)n, out) != 9 * (size_t)n || fwrite(dg, sizeof(double), 8, out) != 8) {
    fprintf(stderr, "write failed\n");
    return 2;
  }
  fclose(out);
  free(f);
  printf("c_abi_program: %ld steps of %lld particles, ke %.17g\n", steps, (long long)n, d.ke);
  return 0;
}
