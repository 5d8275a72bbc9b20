/* Drives every entry point of the FP64 oracle on small boxes so that it can be
 * built with AddressSanitizer and UndefinedBehaviorSanitizer (host code only):
 * the step in each variant (both kernels, both momentum forms, the lambda
 * stress, both correctors, the quasi-2D Q), the neighbour searches (cell list,
 * brute force, FP32 predicate, offsets), the operators, the step fields, the
 * diagnostics and the grid deposit. Exits 0 when every call succeeded; a
 * sanitizer report aborts the program with a non-zero status. Test
 * infrastructure, like the oracle itself. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "orc.h"

static uint64_t rng_state = 88172645463325252ull;
static double urand(void) {
  rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static void fail(const char* what, long long rc) {
  fprintf(stderr, "oracle_sanitize: %s returned %lld\n", what, rc);
  exit(2);
}

typedef struct {
  int n;
  double *x, *y, *ux, *uy, *q, *rho, *ax, *ay, *qzz;
} arrays;

static void fill(arrays* a, int side, int q3d) {
  const int n = side * side;
  a->n = n;
  a->x = malloc(sizeof(double) * n); a->y = malloc(sizeof(double) * n);
  a->ux = malloc(sizeof(double) * n); a->uy = malloc(sizeof(double) * n);
  a->q = malloc(sizeof(double) * 4 * n); a->rho = malloc(sizeof(double) * n);
  a->ax = calloc(n, sizeof(double)); a->ay = calloc(n, sizeof(double));
  a->qzz = q3d ? malloc(sizeof(double) * n) : NULL;
  for (int j = 0; j < side; ++j)
    for (int i = 0; i < side; ++i) {
      const int k = j * side + i;
      a->x[k] = fmod(i + 0.5 + 0.4 * (urand() - 0.5) + side, side);
      a->y[k] = fmod(j + 0.5 + 0.4 * (urand() - 0.5) + side, side);
      a->ux[k] = 1e-3 * (urand() - 0.5);
      a->uy[k] = 1e-3 * (urand() - 0.5);
      const double th = 3.14159265358979323846 * urand();
      const double c = cos(2 * th), s = sin(2 * th);
      if (q3d) {  /* (3/2)(nn - I/3) for an in-plane director */
        const double nx = cos(th), ny = sin(th);
        a->q[4 * k + 0] = 1.5 * (nx * nx - 1.0 / 3.0);
        a->q[4 * k + 1] = a->q[4 * k + 2] = 1.5 * nx * ny;
        a->q[4 * k + 3] = 1.5 * (ny * ny - 1.0 / 3.0);
        a->qzz[k] = -0.5;
      } else {
        a->q[4 * k + 0] = c; a->q[4 * k + 1] = a->q[4 * k + 2] = s; a->q[4 * k + 3] = -c;
      }
      a->rho[k] = 1.0 + 1e-4 * (urand() - 0.5);
    }
}

static void release(arrays* a) {
  free(a->x); free(a->y); free(a->ux); free(a->uy); free(a->q); free(a->rho); free(a->ax); free(a->ay);
  free(a->qzz);
}

static orc_params params(int side, int kernel) {
  orc_params p = {0};
  p.L = side; p.dx = 1.0; p.h = 1.3; p.rho0 = 1.0; p.eta = 1.0; p.Gamma = 0.34; p.lam = 0.7;
  p.A = 0.0; p.B = 0.0; p.C = 0.5; p.K = 0.02; p.zeta = 0.02; p.dt = 1e-3; p.gamma_eos = 7.0;
  p.beta = 1.0; p.c0_factor = 10.0; p.skin = 0.1; p.apd = 1; p.kernel = kernel;
  return p;
}

int main(void) {
  int runs = 0;
  for (int kernel = 0; kernel <= 1; ++kernel) {
    const int side = kernel == 0 ? 16 : 12;
    for (int variant = 0; variant < 7; ++variant) {
      /* 0 plain, 1 conservative form, 2 lambda stress, 3 midpoint corrector,
       * 4 quasi-2D Q, 5 brute-force search, 6 FP32 pair decisions */
      orc_params p = params(side, kernel);
      if (variant == 1) p.form = 1;
      if (variant == 2) p.elastic = 1;
      if (variant == 3) p.integrator = 1;
      if (variant == 4) p.q3d = 1;
      if (variant == 5) p.search = 1;
      if (variant == 6) p.search = 2;
      arrays a;
      fill(&a, side, p.q3d);
      orc_state s = {a.n, a.x, a.y, a.ux, a.uy, a.q, a.rho, a.ax, a.ay, a.qzz};
      orc_diag d;
      int rc = orc_step(&p, &s, 3, &d);
      if (rc != 0) fail("orc_step", rc);
      rc = orc_diagnostics(&p, &s, &d);
      if (rc != 0) fail("orc_diagnostics", rc);
      double* f = malloc(sizeof(double) * 12 * a.n);
      rc = orc_step_fields(&p, &s, f, f + a.n, f + 2 * a.n, f + 3 * a.n, f + 4 * a.n, f + 8 * a.n, f + 10 * a.n);
      if (rc < 0) fail("orc_step_fields", rc);
      free(f);
      release(&a);
      ++runs;
    }
    /* neighbour searches: cell list, brute force, FP32 predicate, FP32 offsets */
    orc_params p = params(side, kernel);
    arrays a;
    fill(&a, side, 0);
    const int64_t cap = 64 * (int64_t)a.n;
    int64_t* rp = malloc(sizeof(int64_t) * (a.n + 1));
    int32_t* col = malloc(sizeof(int32_t) * cap);
    const int nc = (int)floor(side / (orc_kappa(kernel) * p.h + p.skin));
    for (int mode = 0; mode <= 3; ++mode) {
      const int64_t nnz = orc_neighbors(&p, a.n, a.x, a.y, mode, nc, rp, col, cap);
      if (nnz <= 0) fail("orc_neighbors", nnz);
    }
    if (orc_neighbors(&p, a.n, a.x, a.y, 0, nc, rp, col, 1) != -2) fail("orc_neighbors (small cap)", 0);
    int32_t* cxy = malloc(sizeof(int32_t) * 2 * a.n);
    float* oxy = malloc(sizeof(float) * 2 * a.n);
    const double cs = (double)side / nc;
    for (int k = 0; k < a.n; ++k) {
      const int cx = (int)floor(a.x[k] / cs) % nc, cy = (int)floor(a.y[k] / cs) % nc;
      cxy[2 * k] = cx; cxy[2 * k + 1] = cy;
      oxy[2 * k] = (float)(a.x[k] - cx * cs); oxy[2 * k + 1] = (float)(a.y[k] - cy * cs);
    }
    if (orc_neighbors_offsets(&p, a.n, nc, cxy, oxy, rp, col, cap) <= 0) fail("orc_neighbors_offsets", 0);
    /* operators and deposit */
    double *V = malloc(sizeof(double) * a.n), *Bt = malloc(sizeof(double) * 4 * a.n);
    double *gr = malloc(sizeof(double) * 2 * a.n), *lap = malloc(sizeof(double) * a.n);
    int rc = orc_operators(&p, a.n, a.x, a.y, a.rho, V, Bt, gr, lap);
    if (rc != 0) fail("orc_operators", rc);
    const int M = 16;
    double* grid = malloc(sizeof(double) * 2 * M * M);
    const double* fields[2] = {a.ux, a.uy};
    rc = orc_deposit(&p, a.n, a.x, a.y, 2, fields, M, grid);
    if (rc != 0) fail("orc_deposit", rc);
    free(grid); free(V); free(Bt); free(gr); free(lap); free(cxy); free(oxy); free(rp); free(col);
    release(&a);
  }
  printf("oracle_sanitize: %d step runs and every search, operator and deposit call succeeded\n", runs);
  return 0;
}
