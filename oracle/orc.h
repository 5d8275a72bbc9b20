/* orc.h -- FP64 CPU oracle of the SPH Beris-Edwards active-nematic step.
 *
 * TEST INFRASTRUCTURE. This library exists only so that the tests, the smoke
 * check and the benchmark's CPU-baseline leg can compare the HIP path with a
 * plain, slow, obviously correct implementation. No product code may call it.
 * It shares no code, header or constant table with the HIP library.
 *
 * Everything is double precision, built without FMA contraction, OpenMP over
 * particles with static schedules (results do not depend on the thread count).
 * The order tensor is kept with all four components so that symmetry and
 * tracelessness are real invariants, not structural ones.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_params {
  double L, dx, h, rho0, eta, Gamma, lam, A, B, C, K, zeta;
  double dt, gamma_eos, beta, c0_factor, skin;
  int32_t form;    /* 0 corrected momentum (Eq. sphMomentum), 1 conservative pair forces */
  int32_t elastic; /* 1 adds the lambda terms of Eq. elasticstress */
  int32_t apd;     /* artificial particle displacement (Eq. APD) */
  int32_t search;  /* 0 cell list, 1 brute force O(N^2), 2 cell list with the pair decision in FP32 */
  int32_t kernel;  /* 0 quintic spline (Eq. quintic, support 3h), 1 Wendland C2 (support 2h) */
  int32_t integrator; /* corrector: 0 kick-drift-kick, 1 midpoint (u^n + a dt, r^n + u^{n+1/2} dt) */
  int32_t q3d;     /* 0: d = 2 (2x2 Q, I/2); 1: quasi-2D 3x3 Q with the printed I/3 (needs qzz) */
} orc_params;

typedef struct orc_state {
  int64_t n;
  double *x, *y, *ux, *uy;
  double *q;       /* 4 per particle: Qxx, Qxy, Qyx, Qyy */
  double *rho, *ax, *ay;  /* density and a^{n-1/2} */
  double *qzz;     /* Qzz per particle (quasi-2D 3x3 Q only; NULL otherwise) */
} orc_state;

typedef struct orc_diag {
  double px, py;      /* total momentum sum m u */
  double ke;          /* (1/N) sum 1/2 |u|^2 */
  double F;           /* Laplacian-consistent free energy */
  double F_grad;      /* gradient-squared free energy */
  double umax;        /* max |u| */
  double trq_max;     /* max |tr Q| */
  double asym_max;    /* max |Qxy - Qyx| */
  double c0_last;     /* sound speed used by the last step */
} orc_diag;

/* Smoothing kernel (0 quintic spline of Eq. quintic, 1 Wendland C2; 2D
 * normalisation), its radial derivative and its support in units of h. */
double orc_W(int32_t kernel, double h, double r);
double orc_dWdr(int32_t kernel, double h, double r);
double orc_kappa(int32_t kernel);

/* Literal 3x3 forms (row-major, 9 entries) of Eq. corotation with I/3 and of
 * Eq. molecularfielddis with I/3, for the quasi-2D variant; G is the 2x2
 * in-plane velocity gradient (no z velocity, no z dependence). */
void orc_corotation3(double lam, const double* Q, const double* G, double* S);
void orc_molecular_field3(const orc_params* p, const double* Q, const double* lapQ, double* H);

/* Neighbour lists in CSR by particle index, columns ascending.
 * mode 0: FP64 minimum image, cell list;  1: FP64 minimum image, brute force;
 * 2: FP32 predicate on cell-relative offsets (cells of side L/nc, nc given),
 *    brute force over adjacent cells;  3: the list the step builds with
 *    search = 2 (cell list, the same FP32 decision, nc = floor(L/(kappa h +
 *    skin)); nc argument unused).  Returns nnz or a negative error
 *    (-2 when cap is too small). */
int64_t orc_neighbors(const orc_params* p, int64_t n, const double* x, const double* y,
                      int32_t mode, int32_t nc, int64_t* row_ptr, int32_t* col, int64_t cap);

/* The FP32 predicate of mode 2 on given cell coordinates cell_xy[2i + 0/1]
 * and cell-relative FP32 offsets off_xy[2i + 0/1] (cells of side L/nc), for
 * particles that are kept in a cell they have moved slightly out of. */
int64_t orc_neighbors_offsets(const orc_params* p, int64_t n, int32_t nc, const int32_t* cell_xy,
                              const float* off_xy, int64_t* row_ptr, int32_t* col, int64_t cap);

/* Volume, correction tensor, corrected gradient and Laplacian of a scalar
 * field f at positions x,y (Eqs. sphSum, sphCorrectionMatrix, sph1stDerivative,
 * and the scalar corrected Laplacian). Outputs: V[n], Bt[4n] (row major),
 * grad[2n], lap[n]; any output may be NULL. */
int orc_operators(const orc_params* p, int64_t n, const double* x, const double* y,
                  const double* f, double* V, double* Bt, double* grad, double* lap);

/* Co-rotation tensor S (Eq. corotation with d = 2) for Q (4) and velocity
 * gradient G (4, G_ab = du_a/dx_b). */
void orc_corotation(double lam, const double* Q, const double* G, double* S);

/* Molecular field (Eq. molecularfielddis with d = 2) for Q (4), lapQ (4). */
void orc_molecular_field(const orc_params* p, const double* Q, const double* lapQ, double* H);

/* lambda part of the elastic stress (Eq. elasticstress with d = 2, D = Q + I/2):
 * Pi = 2 lam D (Q:H) - lam H D - lam D H, as literal 2x2 matrix products. */
void orc_elastic_stress(double lam, const double* Q, const double* H, double* Pi);

/* Equation of state (Eq. sphEos). */
double orc_eos(double rho, double rho0, double c0, double gamma_eos);

/* Advance the state by nsteps (Sec. 3.1). Returns 0 or a negative error:
 * -1 invalid parameters, -3 allocation failure, -4 non-finite value. */
int orc_step(const orc_params* p, orc_state* s, int64_t nsteps, orc_diag* info);

/* Diagnostics at the current (integer) time level. */
int orc_diagnostics(const orc_params* p, const orc_state* s, orc_diag* out);

/* Per-particle quantities of one step without advancing: V, k, rho_hat, p,
 * m (4 per particle), a (2 per particle), APD displacement (2). Any may be NULL. */
int orc_step_fields(const orc_params* p, const orc_state* s, double* V, double* k,
                    double* rho_hat, double* pres, double* m, double* a, double* dr_apd);

/* Shepard interpolation of nf fields onto an M x M grid with nodes at
 * ((i+1/2)L/M, (j+1/2)L/M): out[f*M*M + j*M + i]. */
int orc_deposit(const orc_params* p, int64_t n, const double* x, const double* y,
                int32_t nf, const double* const* fields, int32_t M, double* out);

int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
