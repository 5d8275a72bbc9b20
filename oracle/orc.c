/* orc.c -- FP64 CPU oracle of one time step of the SPH Beris-Edwards
 * active-nematic solver in a 2D periodic box.
 *
 * TEST INFRASTRUCTURE ONLY: called by tests, the smoke check and the
 * benchmark's CPU-baseline leg. It shares no code with the HIP library.
 *
 * The step follows the paper's Sec. 3.1 in order: half-step predictor of u and
 * r, one neighbour search at the projected configuration, volumes (Eq. sphSum),
 * correction tensor (Eq. sphCorrectionMatrix), corrected velocity gradient
 * (Eq. sph1stDerivative), continuity (Eq. sphContinuity) and half-step density,
 * density filter (Eq. densityCorrection), equation of state (Eq. sphEos),
 * Q gradient and Laplacian, molecular field (Eq. molecularfielddis), co-rotation
 * (Eq. corotation), Q update (Eq. mi), momentum (Eq. sphMomentum), corrector and
 * artificial particle displacement (Eq. APD), periodic wrap (Eq.
 * boundaryconditions). Readings of the paper where it is garbled or silent are
 * written next to the code that takes them.
 *
 * Built with -O2 -ffp-contract=off -fopenmp; everything is double precision.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------ kernel */

/* Support radius of the kernel in units of h. */
double orc_kappa(int32_t kernel) { return kernel == 1 ? 2.0 : 3.0; }

/* kernel 0: Eq. quintic with kappa = 3 and the 2D normalisation
 * a_d = 7/(478 pi h^2); kernel 1: the Wendland C2 function of support 2h,
 * a_d (1 - q/2)^4 (1 + 2q) with a_d = 7/(4 pi h^2). b = q = r/h. */
double orc_W(int32_t kernel, double h, double r) {
  double b = r / h;
  if (kernel == 1) {
    if (b >= 2.0) return 0.0;
    double ad = 7.0 / (4.0 * PI * h * h);
    double t = 1.0 - 0.5 * b;
    return ad * t * t * t * t * (1.0 + 2.0 * b);
  }
  if (b >= 3.0) return 0.0;
  double ad = 7.0 / (478.0 * PI * h * h);
  double t3 = 3.0 - b, t2 = 2.0 - b, t1 = 1.0 - b;
  double s = t3 * t3 * t3 * t3 * t3;
  if (b < 2.0) s -= 6.0 * t2 * t2 * t2 * t2 * t2;
  if (b < 1.0) s += 15.0 * t1 * t1 * t1 * t1 * t1;
  return ad * s;
}

/* dW/dr of either kernel (for Wendland C2 the product rule on
 * t^4 (1 + 2q), t = 1 - q/2, then dq/dr = 1/h). */
double orc_dWdr(int32_t kernel, double h, double r) {
  double b = r / h;
  if (kernel == 1) {
    if (b >= 2.0) return 0.0;
    double ad = 7.0 / (4.0 * PI * h * h);
    double t = 1.0 - 0.5 * b;
    double dq = 4.0 * t * t * t * (-0.5) * (1.0 + 2.0 * b) + t * t * t * t * 2.0;
    return ad * dq / h;
  }
  if (b >= 3.0) return 0.0;
  double ad = 7.0 / (478.0 * PI * h * h);
  double t3 = 3.0 - b, t2 = 2.0 - b, t1 = 1.0 - b;
  double s = -5.0 * t3 * t3 * t3 * t3;
  if (b < 2.0) s += 30.0 * t2 * t2 * t2 * t2;
  if (b < 1.0) s -= 75.0 * t1 * t1 * t1 * t1;
  return ad * s / h;
}

/* Eq. sphEos as printed. */
double orc_eos(double rho, double rho0, double c0, double gamma_eos) {
  return rho0 * c0 * c0 / gamma_eos * (pow(rho / rho0, gamma_eos) - 1.0);
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------ 2x2 algebra */
/* Row-major 2x2: m[0]=xx m[1]=xy m[2]=yx m[3]=yy. */
static void mm(const double* a, const double* b, double* c) {
  double r0 = a[0] * b[0] + a[1] * b[2];
  double r1 = a[0] * b[1] + a[1] * b[3];
  double r2 = a[2] * b[0] + a[3] * b[2];
  double r3 = a[2] * b[1] + a[3] * b[3];
  c[0] = r0; c[1] = r1; c[2] = r2; c[3] = r3;
}
static double ddot(const double* a, const double* b) {  /* a : b */
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
}
static double tr2(const double* a) { return a[0] + a[3]; }

/* Eq. corotation read for d = 2 (the identity is I/2, not I/3):
 * S = (lam E + W) D + D (lam E - W) - 2 lam D (Q : G), D = Q + I/2,
 * E = (G + G^T)/2, W = (G - G^T)/2 with G_ab = du_a/dx_b. */
void orc_corotation(double lam, const double* Q, const double* G, double* S) {
  double E[4] = {G[0], 0.5 * (G[1] + G[2]), 0.5 * (G[2] + G[1]), G[3]};
  double W[4] = {0.0, 0.5 * (G[1] - G[2]), 0.5 * (G[2] - G[1]), 0.0};
  double D[4] = {Q[0] + 0.5, Q[1], Q[2], Q[3] + 0.5};
  double P[4], M[4], t1[4], t2[4];
  for (int k = 0; k < 4; ++k) { P[k] = lam * E[k] + W[k]; M[k] = lam * E[k] - W[k]; }
  mm(P, D, t1);
  mm(D, M, t2);
  double qg = ddot(Q, G);
  for (int k = 0; k < 4; ++k) S[k] = t1[k] + t2[k] - 2.0 * lam * D[k] * qg;
}

/* Eq. molecularfielddis with d = 2 and with the coefficients C and K that the
 * printed Eq. mi carries: H = -A Q + B (Q^2 - tr(Q^2) I/2) - C Q tr(Q^2) + K lapQ. */
void orc_molecular_field(const orc_params* p, const double* Q, const double* lapQ, double* H) {
  double Q2[4];
  mm(Q, Q, Q2);
  double t = tr2(Q2);
  double I[4] = {1, 0, 0, 1};
  for (int k = 0; k < 4; ++k)
    H[k] = -p->A * Q[k] + p->B * (Q2[k] - 0.5 * t * I[k]) - p->C * Q[k] * t + p->K * lapQ[k];
}

/* lambda terms of Eq. elasticstress with D = Q + I/2 and the parenthesis closed
 * after Q:H, written as the literal matrix products:
 * Pi = 2 lam D (Q:H) - lam H D - lam D H. */
void orc_elastic_stress(double lam, const double* Q, const double* H, double* Pi) {
  double D[4] = {Q[0] + 0.5, Q[1], Q[2], Q[3] + 0.5}, HD[4], DH[4];
  mm(H, D, HD);
  mm(D, H, DH);
  double qh = ddot(Q, H);
  for (int c = 0; c < 4; ++c) Pi[c] = 2.0 * lam * D[c] * qh - lam * HD[c] - lam * DH[c];
}

/* ------------------------------------------------------------ 3x3 algebra */
/* Row-major 3x3, quasi-2D variant: the flow is in the plane (no u_z, no z
 * dependence), Q is a full 3x3 tensor and the identity is I/3 as printed. */
static void mm3(const double* a, const double* b, double* c) {
  double r[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += a[3 * i + k] * b[3 * k + j];
      r[3 * i + j] = s;
    }
  memcpy(c, r, sizeof(r));
}
static double tr3(const double* a) { return a[0] + a[4] + a[8]; }

/* Eq. corotation as printed (D = Q + I/3), E and W of the in-plane G padded
 * with zeros in the z row and column. */
void orc_corotation3(double lam, const double* Q, const double* G, double* S) {
  double G3[9] = {G[0], G[1], 0.0, G[2], G[3], 0.0, 0.0, 0.0, 0.0};
  double E[9], W[9], D[9], P[9], M[9], t1[9], t2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      E[3 * i + j] = 0.5 * (G3[3 * i + j] + G3[3 * j + i]);
      W[3 * i + j] = 0.5 * (G3[3 * i + j] - G3[3 * j + i]);
      D[3 * i + j] = Q[3 * i + j] + (i == j ? 1.0 / 3.0 : 0.0);
    }
  for (int k = 0; k < 9; ++k) { P[k] = lam * E[k] + W[k]; M[k] = lam * E[k] - W[k]; }
  mm3(P, D, t1);
  mm3(D, M, t2);
  double qg = 0.0;
  for (int k = 0; k < 9; ++k) qg += Q[k] * G3[k];
  for (int k = 0; k < 9; ++k) S[k] = t1[k] + t2[k] - 2.0 * lam * D[k] * qg;
}

/* Eq. molecularfielddis with I/3: H = -A Q + B (Q^2 - tr(Q^2) I/3) - C Q tr(Q^2) + K lapQ. */
void orc_molecular_field3(const orc_params* p, const double* Q, const double* lapQ, double* H) {
  double Q2[9];
  mm3(Q, Q, Q2);
  double t = tr3(Q2);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      int k = 3 * i + j;
      H[k] = -p->A * Q[k] + p->B * (Q2[k] - (i == j ? t / 3.0 : 0.0)) - p->C * Q[k] * t + p->K * lapQ[k];
    }
}

/* ------------------------------------------------------- neighbour lists */

typedef struct nlist {
  int64_t n;
  int64_t* ptr;
  int32_t* j;
  double* rx; /* r_ij = r_i - r_j, minimum image */
  double* ry;
} nlist;

static void nlist_free(nlist* nl) {
  free(nl->ptr); free(nl->j); free(nl->rx); free(nl->ry);
  memset(nl, 0, sizeof(*nl));
}

static inline double minimg(double d, double L) { return d - L * nearbyint(d / L); }

static inline double wrapc(double x, double L) {
  double y = x - L * floor(x / L);
  if (y >= L) y -= L;
  if (y < 0.0) y = 0.0;
  return y;
}

/* Sort a row by column index (insertion sort; rows hold ~45 entries). */
static void sort_row(int32_t* j, double* rx, double* ry, int64_t m) {
  for (int64_t a = 1; a < m; ++a) {
    int32_t kj = j[a]; double kx = rx ? rx[a] : 0, ky = ry ? ry[a] : 0;
    int64_t b = a - 1;
    while (b >= 0 && j[b] > kj) {
      j[b + 1] = j[b];
      if (rx) { rx[b + 1] = rx[b]; ry[b + 1] = ry[b]; }
      --b;
    }
    j[b + 1] = kj;
    if (rx) { rx[b + 1] = kx; ry[b + 1] = ky; }
  }
}

/* Particles binned into nc x nc cells of side L/nc (counting sort, by index). */
typedef struct cells { int nc; double cs; int64_t* start; int64_t* idx; int32_t* cx; int32_t* cy; } cells;

static int cells_build(cells* c, int64_t n, const double* x, const double* y, double L, int nc) {
  c->nc = nc; c->cs = L / nc;
  c->start = (int64_t*)calloc((size_t)nc * nc + 1, sizeof(int64_t));
  c->idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  c->cx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  c->cy = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!c->start || !c->idx || !c->cx || !c->cy) return -3;
  for (int64_t i = 0; i < n; ++i) {
    int ix = (int)floor(x[i] / c->cs), iy = (int)floor(y[i] / c->cs);
    if (ix < 0) ix = 0; if (ix >= nc) ix = nc - 1;
    if (iy < 0) iy = 0; if (iy >= nc) iy = nc - 1;
    c->cx[i] = ix; c->cy[i] = iy;
    c->start[(int64_t)iy * nc + ix + 1]++;
  }
  for (int64_t k = 0; k < (int64_t)nc * nc; ++k) c->start[k + 1] += c->start[k];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)nc * nc);
  if (!fill) return -3;
  memcpy(fill, c->start, sizeof(int64_t) * (size_t)nc * nc);
  for (int64_t i = 0; i < n; ++i) c->idx[fill[(int64_t)c->cy[i] * nc + c->cx[i]]++] = i;
  free(fill);
  return 0;
}
static void cells_free(cells* c) { free(c->start); free(c->idx); free(c->cx); free(c->cy); }

static int fp32_pair(float oix, float oiy, float ojx, float ojy, int dxc, int dyc, float csf, float R2f);

/* Neighbour predicate (reading of Eq. quintic's support): j != i with
 * 0 < |r_ij| < kappa h (3h for the quintic spline, 2h for Wendland C2) under
 * the minimum-image convention. W(kappa h) = 0, so pairs at exactly kappa h
 * carry no weight either way.
 * search 2 takes the same decision in FP32, with the arithmetic of
 * fp32_predicate (cells of side L/nc, nc = floor(L/(kappa h + skin)), offsets
 * fl32(x - c cs) of this configuration): a pair decision is an integer that
 * floating point decides, so it is taken in the precision of the FP32
 * implementation; the pair geometry stored with it stays FP64. */
static int build_nlist(const orc_params* p, int64_t n, const double* x, const double* y,
                       int brute, nlist* nl) {
  const double L = p->L, R = orc_kappa(p->kernel) * p->h, R2 = R * R;
  const int f32 = p->search == 2;
  memset(nl, 0, sizeof(*nl));
  nl->n = n;
  nl->ptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!nl->ptr) return -3;
  int nc = f32 ? (int)floor(L / (R + p->skin)) : (int)floor(L / R);
  if (nc < 3) {
    if (f32) return -1;
    brute = 1;
  }
  if (f32) brute = 0;
  cells c;
  memset(&c, 0, sizeof(c));
  if (!brute && cells_build(&c, n, x, y, L, nc)) { cells_free(&c); return -3; }
  float *ofx = NULL, *ofy = NULL;
  const float csf = (float)(L / nc), R2f = (float)R2;
  if (f32) {
    ofx = (float*)malloc(sizeof(float) * (size_t)(n + 1));
    ofy = (float*)malloc(sizeof(float) * (size_t)(n + 1));
    if (!ofx || !ofy) { free(ofx); free(ofy); cells_free(&c); return -3; }
    for (int64_t i = 0; i < n; ++i) {
      ofx[i] = (float)(x[i] - c.cx[i] * c.cs);
      ofy[i] = (float)(y[i] - c.cy[i] * c.cs);
    }
  }

  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      for (int64_t i = 0; i < n; ++i) nl->ptr[i + 1] += nl->ptr[i];
      int64_t nnz = nl->ptr[n];
      nl->j = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz + 1));
      nl->rx = (double*)malloc(sizeof(double) * (size_t)(nnz + 1));
      nl->ry = (double*)malloc(sizeof(double) * (size_t)(nnz + 1));
      if (!nl->j || !nl->rx || !nl->ry) { free(ofx); free(ofy); cells_free(&c); return -3; }
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      int64_t cnt = 0, base = pass ? nl->ptr[i] : 0;
      if (brute) {
        for (int64_t j = 0; j < n; ++j) {
          if (j == i) continue;
          double dx = minimg(x[i] - x[j], L), dy = minimg(y[i] - y[j], L);
          double r2 = dx * dx + dy * dy;
          if (r2 > 0.0 && r2 < R2) {
            if (pass) { nl->j[base + cnt] = (int32_t)j; nl->rx[base + cnt] = dx; nl->ry[base + cnt] = dy; }
            ++cnt;
          }
        }
      } else {
        for (int oy = -1; oy <= 1; ++oy)
          for (int ox = -1; ox <= 1; ++ox) {
            int cx = (c.cx[i] + ox + nc) % nc, cy = (c.cy[i] + oy + nc) % nc;
            int64_t cc = (int64_t)cy * nc + cx;
            for (int64_t k = c.start[cc]; k < c.start[cc + 1]; ++k) {
              int64_t j = c.idx[k];
              if (j == i) continue;
              double dx = minimg(x[i] - x[j], L), dy = minimg(y[i] - y[j], L);
              double r2 = dx * dx + dy * dy;
              const int in = f32 ? fp32_pair(ofx[i], ofy[i], ofx[j], ofy[j], ox, oy, csf, R2f)
                                 : (r2 > 0.0 && r2 < R2);
              if (in) {
                if (pass) { nl->j[base + cnt] = (int32_t)j; nl->rx[base + cnt] = dx; nl->ry[base + cnt] = dy; }
                ++cnt;
              }
            }
          }
      }
      if (pass == 0) nl->ptr[i + 1] = cnt;
      else sort_row(nl->j + base, nl->rx + base, nl->ry + base, cnt);
    }
  }
  free(ofx);
  free(ofy);
  if (!brute) cells_free(&c);
  return 0;
}

/* The FP32 pair decision of fp32_predicate below, for j in the stencil cell
 * displaced by (dxc, dyc) from i's cell. volatile keeps every operation a
 * separately rounded FP32 operation. */
static int fp32_pair(float oix, float oiy, float ojx, float ojy, int dxc, int dyc, float csf, float R2f) {
  volatile float tx = oix - ojx;
  volatile float ty = oiy - ojy;
  volatile float sx = (float)(-dxc) * csf;
  volatile float sy = (float)(-dyc) * csf;
  volatile float rx = tx + sx;
  volatile float ry = ty + sy;
  volatile float xx = rx * rx;
  volatile float yy = ry * ry;
  volatile float r2 = xx + yy;
  return r2 > 0.0f && r2 < R2f;
}

/* FP32 predicate on cell-relative offsets, the search rule of a cell-list
 * implementation that stores single-precision positions relative to cells of
 * side cs = L/nc: off = fl32(x - c*cs) with c = floor(x/cs); for j in a cell
 * displaced by d in {-1,0,1} from i's cell (periodic),
 *   rx = fl32( fl32(offx_i - offx_j) + fl32(-d_x) * fl32(cs) ),
 *   r2 = fl32( fl32(rx*rx) + fl32(ry*ry) ),
 * accepted when 0 < r2 < fl32((kappa h)^2). No fused multiply-add anywhere. */
static int64_t fp32_predicate(const orc_params* p, int64_t n, int nc, const int32_t* cx, const int32_t* cy,
                              const float* ox, const float* oy, int64_t* row_ptr, int32_t* col, int64_t cap) {
  const float csf = (float)(p->L / nc);
  const double Rs = orc_kappa(p->kernel) * p->h;
  const float R2f = (float)(Rs * Rs);
  int64_t nnz = 0;
  for (int64_t i = 0; i < n; ++i) {
    row_ptr[i] = nnz;
    for (int64_t j = 0; j < n; ++j) {
      int dxc = ((cx[j] - cx[i]) % nc + nc) % nc; if (dxc == nc - 1) dxc = -1;
      int dyc = ((cy[j] - cy[i]) % nc + nc) % nc; if (dyc == nc - 1) dyc = -1;
      if (dxc > 1 || dyc > 1) continue;
      if (fp32_pair(ox[i], oy[i], ox[j], oy[j], dxc, dyc, csf, R2f)) {
        if (nnz < cap) col[nnz] = (int32_t)j;
        ++nnz;
      }
    }
  }
  row_ptr[n] = nnz;
  return nnz > cap ? -2 : nnz;
}

static int64_t fp32_neighbors(const orc_params* p, int64_t n, const double* x, const double* y,
                              int nc, int64_t* row_ptr, int32_t* col, int64_t cap) {
  if (nc < 3) return -1;
  const double csd = p->L / nc;
  int32_t* cx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t* cy = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  float* ox = (float*)malloc(sizeof(float) * (size_t)(n + 1));
  float* oy = (float*)malloc(sizeof(float) * (size_t)(n + 1));
  if (!cx || !cy || !ox || !oy) { free(cx); free(cy); free(ox); free(oy); return -3; }
  for (int64_t i = 0; i < n; ++i) {
    int ix = (int)floor(x[i] / csd), iy = (int)floor(y[i] / csd);
    if (ix < 0) ix = 0; if (ix >= nc) ix = nc - 1;
    if (iy < 0) iy = 0; if (iy >= nc) iy = nc - 1;
    cx[i] = ix; cy[i] = iy;
    ox[i] = (float)(x[i] - ix * csd);
    oy[i] = (float)(y[i] - iy * csd);
  }
  int64_t nnz = fp32_predicate(p, n, nc, cx, cy, ox, oy, row_ptr, col, cap);
  free(cx); free(cy); free(ox); free(oy);
  return nnz;
}

int64_t orc_neighbors_offsets(const orc_params* p, int64_t n, int32_t nc, const int32_t* cell_xy,
                              const float* off_xy, int64_t* row_ptr, int32_t* col, int64_t cap) {
  if (nc < 3) return -1;
  int32_t* cx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t* cy = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  float* ox = (float*)malloc(sizeof(float) * (size_t)(n + 1));
  float* oy = (float*)malloc(sizeof(float) * (size_t)(n + 1));
  if (!cx || !cy || !ox || !oy) { free(cx); free(cy); free(ox); free(oy); return -3; }
  for (int64_t i = 0; i < n; ++i) {
    cx[i] = cell_xy[2 * i]; cy[i] = cell_xy[2 * i + 1];
    ox[i] = off_xy[2 * i]; oy[i] = off_xy[2 * i + 1];
  }
  int64_t nnz = fp32_predicate(p, n, nc, cx, cy, ox, oy, row_ptr, col, cap);
  free(cx); free(cy); free(ox); free(oy);
  return nnz;
}

int64_t orc_neighbors(const orc_params* p, int64_t n, const double* x, const double* y,
                      int32_t mode, int32_t nc, int64_t* row_ptr, int32_t* col, int64_t cap) {
  if (mode == 2) return fp32_neighbors(p, n, x, y, nc, row_ptr, col, cap);
  nlist nl;
  orc_params q = *p;
  q.search = mode == 3 ? 2 : q.search == 2 ? 0 : q.search;   /* mode 3: the step's list under search 2 */
  int rc = build_nlist(&q, n, x, y, mode == 1, &nl);
  if (rc) { nlist_free(&nl); return rc; }
  int64_t nnz = nl.ptr[n];
  if (nnz > cap) { nlist_free(&nl); return -2; }
  memcpy(row_ptr, nl.ptr, sizeof(int64_t) * (size_t)(n + 1));
  memcpy(col, nl.j, sizeof(int32_t) * (size_t)nnz);
  nlist_free(&nl);
  return nnz;
}

/* ------------------------------------------------------------- operators */

/* Eq. sphSum: V_i = 1 / sum_j W_ij, the sum including the particle itself. */
static void op_volume(const orc_params* p, const nlist* nl, double* V) {
  const double W0 = orc_W(p->kernel, p->h, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nl->n; ++i) {
    double s = W0;
    for (int64_t k = nl->ptr[i]; k < nl->ptr[i + 1]; ++k)
      s += orc_W(p->kernel, p->h, hypot(nl->rx[k], nl->ry[k]));
    V[i] = 1.0 / s;
  }
}

/* Eq. sphCorrectionMatrix: alpha^{sl} = sum_j r_ji^s V_j dW_ij/dx_i^l, with
 * grad_i W_ij = W'(r) r_ij / r; B = alpha^{-1}. When alpha is numerically
 * singular B falls back to the identity and the flag is raised. */
static int op_correction(const orc_params* p, const nlist* nl, const double* V, double* Bt) {
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t i = 0; i < nl->n; ++i) {
    double a[4] = {0, 0, 0, 0};
    for (int64_t k = nl->ptr[i]; k < nl->ptr[i + 1]; ++k) {
      double rx = nl->rx[k], ry = nl->ry[k], r = hypot(rx, ry);
      double dW = orc_dWdr(p->kernel, p->h, r);
      double gx = dW * rx / r, gy = dW * ry / r;   /* grad_i W_ij */
      double Vj = V[nl->j[k]];
      double jx = -rx, jy = -ry;                   /* r_ji */
      a[0] += jx * Vj * gx; a[1] += jx * Vj * gy;
      a[2] += jy * Vj * gx; a[3] += jy * Vj * gy;
    }
    double det = a[0] * a[3] - a[1] * a[2];
    double nrm = a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3];
    double* B = Bt + 4 * i;
    if (!(fabs(det) > 1e-12 * nrm) || !isfinite(det)) {
      B[0] = 1; B[1] = 0; B[2] = 0; B[3] = 1; bad = 1;
    } else {
      B[0] = a[3] / det; B[1] = -a[1] / det; B[2] = -a[2] / det; B[3] = a[0] / det;
    }
  }
  return bad;
}

/* Corrected kernel gradient g_ij: from Eq. sph1stDerivative,
 * df/dx^k = sum_l R^l B^{lk} with R^l = sum_j V_j (f_j - f_i) dW/dx_i^l, so
 * g^k = sum_l dW/dx_i^l B^{lk} (for symmetric alpha this is B_i . grad_i W_ij). */
static inline void corr_grad(const double* B, double rx, double ry, double r, double dW,
                             double* gx, double* gy) {
  double wx = dW * rx / r, wy = dW * ry / r;
  *gx = wx * B[0] + wy * B[2];
  *gy = wx * B[1] + wy * B[3];
}

int orc_operators(const orc_params* p, int64_t n, const double* x, const double* y,
                  const double* f, double* Vout, double* Bout, double* grad, double* lap) {
  nlist nl;
  int rc = build_nlist(p, n, x, y, p->search == 1, &nl);
  if (rc) { nlist_free(&nl); return rc; }
  double* V = (double*)malloc(sizeof(double) * (size_t)(n + 1));
  double* Bt = (double*)malloc(sizeof(double) * 4 * (size_t)(n + 1));
  if (!V || !Bt) { free(V); free(Bt); nlist_free(&nl); return -3; }
  op_volume(p, &nl, V);
  op_correction(p, &nl, V, Bt);
  if (f) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double sx = 0, sy = 0, sl = 0;
      for (int64_t k = nl.ptr[i]; k < nl.ptr[i + 1]; ++k) {
        int32_t j = nl.j[k];
        double rx = nl.rx[k], ry = nl.ry[k], r = hypot(rx, ry);
        double gx, gy;
        corr_grad(Bt + 4 * i, rx, ry, r, orc_dWdr(p->kernel, p->h, r), &gx, &gy);
        sx += V[j] * (f[j] - f[i]) * gx;
        sy += V[j] * (f[j] - f[i]) * gy;
        sl += V[j] * (f[i] - f[j]) * (rx * gx + ry * gy) / (r * r);
      }
      if (grad) { grad[2 * i] = sx; grad[2 * i + 1] = sy; }
      if (lap) lap[i] = 2.0 * sl;
    }
  }
  if (Vout) memcpy(Vout, V, sizeof(double) * (size_t)n);
  if (Bout) memcpy(Bout, Bt, sizeof(double) * 4 * (size_t)n);
  free(V); free(Bt); nlist_free(&nl);
  return 0;
}

/* ----------------------------------------------------------------- step */

typedef struct work {
  nlist nl;
  double *V, *Bt, *G, *k, *rh, *rhat, *pr, *gq, *lq, *H, *qn, *Pi, *ax, *ay, *dr;
  double *qzn;   /* Qzz^{n+1} (quasi-2D variant only) */
  double c0;
  int singular;
} work;

static void work_free(work* w) {
  nlist_free(&w->nl);
  free(w->V); free(w->Bt); free(w->G); free(w->k); free(w->rh); free(w->rhat); free(w->pr);
  free(w->gq); free(w->lq); free(w->H); free(w->qn); free(w->Pi); free(w->ax); free(w->ay); free(w->dr);
  free(w->qzn);
}

/* Evaluate all rates of one step at the projected (half-step) configuration.
 * xh, yh, uxh, uyh are r^{n+1/2}, u^{n+1/2}; the state supplies rho^n and Q^n. */
static int eval_rates(const orc_params* p, const orc_state* s, const double* xh, const double* yh,
                      const double* uxh, const double* uyh, work* w) {
  const int64_t n = s->n;
  const double h = p->h, W0 = orc_W(p->kernel, h, 0.0), dt = p->dt;
  const double m = p->rho0 * p->dx * p->dx;   /* particle mass, constant */
  memset(w, 0, sizeof(*w));
  int rc = build_nlist(p, n, xh, yh, p->search == 1, &w->nl);
  if (rc) return rc;
  size_t N1 = (size_t)n + 1;
  w->V = malloc(sizeof(double) * N1); w->Bt = malloc(sizeof(double) * 4 * N1);
  w->G = malloc(sizeof(double) * 4 * N1); w->k = malloc(sizeof(double) * N1);
  w->rh = malloc(sizeof(double) * N1); w->rhat = malloc(sizeof(double) * N1);
  w->pr = malloc(sizeof(double) * N1); w->gq = malloc(sizeof(double) * 8 * N1);
  w->lq = malloc(sizeof(double) * 4 * N1); w->H = malloc(sizeof(double) * 4 * N1);
  w->qn = malloc(sizeof(double) * 4 * N1); w->Pi = malloc(sizeof(double) * 4 * N1);
  w->ax = malloc(sizeof(double) * N1); w->ay = malloc(sizeof(double) * N1);
  w->dr = malloc(sizeof(double) * 2 * N1);
  if (p->q3d) w->qzn = malloc(sizeof(double) * N1);
  if (!w->V || !w->Bt || !w->G || !w->k || !w->rh || !w->rhat || !w->pr || !w->gq || !w->lq ||
      !w->H || !w->qn || !w->Pi || !w->ax || !w->ay || !w->dr || (p->q3d && !w->qzn))
    return -3;
  const nlist* nl = &w->nl;

  /* Eq. sphSum, Eq. sphCorrectionMatrix */
  op_volume(p, nl, w->V);
  w->singular = op_correction(p, nl, w->V, w->Bt);
  const double* V = w->V;
  const double* Bt = w->Bt;

  /* Velocity gradient G_ab = du_a/dx_b (Eq. sph1stDerivative applied to u at
   * the projected configuration), continuity (Eq. sphContinuity, with rho^n)
   * and the half-step density rho^{n+1/2} = rho^n + k dt/2. */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double G[4] = {0, 0, 0, 0}, kk = 0;
    for (int64_t q = nl->ptr[i]; q < nl->ptr[i + 1]; ++q) {
      int32_t j = nl->j[q];
      double rx = nl->rx[q], ry = nl->ry[q], r = hypot(rx, ry), dW = orc_dWdr(p->kernel, h, r);
      double du[2] = {uxh[j] - uxh[i], uyh[j] - uyh[i]};
      if (p->form == 0) {
        double gx, gy;
        corr_grad(Bt + 4 * i, rx, ry, r, dW, &gx, &gy);
        G[0] += V[j] * du[0] * gx; G[1] += V[j] * du[0] * gy;
        G[2] += V[j] * du[1] * gx; G[3] += V[j] * du[1] * gy;
        kk += V[j] * (-du[0] * gx - du[1] * gy);
      } else {
        double gx, gy;
        corr_grad(Bt + 4 * i, rx, ry, r, dW, &gx, &gy);
        G[0] += V[j] * du[0] * gx; G[1] += V[j] * du[0] * gy;
        G[2] += V[j] * du[1] * gx; G[3] += V[j] * du[1] * gy;
        /* conservative continuity: drho_i/dt = sum_j m (u_i - u_j) . grad_i W_ij */
        kk += m * (-du[0] * dW * rx / r - du[1] * dW * ry / r);
      }
    }
    memcpy(w->G + 4 * i, G, sizeof(G));
    w->k[i] = (p->form == 0) ? s->rho[i] * kk : kk;
    w->rh[i] = s->rho[i] + 0.5 * w->k[i] * dt;
  }

  /* Eq. densityCorrection with the self term in both sums. */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double num = 0.0, den = W0;
    for (int64_t q = nl->ptr[i]; q < nl->ptr[i + 1]; ++q) {
      double Wij = orc_W(p->kernel, h, hypot(nl->rx[q], nl->ry[q]));
      num += (w->rh[i] - w->rh[nl->j[q]]) * Wij;
      den += Wij;
    }
    w->rhat[i] = w->rh[i] - p->beta * num / den;
  }

  /* Eq. sphEos with c0 = c0_factor * max |u^{n+1/2}| over the box (no floor). */
  double umax = 0.0;
#pragma omp parallel for schedule(static) reduction(max : umax)
  for (int64_t i = 0; i < n; ++i) {
    double u = hypot(uxh[i], uyh[i]);
    if (u > umax) umax = u;
  }
  w->c0 = p->c0_factor * umax;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) w->pr[i] = orc_eos(w->rhat[i], p->rho0, w->c0, p->gamma_eos);

  /* Gradient and Laplacian of each Q component (Eq. sph1stDerivative and the
   * scalar corrected Laplacian 2 sum_j V_j (f_i - f_j) (r_ij . g_ij)/r^2),
   * molecular field, co-rotation, rate m and Q^{n+1} = Q^n + m dt (Eq. mi). */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double gq[8] = {0}, lq[4] = {0};
    const double* Qi = s->q + 4 * i;
    for (int64_t q = nl->ptr[i]; q < nl->ptr[i + 1]; ++q) {
      int32_t j = nl->j[q];
      const double* Qj = s->q + 4 * j;
      double rx = nl->rx[q], ry = nl->ry[q], r = hypot(rx, ry), gx, gy;
      corr_grad(Bt + 4 * i, rx, ry, r, orc_dWdr(p->kernel, h, r), &gx, &gy);
      double rg = (rx * gx + ry * gy) / (r * r);
      for (int c = 0; c < 4; ++c) {
        gq[2 * c] += V[j] * (Qj[c] - Qi[c]) * gx;
        gq[2 * c + 1] += V[j] * (Qj[c] - Qi[c]) * gy;
        lq[c] += V[j] * (Qi[c] - Qj[c]) * rg;
      }
    }
    for (int c = 0; c < 4; ++c) lq[c] *= 2.0;
    memcpy(w->gq + 8 * i, gq, sizeof(gq));
    memcpy(w->lq + 4 * i, lq, sizeof(lq));
    double H[4], S[4], mr[4];
    if (p->q3d) {
      /* quasi-2D: 3x3 Q with Qzz, the literal I/3 forms, then the rate is
       * projected onto symmetric traceless 3x3 tensors */
      double lz = 0.0;
      for (int64_t q = nl->ptr[i]; q < nl->ptr[i + 1]; ++q) {
        int32_t j = nl->j[q];
        double rx = nl->rx[q], ry = nl->ry[q], r = hypot(rx, ry), gx, gy;
        corr_grad(Bt + 4 * i, rx, ry, r, orc_dWdr(p->kernel, h, r), &gx, &gy);
        lz += V[j] * (s->qzz[i] - s->qzz[j]) * (rx * gx + ry * gy) / (r * r);
      }
      lz *= 2.0;
      double Q3[9] = {Qi[0], Qi[1], 0.0, Qi[2], Qi[3], 0.0, 0.0, 0.0, s->qzz[i]};
      double L3[9] = {lq[0], lq[1], 0.0, lq[2], lq[3], 0.0, 0.0, 0.0, lz};
      double H3[9], S3[9], m3[9];
      orc_molecular_field3(p, Q3, L3, H3);
      orc_corotation3(p->lam, Q3, w->G + 4 * i, S3);
      for (int c = 0; c < 9; ++c) m3[c] = S3[c] + p->Gamma * H3[c];
      double t = tr3(m3) / 3.0, mp[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) mp[3 * a + b] = 0.5 * (m3[3 * a + b] + m3[3 * b + a]) - (a == b ? t : 0.0);
      H[0] = H3[0]; H[1] = H3[1]; H[2] = H3[3]; H[3] = H3[4];
      memcpy(w->H + 4 * i, H, sizeof(H));
      w->qn[4 * i + 0] = Qi[0] + mp[0] * dt; w->qn[4 * i + 1] = Qi[1] + mp[1] * dt;
      w->qn[4 * i + 2] = Qi[2] + mp[3] * dt; w->qn[4 * i + 3] = Qi[3] + mp[4] * dt;
      w->qzn[i] = s->qzz[i] + mp[8] * dt;
      for (int c = 0; c < 4; ++c) w->Pi[4 * i + c] = 0.0;
      continue;
    }
    orc_molecular_field(p, Qi, lq, H);
    orc_corotation(p->lam, Qi, w->G + 4 * i, S);
    for (int c = 0; c < 4; ++c) mr[c] = S[c] + p->Gamma * H[c];
    /* project the rate onto symmetric traceless tensors (d = 2 reading) */
    double off = 0.5 * (mr[1] + mr[2]), t = 0.5 * (mr[0] + mr[3]);
    double mp[4] = {mr[0] - t, off, off, mr[3] - t};
    memcpy(w->H + 4 * i, H, sizeof(H));
    for (int c = 0; c < 4; ++c) w->qn[4 * i + c] = Qi[c] + mp[c] * dt;
    /* lambda terms of Eq. elasticstress (literal matrix products) */
    orc_elastic_stress(p->lam, Qi, H, w->Pi + 4 * i);
  }

  /* Eq. sphMomentum at the half step, with rho_hat for rho, eta = nu rho0 and
   * the active stress -zeta Q written as -(zeta/rho_i) sum_j V_j (Q_j - Q_i) g_ij.
   * form 1: conservative (antisymmetric) pair forces with m_j = rho0 dx^2. */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double pr[2] = {0, 0}, vi[2] = {0, 0}, ac[2] = {0, 0}, el[2] = {0, 0};
    const double* Qi = s->q + 4 * i;
    const double ri = w->rhat[i], Pi_i = w->pr[i] / (ri * ri);
    double uv[2] = {0, 0}, sr = 0.0, srx = 0.0, sry = 0.0;
    int64_t cnt = 0;
    for (int64_t q = nl->ptr[i]; q < nl->ptr[i + 1]; ++q) {
      int32_t j = nl->j[q];
      const double* Qj = s->q + 4 * j;
      double rx = nl->rx[q], ry = nl->ry[q], r = hypot(rx, ry);
      double dW = orc_dWdr(p->kernel, h, r), Wij = orc_W(p->kernel, h, r);
      double rj = w->rhat[j], Pj = w->pr[j] / (rj * rj);
      double uij[2] = {uxh[i] - uxh[j], uyh[i] - uyh[j]};
      double ur = (uij[0] * rx + uij[1] * ry) / (r * r);
      if (p->form == 0) {
        double gx, gy;
        corr_grad(Bt + 4 * i, rx, ry, r, dW, &gx, &gy);
        pr[0] += V[j] * (Pi_i + Pj) * gx;  pr[1] += V[j] * (Pi_i + Pj) * gy;
        vi[0] += V[j] * ur * gx;           vi[1] += V[j] * ur * gy;
        double dq[4];
        for (int c = 0; c < 4; ++c) dq[c] = Qj[c] - Qi[c];
        ac[0] += V[j] * (dq[0] * gx + dq[1] * gy);
        ac[1] += V[j] * (dq[2] * gx + dq[3] * gy);
        if (p->elastic) {
          const double* Pa = w->Pi + 4 * i; const double* Pb = w->Pi + 4 * j;
          el[0] += V[j] * ((Pb[0] - Pa[0]) * gx + (Pb[1] - Pa[1]) * gy);
          el[1] += V[j] * ((Pb[2] - Pa[2]) * gx + (Pb[3] - Pa[3]) * gy);
        }
      } else {
        double wx = dW * rx / r, wy = dW * ry / r;  /* grad_i W_ij, antisymmetric */
        double rni = s->rho[i], rnj = s->rho[j];
        pr[0] += m * (Pi_i + Pj) * wx;  pr[1] += m * (Pi_i + Pj) * wy;
        vi[0] += m / (rni * rnj) * ur * wx;  vi[1] += m / (rni * rnj) * ur * wy;
        double cq[4];
        for (int c = 0; c < 4; ++c) cq[c] = Qi[c] / (rni * rni) + Qj[c] / (rnj * rnj);
        ac[0] += m * (cq[0] * wx + cq[1] * wy);
        ac[1] += m * (cq[2] * wx + cq[3] * wy);
        if (p->elastic) {
          const double* Pa = w->Pi + 4 * i; const double* Pb = w->Pi + 4 * j;
          double ce[4];
          for (int c = 0; c < 4; ++c) ce[c] = Pa[c] / (rni * rni) + Pb[c] / (rnj * rnj);
          el[0] += m * (ce[0] * wx + ce[1] * wy);
          el[1] += m * (ce[2] * wx + ce[3] * wy);
        }
      }
      /* Eq. APD ingredients at the projected configuration */
      uv[0] += uij[0] * Wij; uv[1] += uij[1] * Wij;
      sr += r; srx += rx / (r * r * r); sry += ry / (r * r * r);
      ++cnt;
    }
    double ax, ay;
    if (p->form == 0) {
      ax = -ri * pr[0] + 8.0 * p->eta / ri * vi[0] - p->zeta / ri * ac[0] + (p->elastic ? el[0] / ri : 0.0);
      ay = -ri * pr[1] + 8.0 * p->eta / ri * vi[1] - p->zeta / ri * ac[1] + (p->elastic ? el[1] / ri : 0.0);
    } else {
      ax = -pr[0] + 8.0 * p->eta * vi[0] - p->zeta * ac[0] + (p->elastic ? el[0] : 0.0);
      ay = -pr[1] + 8.0 * p->eta * vi[1] - p->zeta * ac[1] + (p->elastic ? el[1] : 0.0);
    }
    w->ax[i] = ax; w->ay[i] = ay;
    /* Eq. APD: u_v = |sum_j (u_i - u_j) W_ij| / sum_j W_ij (self included in
     * the denominator, i.e. times V_i); r0 = mean neighbour distance. */
    double dx = 0.0, dy = 0.0;
    if (p->apd && cnt > 0) {
      double u_v = hypot(uv[0], uv[1]) * V[i];
      double r0 = sr / (double)cnt;
      dx = r0 * r0 * u_v * dt * srx;
      dy = r0 * r0 * u_v * dt * sry;
    }
    w->dr[2 * i] = dx; w->dr[2 * i + 1] = dy;
  }
  return w->singular ? 1 : 0;
}

static int check_params(const orc_params* p) {
  if (!(p->L > 2.0 * orc_kappa(p->kernel) * p->h) || !(p->h > 0) || !(p->dx > 0) || !(p->rho0 > 0) || !(p->dt > 0))
    return -1;
  if (p->q3d && (p->form != 0 || p->elastic != 0)) return -1;  /* quasi-2D: corrected form, no lambda terms */
  return 0;
}

int orc_step(const orc_params* p, orc_state* s, int64_t nsteps, orc_diag* info) {
  if (check_params(p) || (p->q3d && !s->qzz)) return -1;
  const int64_t n = s->n;
  const double dt = p->dt, L = p->L;
  size_t N1 = (size_t)n + 1;
  double* xh = malloc(sizeof(double) * N1); double* yh = malloc(sizeof(double) * N1);
  double* uxh = malloc(sizeof(double) * N1); double* uyh = malloc(sizeof(double) * N1);
  if (!xh || !yh || !uxh || !uyh) { free(xh); free(yh); free(uxh); free(uyh); return -3; }
  int status = 0;
  for (int64_t st = 0; st < nsteps; ++st) {
    /* predictor (Sec. 3.1): u^{n+1/2} = u^n + a dt/2 with a = a^{n-1/2}
     * (zero before the first step); r^{n+1/2} = r^n + u^{n+1/2} dt/2 */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      uxh[i] = s->ux[i] + 0.5 * s->ax[i] * dt;
      uyh[i] = s->uy[i] + 0.5 * s->ay[i] * dt;
      xh[i] = wrapc(s->x[i] + 0.5 * uxh[i] * dt, L);
      yh[i] = wrapc(s->y[i] + 0.5 * uyh[i] * dt, L);
    }
    work w;
    int rc = eval_rates(p, s, xh, yh, uxh, uyh, &w);
    if (rc < 0) { work_free(&w); status = rc; break; }
    /* corrector (reading of Sec. 3.1), kick-drift-kick:
     * u^{n+1} = u^{n+1/2} + a^{n+1/2} dt/2, r^{n+1} = r^{n+1/2} + u^{n+1} dt/2;
     * or the midpoint alternative: u^{n+1} = u^n + a^{n+1/2} dt,
     * r^{n+1} = r^n + u^{n+1/2} dt. Both: rho^{n+1} = rho_hat^{n+1/2} + k^{n+1/2} dt/2,
     * then APD and wrap. */
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < n; ++i) {
      double ux, uy, x, y;
      if (p->integrator == 1) {
        ux = s->ux[i] + w.ax[i] * dt;
        uy = s->uy[i] + w.ay[i] * dt;
        x = s->x[i] + uxh[i] * dt + w.dr[2 * i];
        y = s->y[i] + uyh[i] * dt + w.dr[2 * i + 1];
      } else {
        ux = uxh[i] + 0.5 * w.ax[i] * dt;
        uy = uyh[i] + 0.5 * w.ay[i] * dt;
        x = xh[i] + 0.5 * ux * dt + w.dr[2 * i];
        y = yh[i] + 0.5 * uy * dt + w.dr[2 * i + 1];
      }
      s->ux[i] = ux; s->uy[i] = uy;
      s->x[i] = wrapc(x, L); s->y[i] = wrapc(y, L);
      s->rho[i] = w.rhat[i] + 0.5 * w.k[i] * dt;
      s->ax[i] = w.ax[i]; s->ay[i] = w.ay[i];
      for (int c = 0; c < 4; ++c) s->q[4 * i + c] = w.qn[4 * i + c];
      if (p->q3d) s->qzz[i] = w.qzn[i];
      if (!isfinite(ux) || !isfinite(uy) || !isfinite(s->rho[i]) || !isfinite(w.qn[4 * i]) || !isfinite(w.qn[4 * i + 1]))
        bad = 1;
    }
    if (info) info->c0_last = w.c0;
    work_free(&w);
    if (bad) { status = -4; break; }
  }
  free(xh); free(yh); free(uxh); free(uyh);
  return status;
}

int orc_step_fields(const orc_params* p, const orc_state* s, double* V, double* k,
                    double* rho_hat, double* pres, double* mrate, double* a, double* dr_apd) {
  if (check_params(p) || (p->q3d && !s->qzz)) return -1;
  const int64_t n = s->n;
  const double dt = p->dt, L = p->L;
  size_t N1 = (size_t)n + 1;
  double* xh = malloc(sizeof(double) * N1); double* yh = malloc(sizeof(double) * N1);
  double* uxh = malloc(sizeof(double) * N1); double* uyh = malloc(sizeof(double) * N1);
  if (!xh || !yh || !uxh || !uyh) { free(xh); free(yh); free(uxh); free(uyh); return -3; }
  for (int64_t i = 0; i < n; ++i) {
    uxh[i] = s->ux[i] + 0.5 * s->ax[i] * dt;
    uyh[i] = s->uy[i] + 0.5 * s->ay[i] * dt;
    xh[i] = wrapc(s->x[i] + 0.5 * uxh[i] * dt, L);
    yh[i] = wrapc(s->y[i] + 0.5 * uyh[i] * dt, L);
  }
  work w;
  int rc = eval_rates(p, s, xh, yh, uxh, uyh, &w);
  if (rc >= 0) {
    for (int64_t i = 0; i < n; ++i) {
      if (V) V[i] = w.V[i];
      if (k) k[i] = w.k[i];
      if (rho_hat) rho_hat[i] = w.rhat[i];
      if (pres) pres[i] = w.pr[i];
      if (mrate) for (int c = 0; c < 4; ++c) mrate[4 * i + c] = (w.qn[4 * i + c] - s->q[4 * i + c]) / dt;
      if (a) { a[2 * i] = w.ax[i]; a[2 * i + 1] = w.ay[i]; }
      if (dr_apd) { dr_apd[2 * i] = w.dr[2 * i]; dr_apd[2 * i + 1] = w.dr[2 * i + 1]; }
    }
  }
  work_free(&w);
  free(xh); free(yh); free(uxh); free(uyh);
  return rc;
}

/* ---------------------------------------------------------- diagnostics */

/* Diagnostics at the integer time level (r^n, u^n, Q^n): total momentum with
 * m = rho0 dx^2, kinetic energy per particle (Eq. kineticenergy as a particle
 * average), free energy of Eq. freeenergy with the elastic part written with
 * the discrete Laplacian (F = sum V [A/2 trQ^2 + B/3 trQ^3 + C/4 (trQ^2)^2]
 * - K/2 sum V Q:lapQ) and with the squared corrected gradient (F_grad). */
int orc_diagnostics(const orc_params* p, const orc_state* s, orc_diag* out) {
  if (p->q3d && !s->qzz) return -1;
  const int64_t n = s->n;
  const double m = p->rho0 * p->dx * p->dx, h = p->h;
  nlist nl;
  int rc = build_nlist(p, n, s->x, s->y, p->search == 1, &nl);
  if (rc) { nlist_free(&nl); return rc; }
  double* V = malloc(sizeof(double) * (size_t)(n + 1));
  double* Bt = malloc(sizeof(double) * 4 * (size_t)(n + 1));
  if (!V || !Bt) { free(V); free(Bt); nlist_free(&nl); return -3; }
  op_volume(p, &nl, V);
  op_correction(p, &nl, V, Bt);
  double px = 0, py = 0, ke = 0, F = 0, Fg = 0, umax = 0, trq = 0, asym = 0;
#pragma omp parallel for schedule(static) reduction(+ : px, py, ke, F, Fg) reduction(max : umax, trq, asym)
  for (int64_t i = 0; i < n; ++i) {
    const double* Qi = s->q + 4 * i;
    double gq[8] = {0}, lq[4] = {0};
    for (int64_t q = nl.ptr[i]; q < nl.ptr[i + 1]; ++q) {
      int32_t j = nl.j[q];
      const double* Qj = s->q + 4 * j;
      double rx = nl.rx[q], ry = nl.ry[q], r = hypot(rx, ry), gx, gy;
      corr_grad(Bt + 4 * i, rx, ry, r, orc_dWdr(p->kernel, h, r), &gx, &gy);
      double rg = (rx * gx + ry * gy) / (r * r);
      for (int c = 0; c < 4; ++c) {
        gq[2 * c] += V[j] * (Qj[c] - Qi[c]) * gx;
        gq[2 * c + 1] += V[j] * (Qj[c] - Qi[c]) * gy;
        lq[c] += 2.0 * V[j] * (Qi[c] - Qj[c]) * rg;
      }
    }
    double t2, t3, g2 = 0, ql;
    for (int c = 0; c < 8; ++c) g2 += gq[c] * gq[c];
    ql = ddot(Qi, lq);
    if (p->q3d) {
      /* quasi-2D: Qzz enters the invariants, its gradient and Laplacian */
      double gz[2] = {0, 0}, lz = 0;
      for (int64_t q = nl.ptr[i]; q < nl.ptr[i + 1]; ++q) {
        int32_t j = nl.j[q];
        double rx = nl.rx[q], ry = nl.ry[q], r = hypot(rx, ry), gx, gy;
        corr_grad(Bt + 4 * i, rx, ry, r, orc_dWdr(p->kernel, h, r), &gx, &gy);
        gz[0] += V[j] * (s->qzz[j] - s->qzz[i]) * gx;
        gz[1] += V[j] * (s->qzz[j] - s->qzz[i]) * gy;
        lz += 2.0 * V[j] * (s->qzz[i] - s->qzz[j]) * (rx * gx + ry * gy) / (r * r);
      }
      double Q3[9] = {Qi[0], Qi[1], 0.0, Qi[2], Qi[3], 0.0, 0.0, 0.0, s->qzz[i]}, A2[9], A3[9];
      mm3(Q3, Q3, A2); mm3(A2, Q3, A3);
      t2 = tr3(A2); t3 = tr3(A3);
      g2 += gz[0] * gz[0] + gz[1] * gz[1];
      ql += s->qzz[i] * lz;
    } else {
      double Q2[4], Q3[4];
      mm(Qi, Qi, Q2); mm(Q2, Qi, Q3);
      t2 = tr2(Q2); t3 = tr2(Q3);
    }
    double bulk = 0.5 * p->A * t2 + p->B / 3.0 * t3 + 0.25 * p->C * t2 * t2;
    F += V[i] * (bulk - 0.5 * p->K * ql);
    Fg += V[i] * (bulk + 0.5 * p->K * g2);
    px += m * s->ux[i]; py += m * s->uy[i];
    double u2 = s->ux[i] * s->ux[i] + s->uy[i] * s->uy[i];
    ke += 0.5 * u2;
    if (sqrt(u2) > umax) umax = sqrt(u2);
    double tq = Qi[0] + Qi[3] + (p->q3d ? s->qzz[i] : 0.0);
    if (fabs(tq) > trq) trq = fabs(tq);
    if (fabs(Qi[1] - Qi[2]) > asym) asym = fabs(Qi[1] - Qi[2]);
  }
  out->px = px; out->py = py; out->ke = n > 0 ? ke / (double)n : 0.0;
  out->F = F; out->F_grad = Fg; out->umax = umax; out->trq_max = trq; out->asym_max = asym;
  free(V); free(Bt); nlist_free(&nl);
  return 0;
}

/* Shepard interpolation onto grid nodes: f_g = sum_j f_j W_gj / sum_j W_gj over
 * particles within the kernel support kappa h of the node (minimum image).
 * Nodes with no particle within the support get 0. */
int orc_deposit(const orc_params* p, int64_t n, const double* x, const double* y,
                int32_t nf, const double* const* fields, int32_t M, double* out) {
  const double L = p->L, h = p->h, R = orc_kappa(p->kernel) * h;
  int nc = (int)floor(L / R);
  if (nc < 3) nc = 1;
  cells c;
  memset(&c, 0, sizeof(c));
  if (cells_build(&c, n, x, y, L, nc)) { cells_free(&c); return -3; }
  const double dg = L / M;
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < (int64_t)M * M; ++g) {
    int gi = (int)(g % M), gj = (int)(g / M);
    double gx = (gi + 0.5) * dg, gy = (gj + 0.5) * dg;
    int cx = (int)floor(gx / c.cs), cy = (int)floor(gy / c.cs);
    if (cx >= nc) cx = nc - 1; if (cy >= nc) cy = nc - 1;
    double den = 0.0, num[16] = {0};
    int span = nc >= 3 ? 1 : 0;
    for (int oy = -span; oy <= span; ++oy)
      for (int ox = -span; ox <= span; ++ox) {
        int ccx = (cx + ox + nc) % nc, ccy = (cy + oy + nc) % nc;
        int64_t cc = (int64_t)ccy * nc + ccx;
        for (int64_t k = c.start[cc]; k < c.start[cc + 1]; ++k) {
          int64_t j = c.idx[k];
          double dx = minimg(gx - x[j], L), dy = minimg(gy - y[j], L);
          double r = hypot(dx, dy);
          if (r >= R) continue;
          double Wg = orc_W(p->kernel, h, r);
          den += Wg;
          for (int f = 0; f < nf && f < 16; ++f) num[f] += fields[f][j] * Wg;
        }
      }
    for (int f = 0; f < nf && f < 16; ++f) out[(int64_t)f * M * M + g] = den > 0 ? num[f] / den : 0.0;
  }
  cells_free(&c);
  return 0;
}
