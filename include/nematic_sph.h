/* nematic_sph.h -- C ABI of the MI355X (gfx950) SPH Beris-Edwards active-nematic
 * solver in 2D periodic boxes.
 *
 * Problem statement (paper arXiv 2108.08919):
 *   * a periodic L x L box (Sec. 3.1, Eq. boundaryconditions);
 *   * per-particle state r, u, Q, rho advanced by the modified-Euler
 *     predictor-corrector of Sec. 3.1 (Eq. sphTimeIntegrationDerivatives);
 *   * rates from Eqs. sphMomentum, mi, sphContinuity, sphEos and
 *     densityCorrection, positions corrected by Eq. APD;
 *   * parameters of Table 2 plus h (Eq. quintic), gamma and c0 (Eq. sphEos)
 *     and beta (Eq. densityCorrection);
 *   * fields read back only at output times (Sec. 4).
 *
 * Conventions
 *   * Every function returns an int status: NEM_OK (0) or a negative NEM_E_*.
 *   * Host arrays are caller-owned and are in particle-id order (the id of a
 *     particle is its index in the arrays passed to nem_set_state); the library
 *     copies them in and out. The internal cell order is hidden.
 *   * Fields read back are at integer time levels (r^n, u^n, Q^n, rho^n).
 *   * Device memory: the caller may pass an arena of nem_arena_bytes() bytes
 *     (any device allocation, e.g. a torch uint8 tensor) and must keep it alive
 *     until nem_destroy; with arena == NULL the library allocates and owns it.
 *   * Stream: all work is enqueued on the hipStream_t passed to nem_create
 *     (NULL = the null stream). nem_step is asynchronous; device-side errors
 *     are sticky and are returned by nem_sync and by the read calls.
 *   * One nem_sim must not be used from two host threads at once.
 */
#ifndef NEMATIC_SPH_H
#define NEMATIC_SPH_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NEM_OK 0
#define NEM_E_INVAL (-1)     /* bad parameters, sizes or replica index */
#define NEM_E_NOMEM (-2)     /* arena too small or allocation failed */
#define NEM_E_HIP (-3)       /* HIP runtime error */
#define NEM_E_NUMERIC (-4)   /* a non-finite value appeared in the state */
#define NEM_E_OVERFLOW (-5)  /* a cell tile exceeds the LDS staging capacity (on average 24 particles
                                per cell of the quintic spline, 10 per cell of Wendland C2), a cell
                                holds more than 48 particles, or a particle has more than 96
                                pairs within the Verlet radius kappa h + 0.075 h */
#define NEM_E_SINGULAR (-6)  /* correction tensor not invertible; B = I was used */
#define NEM_E_STATE (-7)     /* call order (e.g. step before set_state) */
#define NEM_E_RANGE (-8)     /* an index fell outside its buffer; the access was skipped */

/* Parameters of one periodic box (one replica). Symbols of the paper:
 * Table 2 (Gamma, lambda, A, B, C, K, zeta, rho), Eq. sphMomentum (nu = eta/rho0),
 * Eq. quintic (h; support kappa h, kappa = 3, or 2 for the Wendland C2
 * variant), Eq. sphEos (gamma_eos, c0 = c0_factor max|u|),
 * Eq. densityCorrection (beta). */
typedef struct nem_params {
  double L;          /* box side */
  double dx;         /* initial lattice spacing; particle mass m = rho0 dx^2 */
  double h;          /* smoothing length */
  double rho0;       /* reference density */
  double eta;        /* dynamic viscosity */
  double Gamma;      /* rotational diffusivity */
  double lam;        /* flow-alignment (tumbling) parameter lambda */
  double A, B, C;    /* Landau coefficients (B drops out with the 2x2 Q of d = 2) */
  double K;          /* elastic constant */
  double zeta;       /* activity */
  double dt;         /* time step */
  double gamma_eos;  /* EoS exponent (7) */
  double beta;       /* density filter coefficient (1) */
  double c0_factor;  /* c0 = c0_factor * max |u^{n+1/2}| (10) */
  double skin;       /* cell side >= kappa h + skin; rebinning when a particle leaves its cell by skin/2 */
  int32_t form;      /* 0: B-corrected momentum of Eq. sphMomentum; 1: conservative pair forces */
  int32_t elastic;   /* 0: stress of Eq. mainstress; 1: also the lambda terms of Eq. elasticstress */
  int32_t apd;       /* 1: artificial particle displacement (Eq. APD) */
  int32_t kernel;    /* smoothing kernel: 0 quintic spline of support kappa h = 3h (Eq. quintic);
                        1 Wendland C2, W = 7/(4 pi h^2) (1 - q/2)^4 (1 + 2q), q = r/h < 2 (kappa = 2).
                        Every replica of one simulation uses the same form, elastic, kernel,
                        integrator and q3d (one compiled variant serves all replicas of a launch). */
  int32_t integrator;/* corrector (Sec. 3.1): 0 kick-drift-kick, u^{n+1} = u^{n+1/2} + a^{n+1/2} dt/2,
                        r^{n+1} = r^{n+1/2} + u^{n+1} dt/2; 1 midpoint, u^{n+1} = u^n + a^{n+1/2} dt,
                        r^{n+1} = r^n + u^{n+1/2} dt. Both add the APD shift to r and use the same
                        predictor and density update. */
  int32_t q3d;       /* order tensor: 0 the 2x2 Q of d = 2 (I/2); 1 quasi-2D, a 3x3 Q in the in-plane
                        flow with the printed I/3 in Eqs. corotation and molecularfielddis, the rate
                        projected on traceless tensors; Qxx, Qxy, Qyy are stored (Qzz = -Qxx - Qyy,
                        set with nem_set_qyy; default Qyy = -Qxx). Needs form 0 and elastic 0; the
                        learned step is not available for it. */
} nem_params;

/* FP64 global reductions at the current integer time level. */
typedef struct nem_diag {
  double px, py;     /* total momentum sum m u, m = rho0 dx^2 */
  double ke;         /* (1/N) sum |u|^2 / 2 (Eq. kineticenergy) */
  double F;          /* free energy with the discrete Laplacian: sum V[bulk] - K/2 sum V Q:lapQ */
  double F_grad;     /* free energy with squared corrected gradients */
  double umax;       /* max |u| */
  double c0;         /* sound speed of the last step */
  double qmax;       /* max Frobenius norm of Q */
} nem_diag;

typedef struct nem_sim nem_sim;

/* Library version (major*10000 + minor*100 + patch): 200 is version 0.2.0, the
 * first with the kernel, integrator and q3d fields of nem_params. */
int nem_version(void);

/* Device bytes needed for R replicas with n[r] particles each. */
int nem_arena_bytes(const nem_params* per_replica, const int64_t* n, int32_t R, uint64_t* bytes);

/* Create a solver for R replicas (R = 1 for a single box). per_replica[r] and
 * n[r] give each box's parameters and particle count (n[r] >= 1; the box side
 * must hold at least three cells of side >= 3h + skin). dev_arena/arena_bytes:
 * caller device memory or NULL. hip_stream: a hipStream_t or NULL. */
int nem_create(const nem_params* per_replica, const int64_t* n, int32_t R, void* dev_arena,
               uint64_t arena_bytes, void* hip_stream, nem_sim** out);

/* Set the state of replica r from host FP64 arrays of n[r] entries in id
 * order: positions (wrapped into [0, L)), velocity, Q components Qxx, Qxy
 * (Q symmetric traceless), density and the previous half-step acceleration
 * a^{n-1/2} (zero at the start of a run; may be NULL for zero). The particles
 * are binned by cell and the first predictor half-step is taken on the device. */
int nem_set_state(nem_sim* s, int32_t r, const double* x, const double* y, const double* ux,
                  const double* uy, const double* qxx, const double* qxy, const double* rho,
                  const double* ax, const double* ay);

/* Read the state of replica r into caller host arrays (any may be NULL). */
int nem_get_state(nem_sim* s, int32_t r, double* x, double* y, double* ux, double* uy, double* qxx,
                  double* qxy, double* rho, double* ax, double* ay);

/* Quasi-2D variant (q3d = 1) only: Qyy of replica r from or to caller host
 * arrays of n[r] doubles in id order (Qzz = -Qxx - Qyy). nem_set_state sets
 * Qyy = -Qxx (no out-of-plane part); call nem_set_qyy after it. NEM_E_INVAL
 * for a simulation with q3d = 0, NEM_E_STATE before nem_set_state. */
int nem_set_qyy(nem_sim* s, int32_t r, const double* qyy);
int nem_get_qyy(nem_sim* s, int32_t r, double* qyy);

/* Advance every replica by nsteps time steps (asynchronous). */
int nem_step(nem_sim* s, int64_t nsteps);

/* Wait for the stream; return the first sticky device error (and clear nothing). */
int nem_sync(nem_sim* s);

/* Checkpoints of the whole simulation (every replica) between steps, for
 * resuming a run bit for bit: continuing from a loaded checkpoint gives
 * exactly the fields the saved simulation would have produced (nem_get_state
 * and nem_set_state go through FP64 fields at the integer time level and
 * restart the Verlet list, which is close to but not bitwise that). The
 * checkpoint holds the device state the next step reads (current offsets and
 * their low parts, u^{n+1/2}, Q, a^{n-1/2}, rho - rho0, ids, cells, image
 * counters, cell starts, the max-speed slots, the status and request flags,
 * the Verlet list), the step parity and the tile, lanes-per-particle and
 * compensation options, and each replica's particle count and parameters.
 *   nem_raw_bytes: the checkpoint's size in bytes (about 270 per particle, 192 of them the Verlet list).
 *   nem_save_raw: waits for the stream and copies the checkpoint into the
 *     caller's host buffer of `bytes` bytes (NEM_E_NOMEM if it is smaller than
 *     nem_raw_bytes; NEM_E_STATE before every replica has a state).
 *   nem_load_raw: loads a checkpoint into a simulation created with the same
 *     replica count, particle counts and parameters (compared field by field;
 *     NEM_E_INVAL when anything differs or the buffer is not a checkpoint,
 *     NEM_E_NOMEM when it is shorter than the checkpoint; the simulation is
 *     unchanged in those cases). It sets the saved options and drops captured
 *     graphs. The buffer is the caller's and is only read. */
int nem_raw_bytes(nem_sim* s, uint64_t* bytes);
int nem_save_raw(nem_sim* s, void* host, uint64_t bytes);
int nem_load_raw(nem_sim* s, const void* host, uint64_t bytes);

/* Neighbour lists of replica r as the next step's pair passes walk them, at
 * the configuration that step uses (r^{n+1/2}), in CSR by particle id with
 * ascending columns (Eq. quintic: neighbours are the particles within the
 * kernel support 3h; 2h for the Wendland C2 variant).
 *
 * The library keeps a Verlet list per particle: every pair of the 3 x 3 cell
 * stencil closer than kappa h + delta (delta = 0.075 h) when it was last built;
 * it is rebuilt on the device when some particle has moved 0.45 delta since,
 * after a rebin, a new state, a tile change or a snapshot restore. Every pair
 * pass (volume, rates, filter, stress) walks that list and keeps an entry when
 * 0 < r2 < fl32((kappa h)^2), where, with positions held as FP32 offsets o from
 * the corner of the particle's cell (cells of side cs = fl32(L/nc),
 * nc = floor(L/(kappa h + skin))) and j in the cell displaced by d in
 * {-1,0,1}^2 from i's cell, r = fl(fl(o_i - o_j) + fl32(-d cs)) per component
 * and r2 = fl(fl(rx*rx) + fl(ry*ry)), without fused multiply-add.
 *
 * This call first runs the start of the next step on the stream (the rebin if
 * one is pending, the decision to rebuild, and the Verlet build or walk of the
 * volume pass; the next nem_step then walks the same list), then decodes the
 * list with the passes' own predicate:
 *   which = 0: the neighbours the passes sum over;
 *   which = 1: every entry of the Verlet list (a superset).
 * row_ptr has n[r]+1 entries; col has cap entries; *nnz receives the count.
 * cell_xy (2 n[r] int32, may be NULL) and off_xy (2 n[r] floats, may be NULL)
 * receive, in id order, each particle's cell coordinates and FP32 offsets, the
 * exact inputs of the predicate. Returns NEM_E_NOMEM (with *nnz set) when cap
 * is too small, NEM_E_INVAL for which outside {0, 1}. Allocates a device
 * buffer for the columns (hipMalloc) and synchronises the stream. */
int nem_neighbor_list(nem_sim* s, int32_t r, int32_t which, int64_t* row_ptr, int32_t* col, int64_t cap,
                      int64_t* nnz, int32_t* cell_xy, float* off_xy);

/* nem_neighbor_list with which = 0 and no offsets. */
int nem_neighbors(nem_sim* s, int32_t r, int64_t* row_ptr, int32_t* col, int64_t cap, int64_t* nnz);

/* FP64 reductions of replica r at the current integer time level: momentum,
 * kinetic energy, max |u|, max |Q| (from the stored state), and the free energy
 * of Eq. freeenergy with the elastic part through the discrete Laplacian (F)
 * and through squared corrected gradients (F_grad), whose pair sums are taken
 * at r^n (this reuses the per-step work arrays, so call it between steps). */
int nem_diagnostics(nem_sim* s, int32_t r, nem_diag* out);

/* Grid diagnostics of replica r at the integer time level (paper Sec. 5).
 * All three first Shepard-interpolate u and Q onto an M x M grid (M a power of
 * two in [8, 2048]; nodes at ((i+1/2) L/M, (j+1/2) L/M)): f_g = sum_j f_j W_gj /
 * sum_j W_gj over particles within the kernel support. These calls allocate grid buffers on the
 * device on first use (freed by nem_destroy) and synchronise the stream.
 *
 * nem_deposit: copies the grid to out[4*M*M] = (ux, uy, Qxx, Qxy), each row major
 *   (out[f*M*M + j*M + i]); with q3d = 1 the third field is (Qxx - Qyy)/2, the
 *   in-plane traceless part, so the director angle reads the same way.
 * nem_spectrum: kinetic-energy spectrum E(n) = 1/2 sum_{shell n} |u^(k)|^2 / M^4
 *   with shell n = floor(|k| L/2pi + 1/2) (so sum_n E(n) = <|u|^2>/2 over the grid),
 *   from a double-precision 2D FFT; E has nbins entries (shells beyond
 *   floor(sqrt(2) M/2 + 1/2) are zero); *slope (may be NULL) is the least-squares
 *   slope of ln E on ln n over k_lo..k_hi (<= 0 selects 4 and M/8).
 * nem_defects: counts of +1/2 and -1/2 defects: director angle atan2(Qxy,Qxx)/2
 *   per node, winding around each unit plaquette with edge differences wrapped
 *   into (-pi/2, pi/2]; a total of +pi (-pi) is a +1/2 (-1/2) defect.
 * nem_vorticity_correlation: normalised vorticity-vorticity correlation
 *   (paper Sec. 5, Eq. corr) of the grid field omega = d uy/dx - d ux/dy, taken
 *   spectrally (omega^ = i (kx u^y - ky u^x), the Nyquist wavenumber set to
 *   zero), averaged over all points of the periodic grid:
 *   C(r) = <omega(x + r) omega(x)> / <omega^2>, from a second FFT of |omega^|^2.
 *   c_x[n] and c_y[n] (caller arrays of M/2 + 1 doubles) hold C at separations
 *   n L/M along x and along y; *l_x, *l_y (may be NULL) the first zero crossing
 *   of each, linearly interpolated, in length units (-1 if C stays positive up
 *   to L/2). A field with omega = 0 gives NaN. */
int nem_deposit(nem_sim* s, int32_t r, int32_t M, double* out);
int nem_spectrum(nem_sim* s, int32_t r, int32_t M, double* E, int32_t nbins, int32_t k_lo, int32_t k_hi,
                 double* slope);
int nem_defects(nem_sim* s, int32_t r, int32_t M, int64_t* n_plus, int64_t* n_minus);
int nem_vorticity_correlation(nem_sim* s, int32_t r, int32_t M, double* c_x, double* c_y, double* l_x,
                              double* l_y);

/* For callers that cannot allocate device memory during the call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * nem_defects without its first-use grid allocation. The same kernels write
 * the M x M deposit grid and the two counters into a static device array of
 * the library, 8 MiB + 256 bytes per GPU, held from the library's load until
 * the process ends (its address is looked up once per device by nem_create).
 * M must be a power of two in [8, NEM_NOALLOC_MAX_GRID]; larger grids return
 * NEM_E_INVAL with an explanation in nem_last_error. The call allocates
 * nothing (no hipMalloc, no hipFree); the counters are cleared by a kernel on
 * every call. All calls on one GPU share the array: calls that overlap on one
 * GPU (several threads, or several streams in flight) race and must be
 * serialised by the caller. Synchronises the stream, like nem_defects. */
#define NEM_NOALLOC_MAX_GRID 512
int nem_defects_noalloc(nem_sim* s, int32_t r, int32_t M, int64_t* n_plus, int64_t* n_minus);

/* Lagrangian diagnostics (paper Sec. 5: pathlines of tagged particles, mixing
 * of colour-marked regions).
 *
 * nem_track: unwrapped positions at the integer time level of the particles
 *   ids[0..n_ids) of replica r (ids are the indices of nem_set_state), written
 *   to the caller's x[n_ids], y[n_ids]. Each particle carries a periodic image
 *   counter: it is set by nem_set_state from the coordinates given (positions
 *   outside [0, L) count as images, so a state set from unwrapped coordinates
 *   reads back unwrapped) and changes by one each time the particle crosses the
 *   periodic boundary, so x + L img_x follows the particle through any number
 *   of crossings. NEM_E_INVAL for ids out of [0, n) or n_ids > n.
 * nem_mixing: colour histogram and mixing index of replica r. colour[id]
 *   (caller array of n bytes, values < ncol <= 255) marks each particle, for
 *   instance by the quadrant of its initial position. The box is cut into
 *   B x B equal bins (B <= 1024) and counts[(by B + bx) ncol + c] (caller array
 *   of B*B*ncol, may be NULL) receives the number of particles of colour c in
 *   bin (bx, by), bx = floor(x B / L) of the wrapped position. *index (may be
 *   NULL) = 1 - I with I Danckwerts' intensity of segregation,
 *   I = sum_b sum_c N_b (phi_cb - phi_c)^2 / sum_c N phi_c (1 - phi_c),
 *   phi_cb = N_cb / N_b the colour fractions of bin b and phi_c = N_c / N the
 *   box fractions: 0 while every bin holds one colour, 1 when every bin holds
 *   the box's mixture; NaN with a single colour. */
int nem_track(nem_sim* s, int32_t r, const int32_t* ids, int32_t n_ids, double* x, double* y);
int nem_mixing(nem_sim* s, int32_t r, const uint8_t* colour, int32_t ncol, int32_t B, int64_t* counts,
               double* index);

/* Tuning and instrumentation options (key, value):
 *   NEM_OPT_TILE       cells per tile side (4 or 8)
 *   NEM_OPT_LPP        lanes per particle in the pair loops (1, 2 or 4)
 *   NEM_OPT_COMP       pair-sum compensation: 0 none, 1 Kahan over chunks of 16 pairs
 *                      (default), 2 Kahan on every pair term
 *   NEM_OPT_TIMING     1: record HIP events around every pass launch
 *   NEM_OPT_GRAPH      k > 0: capture k consecutive steps per buffer parity into
 *                      a hipGraph and replay it (steps left over run eagerly;
 *                      ignored while timing is on); 0: eager launches
 *   NEM_OPT_PERSIST    g > 0: pair passes run as g workgroups looping over the
 *                      tile work list of all replicas; 0: one workgroup per tile
 * Changing an option drops captured graphs. */
#define NEM_OPT_TILE 1
#define NEM_OPT_LPP 2
#define NEM_OPT_COMP 3
#define NEM_OPT_TIMING 4
#define NEM_OPT_GRAPH 5
#define NEM_OPT_PERSIST 6
int nem_set_option(nem_sim* s, int32_t key, int64_t value);
/* Current value of an option (NEM_E_INVAL for an unknown key). */
int nem_get_option(nem_sim* s, int32_t key, int64_t* value);

/* Autotuner: times `steps` steps of every supported combination of tile side
 * (4, 8), lanes per particle (1, 2, 4) and persistent grid (0 = one workgroup
 * per tile; 512, 1024, 2048 workgroups looping over the tiles) on the current
 * state of all replicas (restoring the state after each trial), keeps the
 * fastest and returns it (*tile, *lpp, and the best ms per step; each may be
 * NULL; the grid is read back with nem_get_option(NEM_OPT_PERSIST)). Each
 * trial is the fastest of three timings of `steps` steps after a warm-up step;
 * the search starts with 8 untimed steps. Allocates a state snapshot
 * (hipMalloc). */
int nem_autotune(nem_sim* s, int32_t steps, int32_t* tile, int32_t* lpp, double* ms_per_step);

/* Accumulated kernel times (ms, from HIP events recorded on the library's
 * stream around each launch group) and launch counts since the last reset,
 * per pass: 0 rebin (five kernels that return at once unless a rebin was
 * requested), 1 pass A (volume), 2 pass B (gradients and rates), 3 pass C
 * (filter and EoS), 4 pass D (stress and update). Requires NEM_OPT_TIMING;
 * synchronises the stream. */
#define NEM_NPASS 5
int nem_pass_times(nem_sim* s, double* ms, int64_t* launches, int32_t reset);

/* ---------------------------------------------------------------------------
 * Learned corrector: macro steps of mult*dt whose Q and u are corrected by a
 * 12 -> 64 -> 64 -> 5 perceptron (tanh, linear output) on BF16 matrix cores
 * with FP32 accumulation, trained on samples the solver generates, with mult
 * plain steps of dt as the fallback.
 *
 * Inputs per particle (12): Qxx, Qxy, du_x/dx, du_x/dy, du_y/dx, du_y/dy,
 * Hxx, Hxy, (rho - rho0)/rho0, zeta (taken in pass B of the macro step) and
 * the step's change of acceleration a^{n+1/2} - a^{n-1/2} (x, y; from pass D),
 * which drives the velocity error of the lagged predictor; outputs (5):
 * corrections of Qxx, Qxy, Qyy, u_x, u_y (Q projected traceless).
 * Inputs and targets are z-scored with stored means and standard deviations.
 * Weights: flat FP32 vector W1 (12x64, input-major), b1, W2 (64x64), b2,
 * W3 (64x5), b3 (nem_mlp_nparams() values). Device pointers (X, T, Y) are
 * caller-owned device memory; they must stay valid during the call.
 * ------------------------------------------------------------------------- */
typedef struct nem_mlp nem_mlp;
int nem_mlp_nparams(void);
/* Network with zero weights and identity normalisation on hip_stream. */
int nem_mlp_create(void* hip_stream, nem_mlp** out);
int nem_mlp_set_weights(nem_mlp* m, const float* w);   /* host, resets Adam */
int nem_mlp_get_weights(nem_mlp* m, float* w);         /* host */
/* norm[34]: input means (12), input std (12), target means (5), target std (5). */
int nem_mlp_set_norm(nem_mlp* m, const float* norm);
int nem_mlp_get_norm(nem_mlp* m, float* norm);
/* Normalisation fitted (FP64 on the device) to X (n x 12) and T (n x 5). */
int nem_mlp_fit_norm(nem_mlp* m, const float* X, const float* T, int64_t n);
/* Y (n x 5, physical units) = network(X (n x 12)). */
int nem_mlp_forward(nem_mlp* m, const float* X, int64_t n, float* Y);
/* Gradient (host, nem_mlp_nparams() values) of L = (1/2n) sum |y - t|^2 in
 * normalised units over all n samples; *loss may be NULL. */
int nem_mlp_grad(nem_mlp* m, const float* X, const float* T, int64_t n, float* grad, double* loss);
/* Adam (0.9, 0.999, 1e-8) over `epochs` passes of minibatches of `batch`
 * samples (a deterministic per-epoch permutation); *final_loss = last batch. */
int nem_mlp_train(nem_mlp* m, const float* X, const float* T, int64_t n, int32_t epochs, int32_t batch,
                  double lr, double* final_loss);
/* Network evaluated on X (n x 12): *max_norm (may be NULL) = the largest norm
 * of its correction in normalised output units (the quantity nem_step_learned
 * compares with tau); rel_mse[5] (may be NULL; then T may be NULL) = per output
 * the mean squared error against T (n x 5) relative to T's variance (1: no
 * better than no correction). FP64 sums in a fixed order. Allocates a buffer
 * for the predictions (hipMalloc). */
int nem_mlp_eval(nem_mlp* m, const float* X, const float* T, int64_t n, double* rel_mse, double* max_norm);
/* Switch off the outputs o with off[o] != 0 (5 flags): their last-layer weights,
 * bias and output mean become zero, so the network returns exactly zero for
 * them. Resets Adam. */
int nem_mlp_mask_outputs(nem_mlp* m, const int32_t* off);
void nem_mlp_destroy(nem_mlp* m);

/* Training samples at the current state of every replica, particle
 * (part_base(r) + id): X (ntot x 12) inputs of a step of mult*dt, T (ntot x 5)
 * = (Q, u after mult steps of dt) - (Q, u after one step of mult*dt). The
 * state is left unchanged. Allocates a scratch buffer (hipMalloc). */
int nem_samples(nem_sim* s, int32_t mult, float* X, float* T);
/* The same for the selected rows only: row k of X (nrows x 12) and T
 * (nrows x 5) is particle rows[k] (host array, part_base(r) + id, each in
 * [0, total particles)). Allocates scratch buffers (hipMalloc). */
int nem_samples_rows(nem_sim* s, int32_t mult, const int64_t* rows, int64_t nrows, float* X, float* T);
/* n_macro macro steps of mult*dt with corrections; a macro step whose largest
 * correction norm (normalised units) exceeds tau is replayed as mult steps of
 * dt. Synchronises once per macro step (one word read back); allocates
 * scratch buffers (hipMalloc). *n_fallback and *max_norm may be NULL. */
int nem_step_learned(nem_sim* s, nem_mlp* m, int64_t n_macro, int32_t mult, double tau, int64_t* n_fallback,
                     double* max_norm);

/* Error text for a status code, and the last error recorded on a solver. */
const char* nem_strerror(int code);
const char* nem_last_error(const nem_sim* s);

void nem_destroy(nem_sim* s);

#ifdef __cplusplus
}
#endif
#endif
