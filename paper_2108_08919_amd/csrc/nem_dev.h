// nem_dev.h -- device-side data structures shared by the HIP kernels and the
// host runtime of the nematic SPH library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nem {

constexpr int WG = 256;          // threads per workgroup of every pair pass
constexpr int MAXT = 8;          // largest tile side in cells
constexpr int MAXSC = (MAXT + 2) * (MAXT + 2);  // staged cells per tile (interior + halo)
constexpr int KMAX = 96;         // list capacity: entries per particle of the Verlet and direct-search lists
constexpr int UMAX_SLOTS = 64;   // per-replica slots of the max-speed reduction

// Sticky device error bits (flags[0]).
enum : unsigned {
  ERR_NUMERIC = 1u,
  ERR_OVERFLOW = 2u,
  ERR_SINGULAR = 4u,
  ERR_RANGE = 8u,
};

// One periodic box. All per-pair constants are FP32; csd and Ld keep the
// double-precision geometry used when positions enter or leave the library.
struct RepDev {
  int nc;          // cells per side
  int cell_base;   // first global cell of this replica
  int part_base;   // first particle (sorted arrays) of this replica
  int n;           // particles
  int tiles_x, tiles_y, tile_base, form;
  float cs, cs_lo; // cell side as a float pair (cs + cs_lo = L/nc to ~1e-14 relative)
  float h, hinv;
  float R2;        // fl32((kappa h)^2), kappa = 3 (quintic) or 2 (Wendland C2): pair accepted when 0 < r^2 < R2
  float a2;        // normalisation: 7 / (478 pi h^2) (quintic), 7 / (4 pi h^2) (Wendland C2)
  float W0;        // W(0): 66 a2 (quintic), a2 (Wendland C2)
  float dWc;       // quintic: dW/dr = dWc (t3^4 - 6 t2^4 + 15 t1^4), dWc = -5 a2 / h;
                   // Wendland C2: (dW/dr)/r = dWc (1 - q/2)^3, dWc = -5 a2 / h^2
  float skin_half, rho0, eta, Gamma;
  float lam, A, C, K;
  float zeta, dt, gamma_eos, beta;
  float c0_factor, mass, inv_rho0, B;
  int elastic, apd;
  int kern;        // smoothing kernel: 0 quintic spline (support 3h), 1 Wendland C2 (support 2h)
  int integ;       // corrector: 0 kick-drift-kick, 1 midpoint
  int q3d;         // 0: 2x2 Q (d = 2); 1: quasi-2D 3x3 Q with I/3 (Qyy stored, Qzz = -Qxx - Qyy)
  float R2v;       // Verlet list radius: fl32((kappa h + delta)^2), delta = 0.075 h
  float disp2;     // rebuild the Verlet list when a particle moved more than 0.45 delta: (0.45 delta)^2
  double csd, Ld;
};

// Pointers of one step. *_cur / *_nxt alternate between steps.
struct StepArgs {
  const RepDev* reps;
  const int* work;        // 2 ints per work item: replica, tile index
  int nwork, T;           // work items, tile side in cells
  int lpp;                // lanes per particle in passes B-D (1, 2, 4)
  int grid;               // 0: one workgroup per tile; > 0: persistent grid size
  const int* cell_start;  // [ncells + 1], particles sorted by (replica, cell, id)
  int ncells, ntot;
  const float2* off_cur;  // cell-relative position (high part) at r^{n+1/2}
  float2* off_nxt;        // same for the next step
  float2* offlo;          // low part of the position (compensation)
  float2* u;              // u^{n+1/2}
  const float2* q_cur;    // (Qxx, Qxy) at Q^n
  float2* q_nxt;          // Q^{n+1}
  const float* qyy_cur;   // Qyy^n (quasi-2D variant only)
  float* qyy_nxt;         // Qyy^{n+1}
  float2* acc;            // a^{n+1/2} (kept for read-back and restart)
  float* drho;            // rho^n - rho0, then rho^{n+1} - rho0
  int* cell;              // global cell of each particle (from the last binning)
  float* V;               // particle volume
  float4* bk;             // (Bxx, Bxy, Byy, k)
  float* dh;              // rho^{n+1/2} - rho0
  float2* apart;          // viscous + active acceleration before division by rho_hat
  float* uv;              // APD velocity-variance coefficient
  float2* pi;             // lambda part of the elastic stress (Pi_xx, Pi_xy)
  float* P;               // p / rho_hat^2
  float* drhat;           // rho_hat - rho0
  unsigned* flags;        // [0] error bits, [1] rebin request, [2] Verlet rebuild request, [3] rebuild this step
  const unsigned* umax_cur;  // [R][UMAX_SLOTS]: max |u^{n+1/2}| (float bits)
  unsigned* umax_nxt;        // [R][UMAX_SLOTS]: max |u^{n+3/2}| being accumulated
  uint32_t* nl;              // neighbour list of the direct search (diagnostics): word w of particle g
                             // at nl[w*ntot + g], two 16-bit entries (LDS slot | (dx+1)<<12 | (dy+1)<<14)
  int* ncnt;                 // its length per particle
  float* feat;               // NULL, or 12 features per particle at [g] (storage order)
  uint32_t* vl;              // Verlet list (pairs within the Verlet radius at the last build), layout as nl;
                             // every pass walks it through the neighbour predicate
  int* vcnt;                 // Verlet list length
  float2* off_build;         // offset of each particle when the Verlet list was built
  const int* id;             // particle ids (sorted order)
};

// Kernel variant of the pair passes.
struct PassCfg { int T, LPP, COMP, FORM, EL, KERN, Q3, INTEG; };

// Arguments of the binning, ingest, export and reduction kernels.
struct SortArgs {
  const RepDev* reps;
  int R;
  int ncells, ntot;
  int* cell_start;       // [ncells + 1]
  int* count;            // [ncells], zero between sorts
  int* cursor;           // [ncells], zero between sorts
  int* perm;             // [ntot]
  // unsorted staging copy of the persistent fields
  int* t_key; float2* t_off; float2* t_lo; float2* t_u; float2* t_q; float* t_drho; float2* t_acc; int* t_id;
  int2* t_img; float* t_qyy;
  // persistent sorted fields
  float2* off; float2* offlo; float2* u; float2* q; float* drho; float2* acc; int* id; int* cell;
  int2* img;             // periodic image of each particle: unwrapped r = r + img * L
  float* qyy;            // Qyy (quasi-2D variant), current parity
  unsigned* flags;
  const unsigned* gate;  // run only when *gate != 0 (NULL: always)
  const float2* off_build;  // offsets at the last Verlet build (displacement checks)
};

// Launchers (nem_passes.hip, nem_sort.hip).
bool launch_pass(int pass, const PassCfg& c, const StepArgs& a, hipStream_t s);
bool launch_pass_a_verlet(const PassCfg& c, const StepArgs& a, hipStream_t s);
void launch_request_relist(unsigned* flags, hipStream_t st);
void launch_list_export(int T, int kern, const StepArgs& a, int rep, int which, int mode, int* cnt,
                        const int64_t* row_ptr, int32_t* col, int64_t cap, hipStream_t s);
void launch_export_offsets(const SortArgs& s, int r, int n, int* cxy, float* oxy, hipStream_t st);
void launch_ingest(const SortArgs& s, int r, const double* in, int n, unsigned* umax, hipStream_t st);
void launch_rebin_key(const SortArgs& s, hipStream_t st);
void launch_sort_tail(const SortArgs& s, int k0, int n, int c0, int nc, int base, hipStream_t st);
void launch_step_begin(unsigned* flags, unsigned* umax_nxt, int R, hipStream_t st);
void launch_export(const SortArgs& s, int r, double* out, int n, hipStream_t st);
void launch_track(const SortArgs& s, int r, int n, int* inv, const int* ids, int nt, double* out, hipStream_t st);
void launch_qyy_io(const SortArgs& s, int r, int n, double* buf, int to_device, hipStream_t st);
void launch_colour_counts(const SortArgs& s, int r, int n, const uint8_t* colour, int ncol, int B,
                          unsigned long long* counts, hipStream_t st);
void launch_reduce(const SortArgs& s, int r, int n, const double* fe, double* red, hipStream_t st);
void launch_free_energy(int T, int kern, const StepArgs& a, double* fe, hipStream_t s);
void launch_int_offsets(const SortArgs& s, float2* out, hipStream_t st);
void launch_deposit(int T, int kern, const StepArgs& a, int rep, int M, double* grid, hipStream_t s);
void launch_fft2(const double* grid, double2* z, double2* w, int M, int logM, hipStream_t s);
void launch_shells(const double2* Z, int M, int nbins, double* part, double* E, hipStream_t s);
void launch_vort_correlation(const double2* W, int M, int logM, double L, double2* z, double2* w, double* axes,
                             hipStream_t s);
void launch_winding(const double* grid, int M, unsigned long long* counts, hipStream_t s);

}  // namespace nem
