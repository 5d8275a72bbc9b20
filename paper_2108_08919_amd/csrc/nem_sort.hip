// nem_sort.hip -- binning of particles into cells (counting sort), ingest of
// host states, export to id order, and the per-step bookkeeping kernels.
//
// Particles are kept sorted by (replica, cell, id): every cell is a contiguous
// run and the order inside a cell is canonical, so results do not depend on
// the order in which atomics land. Rebinning happens only when some particle
// has left its cell by more than skin/2 (pass D raises flags[1]); the kernels
// below read that flag themselves and return at once when it is clear, so the
// per-step launch sequence is fixed.
#include "nem_dev.h"

namespace nem {



__device__ inline bool gated(const unsigned* gate) { return gate != nullptr && *gate == 0u; }

__device__ inline int rep_of_particle(const RepDev* reps, int R, int k) {
  int lo = 0, hi = R;  // largest r with part_base <= k
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (reps[mid].part_base <= k) lo = mid; else hi = mid;
  }
  return lo;
}

// Host state (FP64, id order) of replica r -> unsorted staging arrays.
// Takes the first predictor half-step in double precision:
// u^{n+1/2} = u^n + a dt/2, r^{n+1/2} = wrap(r^n + u^{n+1/2} dt/2).
__global__ void k_ingest(SortArgs s, int r, const double* __restrict__ in, int n, unsigned* umax) {
  const RepDev R = s.reps[r];
  const double* x = in;
  const double* y = in + n;
  const double* ux = in + 2 * (size_t)n;
  const double* uy = in + 3 * (size_t)n;
  const double* qxx = in + 4 * (size_t)n;
  const double* qxy = in + 5 * (size_t)n;
  const double* rho = in + 6 * (size_t)n;
  const double* ax = in + 7 * (size_t)n;
  const double* ay = in + 8 * (size_t)n;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
#pragma clang fp contract(off)
    const double hdt = 0.5 * (double)R.dt;
    const double uhx = ux[i] + hdt * ax[i], uhy = uy[i] + hdt * ay[i];
    double xh = x[i] + hdt * uhx, yh = y[i] + hdt * uhy;
    // wrap into [0, L), counting the periodic images taken off
    double ix = floor(xh / R.Ld), iy = floor(yh / R.Ld);
    xh = xh - R.Ld * ix; if (xh >= R.Ld) { xh -= R.Ld; ix += 1.0; } if (xh < 0.0) xh = 0.0;
    yh = yh - R.Ld * iy; if (yh >= R.Ld) { yh -= R.Ld; iy += 1.0; } if (yh < 0.0) yh = 0.0;
    if (!(fabs(ix) < 1e9 && fabs(iy) < 1e9)) { atomicOr(s.flags, ERR_RANGE); ix = 0.0; iy = 0.0; }
    int cx = (int)floor(xh / R.csd), cy = (int)floor(yh / R.csd);
    cx = min(max(cx, 0), R.nc - 1);
    cy = min(max(cy, 0), R.nc - 1);
    const double bx = (double)cx * R.csd, by = (double)cy * R.csd;
    const double ox = xh - bx, oy = yh - by;
    const float hx = (float)ox, hy = (float)oy;
    const float lx = (float)(ox - (double)hx), ly = (float)(oy - (double)hy);
    const int k = R.part_base + i;
    const int key = R.cell_base + cy * R.nc + cx;
    s.t_key[k] = key;
    s.t_off[k] = make_float2(hx, hy);
    s.t_lo[k] = make_float2(lx, ly);
    const float2 uf = make_float2((float)uhx, (float)uhy);
    s.t_u[k] = uf;
    s.t_q[k] = make_float2((float)qxx[i], (float)qxy[i]);
    s.t_qyy[k] = -(float)qxx[i];   // quasi-2D variant: Qzz = 0 until nem_set_qyy
    s.t_drho[k] = (float)(rho[i] - (double)R.rho0);
    s.t_acc[k] = make_float2((float)ax[i], (float)ay[i]);
    s.t_id[k] = i;
    s.t_img[k] = make_int2((int)ix, (int)iy);
    atomicAdd(&s.count[key], 1);
    atomicMax(&umax[r * UMAX_SLOTS + (i & (UMAX_SLOTS - 1))], __float_as_uint(sqrtf(uf.x * uf.x + uf.y * uf.y)));
  }
}

// Rebin step 1: re-base every particle into the cell its offset now lies in
// (cells move by at most one per direction between rebins) and copy it to the
// staging arrays.
__global__ void k_rebin_key(SortArgs s) {
  if (gated(s.gate)) return;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < s.ntot; k += gridDim.x * blockDim.x) {
    const int r = rep_of_particle(s.reps, s.R, k);
    const RepDev R = s.reps[r];
    const int c = s.cell[k] - R.cell_base;
    if (c < 0 || c >= R.nc * R.nc) { atomicOr(s.flags, ERR_RANGE); continue; }
    int cx = c % R.nc, cy = c / R.nc;
    const float2 o = s.off[k], lo = s.offlo[k];
    int dx = (o.x < 0.0f) ? -1 : (o.x >= R.cs ? 1 : 0);
    int dy = (o.y < 0.0f) ? -1 : (o.y >= R.cs ? 1 : 0);
    if (o.x < -R.cs || o.x >= 2.0f * R.cs || o.y < -R.cs || o.y >= 2.0f * R.cs) atomicOr(s.flags, ERR_RANGE);
    float2 nh, nl;
    {
#pragma clang fp contract(off)
      // (hi, lo) - d (cs, cs_lo), renormalised
      // TwoSum of hi - d*cs keeps the rounding error of the subtraction
      const float shx = (float)(-dx) * R.cs, slx = (float)(-dx) * R.cs_lo;
      float t = o.x + shx, bp = t - o.x;
      float e = (o.x - (t - bp)) + (shx - bp);
      float l2 = (lo.x + slx) + e;
      nh.x = t + l2; nl.x = l2 - (nh.x - t);
      const float shy = (float)(-dy) * R.cs, sly = (float)(-dy) * R.cs_lo;
      t = o.y + shy; bp = t - o.y;
      e = (o.y - (t - bp)) + (shy - bp);
      l2 = (lo.y + sly) + e;
      nh.y = t + l2; nl.y = l2 - (nh.y - t);
    }
    // crossing the periodic boundary changes the particle's image
    int2 im = s.img[k];
    if (cx + dx < 0) im.x -= 1; else if (cx + dx >= R.nc) im.x += 1;
    if (cy + dy < 0) im.y -= 1; else if (cy + dy >= R.nc) im.y += 1;
    cx = (cx + dx + R.nc) % R.nc;
    cy = (cy + dy + R.nc) % R.nc;
    const int key = R.cell_base + cy * R.nc + cx;
    s.t_key[k] = key;
    s.t_off[k] = nh;
    s.t_lo[k] = nl;
    s.t_u[k] = s.u[k];
    s.t_q[k] = s.q[k];
    s.t_qyy[k] = s.qyy[k];
    s.t_drho[k] = s.drho[k];
    s.t_acc[k] = s.acc[k];
    s.t_id[k] = s.id[k];
    s.t_img[k] = im;
    atomicAdd(&s.count[key], 1);
  }
}

// Exclusive scan of count[c0 .. c0+nc) into cell_start[c0 ..], offset by base;
// cell_start[c0+nc] = base + total. One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan(SortArgs s, int c0, int nc, int base) {
  if (gated(s.gate)) return;
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int chunk = (nc + 1023) / 1024;
  const int b = min(nc, t * chunk), e = min(nc, b + chunk);
  int sum = 0;
  for (int i = b; i < e; ++i) sum += s.count[c0 + i];
  part[t] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // Hillis-Steele inclusive scan
    int v = (t >= d) ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = base + part[t] - sum;
  for (int i = b; i < e; ++i) {
    s.cell_start[c0 + i] = run;
    run += s.count[c0 + i];
  }
  if (t == 1023) s.cell_start[c0 + nc] = base + part[1023];
}

// Place each staged particle in its cell's range (arbitrary order inside).
__global__ void k_scatter(SortArgs s, int k0, int n) {
  if (gated(s.gate)) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int k = k0 + i;
    const int key = s.t_key[k];
    if (key < 0 || key >= s.ncells) { atomicOr(s.flags, ERR_RANGE); continue; }
    const int slot = s.cell_start[key] + atomicAdd(&s.cursor[key], 1);
    if (slot < 0 || slot >= s.ntot) { atomicOr(s.flags, ERR_RANGE); continue; }
    s.perm[slot] = k;
  }
}

// Canonical order inside each cell: ascending particle id (insertion sort of
// the short per-cell runs, one thread per cell).
__global__ void k_cellsort(SortArgs s, int c0, int nc) {
  if (gated(s.gate)) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += gridDim.x * blockDim.x) {
    const int b = s.cell_start[c0 + i], e = s.cell_start[c0 + i + 1];
    if (b < 0 || e > s.ntot || b > e) { atomicOr(s.flags, ERR_RANGE); continue; }
    bool ok = true;
    for (int a = b; a < e; ++a) {
      const int v = s.perm[a];
      if (v < 0 || v >= s.ntot) ok = false;
    }
    if (!ok) { atomicOr(s.flags, ERR_RANGE); continue; }
    for (int a = b + 1; a < e; ++a) {
      const int v = s.perm[a];
      const int kv = s.t_id[v];
      int c = a - 1;
      while (c >= b && s.t_id[s.perm[c]] > kv) { s.perm[c + 1] = s.perm[c]; --c; }
      s.perm[c + 1] = v;
    }
  }
}

// Move staged particles to their sorted slots; clear count/cursor of the cells.
__global__ void k_gather(SortArgs s, int k0, int n, int c0, int nc) {
  if (gated(s.gate)) return;
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int k = k0 + i;
    const int src = s.perm[k];
    if (src < 0 || src >= s.ntot) { atomicOr(s.flags, ERR_RANGE); continue; }
    s.off[k] = s.t_off[src];
    s.offlo[k] = s.t_lo[src];
    s.u[k] = s.t_u[src];
    s.q[k] = s.t_q[src];
    s.qyy[k] = s.t_qyy[src];
    s.drho[k] = s.t_drho[src];
    s.acc[k] = s.t_acc[src];
    s.id[k] = s.t_id[src];
    s.img[k] = s.t_img[src];
    s.cell[k] = s.t_key[src];
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += stride) {
    s.count[c0 + i] = 0;
    s.cursor[c0 + i] = 0;
  }
}

// Start of a step: clear the rebin request (after the gated kernels read it)
// and the next step's max-speed accumulators.
// After the (gated) rebin: decide whether this step rebuilds the Verlet list
// (a rebin happened or a rebuild was requested), clear both requests, and clear
// the max-speed slots that this step's pass D fills.
__global__ void k_step_begin(unsigned* flags, unsigned* umax_nxt, int R) {
  const int t = threadIdx.x;
  if (t == 0) {
    flags[3] = (flags[1] | flags[2]) ? 1u : 0u;
    flags[2] = 0u;
    flags[1] = 0u;
  }
  for (int r = t; r < R * UMAX_SLOTS; r += blockDim.x) umax_nxt[r] = 0u;
}

// Request a Verlet rebuild at the next step (new state, tile change, restore).
__global__ void k_request_relist(unsigned* flags) {
  if (blockIdx.x == 0 && threadIdx.x == 0) flags[2] = 1u;
}

// Position of sorted particle k at the integer time level,
// r^n = r^{n+1/2} - u^{n+1/2} dt/2, relative to the box of its image (may lie
// just outside [0, L) after the half-step back).
__device__ inline void position_n(const SortArgs& s, const RepDev& R, int k, double& x, double& y) {
#pragma clang fp contract(off)
  const int c = s.cell[k] - R.cell_base;
  const int cx = c % R.nc, cy = c / R.nc;
  const float2 o = s.off[k], lo = s.offlo[k], uh = s.u[k];
  const double hdt = 0.5 * (double)R.dt;
  x = (double)cx * R.csd + ((double)o.x + (double)lo.x) - hdt * (double)uh.x;
  y = (double)cy * R.csd + ((double)o.y + (double)lo.y) - hdt * (double)uh.y;
}

// The same wrapped into [0, L).
__device__ inline void position_n_wrapped(const SortArgs& s, const RepDev& R, int k, double& x, double& y) {
#pragma clang fp contract(off)
  position_n(s, R, k, x, y);
  x = x - R.Ld * floor(x / R.Ld); if (x >= R.Ld) x -= R.Ld;
  y = y - R.Ld * floor(y / R.Ld); if (y >= R.Ld) y -= R.Ld;
}

// Sorted state of replica r -> FP64 arrays in id order at the integer time
// level: r^n = r^{n+1/2} - u^{n+1/2} dt/2, u^n = u^{n+1/2} - a dt/2.
__global__ void k_export(SortArgs s, int r, double* out, int n) {
  const RepDev R = s.reps[r];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
#pragma clang fp contract(off)
    const int k = R.part_base + i;
    const int id = s.id[k];
    if (id < 0 || id >= n) { atomicOr(s.flags, ERR_RANGE); continue; }
    const float2 uh = s.u[k], ac = s.acc[k], q = s.q[k];
    const double hdt = 0.5 * (double)R.dt;
    const double uxn = (double)uh.x - hdt * (double)ac.x;
    const double uyn = (double)uh.y - hdt * (double)ac.y;
    double x, y;
    position_n_wrapped(s, R, k, x, y);
    out[id] = x;
    out[(size_t)n + id] = y;
    out[2 * (size_t)n + id] = uxn;
    out[3 * (size_t)n + id] = uyn;
    out[4 * (size_t)n + id] = (double)q.x;
    out[5 * (size_t)n + id] = (double)q.y;
    out[6 * (size_t)n + id] = (double)R.rho0 + (double)s.drho[k];
    out[7 * (size_t)n + id] = (double)ac.x;
    out[8 * (size_t)n + id] = (double)ac.y;
  }
}

// Cell coordinates and FP32 offsets (high part) of every particle of replica r
// at r^{n+1/2}, the values the neighbour predicate of the next step reads:
// cxy[2 id + 0/1] = cell x/y, oxy[2 id + 0/1] = offset x/y from the cell corner.
__global__ void k_export_offsets(SortArgs s, int r, int n, int* cxy, float* oxy) {
  const RepDev R = s.reps[r];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int k = R.part_base + i;
    const int id = s.id[k];
    const int c = s.cell[k] - R.cell_base;
    if (id < 0 || id >= n || c < 0 || c >= R.nc * R.nc) { atomicOr(s.flags, ERR_RANGE); continue; }
    const float2 o = s.off[k];
    cxy[2 * (size_t)id] = c % R.nc;
    cxy[2 * (size_t)id + 1] = c / R.nc;
    oxy[2 * (size_t)id] = o.x;
    oxy[2 * (size_t)id + 1] = o.y;
  }
}

// Qyy of replica r (quasi-2D variant) to or from an FP64 array in id order:
// to_device != 0 copies buf[id] into the sorted array, else the reverse.
__global__ void k_qyy_io(SortArgs s, int r, int n, double* buf, int to_device) {
  const RepDev R = s.reps[r];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int k = R.part_base + i;
    const int id = s.id[k];
    if (id < 0 || id >= n) { atomicOr(s.flags, ERR_RANGE); continue; }
    if (to_device) s.qyy[k] = (float)buf[id];
    else buf[id] = (double)s.qyy[k];
  }
}

// Pathlines: inv[id] = sorted slot of every particle of replica r.
__global__ void k_track_inv(SortArgs s, int r, int n, int* inv) {
  const RepDev R = s.reps[r];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int k = R.part_base + i;
    const int id = s.id[k];
    if (id < 0 || id >= n) { atomicOr(s.flags, ERR_RANGE); continue; }
    inv[id] = k;
  }
}

// Unwrapped integer-level positions of the particles ids[0..nt):
// out[t] = x + img_x L, out[nt + t] = y + img_y L.
__global__ void k_track(SortArgs s, int r, int n, const int* inv, const int* ids, int nt, double* out) {
  const RepDev R = s.reps[r];
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += gridDim.x * blockDim.x) {
#pragma clang fp contract(off)
    const int id = ids[t];
    const int k = (id >= 0 && id < n) ? inv[id] : -1;
    if (k < R.part_base || k >= R.part_base + n) {
      atomicOr(s.flags, ERR_RANGE);
      out[t] = NAN; out[(size_t)nt + t] = NAN;
      continue;
    }
    double x, y;
    position_n(s, R, k, x, y);
    const int2 im = s.img[k];
    out[t] = x + (double)im.x * R.Ld;
    out[(size_t)nt + t] = y + (double)im.y * R.Ld;
  }
}

// Mixing: counts[(by * B + bx) * ncol + c] = particles of colour c (by id) in
// bin (bx, by) of a B x B partition of the box, from the wrapped integer-level
// positions, bx = floor(x B / L).
__global__ void k_colour_counts(SortArgs s, int r, int n, const uint8_t* colour, int ncol, int B,
                                unsigned long long* counts) {
  const RepDev R = s.reps[r];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
#pragma clang fp contract(off)
    const int k = R.part_base + i;
    const int id = s.id[k];
    if (id < 0 || id >= n) { atomicOr(s.flags, ERR_RANGE); continue; }
    const int c = colour[id];
    if (c >= ncol) { atomicOr(s.flags, ERR_RANGE); continue; }
    double x, y;
    position_n_wrapped(s, R, k, x, y);
    const int bx = min(max((int)floor(x * (double)B / R.Ld), 0), B - 1);
    const int by = min(max((int)floor(y * (double)B / R.Ld), 0), B - 1);
    atomicAdd(&counts[((size_t)by * B + bx) * ncol + c], 1ull);
  }
}

// FP64 reductions of replica r at the integer time level (fixed grid, fixed
// tree: the result does not depend on scheduling). Stage 1: one partial per
// block in red[64 + 8*b + k]; stage 2 sums them in order into red[0..6]:
// sum ux, sum uy, sum |u|^2 / 2, max |u|, max |Q|_F, sum F_i, sum F_grad_i
// (fe = per-particle free-energy terms, ntot apart; may be NULL).
constexpr int RED_BLOCKS = 256;
__global__ __launch_bounds__(256) void k_reduce1(SortArgs s, int r, int n, const double* fe, double* red) {
  const RepDev R = s.reps[r];
  __shared__ double sh[7][256];
  double a0 = 0, a1 = 0, a2 = 0, m0 = 0, m1 = 0, f0 = 0, f1 = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int k = R.part_base + i;
    const float2 uh = s.u[k], ac = s.acc[k], q = s.q[k];
    const double hdt = 0.5 * (double)R.dt;
    const double ux = (double)uh.x - hdt * (double)ac.x, uy = (double)uh.y - hdt * (double)ac.y;
    const double u2 = ux * ux + uy * uy;
    a0 += ux; a1 += uy; a2 += 0.5 * u2;
    m0 = fmax(m0, sqrt(u2));
    if (R.q3d) {  // 3x3 Frobenius norm, Qzz = -Qxx - Qyy
      const double qa = q.x, qb = q.y, qc = s.qyy[k], qz = -qa - qc;
      m1 = fmax(m1, sqrt(qa * qa + 2.0 * qb * qb + qc * qc + qz * qz));
    } else {
      m1 = fmax(m1, sqrt(2.0 * ((double)q.x * q.x + (double)q.y * q.y)));
    }
    if (fe) { f0 += fe[k]; f1 += fe[(size_t)s.ntot + k]; }
  }
  const int t = threadIdx.x;
  sh[0][t] = a0; sh[1][t] = a1; sh[2][t] = a2; sh[3][t] = m0; sh[4][t] = m1; sh[5][t] = f0; sh[6][t] = f1;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (t < d) {
      sh[0][t] += sh[0][t + d]; sh[1][t] += sh[1][t + d]; sh[2][t] += sh[2][t + d];
      sh[3][t] = fmax(sh[3][t], sh[3][t + d]); sh[4][t] = fmax(sh[4][t], sh[4][t + d]);
      sh[5][t] += sh[5][t + d]; sh[6][t] += sh[6][t + d];
    }
    __syncthreads();
  }
  if (t < 7) red[64 + 8 * blockIdx.x + t] = sh[t][0];
}
__global__ void k_reduce2(double* red) {
  if (threadIdx.x != 0) return;
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = 0; b < RED_BLOCKS; ++b) {
    for (int k = 0; k < 3; ++k) v[k] += red[64 + 8 * b + k];
    for (int k = 3; k < 5; ++k) v[k] = fmax(v[k], red[64 + 8 * b + k]);
    for (int k = 5; k < 7; ++k) v[k] += red[64 + 8 * b + k];
  }
  for (int k = 0; k < 7; ++k) red[k] = v[k];
}

// Integer-level offsets r^n = r^{n+1/2} - u^{n+1/2} dt/2 relative to the binned
// cells (FP32), for diagnostics that need the pair geometry at r^n.
__global__ void k_int_offsets(SortArgs s, float2* out) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < s.ntot; k += gridDim.x * blockDim.x) {
    const int r = rep_of_particle(s.reps, s.R, k);
    const float hdt = 0.5f * s.reps[r].dt;
    const float2 o = s.off[k], lo = s.offlo[k], u = s.u[k];
    out[k] = make_float2(o.x + (lo.x - hdt * u.x), o.y + (lo.y - hdt * u.y));
  }
}

// -------------------------------------------------------------- launchers
static int grid_for(int n) { return max(1, min((n + 255) / 256, 2048)); }

void launch_ingest(const SortArgs& s, int r, const double* in, int n, unsigned* umax, hipStream_t st) {
  hipLaunchKernelGGL(k_ingest, dim3(grid_for(n)), dim3(256), 0, st, s, r, in, n, umax);
}
void launch_rebin_key(const SortArgs& s, hipStream_t st) {
  hipLaunchKernelGGL(k_rebin_key, dim3(grid_for(s.ntot)), dim3(256), 0, st, s);
}
void launch_sort_tail(const SortArgs& s, int k0, int n, int c0, int nc, int base, hipStream_t st) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, s, c0, nc, base);
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(n)), dim3(256), 0, st, s, k0, n);
  hipLaunchKernelGGL(k_cellsort, dim3(grid_for(nc)), dim3(256), 0, st, s, c0, nc);
  hipLaunchKernelGGL(k_gather, dim3(grid_for(max(n, nc))), dim3(256), 0, st, s, k0, n, c0, nc);
}
void launch_step_begin(unsigned* flags, unsigned* umax_nxt, int R, hipStream_t st) {
  hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(256), 0, st, flags, umax_nxt, R);
}
void launch_request_relist(unsigned* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_request_relist, dim3(1), dim3(64), 0, st, flags);
}
void launch_int_offsets(const SortArgs& s, float2* out, hipStream_t st) {
  hipLaunchKernelGGL(k_int_offsets, dim3(grid_for(s.ntot)), dim3(256), 0, st, s, out);
}
void launch_reduce(const SortArgs& s, int r, int n, const double* fe, double* red, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce1, dim3(RED_BLOCKS), dim3(256), 0, st, s, r, n, fe, red);
  hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(64), 0, st, red);
}
void launch_export(const SortArgs& s, int r, double* out, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_export, dim3(grid_for(n)), dim3(256), 0, st, s, r, out, n);
}

void launch_export_offsets(const SortArgs& s, int r, int n, int* cxy, float* oxy, hipStream_t st) {
  hipLaunchKernelGGL(k_export_offsets, dim3(grid_for(n)), dim3(256), 0, st, s, r, n, cxy, oxy);
}

void launch_qyy_io(const SortArgs& s, int r, int n, double* buf, int to_device, hipStream_t st) {
  hipLaunchKernelGGL(k_qyy_io, dim3(grid_for(n)), dim3(256), 0, st, s, r, n, buf, to_device);
}

void launch_track(const SortArgs& s, int r, int n, int* inv, const int* ids, int nt, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_track_inv, dim3(grid_for(n)), dim3(256), 0, st, s, r, n, inv);
  hipLaunchKernelGGL(k_track, dim3(grid_for(nt)), dim3(256), 0, st, s, r, n, (const int*)inv, ids, nt, out);
}

void launch_colour_counts(const SortArgs& s, int r, int n, const uint8_t* colour, int ncol, int B,
                          unsigned long long* counts, hipStream_t st) {
  hipLaunchKernelGGL(k_colour_counts, dim3(grid_for(n)), dim3(256), 0, st, s, r, n, colour, ncol, B, counts);
}

}  // namespace nem
