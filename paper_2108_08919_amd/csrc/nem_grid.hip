// nem_grid.hip -- grid diagnostics of one replica: Shepard deposit of the
// particle fields onto an M x M grid, the kinetic-energy spectrum through a
// double-precision 2D FFT, and the count of +-1/2 defects (paper Sec. 5:
// Eq. kineticenergy and the energy spectrum; defect maps).
//
//   deposit  f_g = sum_j f_j W(|x_g - x_j|) / sum_j W(|x_g - x_j|) over particles
//            within 3h of node g, nodes at ((i+1/2) L/M, (j+1/2) L/M), fields
//            at the integer time level (u^n, Q^n); FP32 pair sums, FP64 out
//   spectrum z = u_x + i u_y, 2D FFT (radix-2, in LDS, rows then transposed
//            rows), E(n) = 1/2 sum_{shell n} (|u_x^|^2 + |u_y^|^2) / M^4 with
//            |u_x^(k)|^2 + |u_y^(k)|^2 = (|z^(k)|^2 + |z^(-k)|^2) / 2,
//            shell n = floor(|k| L/2pi + 1/2); per-row partial histograms are
//            summed in row order, so the result is deterministic
//   defects  theta = atan2(Qxy, Qxx)/2 per node; around each unit plaquette the
//            four edge differences wrapped into (-pi/2, pi/2] add to +-pi at a
//            +-1/2 defect; counted with integer atomics
#include "nem_dev.h"
#include "nem_pair.h"

namespace nem {

// --------------------------------------------------------------- deposit
template <int T, int KERN>
__global__ __launch_bounds__(WG) void k_deposit(const StepArgs a, int rep_only, int M, double* grid) {
  __shared__ TileLDS<T> L;
  constexpr int MP = TileCfg<T, KERN>::MAXP;
  __shared__ float2 s_off[MP];
  __shared__ float4 s_f[MP];   // ux, uy, qxx, qxy at the integer level
  RepDev R;
  int rep;
  if (!tile_begin<T, KERN>(a, blockIdx.x, L, R, rep)) return;
  if (rep != rep_only) return;
  const int ni = L.hdr[0], nj = L.hdr[1], nreg = L.hdr[3];
  const int S = L.cstart[nreg];
  const float hdt = 0.5f * R.dt;
  for (int t = threadIdx.x; t < S; t += WG) {
    const int g = staged_global<T>(a, L, t);
    s_off[t] = a.off_cur[g];
    const float2 u = a.u[g], ac = a.acc[g], q = a.q_cur[g];
    // third field: Qxx in d = 2; (Qxx - Qyy)/2, the in-plane traceless part, in
    // the quasi-2D variant (the same director angle atan2(Qxy, .)/2)
    const float qa = R.q3d ? 0.5f * (q.x - a.qyy_cur[g]) : q.x;
    s_f[t] = make_float4(u.x - hdt * ac.x, u.y - hdt * ac.y, qa, q.y);
  }
  __syncthreads();
  const int tile = a.work[2 * blockIdx.x + 1];
  const int cx0 = (tile % R.tiles_x) * T, cy0 = (tile / R.tiles_x) * T;
  const double hg = R.Ld / M;
  // nodes whose centre lies in the tile's cells: node i belongs to cell
  // floor((i + 1/2) hg / csd), the same rule for every tile
  const int ix0 = max(0, (int)floor(cx0 * R.csd / hg - 0.5) - 1);
  const int ix1 = min(M - 1, (int)ceil((cx0 + ni) * R.csd / hg - 0.5) + 1);
  const int iy0 = max(0, (int)floor(cy0 * R.csd / hg - 0.5) - 1);
  const int iy1 = min(M - 1, (int)ceil((cy0 + nj) * R.csd / hg - 0.5) + 1);
  const int nx = ix1 - ix0 + 1, nn = nx * (iy1 - iy0 + 1);
  for (int t = threadIdx.x; t < nn; t += WG) {
#pragma clang fp contract(off)
    const int ix = ix0 + t % nx, iy = iy0 + t / nx;
    const double gx = (ix + 0.5) * hg, gy = (iy + 0.5) * hg;
    int cx = (int)floor(gx / R.csd), cy = (int)floor(gy / R.csd);
    cx = min(cx, R.nc - 1); cy = min(cy, R.nc - 1);
    const int li = cx - cx0, lj = cy - cy0;
    if (li < 0 || li >= ni || lj < 0 || lj >= nj) continue;
    const float ox = (float)(gx - cx * R.csd), oy = (float)(gy - cy * R.csd);
    Acc<1> den, fx, fy, fa, fb;
    den.init(); fx.init(); fy.init(); fa.init(); fb.init();
    for (int cidx = 0; cidx < 9; ++cidx) {
      const int dy = cidx / 3 - 1, dx = cidx % 3 - 1;
      const int sc = L.slot[(lj + dy + 1) * (ni + 2) + (li + dx + 1)];
      const float sx = (float)(-dx) * R.cs, sy = (float)(-dy) * R.cs;
      for (int j = L.cstart[sc]; j < L.cstart[sc + 1]; ++j) {
        const float2 oj = s_off[j];
        float rx, ry, r2;
        pair_accept(ox, oy, oj.x, oj.y, sx, sy, R.R2, rx, ry, r2);
        if (!(r2 < R.R2)) continue;
        const float w = (r2 > 0.0f) ? kernel_w<KERN>(R, r2) : R.W0;
        const float4 f = s_f[j];
        den.add(w); fx.fma(f.x, w); fy.fma(f.y, w); fa.fma(f.z, w); fb.fma(f.w, w);
      }
      den.end_cell(); fx.end_cell(); fy.end_cell(); fa.end_cell(); fb.end_cell();
    }
    const double d = den.value();
    const size_t o = (size_t)iy * M + ix, MM = (size_t)M * M;
    const bool ok = d > 0.0;
    grid[o] = ok ? fx.value() / d : 0.0;
    grid[MM + o] = ok ? fy.value() / d : 0.0;
    grid[2 * MM + o] = ok ? fa.value() / d : 0.0;
    grid[3 * MM + o] = ok ? fb.value() / d : 0.0;
  }
}

// ------------------------------------------------------------------- FFT
// z[r][c] = ux + i uy from the deposit grid.
__global__ void k_pack_complex(const double* grid, double2* z, int M) {
  const size_t MM = (size_t)M * M;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < MM; k += (size_t)gridDim.x * blockDim.x)
    z[k] = make_double2(grid[k], grid[MM + k]);
}

__device__ inline unsigned bitrev(unsigned v, int bits) { return __brev(v) >> (32 - bits); }

// In-place radix-2 decimation-in-time FFT of each row (length M = 2^logM,
// forward sign), one workgroup per row, the row held in LDS.
__global__ __launch_bounds__(256) void k_fft_rows(double2* z, int M, int logM) {
  extern __shared__ double2 buf[];
  double2* row = z + (size_t)blockIdx.x * M;
  for (int i = threadIdx.x; i < M; i += blockDim.x) buf[bitrev(i, logM)] = row[i];
  __syncthreads();
  for (int s = 1; s <= logM; ++s) {
    const int half = 1 << (s - 1);
    for (int b = threadIdx.x; b < M / 2; b += blockDim.x) {
      const int grp = b / half, pos = b % half;
      const int i0 = grp * 2 * half + pos, i1 = i0 + half;
      double sn, cs;
      sincospi(-(double)pos / half, &sn, &cs);   // exp(-2 pi i pos / (2 half))
      const double2 x0 = buf[i0], x1 = buf[i1];
      const double tr = x1.x * cs - x1.y * sn, ti = x1.x * sn + x1.y * cs;
      buf[i0] = make_double2(x0.x + tr, x0.y + ti);
      buf[i1] = make_double2(x0.x - tr, x0.y - ti);
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < M; i += blockDim.x) row[i] = buf[i];
}

// out[c][r] = in[r][c] through 32 x 32 LDS tiles.
__global__ void k_transpose(const double2* in, double2* out, int M) {
  __shared__ double2 t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int r = by + k, c = bx + threadIdx.x;
    if (r < M && c < M) t[k][threadIdx.x] = in[(size_t)r * M + c];
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int r = bx + k, c = by + threadIdx.x;
    if (r < M && c < M) out[(size_t)r * M + c] = t[threadIdx.x][k];
  }
}

// Per-row shell histogram (one thread per row) of the energy of each mode.
__global__ void k_shell_rows(const double2* Z, int M, int nbins, double* part) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= M) return;
  double* h = part + (size_t)r * nbins;
  for (int n = 0; n < nbins; ++n) h[n] = 0.0;
  const double M4 = (double)M * M * (double)M * M;
  const int kr = (r < M / 2) ? r : r - M;
  const int rm = (M - r) % M;
  for (int c = 0; c < M; ++c) {
    const int kc = (c < M / 2) ? c : c - M;
    const int cm = (M - c) % M;
    const double2 a = Z[(size_t)r * M + c], b = Z[(size_t)rm * M + cm];
    const double e = 0.25 * ((a.x * a.x + a.y * a.y) + (b.x * b.x + b.y * b.y)) / M4;
    const int n = (int)floor(sqrt((double)kr * kr + (double)kc * kc) + 0.5);
    if (n < nbins) h[n] += e;
  }
}

__global__ void k_shell_sum(const double* part, int M, int nbins, double* E) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nbins) return;
  double s = 0.0;
  for (int r = 0; r < M; ++r) s += part[(size_t)r * nbins + n];
  E[n] = s;
}

// --------------------------------------------------------------- defects
__device__ inline double wrap_half_pi(double d) {
  const double pi = 3.14159265358979323846;
  double w = d - pi * floor(d / pi + 0.5);
  if (w <= -0.5 * pi) w += pi;
  return w;
}

__global__ void k_winding(const double* grid, int M, unsigned long long* counts) {
  const size_t MM = (size_t)M * M;
  const double* qxx = grid + 2 * MM;
  const double* qxy = grid + 3 * MM;
  const double pi = 3.14159265358979323846;
  unsigned long long np = 0, nm = 0;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < MM; k += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(k % M), j = (int)(k / M);
    const int i1 = (i + 1) % M, j1 = (j + 1) % M;
    const double ta = 0.5 * atan2(qxy[(size_t)j * M + i], qxx[(size_t)j * M + i]);
    const double tb = 0.5 * atan2(qxy[(size_t)j * M + i1], qxx[(size_t)j * M + i1]);
    const double tc = 0.5 * atan2(qxy[(size_t)j1 * M + i1], qxx[(size_t)j1 * M + i1]);
    const double td = 0.5 * atan2(qxy[(size_t)j1 * M + i], qxx[(size_t)j1 * M + i]);
    const double w = wrap_half_pi(tb - ta) + wrap_half_pi(tc - tb) + wrap_half_pi(td - tc) + wrap_half_pi(ta - td);
    if (w > 0.5 * pi) ++np;
    else if (w < -0.5 * pi) ++nm;
  }
  if (np) atomicAdd(&counts[0], np);
  if (nm) atomicAdd(&counts[1], nm);
}

// -------------------------------------------------------------- launchers
void launch_deposit(int T, int kern, const StepArgs& a, int rep, int M, double* grid, hipStream_t s) {
  const dim3 grid_(a.nwork), block(WG);
  if (kern == 1) {
    if (T == 8) hipLaunchKernelGGL((k_deposit<8, 1>), grid_, block, 0, s, a, rep, M, grid);
    else hipLaunchKernelGGL((k_deposit<4, 1>), grid_, block, 0, s, a, rep, M, grid);
  } else {
    if (T == 8) hipLaunchKernelGGL((k_deposit<8, 0>), grid_, block, 0, s, a, rep, M, grid);
    else hipLaunchKernelGGL((k_deposit<4, 0>), grid_, block, 0, s, a, rep, M, grid);
  }
}

// |omega^(k)|^2 of the vorticity omega = d uy/dx - d ux/dy from the 2D FFT
// W of z = ux + i uy (W[a*M + b] = Z(kx index a, ky index b), as launch_fft2
// leaves it): u^x(k) = (Z(k) + conj Z(-k))/2, u^y(k) = (Z(k) - conj Z(-k))/(2i),
// omega^ = i (kx u^y - ky u^x) with k = 2 pi n / L; the Nyquist wavenumber
// (n = -M/2) has no derivative on the grid and is set to zero. P keeps the
// (kx, ky) layout, as a complex array with zero imaginary part.
__global__ void k_vort_power(const double2* W, int M, double L, double2* P) {
  const size_t MM = (size_t)M * M;
  const double tpl = 2.0 * M_PI / L;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < MM; k += (size_t)gridDim.x * blockDim.x) {
    const int a = (int)(k / M), b = (int)(k % M);
    const int na = (a < M / 2) ? a : a - M, nb = (b < M / 2) ? b : b - M;
    const double kx = (na == -M / 2) ? 0.0 : tpl * na, ky = (nb == -M / 2) ? 0.0 : tpl * nb;
    const double2 z = W[k], zm = W[(size_t)((M - a) % M) * M + (M - b) % M];
    const double uxr = 0.5 * (z.x + zm.x), uxi = 0.5 * (z.y - zm.y);  // (Z + conj Zm) / 2
    const double uyr = 0.5 * (z.y + zm.y), uyi = -0.5 * (z.x - zm.x);  // (Z - conj Zm) / (2i)
    // omega^ = i (kx u^y - ky u^x): |omega^|^2 = |kx u^y - ky u^x|^2
    const double wr = kx * uyr - ky * uxr, wi = kx * uyi - ky * uxi;
    P[k] = make_double2(wr * wr + wi * wi, 0.0);
  }
}

// Row 0 and column 0 of the M x M grid V (real parts): out[0..M/2] = V[0][n],
// out[M/2+1..M+1] = V[n][0].
__global__ void k_grid_axes(const double2* V, int M, double* out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n > M / 2) return;
  out[n] = V[n].x;
  out[M / 2 + 1 + n] = V[(size_t)n * M].x;
}

void launch_vort_correlation(const double2* W, int M, int logM, double L, double2* z, double2* w, double* axes,
                             hipStream_t s) {
  const size_t MM = (size_t)M * M;
  const int nb = (int)std::min<size_t>((MM + 255) / 256, 4096);
  hipLaunchKernelGGL(k_vort_power, dim3(nb), dim3(256), 0, s, W, M, L, z);
  // second 2D FFT: rows of P (along ky), transpose, rows (along kx); the result
  // V[ry*M + rx] = sum_k P(k) e^{-i k.r} is M^4 times the periodic autocorrelation
  const size_t lds = sizeof(double2) * M;
  hipLaunchKernelGGL(k_fft_rows, dim3(M), dim3(256), lds, s, z, M, logM);
  const dim3 tg((M + 31) / 32, (M + 31) / 32), tb(32, 8);
  hipLaunchKernelGGL(k_transpose, tg, tb, 0, s, (const double2*)z, w, M);
  hipLaunchKernelGGL(k_fft_rows, dim3(M), dim3(256), lds, s, w, M, logM);
  hipLaunchKernelGGL(k_grid_axes, dim3((M / 2 + 1 + 255) / 256), dim3(256), 0, s, (const double2*)w, M, axes);
}

void launch_fft2(const double* grid, double2* z, double2* w, int M, int logM, hipStream_t s) {
  const size_t MM = (size_t)M * M;
  const int nb = (int)std::min<size_t>((MM + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pack_complex, dim3(nb), dim3(256), 0, s, grid, z, M);
  const size_t lds = sizeof(double2) * M;
  hipLaunchKernelGGL(k_fft_rows, dim3(M), dim3(256), lds, s, z, M, logM);
  const dim3 tg((M + 31) / 32, (M + 31) / 32), tb(32, 8);
  hipLaunchKernelGGL(k_transpose, tg, tb, 0, s, z, w, M);
  hipLaunchKernelGGL(k_fft_rows, dim3(M), dim3(256), lds, s, w, M, logM);
}

void launch_shells(const double2* Z, int M, int nbins, double* part, double* E, hipStream_t s) {
  hipLaunchKernelGGL(k_shell_rows, dim3((M + 63) / 64), dim3(64), 0, s, Z, M, nbins, part);
  hipLaunchKernelGGL(k_shell_sum, dim3((nbins + 255) / 256), dim3(256), 0, s, part, M, nbins, E);
}

void launch_winding(const double* grid, int M, unsigned long long* counts, hipStream_t s) {
  const size_t MM = (size_t)M * M;
  const int nb = (int)std::min<size_t>((MM + 255) / 256, 4096);
  hipLaunchKernelGGL(k_winding, dim3(nb), dim3(256), 0, s, grid, M, counts);
}

}  // namespace nem
