// nem_pair.h -- tile staging, neighbour predicate, smoothing kernels and
// compensated sums used by every pair pass (gfx950, wave64).
#pragma once
#include "nem_dev.h"

namespace nem {

// Tile geometry for a tile side of T cells. A workgroup stages the T x T
// interior cells of its tile plus a one-cell periodic halo into LDS; interior
// cells come first so that interior particles occupy LDS slots [0, nin).
// LDS particle capacity per staged cell: 24 for the quintic spline's cells
// (side >= 3h + skin = 4 dx, 16 particles on the lattice), 10 for Wendland C2's
// (side >= 2h + skin = 2.7 dx, 7.3 on the lattice), small enough that five
// workgroups of the 8 x 8 tile fit in one CU's LDS. A tile holding more sets
// ERR_OVERFLOW.
template <int T, int KERN = 0>
struct TileCfg {
  static constexpr int NSC = (T + 2) * (T + 2);
  static constexpr int MAXP = NSC * (KERN == 1 ? 10 : 24);
};

template <int T>
struct TileLDS {
  int cstart[TileCfg<T>::NSC + 1];  // prefix of staged counts (staged-cell order)
  int gstart[TileCfg<T>::NSC];      // first global particle of each staged cell
  int slot[TileCfg<T>::NSC];        // region index (lj+1)*(ni+2)+(li+1) -> staged cell
  int hdr[8];                       // ni, nj, nint, nreg
  float2 shift[16];                 // image shift of stencil direction (dx+1) | (dy+1) << 2
};

// Staged-cell index of region cell (li, lj), li in [-1, ni], lj in [-1, nj].
__device__ inline int staged_index(int li, int lj, int ni, int nj) {
  if (li >= 0 && li < ni && lj >= 0 && lj < nj) return lj * ni + li;
  int nint = ni * nj, rank;
  if (lj == -1) rank = li + 1;
  else if (lj < nj) rank = (ni + 2) + 2 * lj + (li == -1 ? 0 : 1);
  else rank = (ni + 2) + 2 * nj + (li + 1);
  return nint + rank;
}

// Fill the tile header and cell tables; returns the replica index. Every
// thread of the workgroup must call it.
template <int T>
__device__ int tile_setup(const StepArgs& a, int w, TileLDS<T>& L, RepDev& R) {
  const int rep = a.work[2 * w];
  const int tile = a.work[2 * w + 1];
  R = a.reps[rep];
  const int tx = tile % R.tiles_x, ty = tile / R.tiles_x;
  const int cx0 = tx * T, cy0 = ty * T;
  const int ni = min(T, R.nc - cx0), nj = min(T, R.nc - cy0);
  const int nreg = (ni + 2) * (nj + 2);
  const int t = threadIdx.x;
  __shared__ int cnt[TileCfg<T>::NSC];
  if (t < nreg) {
    const int li = t % (ni + 2) - 1, lj = t / (ni + 2) - 1;
    const int st = staged_index(li, lj, ni, nj);
    const int gx = (cx0 + li + R.nc) % R.nc, gy = (cy0 + lj + R.nc) % R.nc;
    const int gc = R.cell_base + gy * R.nc + gx;
    int s0 = 0, s1 = 0;
    if (gc >= 0 && gc < a.ncells) { s0 = a.cell_start[gc]; s1 = a.cell_start[gc + 1]; }
    else atomicOr(a.flags, ERR_RANGE);
    L.slot[t] = st;
    L.gstart[st] = s0;
    cnt[st] = max(s1 - s0, 0);
  }
  if (t == 0) { L.hdr[0] = ni; L.hdr[1] = nj; L.hdr[2] = ni * nj; L.hdr[3] = nreg; }
  if (t < 16) L.shift[t] = make_float2((float)(1 - (t & 3)) * R.cs, (float)(1 - (t >> 2)) * R.cs);
  __syncthreads();
  if (t < 64) {  // wave 0: exclusive scan of up to 128 counts, two per lane
    const int i0 = 2 * t, i1 = 2 * t + 1;
    const int v0 = i0 < nreg ? cnt[i0] : 0, v1 = i1 < nreg ? cnt[i1] : 0;
    int s = v0 + v1, inc = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      int o = __shfl_up(inc, d, 64);
      if (t >= d) inc += o;
    }
    const int ex = inc - s;
    if (t == 0) L.cstart[0] = 0;
    if (i0 < nreg) L.cstart[i0 + 1] = ex + v0;
    if (i1 < nreg) L.cstart[i1 + 1] = ex + v0 + v1;
  }
  __syncthreads();
  return rep;
}

// Staged cell containing LDS slot p, searching cstart[lo..hi).
__device__ inline int find_cell(const int* cstart, int hi, int p) {
  int lo = 0;  // invariant: cstart[lo] <= p < cstart[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (cstart[mid] <= p) lo = mid; else hi = mid;
  }
  return lo;
}

// Neighbour predicate on FP32 cell-relative offsets. For j in the stencil cell
// displaced by (dx, dy) from i's cell, sx = -dx*cs, sy = -dy*cs and
//   rx = fl(fl(oix - ojx) + sx), r2 = fl(fl(rx*rx) + fl(ry*ry)),
// accepted when 0 < r2 < R2 = fl32((3h)^2). No contraction, so the decision is
// reproducible bit for bit from the documented rule.
__device__ __forceinline__ bool pair_accept(float oix, float oiy, float ojx, float ojy, float sx,
                                            float sy, float R2, float& rx, float& ry, float& r2) {
#pragma clang fp contract(off)
  const float tx = oix - ojx;
  const float ty = oiy - ojy;
  rx = tx + sx;
  ry = ty + sy;
  const float xx = rx * rx;
  const float yy = ry * ry;
  r2 = xx + yy;
  return (r2 > 0.0f) & (r2 < R2);
}

// Smoothing kernels of support kappa h (2D), selected at compile time:
//   KERN 0: quintic spline, kappa = 3 (Eq. quintic; the paper's kernel),
//   KERN 1: Wendland C2, kappa = 2, W = a2 (1 - q/2)^4 (1 + 2q), a2 = 7/(4 pi h^2).
// F = (dW/dr)/r, so that grad_i W_ij = F r_ij.
// kernel_raw returns W and F without the replica's constant factors,
// Wr = W / a2 and Fr = F / dWc: the pair loops apply a2 once per particle after
// the sum and fold dWc into a staged per-particle factor (the volume), which
// takes two multiplies out of every pair.
//   quintic:     Wr = t3^5 - 6 t2^5 + 15 t1^5, Fr = (t3^4 - 6 t2^4 + 15 t1^4) / r,
//                t_m = (m - q)_+, q = r/h (dW/dr = dWc (...), dWc = -5 a2 / h);
//   Wendland C2: Wr = (1 - q/2)^4 (1 + 2q), Fr = (1 - q/2)^3 (dWc = -5 a2 / h^2).
// r2 is positive and far above the FP32 denormal range for every accepted pair
// (particles never come within 1e-19 of each other), so the hardware
// reciprocal square root is used without the denormal rescaling of rsqrtf.
// Every listed pair has r < 3h up to rounding, so t3 needs no clamp.
struct KW { float rinv, r, W, F; };
template <int KERN>
__device__ __forceinline__ KW kernel_raw(const RepDev& R, float r2) {
  KW k;
  k.rinv = __builtin_amdgcn_rsqf(r2);
  k.r = r2 * k.rinv;
  const float b = k.r * R.hinv;   // q
  // (1 - q)_+ and (2 - q)_+ / 2 lie in [0, 1] (q >= 0), so each is one
  // instruction with the result clamp. t2 = 2 u exactly (scaling by 2 commutes
  // with rounding), so -6 t2^4 = -96 u^4 and -6 t2^5 = -192 u^4 u give the same
  // bits as the unscaled form.
  if constexpr (KERN == 0) {
    const float t3 = 3.0f - b;
    const float u = fminf(fmaxf(fmaf(-0.5f, b, 1.0f), 0.0f), 1.0f);   // (2 - q)_+ / 2
    const float t1 = fminf(fmaxf(1.0f - b, 0.0f), 1.0f);               // (1 - q)_+
    const float t3s = t3 * t3, us = u * u, t1s = t1 * t1;
    const float t34 = t3s * t3s, u4 = us * us, t14 = t1s * t1s;
    k.W = fmaf(15.0f * t14, t1, fmaf(-192.0f * u4, u, t34 * t3));
    k.F = fmaf(15.0f, t14, fmaf(-96.0f, u4, t34)) * k.rinv;
  } else {
    const float t = fminf(fmaxf(fmaf(-0.5f, b, 1.0f), 0.0f), 1.0f);
    const float t2 = t * t;
    k.W = (t2 * t2) * fmaf(2.0f, b, 1.0f);
    k.F = t2 * t;
  }
  return k;
}

// W(0) / a2: the self term of the kernel sums in units of a2.
template <int KERN>
constexpr float kernel_w0_raw() { return KERN == 0 ? 66.0f : 1.0f; }

// W and F with their constant factors (passes off the step's hot path).
template <int KERN>
__device__ __forceinline__ KW kernel_wf(const RepDev& R, float r2) {
  KW k = kernel_raw<KERN>(R, r2);
  k.W *= R.a2;
  k.F *= R.dWc;
  return k;
}

// W only.
template <int KERN>
__device__ __forceinline__ float kernel_w(const RepDev& R, float r2) {
  return R.a2 * kernel_raw<KERN>(R, r2).W;
}

// A pair-sum accumulator. COMP 0: plain FP32 sum. COMP 1: Kahan summation over
// short chunks of pairs (a chunk is 16 listed pairs): terms are added plainly
// into the chunk partial p, and at the end of the chunk p is added to the
// running sum s with its rounding error recovered exactly (Fast2Sum) and
// carried into the next chunk's partial. That is Kahan's update applied to the
// chunk sums with the compensation held in p, so it costs two registers and
// three operations per chunk. COMP 2: Kahan compensation on every pair term.
template <int COMP>
struct Acc {
  float s, c, p;
  __device__ __forceinline__ void init() { s = 0.0f; c = 0.0f; p = 0.0f; }
  __device__ __forceinline__ static void kahan(float& s_, float& c_, float x) {
    const float y = x - c_;
    const float t = s_ + y;
    c_ = (t - s_) - y;
    s_ = t;
  }
  __device__ __forceinline__ void add(float x) {
    if constexpr (COMP == 0) s += x;
    else if constexpr (COMP == 1) p += x;
    else kahan(s, c, x);
  }
  __device__ __forceinline__ void fma(float a, float b) {
    if constexpr (COMP == 0) s = fmaf(a, b, s);
    else if constexpr (COMP == 1) p = fmaf(a, b, p);
    else { const float x = a * b; kahan(s, c, x); }
  }
  __device__ __forceinline__ void end_cell() {
    if constexpr (COMP == 1) {
#pragma clang fp contract(off)
      const float t = s + p;
      p = (s - t) + p;
      s = t;
    }
  }
  // This lane's compensated value. For COMP 1, s + p is also what closing an
  // open chunk would give (its rounded sum), so none is closed before this.
  __device__ __forceinline__ float value() const {
    if constexpr (COMP == 0) return s;
    else if constexpr (COMP == 1) return s + p;
    else return s - c;
  }
};

__device__ __forceinline__ void flag(unsigned* flags, unsigned bit) { atomicOr(flags, bit); }

// Common prologue: set up the tile, check LDS capacity. Returns false when the
// workgroup has nothing to do (uniform across the workgroup).
template <int T, int KERN = 0>
__device__ __forceinline__ bool tile_begin(const StepArgs& a, int w, TileLDS<T>& L, RepDev& R, int& rep) {
  if (w >= a.nwork) return false;
  rep = tile_setup<T>(a, w, L, R);
  const int S = L.cstart[L.hdr[3]];
  if (S > TileCfg<T, KERN>::MAXP) {
    if (threadIdx.x == 0) flag(a.flags, ERR_OVERFLOW);
    return false;
  }
  return true;
}

// Global index of LDS slot t (staging loop).
template <int T>
__device__ __forceinline__ int staged_global(const StepArgs& a, const TileLDS<T>& L, int t) {
  const int st = find_cell(L.cstart, L.hdr[3], t);
  int g = L.gstart[st] + (t - L.cstart[st]);
  if (g < 0 || g >= a.ntot) { flag(a.flags, ERR_RANGE); g = 0; }
  return g;
}


}  // namespace nem
