// nem_passes.hip -- the four pair passes of one SPH time step on gfx950.
//
// Each workgroup owns a tile of T x T cells of one replica and stages the tile
// plus its one-cell periodic halo into LDS (particles are sorted by cell, so
// every cell is a contiguous run). Positions are FP32 offsets from the
// particle's cell corner; the periodic image shift of a stencil cell is a whole
// number of cell sides, so pair vectors keep the precision of the offsets
// anywhere in the box.
//
// Every pass walks the particle's Verlet list: the pairs of the 3 x 3 cell
// stencil closer than 3h + delta when the list was built, as 16-bit entries
// (LDS slot of the neighbour in the tile's staging order + stencil direction).
// Each pass stages the same tile in the same order and puts every entry
// through the same FP32 predicate (0 < r^2 < (3h)^2), so all four passes sum
// over exactly the same neighbour set. Several lanes may share a particle
// (each takes every lpp-th entry; sums are combined with wave shuffles); a
// tile's short tail of particles is spread over more lanes.
//
//   pass A  Verlet list (rebuilt from the ~144 candidates of the stencil when
//           particles have moved too far); volume V_i = 1 / sum_j W_ij
//           (Eq. sphSum, self included)
//   pass B  correction tensor and B = alpha^{-1} (Eq. sphCorrectionMatrix),
//           velocity gradient and continuity (Eqs. sph1stDerivative,
//           sphContinuity), Q gradient and Laplacian, molecular field
//           (Eq. molecularfielddis), co-rotation (Eq. corotation), Q update
//           (Eq. mi), viscous and active accelerations (Eq. sphMomentum)
//   pass C  density filter (Eq. densityCorrection) and EoS (Eq. sphEos); APD
//           velocity variance (Eq. APD: u^{n+1/2} is the same as in pass B,
//           and this pass evaluates W anyway)
//   pass D  pressure term (Eq. sphMomentum), corrector, APD geometry sums and
//           displacement (Eq. APD) and the next step's predictor (Sec. 3.1),
//           fused
#include <algorithm>

#include "nem_dev.h"
#include "nem_pair.h"

namespace nem {

// Lanes per particle for an iteration with `rem` particles left: the base
// value, doubled while the particles still fill the workgroup (at most 16).
__device__ __forceinline__ int lanes_for(int rem, int base_lpp) {
  int l = base_lpp;
  while (l < 16 && rem * l * 2 <= WG) l <<= 1;
  return l;
}

__device__ __forceinline__ float wave_sum(float v, int lpp) {
  for (int o = 1; o < lpp; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_sum_int(int v, int lpp) {
  for (int o = 1; o < lpp; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Pair geometry of a list entry (LDS slot | direction code << 12) through the
// neighbour predicate: true when the pair is a neighbour at this step's
// positions. Every pass, and the list export, decides with this one function.
__device__ __forceinline__ bool verlet_pair(uint32_t e, const float2* shift, int jmax, const float2* s_off,
                                            float2 oi, float R2, int& j, float& rx, float& ry, float& r2) {
  j = min((int)(e & 0xFFFu), jmax);
  const float2 sh = shift[(e >> 12) & 15u];
  const float2 oj = s_off[j];
  return pair_accept(oi.x, oi.y, oj.x, oj.y, sh.x, sh.y, R2, rx, ry, r2);
}

// The 32-bit words of one particle's list (two 16-bit entries each, rows
// `stride` words apart), each loaded DEPTH words before it is used. The
// register copies w[i] = w[i + 1] make the compiler wait for a load DEPTH - 1
// iterations after issuing it, so pair work overlaps each load's latency (a
// load waited for at once left the passes stalled on HBM). Rows past the
// particle's nw words are not loaded.
template <int DEPTH>
struct ListStream {
  const uint32_t* p;
  size_t stride;
  int nw, m;
  uint32_t w[DEPTH];
  __device__ __forceinline__ ListStream(const uint32_t* p_, size_t stride_, int nwords)
      : p(p_), stride(stride_), nw(nwords), m(DEPTH) {
#pragma unroll
    for (int i = 0; i < DEPTH; ++i) w[i] = nw > i ? p[(size_t)i * stride] : 0u;
  }
  __device__ __forceinline__ uint32_t next() {
    const uint32_t r = w[0];
#pragma unroll
    for (int i = 0; i + 1 < DEPTH; ++i) w[i] = w[i + 1];
    w[DEPTH - 1] = m < nw ? p[(size_t)m * stride] : 0u;
    ++m;
    return r;
  }
};

// Walk the list of particle g: lane `sub` of `lpp` takes entries sub,
// sub+lpp, ...; flush() closes a compensation chunk every 16 entries (the
// last, open chunk is summed by the accumulators' value()).
// WPI: list words per iteration of the one-lane walk (2 puts four pairs of
// work behind each load; the chunking of the compensated sums is the same).
template <int WPI = 1, typename Body, typename Flush>
__device__ __forceinline__ void each_listed(const uint32_t* __restrict__ nl, int ntot, int g, int cnt, int lpp,
                                            int sub, Body&& body, Flush&& flush) {
  const uint32_t* p = nl + g;
  if (lpp == 1) {
    ListStream<WPI == 2 ? 3 : 2> ls(p, (size_t)ntot, (cnt + 1) >> 1);
    int k = 0;
    if constexpr (WPI == 2) {
      for (; k + 3 < cnt; k += 4) {
        const uint32_t wa = ls.next();
        const uint32_t wb = ls.next();
        body(wa & 0xFFFFu);
        body(wa >> 16);
        body(wb & 0xFFFFu);
        body(wb >> 16);
        if ((k & 15) == 12) flush();
      }
    }
    for (; k + 1 < cnt; k += 2) {
      const uint32_t w = ls.next();
      body(w & 0xFFFFu);
      body(w >> 16);
      if ((k & 15) == 14) flush();
    }
    if (k < cnt) body(ls.next() & 0xFFFFu);
  } else {
    int it = 0;
    for (int k = sub; k < cnt; k += lpp, ++it) {
      const uint32_t w = p[(size_t)(k >> 1) * ntot];
      body((k & 1) ? (w >> 16) : (w & 0xFFFFu));
      if ((it & 15) == 15) flush();
    }
  }
}

// --------------------------------------------- direct search (diagnostics)
// Volumes and an explicit neighbour list (nl, ncnt) at given offsets, for the
// free-energy kernel of the diagnostics, which runs between steps on the
// integer-level positions. The step itself uses the Verlet list below.
// Phase 1 runs the predicate over the candidates of the nine stencil cells and
// records, per cell, one 64-bit word: the accepted particles as a mask in bits
// 0-47 (bit b = b-th particle of the cell; a cell holds at most 48), the
// cell's first LDS slot in bits 48-59 and the stencil direction code in bits
// 60-63. Phase 2 walks the accepted pairs in cell order, all lanes taking their
// k-th pair together: it sums the kernel terms and emits the list entries
// (coalesced stores), so the kernel is evaluated for accepted pairs only.
constexpr int CELL_MAX = 48;
constexpr unsigned long long MASK48 = (1ull << 48) - 1ull;

template <int T, int COMP, int KERN>
__device__ __forceinline__ void tile_pass_a(const StepArgs& a, int w) {
  __shared__ TileLDS<T> L;
  __shared__ float2 s_off[TileCfg<T, KERN>::MAXP];
  __shared__ unsigned long long s_mask[9 * WG];  // lane-private, cell-major
  static_assert(TileCfg<T, KERN>::MAXP <= 4096, "LDS slot must fit 12 bits");
  RepDev R;
  int rep;
  if (!tile_begin<T, KERN>(a, w, L, R, rep)) return;
  const int ni = L.hdr[0], nint = L.hdr[2], nreg = L.hdr[3];
  const int S = L.cstart[nreg];
  for (int t = threadIdx.x; t < S; t += WG) s_off[t] = a.off_cur[staged_global<T>(a, L, t)];
  __syncthreads();
  const int nin = L.cstart[nint];
  const int tid = threadIdx.x;
  for (int base = 0; base < nin; base += WG) {
    const int p = base + tid;
    if (p >= nin) break;
    const int st = find_cell(L.cstart, nint, p);
    const int li = st % ni, lj = st / ni;
    const float2 oi = s_off[p];
    int cnt = 0;
    bool big = false;
#pragma unroll 1
    for (int cidx = 0; cidx < 9; ++cidx) {
      const int dy = cidx / 3, dx = cidx % 3;  // direction + 1
      const int sc = L.slot[(lj + dy) * (ni + 2) + (li + dx)];
      const int j0 = L.cstart[sc];
      const int nj = L.cstart[sc + 1] - j0;
      if (nj > CELL_MAX) big = true;
      const uint32_t code = (uint32_t)dx | ((uint32_t)dy << 2);
      const float2 sh = L.shift[code];
      uint32_t mlo = 0u, mhi = 0u;
      const int n0 = min(nj, 32), n1 = min(nj, CELL_MAX);
      for (int b = 0; b < n0; ++b) {
        const float2 oj = s_off[j0 + b];
        float rx, ry, r2;
        if (pair_accept(oi.x, oi.y, oj.x, oj.y, sh.x, sh.y, R.R2, rx, ry, r2)) mlo |= 1u << b;
      }
      for (int b = 32; b < n1; ++b) {
        const float2 oj = s_off[j0 + b];
        float rx, ry, r2;
        if (pair_accept(oi.x, oi.y, oj.x, oj.y, sh.x, sh.y, R.R2, rx, ry, r2)) mhi |= 1u << (b - 32);
      }
      s_mask[cidx * WG + tid] = ((unsigned long long)code << 60) | ((unsigned long long)j0 << 48) |
                                ((unsigned long long)mhi << 32) | mlo;
      cnt += __popc(mlo) + __popc(mhi);
    }
    const int kept = min(cnt, KMAX);
    const int g = L.gstart[st] + (p - L.cstart[st]);
    if (g < 0 || g >= a.ntot) { flag(a.flags, ERR_RANGE); continue; }
    if (cnt > KMAX || big) flag(a.flags, ERR_OVERFLOW);
    Acc<COMP> sw;
    sw.init();
    int c = -1;
    unsigned long long m = 0ull, x = 0ull;
    uint32_t word = 0u;
    uint32_t* dst = a.nl + g;
    for (int k = 0; k < kept; ++k) {
      while (m == 0ull && c < 8) {
        ++c;
        x = s_mask[c * WG + tid];
        m = x & MASK48;
      }
      const uint32_t hi = (uint32_t)(x >> 48);  // code << 12 | first slot
      const int j = (int)(hi & 0xFFFu) + __builtin_ctzll(m);
      m &= m - 1ull;
      const float2 sh = L.shift[hi >> 12];
      const float2 oj = s_off[j];
      float rx, ry, r2;
      pair_accept(oi.x, oi.y, oj.x, oj.y, sh.x, sh.y, R.R2, rx, ry, r2);
      sw.add(kernel_raw<KERN>(R, r2).W);
      const uint32_t e = (uint32_t)j | (hi & 0xF000u);
      if (k & 1) dst[(size_t)(k >> 1) * a.ntot] = word | (e << 16);
      else word = e;
      if ((k & 15) == 15) sw.end_cell();
    }
    if (kept & 1) dst[(size_t)(kept >> 1) * a.ntot] = word;
    a.V[g] = 1.0f / (R.a2 * (kernel_w0_raw<KERN>() + sw.value()));
    a.ncnt[g] = kept;
  }
}

// ------------------------------------------------------------- pass A, Verlet
// The Verlet list holds every pair of the 3 x 3 stencil closer than 3h + delta
// (delta = 0.075 h) at the last build. It stays a superset of the neighbour
// set while no particle has moved more than 0.45 delta since the build (pass D
// checks and requests a rebuild, as does every rebin, new state, tile change
// or snapshot restore): a pair left out was at least 3h + delta apart, so it is
// still more than 3h + 0.1 delta apart; pairs outside the stencil are excluded
// by the rebin criterion. Every pass walks it and applies the exact predicate,
// so the candidate search of the ~144 stencil particles runs only on rebuild
// steps. Pass A sums the kernel over the accepted pairs (the volume).

// Build: candidate search with the Verlet radius (masks as in the direct
// search), then one walk over the Verlet pairs in cell order that writes the
// list and sums W over the pairs that pass the exact predicate.
template <int T, int COMP, int KERN>
__device__ __forceinline__ void tile_pass_a_build(const StepArgs& a, int w) {
  __shared__ TileLDS<T> L;
  __shared__ float2 s_off[TileCfg<T, KERN>::MAXP];
  __shared__ unsigned long long s_mask[9 * WG];
  RepDev R;
  int rep;
  if (!tile_begin<T, KERN>(a, w, L, R, rep)) return;
  const int ni = L.hdr[0], nint = L.hdr[2], nreg = L.hdr[3];
  const int S = L.cstart[nreg];
  for (int t = threadIdx.x; t < S; t += WG) s_off[t] = a.off_cur[staged_global<T>(a, L, t)];
  __syncthreads();
  const int nin = L.cstart[nint];
  const int tid = threadIdx.x;
  for (int base = 0; base < nin; base += WG) {
    const int p = base + tid;
    if (p >= nin) break;
    const int st = find_cell(L.cstart, nint, p);
    const int li = st % ni, lj = st / ni;
    const float2 oi = s_off[p];
    int cnt = 0;
    bool big = false;
#pragma unroll 1
    for (int cidx = 0; cidx < 9; ++cidx) {
      const int dy = cidx / 3, dx = cidx % 3;
      const int sc = L.slot[(lj + dy) * (ni + 2) + (li + dx)];
      const int j0 = L.cstart[sc];
      const int nj = L.cstart[sc + 1] - j0;
      if (nj > CELL_MAX) big = true;
      const uint32_t code = (uint32_t)dx | ((uint32_t)dy << 2);
      const float2 sh = L.shift[code];
      uint32_t mlo = 0u, mhi = 0u;
      const int n0 = min(nj, 32), n1 = min(nj, CELL_MAX);
      for (int b = 0; b < n0; ++b) {
        const float2 oj = s_off[j0 + b];
        float rx, ry, r2;
        if (pair_accept(oi.x, oi.y, oj.x, oj.y, sh.x, sh.y, R.R2v, rx, ry, r2)) mlo |= 1u << b;
      }
      for (int b = 32; b < n1; ++b) {
        const float2 oj = s_off[j0 + b];
        float rx, ry, r2;
        if (pair_accept(oi.x, oi.y, oj.x, oj.y, sh.x, sh.y, R.R2v, rx, ry, r2)) mhi |= 1u << (b - 32);
      }
      s_mask[cidx * WG + tid] = ((unsigned long long)code << 60) | ((unsigned long long)j0 << 48) |
                                ((unsigned long long)mhi << 32) | mlo;
      cnt += __popc(mlo) + __popc(mhi);
    }
    const int vk = min(cnt, KMAX);
    const int g = L.gstart[st] + (p - L.cstart[st]);
    if (g < 0 || g >= a.ntot) { flag(a.flags, ERR_RANGE); continue; }
    if (cnt > KMAX || big) flag(a.flags, ERR_OVERFLOW);
    Acc<COMP> sw;
    sw.init();
    int c = -1;
    unsigned long long m = 0ull, x = 0ull;
    uint32_t vword = 0u;
    uint32_t* vdst = a.vl + g;
    for (int k = 0; k < vk; ++k) {
      while (m == 0ull && c < 8) {
        ++c;
        x = s_mask[c * WG + tid];
        m = x & MASK48;
      }
      const uint32_t hi = (uint32_t)(x >> 48);
      const int j = (int)(hi & 0xFFFu) + __builtin_ctzll(m);
      m &= m - 1ull;
      const uint32_t e = (uint32_t)j | (hi & 0xF000u);
      if (k & 1) vdst[(size_t)(k >> 1) * a.ntot] = vword | (e << 16);
      else vword = e;
      int jj;
      float rx, ry, r2;
      if (verlet_pair(e, L.shift, S - 1, s_off, oi, R.R2, jj, rx, ry, r2)) sw.add(kernel_raw<KERN>(R, r2).W);
      if ((k & 15) == 15) sw.end_cell();
    }
    if (vk & 1) vdst[(size_t)(vk >> 1) * a.ntot] = vword;
    a.vcnt[g] = vk;
    a.off_build[g] = oi;
    a.V[g] = 1.0f / (R.a2 * (kernel_w0_raw<KERN>() + sw.value()));
  }
}

// Walk: the volume over the Verlet entries that pass the exact predicate.
template <int T, int COMP, int KERN>
__device__ __forceinline__ void tile_pass_a_walk(const StepArgs& a, int w) {
  __shared__ TileLDS<T> L;
  __shared__ float2 s_off[TileCfg<T, KERN>::MAXP];
  RepDev R;
  int rep;
  if (!tile_begin<T, KERN>(a, w, L, R, rep)) return;
  const int nint = L.hdr[2], nreg = L.hdr[3];
  const int S = L.cstart[nreg];
  for (int t = threadIdx.x; t < S; t += WG) s_off[t] = a.off_cur[staged_global<T>(a, L, t)];
  __syncthreads();
  const int nin = L.cstart[nint];
  for (int base = 0; base < nin; base += WG) {
    const int p = base + threadIdx.x;
    if (p >= nin) break;
    const int st = find_cell(L.cstart, nint, p);
    const int g = L.gstart[st] + (p - L.cstart[st]);
    if (g < 0 || g >= a.ntot) { flag(a.flags, ERR_RANGE); continue; }
    const float2 oi = s_off[p];
    Acc<COMP> sw;
    sw.init();
    each_listed<2>(a.vl, a.ntot, g, min(a.vcnt[g], KMAX), 1, 0, [&](uint32_t e) {
      int j; float rx, ry, r2;
      const bool in = verlet_pair(e, L.shift, S - 1, s_off, oi, R.R2, j, rx, ry, r2);
      const float W = kernel_raw<KERN>(R, r2).W;
      sw.add(in ? W : 0.0f);                 // exact zero outside the support
    }, [&]() { sw.end_cell(); });
    a.V[g] = 1.0f / (R.a2 * (kernel_w0_raw<KERN>() + sw.value()));
  }
}

// ------------------------------------------------------------------ pass B
// Q3 = 1: quasi-2D variant, a 3x3 order tensor (Qxx, Qxy, Qyy stored,
// Qzz = -Qxx - Qyy) with the printed I/3 in the co-rotation and the molecular
// field; corrected momentum form without the lambda stress terms only.
template <int T, int COMP, int FORM, int EL, int KERN, int Q3>
__device__ __forceinline__ void tile_pass_b(const StepArgs& a, int w) {
  static_assert(Q3 == 0 || (FORM == 0 && EL == 0), "quasi-2D: corrected form, no lambda terms");
  __shared__ TileLDS<T> L;
  constexpr int MP = TileCfg<T, KERN>::MAXP;
  __shared__ float2 s_off[MP];
  __shared__ float2 s_u[MP];
  __shared__ float2 s_q[MP];
  __shared__ float s_V[MP];                  // V dWc: V_j F = s_V[j] Fr
  __shared__ float s_rho[FORM == 1 ? MP : 1];
  __shared__ float s_qc[Q3 == 1 ? MP : 1];   // Qyy of the quasi-2D variant
  RepDev R;
  int rep;
  if (!tile_begin<T, KERN>(a, w, L, R, rep)) return;
  const int nint = L.hdr[2], nreg = L.hdr[3];
  const int S = L.cstart[nreg];
  for (int t = threadIdx.x; t < S; t += WG) {
    const int g = staged_global<T>(a, L, t);
    s_off[t] = a.off_cur[g];
    s_u[t] = a.u[g];
    s_q[t] = a.q_cur[g];
    if constexpr (Q3 == 1) s_qc[t] = a.qyy_cur[g];
    s_V[t] = a.V[g] * R.dWc;
    if constexpr (FORM == 1) s_rho[t] = R.rho0 + a.drho[g];
  }
  __syncthreads();
  const int nin = L.cstart[nint];
  for (int base = 0; base < nin;) {
    const int lpp = lanes_for(nin - base, a.lpp);
    const int p = base + threadIdx.x / lpp;
    const int sub = threadIdx.x & (lpp - 1);
    base += WG / lpp;
    int g = -1;
    if (p < nin) {
      const int st = find_cell(L.cstart, nint, p);
      g = L.gstart[st] + (p - L.cstart[st]);
      if (g < 0 || g >= a.ntot) { flag(a.flags, ERR_RANGE); g = -1; }
    }
    const bool act = g >= 0;
    // raw pair sums (see the epilogue for their meaning)
    Acc<COMP> Sxx, Sxy, Syy, Gxx, Gxy, Gyx, Gyy, Qax, Qay, Qbx, Qby;
    Acc<COMP> Mxx_a, Mxy_a, Myy_a, Mxx_b, Mxy_b, Myy_b, Vsx, Vsy;
    Acc<COMP> Kc, V1x, V1y, A1x, A1y;
    Acc<COMP> Qcx, Qcy, Mxx_c, Mxy_c, Myy_c;   // quasi-2D: gradient and Laplacian sums of Qyy
    Sxx.init(); Sxy.init(); Syy.init(); Gxx.init(); Gxy.init(); Gyx.init(); Gyy.init();
    Qax.init(); Qay.init(); Qbx.init(); Qby.init();
    Mxx_a.init(); Mxy_a.init(); Myy_a.init(); Mxx_b.init(); Mxy_b.init(); Myy_b.init();
    Vsx.init(); Vsy.init();
    Kc.init(); V1x.init(); V1y.init(); A1x.init(); A1y.init();
    Qcx.init(); Qcy.init(); Mxx_c.init(); Mxy_c.init(); Myy_c.init();
    float2 ui = {0.f, 0.f}, qi = {0.f, 0.f};
    float qci = 0.f;
    float ri = 1.0f;
    if (act) {
      const float2 oi = s_off[p];
      ui = s_u[p];
      qi = s_q[p];
      if constexpr (Q3 == 1) qci = s_qc[p];
      if constexpr (FORM == 1) ri = s_rho[p];
      const float ri2inv = 1.0f / (ri * ri);
      const int cnt = min(a.vcnt[g], KMAX);
      each_listed<2>(a.vl, a.ntot, g, cnt, lpp, sub, [&](uint32_t e) {
        int j; float rx, ry, r2;
        // entries outside the support are skipped (a branch measured faster
        // here than zeroing their terms with selects)
        if (!verlet_pair(e, L.shift, S - 1, s_off, oi, R.R2, j, rx, ry, r2)) return;
        const KW k = kernel_raw<KERN>(R, r2);
        const float2 uj = s_u[j], qj = s_q[j];
        const float c = s_V[j] * k.F;          // V_j W'(r)/r
        const float cx = c * rx, cy = c * ry;  // V_j grad_i W_ij
        const float txx = cx * rx, txy = cx * ry, tyy = cy * ry;
        Sxx.add(txx); Sxy.add(txy); Syy.add(tyy);
        const float dux = uj.x - ui.x, duy = uj.y - ui.y;
        const float dqa = qj.x - qi.x, dqb = qj.y - qi.y;
        Gxx.fma(dux, cx); Gxy.fma(dux, cy); Gyx.fma(duy, cx); Gyy.fma(duy, cy);
        Qax.fma(dqa, cx); Qay.fma(dqa, cy); Qbx.fma(dqb, cx); Qby.fma(dqb, cy);
        const float e2 = k.rinv * k.rinv;
        const float la = -dqa * e2, lb = -dqb * e2;   // (Q_i - Q_j)/r^2
        Mxx_a.fma(la, txx); Mxy_a.fma(la, txy); Myy_a.fma(la, tyy);
        Mxx_b.fma(lb, txx); Mxy_b.fma(lb, txy); Myy_b.fma(lb, tyy);
        if constexpr (Q3 == 1) {
          const float dqc = s_qc[j] - qci;
          Qcx.fma(dqc, cx); Qcy.fma(dqc, cy);
          const float lc = -dqc * e2;
          Mxx_c.fma(lc, txx); Mxy_c.fma(lc, txy); Myy_c.fma(lc, tyy);
        }
        const float sv = -(dux * rx + duy * ry) * e2;  // (u_i - u_j).r_ij / r^2
        if constexpr (FORM == 0) {
          Vsx.fma(sv, cx); Vsy.fma(sv, cy);
        } else {
          const float rj = s_rho[j];
          const float Ft = R.dWc * k.F;
          const float fx = Ft * rx, fy = Ft * ry;    // grad_i W_ij
          Kc.add(-(dux * fx + duy * fy));
          const float svr = sv / rj;
          V1x.fma(svr, fx); V1y.fma(svr, fy);
          const float rj2inv = 1.0f / (rj * rj);
          const float ca = qi.x * ri2inv + qj.x * rj2inv, cb = qi.y * ri2inv + qj.y * rj2inv;
          A1x.add(ca * fx + cb * fy); A1y.add(cb * fx - ca * fy);
        }
      }, [&]() {
        Sxx.end_cell(); Sxy.end_cell(); Syy.end_cell();
        Gxx.end_cell(); Gxy.end_cell(); Gyx.end_cell(); Gyy.end_cell();
        Qax.end_cell(); Qay.end_cell(); Qbx.end_cell(); Qby.end_cell();
        Mxx_a.end_cell(); Mxy_a.end_cell(); Myy_a.end_cell();
        Mxx_b.end_cell(); Mxy_b.end_cell(); Myy_b.end_cell();
        Vsx.end_cell(); Vsy.end_cell();
        if constexpr (FORM == 1) { Kc.end_cell(); V1x.end_cell(); V1y.end_cell(); A1x.end_cell(); A1y.end_cell(); }
        if constexpr (Q3 == 1) { Qcx.end_cell(); Qcy.end_cell(); Mxx_c.end_cell(); Mxy_c.end_cell(); Myy_c.end_cell(); }
      });
    }
    const float sxx = wave_sum(Sxx.value(), lpp), sxy = wave_sum(Sxy.value(), lpp), syy = wave_sum(Syy.value(), lpp);
    const float gxx = wave_sum(Gxx.value(), lpp), gxy = wave_sum(Gxy.value(), lpp);
    const float gyx = wave_sum(Gyx.value(), lpp), gyy = wave_sum(Gyy.value(), lpp);
    const float qax = wave_sum(Qax.value(), lpp), qay = wave_sum(Qay.value(), lpp);
    const float qbx = wave_sum(Qbx.value(), lpp), qby = wave_sum(Qby.value(), lpp);
    const float mxxa = wave_sum(Mxx_a.value(), lpp), mxya = wave_sum(Mxy_a.value(), lpp);
    const float myya = wave_sum(Myy_a.value(), lpp);
    const float mxxb = wave_sum(Mxx_b.value(), lpp), mxyb = wave_sum(Mxy_b.value(), lpp);
    const float myyb = wave_sum(Myy_b.value(), lpp);
    float vsx = 0.f, vsy = 0.f, kc = 0.f, v1x = 0.f, v1y = 0.f, a1x = 0.f, a1y = 0.f;
    float qcx = 0.f, qcy = 0.f, mxxc = 0.f, mxyc = 0.f, myyc = 0.f;
    if constexpr (Q3 == 1) {
      qcx = wave_sum(Qcx.value(), lpp); qcy = wave_sum(Qcy.value(), lpp);
      mxxc = wave_sum(Mxx_c.value(), lpp); mxyc = wave_sum(Mxy_c.value(), lpp); myyc = wave_sum(Myy_c.value(), lpp);
    }
    if constexpr (FORM == 0) { vsx = wave_sum(Vsx.value(), lpp); vsy = wave_sum(Vsy.value(), lpp); }
    else {
      kc = wave_sum(Kc.value(), lpp); v1x = wave_sum(V1x.value(), lpp); v1y = wave_sum(V1y.value(), lpp);
      a1x = wave_sum(A1x.value(), lpp); a1y = wave_sum(A1y.value(), lpp);
    }
    if (act && sub == 0) {
      // alpha = -sum_j V_j W'/r r_ij (x) r_ij, B = alpha^{-1}
      const float axx = -sxx, axy = -sxy, ayy = -syy;
      const float det = axx * ayy - axy * axy;
      const float nrm = axx * axx + 2.0f * axy * axy + ayy * ayy;
      float Bxx = 1.f, Bxy = 0.f, Byy = 1.f;
      if (det > 1e-12f * nrm && isfinite(det)) {
        const float id = 1.0f / det;
        Bxx = ayy * id; Bxy = -axy * id; Byy = axx * id;
      } else {
        flag(a.flags, ERR_SINGULAR);
      }
      // velocity gradient G_ab = du_a/dx_b = sum_l Gu[a][l] B^{lb}
      const float G11 = gxx * Bxx + gxy * Bxy, G12 = gxx * Bxy + gxy * Byy;
      const float G21 = gyx * Bxx + gyy * Bxy, G22 = gyx * Bxy + gyy * Byy;
      const float divu = G11 + G22;
      const float drho_n = a.drho[g];
      const float kk = (FORM == 0) ? -(R.rho0 + drho_n) * divu : R.mass * kc;
      a.dh[g] = drho_n + 0.5f * kk * R.dt;
      a.bk[g] = make_float4(Bxx, Bxy, Byy, kk);
      // corrected gradients of Qxx (a) and Qxy (b)
      const float dax = qax * Bxx + qay * Bxy, day = qax * Bxy + qay * Byy;
      const float dbx = qbx * Bxx + qby * Bxy, dby = qbx * Bxy + qby * Byy;
      // Laplacians: 2 sum_j V_j (Q_i - Q_j) (r_ij . g_ij) / r^2
      const float lapa = 2.0f * (Bxx * mxxa + 2.0f * Bxy * mxya + Byy * myya);
      const float lapb = 2.0f * (Bxx * mxxb + 2.0f * Bxy * mxyb + Byy * myyb);
      const float qa = qi.x, qb = qi.y;
      const float e12 = 0.5f * (G12 + G21), w12 = 0.5f * (G12 - G21);
      float Ha, Hb;
      float dcy = 0.f;   // d Qyy / dy (quasi-2D)
      if constexpr (Q3 == 0) {
        // molecular field (2D: the B term vanishes identically)
        const float trq2 = 2.0f * (qa * qa + qb * qb);
        const float cbulk = R.A + R.C * trq2;
        Ha = -cbulk * qa + R.K * lapa; Hb = -cbulk * qb + R.K * lapb;
        // co-rotation projected on symmetric traceless tensors (d = 2)
        const float QG = qa * (G11 - G22) + 2.0f * qb * e12;
        const float Sa = R.lam * (qa * divu + 0.5f * (G11 - G22)) + 2.0f * w12 * qb - 2.0f * R.lam * qa * QG;
        const float Sb = R.lam * (qb * divu + e12) - 2.0f * w12 * qa - 2.0f * R.lam * qb * QG;
        a.q_nxt[g] = make_float2(qa + (Sa + R.Gamma * Ha) * R.dt, qb + (Sb + R.Gamma * Hb) * R.dt);
      } else {
        // quasi-2D: Q = [[qa, qb, 0], [qb, qc, 0], [0, 0, qz]], qz = -qa - qc,
        // D = Q + I/3; E and W in-plane. The rate is projected on traceless
        // tensors (its trace is (2 lambda/3) div u from the weak compressibility).
        const float qc = qci, qz = -qa - qc;
        dcy = qcx * Bxy + qcy * Byy;
        const float lapc = 2.0f * (Bxx * mxxc + 2.0f * Bxy * mxyc + Byy * myyc);
        const float lapz = -lapa - lapc;
        const float t2 = qa * qa + 2.0f * qb * qb + qc * qc + qz * qz;
        const float cb = R.A + R.C * t2, t3 = t2 * (1.0f / 3.0f);
        Ha = -cb * qa + R.B * (qa * qa + qb * qb - t3) + R.K * lapa;
        Hb = -cb * qb + R.B * qb * (qa + qc) + R.K * lapb;
        const float Hc = -cb * qc + R.B * (qb * qb + qc * qc - t3) + R.K * lapc;
        const float Hz = -cb * qz + R.B * (qz * qz - t3) + R.K * lapz;
        const float dxx = qa + (1.0f / 3.0f), dyy = qc + (1.0f / 3.0f), dzz = qz + (1.0f / 3.0f), dxy = qb;
        const float QG = qa * G11 + qb * (G12 + G21) + qc * G22;
        const float l2 = 2.0f * R.lam * QG;
        const float Sxx = 2.0f * R.lam * (G11 * dxx + e12 * dxy) + 2.0f * w12 * dxy - l2 * dxx;
        const float Sxy = R.lam * (e12 * (dxx + dyy) + dxy * divu) + w12 * (dyy - dxx) - l2 * dxy;
        const float Syy = 2.0f * R.lam * (e12 * dxy + G22 * dyy) - 2.0f * w12 * dxy - l2 * dyy;
        const float Szz = -l2 * dzz;
        const float mxx = Sxx + R.Gamma * Ha, mxy = Sxy + R.Gamma * Hb, myy = Syy + R.Gamma * Hc;
        const float mtr = (mxx + myy + Szz + R.Gamma * Hz) * (1.0f / 3.0f);
        a.q_nxt[g] = make_float2(qa + (mxx - mtr) * R.dt, qb + mxy * R.dt);
        a.qyy_nxt[g] = qc + (myy - mtr) * R.dt;
      }
      float apx, apy;
      if constexpr (FORM == 0) {
        const float vcx = vsx * Bxx + vsy * Bxy, vcy = vsx * Bxy + vsy * Byy;
        // div Q: (dQxx/dx + dQxy/dy, dQxy/dx + dQyy/dy), Qyy = -Qxx in d = 2
        const float divqx = dax + dby, divqy = (Q3 == 0) ? dbx - day : dbx + dcy;
        apx = 8.0f * R.eta * vcx - R.zeta * divqx;
        apy = 8.0f * R.eta * vcy - R.zeta * divqy;
      } else {
        const float cv = R.mass * 8.0f * R.eta / ri;
        apx = cv * v1x - R.zeta * R.mass * a1x;
        apy = cv * v1y - R.zeta * R.mass * a1y;
      }
      a.apart[g] = make_float2(apx, apy);
      if constexpr (EL == 1) {
        const float QH = 2.0f * (qa * Ha + qb * Hb);
        a.pi[g] = make_float2(R.lam * (2.0f * QH * qa - Ha), R.lam * (2.0f * QH * qb - Hb));
      }
      if (Q3 == 0 && a.feat) {  // learned-corrector inputs 0-9 (storage order): Q, grad u, H, density, activity
        float* f = a.feat + (size_t)g * 12;
        f[0] = qa; f[1] = qb;
        f[2] = G11; f[3] = G12; f[4] = G21; f[5] = G22;
        f[6] = Ha; f[7] = Hb;
        f[8] = drho_n * R.inv_rho0; f[9] = R.zeta;
      }
    }
  }
}

// ------------------------------------------------------------------ pass C
template <int T, int COMP, int KERN>
__device__ __forceinline__ void tile_pass_c(const StepArgs& a, int w) {
  __shared__ TileLDS<T> L;
  constexpr int MP = TileCfg<T, KERN>::MAXP;
  __shared__ float2 s_off[MP];
  __shared__ float s_dh[MP];
  __shared__ float2 s_u[MP];
  RepDev R;
  int rep;
  if (!tile_begin<T, KERN>(a, w, L, R, rep)) return;
  const int nint = L.hdr[2], nreg = L.hdr[3];
  const int S = L.cstart[nreg];
  for (int t = threadIdx.x; t < S; t += WG) {
    const int g = staged_global<T>(a, L, t);
    s_off[t] = a.off_cur[g];
    s_dh[t] = a.dh[g];
    s_u[t] = a.u[g];
  }
  __syncthreads();
  unsigned umb = 0;
  for (int k = 0; k < UMAX_SLOTS; ++k) umb = max(umb, a.umax_cur[rep * UMAX_SLOTS + k]);
  const float c0 = R.c0_factor * __uint_as_float(umb);
  const float pc = R.rho0 * c0 * c0 / R.gamma_eos;
  const int nin = L.cstart[nint];
  for (int base = 0; base < nin;) {
    const int lpp = lanes_for(nin - base, a.lpp);
    const int p = base + threadIdx.x / lpp;
    const int sub = threadIdx.x & (lpp - 1);
    base += WG / lpp;
    int g = -1;
    if (p < nin) {
      const int st = find_cell(L.cstart, nint, p);
      g = L.gstart[st] + (p - L.cstart[st]);
      if (g < 0 || g >= a.ntot) { flag(a.flags, ERR_RANGE); g = -1; }
    }
    const bool act = g >= 0;
    Acc<COMP> sd, Wux, Wuy;   // in units of a2
    sd.init(); Wux.init(); Wuy.init();
    if (act) {
      const float2 oi = s_off[p], ui = s_u[p];
      const int cnt = min(a.vcnt[g], KMAX);
      each_listed<2>(a.vl, a.ntot, g, cnt, lpp, sub, [&](uint32_t e) {
        int j; float rx, ry, r2;
        // entries outside the support add exact zeros (a select: a branch here
        // splits the four-entry iteration and measured 9% slower); the select
        // also drops the non-finite W of coincident particles
        const bool in = verlet_pair(e, L.shift, S - 1, s_off, oi, R.R2, j, rx, ry, r2);
        const float Wr = kernel_raw<KERN>(R, r2).W;
        const float W = in ? Wr : 0.0f;
        const float2 uj = s_u[j];
        sd.fma(s_dh[j], W);
        Wux.fma(ui.x - uj.x, W); Wuy.fma(ui.y - uj.y, W);   // sum_j (u_i - u_j) W_ij
      }, [&]() { sd.end_cell(); Wux.end_cell(); Wuy.end_cell(); });
    }
    const float tot = wave_sum(sd.value(), lpp);
    const float wux = wave_sum(Wux.value(), lpp), wuy = wave_sum(Wuy.value(), lpp);
    if (act && sub == 0) {
      const float Vi = a.V[g];
      const float dhi = s_dh[p];
      // Shepard filter with the self term, written for rho - rho0
      const float shep = (Vi * R.a2) * fmaf(kernel_w0_raw<KERN>(), dhi, tot);
      const float drh = dhi - R.beta * (dhi - shep);
      const float x = drh * R.inv_rho0;
      float pw;  // (1 + x)^gamma - 1
      if (R.gamma_eos == 7.0f)
        pw = x * (7.0f + x * (21.0f + x * (35.0f + x * (35.0f + x * (21.0f + x * (7.0f + x))))));
      else
        pw = expm1f(R.gamma_eos * log1pf(x));
      const float rh = R.rho0 + drh;
      a.P[g] = pc * pw / (rh * rh);
      a.drhat[g] = drh;
      a.uv[g] = sqrtf(wux * wux + wuy * wuy) * (R.a2 * Vi);
    }
  }
}

// ------------------------------------------------------------------ pass D
// INTEG: corrector, 0 kick-drift-kick, 1 midpoint (the integrator parameter picks the variant at launch).
template <int T, int COMP, int FORM, int EL, int KERN, int INTEG>
__device__ __forceinline__ void tile_pass_d(const StepArgs& a, int w) {
  __shared__ TileLDS<T> L;
  constexpr int MP = TileCfg<T, KERN>::MAXP;
  // FORM 0 stages V dWc (V_j F = s_V[j] Fr); without the lambda stress it also
  // stages s_P = P V dWc, so that (P_i + P_j) V_j F = (P_i s_V[j] + s_P[j]) Fr.
  constexpr bool PV = FORM == 0 && EL == 0;
  __shared__ float2 s_off[MP];
  __shared__ float s_V[MP];
  __shared__ float s_P[MP];
  __shared__ float2 s_pi[EL == 1 ? MP : 1];
  __shared__ float s_wmax[WG / 64];
  RepDev R;
  int rep;
  if (!tile_begin<T, KERN>(a, w, L, R, rep)) return;
  const int nint = L.hdr[2], nreg = L.hdr[3];
  const int S = L.cstart[nreg];
  for (int t = threadIdx.x; t < S; t += WG) {
    const int g = staged_global<T>(a, L, t);
    s_off[t] = a.off_cur[g];
    const float Vd = a.V[g] * R.dWc;
    s_V[t] = Vd;
    s_P[t] = PV ? a.P[g] * Vd : a.P[g];
    if constexpr (EL == 1) s_pi[t] = a.pi[g];
  }
  __syncthreads();
  const int nin = L.cstart[nint];
  float umax_l = 0.0f;
  bool rebin = false, bad = false, relist = false;
  for (int base = 0; base < nin;) {
    const int lpp = lanes_for(nin - base, a.lpp);
    const int p = base + threadIdx.x / lpp;
    const int sub = threadIdx.x & (lpp - 1);
    base += WG / lpp;
    int g = -1;
    if (p < nin) {
      const int st = find_cell(L.cstart, nint, p);
      g = L.gstart[st] + (p - L.cstart[st]);
      if (g < 0 || g >= a.ntot) { flag(a.flags, ERR_RANGE); g = -1; }
    }
    const bool act = g >= 0;
    Acc<COMP> Px, Py, Exx, Exy, Eyx, Eyy;
    Acc<COMP> Gx, Gy, Gr;   // APD geometry: sum r_ij / r^3, sum r
    Px.init(); Py.init(); Exx.init(); Exy.init(); Eyx.init(); Eyy.init();
    Gx.init(); Gy.init(); Gr.init();
    float2 oi = {0.f, 0.f};
    int nacc = 0;   // accepted neighbours taken by this lane
    if (act) {
      oi = s_off[p];
      const float Pi = PV ? a.P[g] : s_P[p];
      float2 pii = {0.f, 0.f};
      if constexpr (EL == 1) pii = s_pi[p];
      const int cnt = min(a.vcnt[g], KMAX);
      each_listed<2>(a.vl, a.ntot, g, cnt, lpp, sub, [&](uint32_t e) {
        int j; float rx, ry, r2;
        if (!verlet_pair(e, L.shift, S - 1, s_off, oi, R.R2, j, rx, ry, r2)) return;   // as in pass B
        ++nacc;
        const KW k = kernel_raw<KERN>(R, r2);
        const float c = (FORM == 0) ? s_V[j] * k.F : R.dWc * k.F;
        const float f = PV ? fmaf(Pi, s_V[j], s_P[j]) * k.F : (Pi + s_P[j]) * c;
        Px.fma(f, rx); Py.fma(f, ry);
        const float r3 = k.rinv * k.rinv * k.rinv;
        Gx.fma(rx, r3); Gy.fma(ry, r3); Gr.add(k.r);
        if constexpr (EL == 1) {
          const float2 pj = s_pi[j];
          const float cx = c * rx, cy = c * ry;
          const float dpa = pj.x - pii.x, dpb = pj.y - pii.y;
          Exx.fma(dpa, cx); Exy.fma(dpa, cy); Eyx.fma(dpb, cx); Eyy.fma(dpb, cy);
        }
      }, [&]() {
        Px.end_cell(); Py.end_cell(); Gx.end_cell(); Gy.end_cell(); Gr.end_cell();
        if constexpr (EL == 1) { Exx.end_cell(); Exy.end_cell(); Eyx.end_cell(); Eyy.end_cell(); }
      });
    }
    const float prx = wave_sum(Px.value(), lpp), pry = wave_sum(Py.value(), lpp);
    const float gx = wave_sum(Gx.value(), lpp), gy = wave_sum(Gy.value(), lpp), gr = wave_sum(Gr.value(), lpp);
    const int cnt = wave_sum_int(nacc, lpp);
    float exx = 0.f, exy = 0.f, eyx = 0.f, eyy = 0.f;
    if constexpr (EL == 1) {
      exx = wave_sum(Exx.value(), lpp); exy = wave_sum(Exy.value(), lpp);
      eyx = wave_sum(Eyx.value(), lpp); eyy = wave_sum(Eyy.value(), lpp);
    }
    if (act && sub == 0) {
      const float4 bk = a.bk[g];
      const float drh = a.drhat[g];
      const float rh = R.rho0 + drh;
      const float2 ap = a.apart[g];
      float ax, ay;
      if constexpr (FORM == 0) {
        ax = -rh * (prx * bk.x + pry * bk.y) + ap.x / rh;
        ay = -rh * (prx * bk.y + pry * bk.z) + ap.y / rh;
        if constexpr (EL == 1) {
          const float dPax = exx * bk.x + exy * bk.y, dPay = exx * bk.y + exy * bk.z;
          const float dPbx = eyx * bk.x + eyy * bk.y, dPby = eyx * bk.y + eyy * bk.z;
          ax += (dPax + dPby) / rh;
          ay += (dPbx - dPay) / rh;
        }
      } else {
        ax = -R.mass * prx + ap.x;
        ay = -R.mass * pry + ap.y;
      }
      const float2 uh = a.u[g];
      const float hdt = 0.5f * R.dt;
      float u1x, u1y;                                              // u^{n+1}
      if constexpr (INTEG == 0) {                                  // kick-drift-kick
        u1x = uh.x + hdt * ax; u1y = uh.y + hdt * ay;
      } else {                                                     // midpoint: u^n + a dt,
        const float2 ap = a.acc[g];                                // u^n = u^{n+1/2} - a^{n-1/2} dt/2
        u1x = (uh.x - hdt * ap.x) + R.dt * ax;
        u1y = (uh.y - hdt * ap.y) + R.dt * ay;
      }
      float drx = 0.f, dry = 0.f;
      if (R.apd && cnt > 0) {
        const float r0 = gr / (float)cnt;   // mean neighbour distance
        const float f = r0 * r0 * a.uv[g] * R.dt;
        drx = f * gx; dry = f * gy;
      }
      if (a.feat) {   // learned-corrector inputs 10-11: the step's change of acceleration a^{n+1/2} - a^{n-1/2}
        const float2 ao = a.acc[g];
        float* f = a.feat + (size_t)g * 12;
        f[10] = ax - ao.x; f[11] = ay - ao.y;
      }
      const float unx = u1x + hdt * ax, uny = u1y + hdt * ay;      // u^{n+3/2}
      // r^{n+1} - r^{n+1/2}: u^{n+1} dt/2 (kick-drift-kick) or u^{n+1/2} dt/2
      // (midpoint, r^n + u^{n+1/2} dt), then the next predictor's u^{n+3/2} dt/2
      const float vdx = INTEG == 0 ? u1x : uh.x, vdy = INTEG == 0 ? u1y : uh.y;
      const float dispx = hdt * vdx + drx + hdt * unx;
      const float dispy = hdt * vdy + dry + hdt * uny;
      // compensated position update: (hi, lo) += disp
      const float2 lo = a.offlo[g];
      float2 nh, nl;
      {
#pragma clang fp contract(off)
        float s = oi.x + dispx, bp = s - oi.x;
        float e = (oi.x - (s - bp)) + (dispx - bp);
        float l2 = lo.x + e;
        nh.x = s + l2; nl.x = l2 - (nh.x - s);
        s = oi.y + dispy; bp = s - oi.y;
        e = (oi.y - (s - bp)) + (dispy - bp);
        l2 = lo.y + e;
        nh.y = s + l2; nl.y = l2 - (nh.y - s);
      }
      const float dn = drh + hdt * bk.w;
      const float2 ob = a.off_build[g];
      const float bx = nh.x - ob.x, by = nh.y - ob.y;
      if (bx * bx + by * by > R.disp2) relist = true;
      a.off_nxt[g] = nh;
      a.offlo[g] = nl;
      a.u[g] = make_float2(unx, uny);
      a.acc[g] = make_float2(ax, ay);
      a.drho[g] = dn;
      umax_l = fmaxf(umax_l, sqrtf(unx * unx + uny * uny));
      if (nh.x < -R.skin_half || nh.x > R.cs + R.skin_half || nh.y < -R.skin_half || nh.y > R.cs + R.skin_half)
        rebin = true;
      if (!(isfinite(unx) && isfinite(uny) && isfinite(nh.x) && isfinite(nh.y) && isfinite(dn))) bad = true;
    }
  }
  // max speed: wave shuffles, LDS across waves, one atomic per workgroup into
  // one of UMAX_SLOTS slots of the replica (pass C takes the max of the slots)
  for (int o = 1; o < 64; o <<= 1) umax_l = fmaxf(umax_l, __shfl_xor(umax_l, o, 64));
  if ((threadIdx.x & 63) == 0) s_wmax[threadIdx.x >> 6] = umax_l;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = 0.0f;
    for (int w = 0; w < WG / 64; ++w) m = fmaxf(m, s_wmax[w]);
    if (m > 0.0f) atomicMax(&a.umax_nxt[rep * UMAX_SLOTS + (w & (UMAX_SLOTS - 1))], __float_as_uint(m));
  }
  if (rebin) atomicOr(&a.flags[1], 1u);
  if (relist) atomicOr(&a.flags[2], 1u);
  if (bad) flag(a.flags, ERR_NUMERIC);
}

// ------------------------------------------------------- free energy (FP64)
// Per-particle contributions to the free energy of Eq. freeenergy at the
// integer time level, with the elastic part written through the discrete
// Laplacian (F) and through squared corrected gradients (F_grad):
//   F_i    = V_i [A/2 trQ^2 + C/4 (trQ^2)^2 - K/2 Q:lapQ]
//   F_grad = V_i [A/2 trQ^2 + C/4 (trQ^2)^2 + K/2 sum_abc (d_c Q_ab)^2]
// (trQ^3 = 0 in 2D). Runs after the direct search on the integer-level offsets
// and walks its list (every entry passes the predicate again, as in the passes).
template <int T, int KERN>
__global__ __launch_bounds__(WG) void k_free_energy(const StepArgs a, double* fe) {
  __shared__ TileLDS<T> L;
  constexpr int MP = TileCfg<T, KERN>::MAXP;
  __shared__ float2 s_off[MP];
  __shared__ float2 s_q[MP];
  __shared__ float s_V[MP];
  __shared__ float s_qc[MP];   // Qyy (quasi-2D variant)
  RepDev R;
  int rep;
  if (!tile_begin<T, KERN>(a, blockIdx.x, L, R, rep)) return;
  const int nint = L.hdr[2], nreg = L.hdr[3];
  const int S = L.cstart[nreg];
  for (int t = threadIdx.x; t < S; t += WG) {
    const int g = staged_global<T>(a, L, t);
    s_off[t] = a.off_cur[g];
    s_q[t] = a.q_cur[g];
    s_V[t] = a.V[g];
    if (R.q3d) s_qc[t] = a.qyy_cur[g];
  }
  __syncthreads();
  const int nin = L.cstart[nint];
  for (int p = threadIdx.x; p < nin; p += WG) {
    const int st = find_cell(L.cstart, nint, p);
    const int g = L.gstart[st] + (p - L.cstart[st]);
    if (g < 0 || g >= a.ntot) { flag(a.flags, ERR_RANGE); continue; }
    const float2 oi = s_off[p], qi = s_q[p];
    Acc<1> Sxx, Sxy, Syy, Qax, Qay, Qbx, Qby, Mxxa, Mxya, Myya, Mxxb, Mxyb, Myyb;
    Acc<1> Qcx, Qcy, Mxxc, Mxyc, Myyc;
    Sxx.init(); Sxy.init(); Syy.init(); Qax.init(); Qay.init(); Qbx.init(); Qby.init();
    Mxxa.init(); Mxya.init(); Myya.init(); Mxxb.init(); Mxyb.init(); Myyb.init();
    Qcx.init(); Qcy.init(); Mxxc.init(); Mxyc.init(); Myyc.init();
    const float qci = R.q3d ? s_qc[p] : 0.0f;
    each_listed(a.nl, a.ntot, g, min(a.ncnt[g], KMAX), 1, 0, [&](uint32_t e) {
      int j; float rx, ry, r2;
      if (!verlet_pair(e, L.shift, S - 1, s_off, oi, R.R2, j, rx, ry, r2)) return;
      const KW k = kernel_wf<KERN>(R, r2);
      const float c = s_V[j] * k.F, cx = c * rx, cy = c * ry;
      const float txx = cx * rx, txy = cx * ry, tyy = cy * ry;
      Sxx.add(txx); Sxy.add(txy); Syy.add(tyy);
      const float2 qj = s_q[j];
      const float dqa = qj.x - qi.x, dqb = qj.y - qi.y, e2 = k.rinv * k.rinv;
      Qax.fma(dqa, cx); Qay.fma(dqa, cy); Qbx.fma(dqb, cx); Qby.fma(dqb, cy);
      const float la = -dqa * e2, lb = -dqb * e2;
      Mxxa.fma(la, txx); Mxya.fma(la, txy); Myya.fma(la, tyy);
      Mxxb.fma(lb, txx); Mxyb.fma(lb, txy); Myyb.fma(lb, tyy);
      if (R.q3d) {
        const float dqc = s_qc[j] - qci, lc = -dqc * e2;
        Qcx.fma(dqc, cx); Qcy.fma(dqc, cy);
        Mxxc.fma(lc, txx); Mxyc.fma(lc, txy); Myyc.fma(lc, tyy);
      }
    }, [&]() {
      Sxx.end_cell(); Sxy.end_cell(); Syy.end_cell(); Qax.end_cell(); Qay.end_cell(); Qbx.end_cell();
      Qby.end_cell(); Mxxa.end_cell(); Mxya.end_cell(); Myya.end_cell(); Mxxb.end_cell(); Mxyb.end_cell();
      Myyb.end_cell(); Qcx.end_cell(); Qcy.end_cell(); Mxxc.end_cell(); Mxyc.end_cell(); Myyc.end_cell();
    });
    const float axx = -Sxx.value(), axy = -Sxy.value(), ayy = -Syy.value();
    const float det = axx * ayy - axy * axy;
    float Bxx = 1.f, Bxy = 0.f, Byy = 1.f;
    if (det > 1e-12f * (axx * axx + 2.0f * axy * axy + ayy * ayy) && isfinite(det)) {
      const float id = 1.0f / det;
      Bxx = ayy * id; Bxy = -axy * id; Byy = axx * id;
    }
    const double dax = Qax.value() * Bxx + Qay.value() * Bxy, day = Qax.value() * Bxy + Qay.value() * Byy;
    const double dbx = Qbx.value() * Bxx + Qby.value() * Bxy, dby = Qbx.value() * Bxy + Qby.value() * Byy;
    const double lapa = 2.0 * (Bxx * Mxxa.value() + 2.0f * Bxy * Mxya.value() + Byy * Myya.value());
    const double lapb = 2.0 * (Bxx * Mxxb.value() + 2.0f * Bxy * Mxyb.value() + Byy * Myyb.value());
    const double qa = qi.x, qb = qi.y;
    double bulk, qlq, g2;
    if (!R.q3d) {
      const double t2 = 2.0 * (qa * qa + qb * qb);
      bulk = 0.5 * (double)R.A * t2 + 0.25 * (double)R.C * t2 * t2;
      // Q:lapQ and sum of squared gradients over the four components of Q
      qlq = 2.0 * (qa * lapa + qb * lapb);
      g2 = 2.0 * (dax * dax + day * day + dbx * dbx + dby * dby);
    } else {
      // quasi-2D: Q = diag-block [[qa, qb], [qb, qc]] + qz e_z e_z, qz = -qa - qc
      const double qc = qci, qz = -qa - qc;
      const double dcx = Qcx.value() * Bxx + Qcy.value() * Bxy, dcy = Qcx.value() * Bxy + Qcy.value() * Byy;
      const double lapc = 2.0 * (Bxx * Mxxc.value() + 2.0f * Bxy * Mxyc.value() + Byy * Myyc.value());
      const double t2 = qa * qa + 2.0 * qb * qb + qc * qc + qz * qz;
      const double t3 = qa * qa * qa + 3.0 * qb * qb * (qa + qc) + qc * qc * qc + qz * qz * qz;
      bulk = 0.5 * (double)R.A * t2 + (double)R.B / 3.0 * t3 + 0.25 * (double)R.C * t2 * t2;
      qlq = qa * lapa + 2.0 * qb * lapb + qc * lapc + qz * (-lapa - lapc);
      const double dzx = -dax - dcx, dzy = -day - dcy;
      g2 = dax * dax + day * day + 2.0 * (dbx * dbx + dby * dby) + dcx * dcx + dcy * dcy + dzx * dzx + dzy * dzy;
    }
    const double Vi = s_V[p];
    fe[g] = Vi * (bulk - 0.5 * (double)R.K * qlq);
    fe[(size_t)a.ntot + g] = Vi * (bulk + 0.5 * (double)R.K * g2);
  }
}

void launch_free_energy(int T, int kern, const StepArgs& a, double* fe, hipStream_t s) {
  const dim3 grid(a.nwork), block(WG);
  if (kern == 1) {
    if (T == 8) hipLaunchKernelGGL((k_free_energy<8, 1>), grid, block, 0, s, a, fe);
    else hipLaunchKernelGGL((k_free_energy<4, 1>), grid, block, 0, s, a, fe);
  } else {
    if (T == 8) hipLaunchKernelGGL((k_free_energy<8, 0>), grid, block, 0, s, a, fe);
    else hipLaunchKernelGGL((k_free_energy<4, 0>), grid, block, 0, s, a, fe);
  }
}

// ---------------------------------------------------------- neighbour export
// The pairs the pair passes sum over, decoded from the Verlet list exactly as
// they walk it: which = 0 keeps the entries that pass the predicate
// (verlet_pair, the passes' own decision), which = 1 every entry of the list.
// mode 0 counts the entries of each particle of replica rep_only into
// cnt[id]; mode 1 writes the neighbours' ids from row_ptr[id] on.
template <int T, int KERN>
__global__ __launch_bounds__(WG) void k_list_export(const StepArgs a, int rep_only, int which, int mode, int* cnt,
                                                    const int64_t* row_ptr, int32_t* col, int64_t cap) {
  __shared__ TileLDS<T> L;
  constexpr int MP = TileCfg<T, KERN>::MAXP;
  __shared__ float2 s_off[MP];
  __shared__ int s_id[MP];
  RepDev R;
  int rep;
  if (!tile_begin<T, KERN>(a, blockIdx.x, L, R, rep)) return;
  if (rep != rep_only) return;
  const int nint = L.hdr[2], nreg = L.hdr[3];
  const int S = L.cstart[nreg];
  for (int t = threadIdx.x; t < S; t += WG) {
    const int g = staged_global<T>(a, L, t);
    s_off[t] = a.off_cur[g];
    s_id[t] = a.id[g];
  }
  __syncthreads();
  const int nin = L.cstart[nint];
  for (int p = threadIdx.x; p < nin; p += WG) {
    const int st = find_cell(L.cstart, nint, p);
    const int g = L.gstart[st] + (p - L.cstart[st]);
    const int idi = s_id[p];
    if (g < 0 || g >= a.ntot || idi < 0 || idi >= R.n) { flag(a.flags, ERR_RANGE); continue; }
    const float2 oi = s_off[p];
    int c = 0;
    const int64_t base = (mode == 1) ? row_ptr[idi] : 0;
    each_listed(a.vl, a.ntot, g, min(a.vcnt[g], KMAX), 1, 0, [&](uint32_t e) {
      int j; float rx, ry, r2;
      const bool in = verlet_pair(e, L.shift, S - 1, s_off, oi, R.R2, j, rx, ry, r2);
      if (which == 0 && !in) return;
      if (mode == 1) {
        if (base + c < cap) col[base + c] = s_id[j];
        else flag(a.flags, ERR_RANGE);
      }
      ++c;
    }, []() {});
    if (mode == 0) cnt[idi] = c;
  }
}

// ---------------------------------------------------------------- kernels
// One workgroup per tile, or fewer workgroups looping over the tiles
// (persistent launch: StepArgs::grid > 0).
template <int T, int COMP, int KERN>
__global__ __launch_bounds__(WG) void k_pass_a(const StepArgs a) {
  for (int w = blockIdx.x; w < a.nwork; w += gridDim.x) { tile_pass_a<T, COMP, KERN>(a, w); __syncthreads(); }
}
// Gated on the rebuild flag of this step (flags[3], set by the step-begin
// kernel): exactly one of the two runs its tiles, the other exits at once.
template <int T, int COMP, int KERN>
__global__ __launch_bounds__(WG) void k_pass_a_build(const StepArgs a) {
  if (a.flags[3] == 0u) return;
  for (int w = blockIdx.x; w < a.nwork; w += gridDim.x) { tile_pass_a_build<T, COMP, KERN>(a, w); __syncthreads(); }
}
template <int T, int COMP, int KERN>
__global__ __launch_bounds__(WG) void k_pass_a_walk(const StepArgs a) {
  if (a.flags[3] != 0u) return;
  for (int w = blockIdx.x; w < a.nwork; w += gridDim.x) { tile_pass_a_walk<T, COMP, KERN>(a, w); __syncthreads(); }
}

// Occupancy targets (waves per SIMD) of the pair passes: more resident waves
// hide the LDS and list latency in each pair's dependency chain; the targets
// are the largest that compile without register spills for the variant.
template <int T, int COMP, int FORM, int EL, int KERN>
struct Waves {
  static constexpr int B = ((T == 4 || KERN == 1) && (COMP == 0 || (COMP == 1 && FORM == 0))) ? 5 : 1;
  static constexpr int C = 8;
  static constexpr int D = ((T == 4 || KERN == 1) && EL == 0) ? 8 : 1;
};

template <int T, int COMP, int FORM, int EL, int KERN, int Q3>
__global__ __launch_bounds__(WG)
__attribute__((amdgpu_waves_per_eu(Q3 == 0 ? Waves<T, COMP, FORM, EL, KERN>::B : 1)))
void k_pass_b(const StepArgs a) {
  for (int w = blockIdx.x; w < a.nwork; w += gridDim.x) { tile_pass_b<T, COMP, FORM, EL, KERN, Q3>(a, w); __syncthreads(); }
}
template <int T, int COMP, int KERN>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(Waves<T, COMP, 0, 0, KERN>::C)))
void k_pass_c(const StepArgs a) {
  for (int w = blockIdx.x; w < a.nwork; w += gridDim.x) { tile_pass_c<T, COMP, KERN>(a, w); __syncthreads(); }
}
template <int T, int COMP, int FORM, int EL, int KERN, int INTEG>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(Waves<T, COMP, FORM, EL, KERN>::D)))
void k_pass_d(const StepArgs a) {
  for (int w = blockIdx.x; w < a.nwork; w += gridDim.x) { tile_pass_d<T, COMP, FORM, EL, KERN, INTEG>(a, w); __syncthreads(); }
}

// ------------------------------------------------------------- dispatch
template <int T, int COMP, int FORM, int EL, int KERN>
static void launch4(int pass, int q3, int integ, const StepArgs& a, hipStream_t s) {
  const dim3 grid(a.grid > 0 ? std::min(a.grid, a.nwork) : a.nwork), block(WG);
  switch (pass) {
    case 1: hipLaunchKernelGGL((k_pass_a<T, COMP, KERN>), grid, block, 0, s, a); break;
    case 2:
      if constexpr (FORM == 0 && EL == 0) {
        if (q3) { hipLaunchKernelGGL((k_pass_b<T, COMP, 0, 0, KERN, 1>), grid, block, 0, s, a); break; }
      }
      hipLaunchKernelGGL((k_pass_b<T, COMP, FORM, EL, KERN, 0>), grid, block, 0, s, a);
      break;
    case 3: hipLaunchKernelGGL((k_pass_c<T, COMP, KERN>), grid, block, 0, s, a); break;
    case 4:
      if (integ) hipLaunchKernelGGL((k_pass_d<T, COMP, FORM, EL, KERN, 1>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_pass_d<T, COMP, FORM, EL, KERN, 0>), grid, block, 0, s, a);
      break;
  }
}

template <int T, int COMP, int KERN>
static bool launch_phys(int pass, const PassCfg& c, const StepArgs& a, hipStream_t s) {
  if (c.Q3 && (c.FORM != 0 || c.EL != 0)) return false;
  if (c.FORM == 0 && c.EL == 0) { launch4<T, COMP, 0, 0, KERN>(pass, c.Q3, c.INTEG, a, s); return true; }
  if (c.FORM == 1 && c.EL == 0) { launch4<T, COMP, 1, 0, KERN>(pass, c.Q3, c.INTEG, a, s); return true; }
  if (c.FORM == 0 && c.EL == 1) { launch4<T, COMP, 0, 1, KERN>(pass, c.Q3, c.INTEG, a, s); return true; }
  return false;
}

template <int T, int KERN>
static bool launch_comp(int pass, const PassCfg& c, const StepArgs& a, hipStream_t s) {
  switch (c.COMP) {
    case 0: return launch_phys<T, 0, KERN>(pass, c, a, s);
    case 1: return launch_phys<T, 1, KERN>(pass, c, a, s);
    case 2: return launch_phys<T, 2, KERN>(pass, c, a, s);
  }
  return false;
}

template <int T, int COMP, int KERN>
static void launch_verlet(const StepArgs& a, hipStream_t s) {
  const int full = a.grid > 0 ? std::min(a.grid, a.nwork) : a.nwork;
  // the build runs rarely: a persistent grid keeps the skipped launch short
  hipLaunchKernelGGL((k_pass_a_build<T, COMP, KERN>), dim3(std::min(full, 2048)), dim3(WG), 0, s, a);
  hipLaunchKernelGGL((k_pass_a_walk<T, COMP, KERN>), dim3(full), dim3(WG), 0, s, a);
}

template <int KERN>
static bool launch_verlet_k(const PassCfg& c, const StepArgs& a, hipStream_t s) {
  switch (c.COMP * 2 + (c.T == 8 ? 1 : 0)) {
    case 0: launch_verlet<4, 0, KERN>(a, s); return true;
    case 1: launch_verlet<8, 0, KERN>(a, s); return true;
    case 2: launch_verlet<4, 1, KERN>(a, s); return true;
    case 3: launch_verlet<8, 1, KERN>(a, s); return true;
    case 4: launch_verlet<4, 2, KERN>(a, s); return true;
    case 5: launch_verlet<8, 2, KERN>(a, s); return true;
  }
  return false;
}

// Pass A of a step: Verlet build (when flagged) or walk.
bool launch_pass_a_verlet(const PassCfg& c, const StepArgs& a, hipStream_t s) {
  if (c.T != 4 && c.T != 8) return false;
  if (c.KERN == 0) return launch_verlet_k<0>(c, a, s);
  if (c.KERN == 1) return launch_verlet_k<1>(c, a, s);
  return false;
}

// Tiles of 4 or 8 cells; lanes per particle (1, 2, 4) is a runtime argument.
bool launch_pass(int pass, const PassCfg& c, const StepArgs& a, hipStream_t s) {
  if (c.LPP != 1 && c.LPP != 2 && c.LPP != 4) return false;
  if (c.KERN == 0) {
    if (c.T == 4) return launch_comp<4, 0>(pass, c, a, s);
    if (c.T == 8) return launch_comp<8, 0>(pass, c, a, s);
  } else if (c.KERN == 1) {
    if (c.T == 4) return launch_comp<4, 1>(pass, c, a, s);
    if (c.T == 8) return launch_comp<8, 1>(pass, c, a, s);
  }
  return false;
}

void launch_list_export(int T, int kern, const StepArgs& a, int rep, int which, int mode, int* cnt,
                        const int64_t* row_ptr, int32_t* col, int64_t cap, hipStream_t s) {
  const dim3 grid(a.nwork), block(WG);
  if (kern == 1) {
    if (T == 8) hipLaunchKernelGGL((k_list_export<8, 1>), grid, block, 0, s, a, rep, which, mode, cnt, row_ptr, col, cap);
    else hipLaunchKernelGGL((k_list_export<4, 1>), grid, block, 0, s, a, rep, which, mode, cnt, row_ptr, col, cap);
  } else {
    if (T == 8) hipLaunchKernelGGL((k_list_export<8, 0>), grid, block, 0, s, a, rep, which, mode, cnt, row_ptr, col, cap);
    else hipLaunchKernelGGL((k_list_export<4, 0>), grid, block, 0, s, a, rep, which, mode, cnt, row_ptr, col, cap);
  }
}
}  // namespace nem
