// nem_passes.hip -- the four pair passes of one SPH time step on gfx950.
//
// Each workgroup owns a tile of T x T cells of one replica, stages the tile and
// its one-cell periodic halo into LDS (particles are sorted by cell, so every
// cell is a contiguous run), and lets LPP lanes cooperate on each interior
// particle: lane `sub` takes every LPP-th candidate of each stencil cell and
// the lane sums are combined with wave shuffles. Positions are FP32 offsets
// from the particle's cell corner; the periodic image shift of a stencil cell
// is a whole number of cell sides, so pair vectors keep the precision of the
// offsets anywhere in the box.
//
//   pass A  volume V_i = 1 / sum_j W_ij (Eq. sphSum, self included)
//   pass B  correction tensor and B = alpha^{-1} (Eq. sphCorrectionMatrix),
//           velocity gradient and continuity (Eqs. sph1stDerivative,
//           sphContinuity), Q gradient and Laplacian, molecular field
//           (Eq. molecularfielddis), co-rotation (Eq. corotation), Q update
//           (Eq. mi), viscous and active accelerations (Eq. sphMomentum),
//           APD velocity variance (Eq. APD)
//   pass C  density filter (Eq. densityCorrection) and EoS (Eq. sphEos)
//   pass D  pressure term (Eq. sphMomentum), corrector, APD (Eq. APD),
//           and the next step's predictor (Sec. 3.1), fused
#include "nem_dev.h"
#include "nem_pair.h"

namespace nem {

// Common prologue: set up the tile, check LDS capacity. Returns false when the
// workgroup has nothing to do.
template <int T>
__device__ __forceinline__ bool tile_begin(const StepArgs& a, TileLDS<T>& L, RepDev& R, int& rep) {
  const int w = blockIdx.x;
  if (w >= a.nwork) return false;
  rep = tile_setup<T>(a, w, L, R);
  const int S = L.cstart[L.hdr[3]];
  if (S > TileCfg<T>::MAXP) {
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

// ------------------------------------------------------------------ pass A
template <int T, int LPP, int COMP>
__global__ __launch_bounds__(WG) void k_pass_a(const StepArgs a) {
  __shared__ TileLDS<T> L;
  __shared__ float2 s_off[TileCfg<T>::MAXP];
  RepDev R;
  int rep;
  if (!tile_begin<T>(a, L, R, rep)) return;
  const int ni = L.hdr[0], nint = L.hdr[2], nreg = L.hdr[3];
  const int S = L.cstart[nreg];
  for (int t = threadIdx.x; t < S; t += WG) s_off[t] = a.off_cur[staged_global<T>(a, L, t)];
  __syncthreads();
  const int nin = L.cstart[nint];
  const int sub = threadIdx.x % LPP;
  for (int base = 0; base < nin; base += WG / LPP) {
    const int p = base + threadIdx.x / LPP;
    const bool act = p < nin;
    int st = 0;
    Acc<COMP> sw;
    sw.init();
    if (act) {
      st = find_cell(L.cstart, nint, p);
      const int li = st % ni, lj = st / ni;
      const float2 oi = s_off[p];
#pragma unroll 1
      for (int cidx = 0; cidx < 9; ++cidx) {
          const int dy = cidx / 3 - 1, dx = cidx % 3 - 1;
          const int sc = L.slot[(lj + dy + 1) * (ni + 2) + (li + dx + 1)];
          const int j1 = L.cstart[sc + 1];
          const float sx = (float)(-dx) * R.cs, sy = (float)(-dy) * R.cs;
          for (int j = L.cstart[sc] + sub; j < j1; j += LPP) {
            const float2 oj = s_off[j];
            float rx, ry, r2;
            if (pair_accept(oi.x, oi.y, oj.x, oj.y, sx, sy, R.R2, rx, ry, r2)) sw.add(quintic_W(R, r2));
          }
          sw.end_cell();
        }
    }
    const float tot = sw.template total<LPP>();
    if (act && sub == 0) {
      const int g = L.gstart[st] + (p - L.cstart[st]);
      if (g < 0 || g >= a.ntot) { flag(a.flags, ERR_RANGE); continue; }
      a.V[g] = 1.0f / (R.W0 + tot);
    }
  }
}

// ------------------------------------------------------------------ pass B
template <int T, int LPP, int COMP, int FORM, int EL>
__global__ __launch_bounds__(WG) void k_pass_b(const StepArgs a) {
  __shared__ TileLDS<T> L;
  constexpr int MP = TileCfg<T>::MAXP;
  __shared__ float2 s_off[MP];
  __shared__ float2 s_u[MP];
  __shared__ float2 s_q[MP];
  __shared__ float s_V[MP];
  __shared__ float s_rho[FORM == 1 ? MP : 1];
  RepDev R;
  int rep;
  if (!tile_begin<T>(a, L, R, rep)) return;
  const int ni = L.hdr[0], nint = L.hdr[2], nreg = L.hdr[3];
  const int S = L.cstart[nreg];
  for (int t = threadIdx.x; t < S; t += WG) {
    const int g = staged_global<T>(a, L, t);
    s_off[t] = a.off_cur[g];
    s_u[t] = a.u[g];
    s_q[t] = a.q_cur[g];
    s_V[t] = a.V[g];
    if constexpr (FORM == 1) s_rho[t] = R.rho0 + a.drho[g];
  }
  __syncthreads();
  const int nin = L.cstart[nint];
  const int sub = threadIdx.x % LPP;
  for (int base = 0; base < nin; base += WG / LPP) {
    const int p = base + threadIdx.x / LPP;
    const bool act = p < nin;
    int st = 0;
    // raw pair sums (see the epilogue for their meaning)
    Acc<COMP> Sxx, Sxy, Syy, Gxx, Gxy, Gyx, Gyy, Qax, Qay, Qbx, Qby;
    Acc<COMP> Mxx_a, Mxy_a, Myy_a, Mxx_b, Mxy_b, Myy_b, Vsx, Vsy, Wux, Wuy;
    Acc<COMP> Kc, V1x, V1y, A1x, A1y;
    Sxx.init(); Sxy.init(); Syy.init(); Gxx.init(); Gxy.init(); Gyx.init(); Gyy.init();
    Qax.init(); Qay.init(); Qbx.init(); Qby.init();
    Mxx_a.init(); Mxy_a.init(); Myy_a.init(); Mxx_b.init(); Mxy_b.init(); Myy_b.init();
    Vsx.init(); Vsy.init(); Wux.init(); Wuy.init();
    Kc.init(); V1x.init(); V1y.init(); A1x.init(); A1y.init();
    float2 ui = {0.f, 0.f}, qi = {0.f, 0.f};
    float ri = 1.0f;
    if (act) {
      st = find_cell(L.cstart, nint, p);
      const int li = st % ni, lj = st / ni;
      const float2 oi = s_off[p];
      ui = s_u[p];
      qi = s_q[p];
      if constexpr (FORM == 1) ri = s_rho[p];
      const float ri2inv = 1.0f / (ri * ri);
#pragma unroll 1
      for (int cidx = 0; cidx < 9; ++cidx) {
          const int dy = cidx / 3 - 1, dx = cidx % 3 - 1;
          const int sc = L.slot[(lj + dy + 1) * (ni + 2) + (li + dx + 1)];
          const int j1 = L.cstart[sc + 1];
          const float sx = (float)(-dx) * R.cs, sy = (float)(-dy) * R.cs;
          for (int j = L.cstart[sc] + sub; j < j1; j += LPP) {
            const float2 oj = s_off[j];
            float rx, ry, r2;
            if (!pair_accept(oi.x, oi.y, oj.x, oj.y, sx, sy, R.R2, rx, ry, r2)) continue;
            const KW k = quintic(R, r2);
            const float Vj = s_V[j];
            const float2 uj = s_u[j], qj = s_q[j];
            const float c = Vj * k.F;              // V_j W'(r)/r
            const float cx = c * rx, cy = c * ry;  // V_j grad_i W_ij
            const float txx = cx * rx, txy = cx * ry, tyy = cy * ry;
            Sxx.add(txx); Sxy.add(txy); Syy.add(tyy);
            const float dux = uj.x - ui.x, duy = uj.y - ui.y;
            const float dqa = qj.x - qi.x, dqb = qj.y - qi.y;
            Gxx.fma(dux, cx); Gxy.fma(dux, cy); Gyx.fma(duy, cx); Gyy.fma(duy, cy);
            Qax.fma(dqa, cx); Qay.fma(dqa, cy); Qbx.fma(dqb, cx); Qby.fma(dqb, cy);
            const float e = k.rinv * k.rinv;
            const float la = -dqa * e, lb = -dqb * e;   // (Q_i - Q_j)/r^2
            Mxx_a.fma(la, txx); Mxy_a.fma(la, txy); Myy_a.fma(la, tyy);
            Mxx_b.fma(lb, txx); Mxy_b.fma(lb, txy); Myy_b.fma(lb, tyy);
            const float sv = -(dux * rx + duy * ry) * e;  // (u_i - u_j).r_ij / r^2
            if constexpr (FORM == 0) {
              Vsx.fma(sv, cx); Vsy.fma(sv, cy);
            } else {
              const float rj = s_rho[j];
              const float fx = k.F * rx, fy = k.F * ry;  // grad_i W_ij
              Kc.add(-(dux * fx + duy * fy));
              const float svr = sv / rj;
              V1x.fma(svr, fx); V1y.fma(svr, fy);
              const float rj2inv = 1.0f / (rj * rj);
              const float ca = qi.x * ri2inv + qj.x * rj2inv, cb = qi.y * ri2inv + qj.y * rj2inv;
              A1x.add(ca * fx + cb * fy); A1y.add(cb * fx - ca * fy);
            }
            Wux.fma(-dux, k.W); Wuy.fma(-duy, k.W);
          }
          Sxx.end_cell(); Sxy.end_cell(); Syy.end_cell();
          Gxx.end_cell(); Gxy.end_cell(); Gyx.end_cell(); Gyy.end_cell();
          Qax.end_cell(); Qay.end_cell(); Qbx.end_cell(); Qby.end_cell();
          Mxx_a.end_cell(); Mxy_a.end_cell(); Myy_a.end_cell();
          Mxx_b.end_cell(); Mxy_b.end_cell(); Myy_b.end_cell();
          Vsx.end_cell(); Vsy.end_cell(); Wux.end_cell(); Wuy.end_cell();
          if constexpr (FORM == 1) { Kc.end_cell(); V1x.end_cell(); V1y.end_cell(); A1x.end_cell(); A1y.end_cell(); }
        }
    }
    const float sxx = Sxx.template total<LPP>(), sxy = Sxy.template total<LPP>(), syy = Syy.template total<LPP>();
    const float gxx = Gxx.template total<LPP>(), gxy = Gxy.template total<LPP>();
    const float gyx = Gyx.template total<LPP>(), gyy = Gyy.template total<LPP>();
    const float qax = Qax.template total<LPP>(), qay = Qay.template total<LPP>();
    const float qbx = Qbx.template total<LPP>(), qby = Qby.template total<LPP>();
    const float mxxa = Mxx_a.template total<LPP>(), mxya = Mxy_a.template total<LPP>(), myya = Myy_a.template total<LPP>();
    const float mxxb = Mxx_b.template total<LPP>(), mxyb = Mxy_b.template total<LPP>(), myyb = Myy_b.template total<LPP>();
    const float wux = Wux.template total<LPP>(), wuy = Wuy.template total<LPP>();
    float vsx = 0.f, vsy = 0.f, kc = 0.f, v1x = 0.f, v1y = 0.f, a1x = 0.f, a1y = 0.f;
    if constexpr (FORM == 0) { vsx = Vsx.template total<LPP>(); vsy = Vsy.template total<LPP>(); }
    else {
      kc = Kc.template total<LPP>(); v1x = V1x.template total<LPP>(); v1y = V1y.template total<LPP>();
      a1x = A1x.template total<LPP>(); a1y = A1y.template total<LPP>();
    }
    if (act && sub == 0) {
      const int g = L.gstart[st] + (p - L.cstart[st]);
      if (g < 0 || g >= a.ntot) { flag(a.flags, ERR_RANGE); continue; }
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
      // molecular field (2D: the B term vanishes identically)
      const float qa = qi.x, qb = qi.y;
      const float trq2 = 2.0f * (qa * qa + qb * qb);
      const float cb = R.A + R.C * trq2;
      const float Ha = -cb * qa + R.K * lapa, Hb = -cb * qb + R.K * lapb;
      // co-rotation projected on symmetric traceless tensors (d = 2)
      const float e12 = 0.5f * (G12 + G21), w12 = 0.5f * (G12 - G21);
      const float QG = qa * (G11 - G22) + 2.0f * qb * e12;
      const float Sa = R.lam * (qa * divu + 0.5f * (G11 - G22)) + 2.0f * w12 * qb - 2.0f * R.lam * qa * QG;
      const float Sb = R.lam * (qb * divu + e12) - 2.0f * w12 * qa - 2.0f * R.lam * qb * QG;
      a.q_nxt[g] = make_float2(qa + (Sa + R.Gamma * Ha) * R.dt, qb + (Sb + R.Gamma * Hb) * R.dt);
      float apx, apy;
      if constexpr (FORM == 0) {
        const float vcx = vsx * Bxx + vsy * Bxy, vcy = vsx * Bxy + vsy * Byy;
        const float divqx = dax + dby, divqy = dbx - day;
        apx = 8.0f * R.eta * vcx - R.zeta * divqx;
        apy = 8.0f * R.eta * vcy - R.zeta * divqy;
      } else {
        const float cv = R.mass * 8.0f * R.eta / ri;
        apx = cv * v1x - R.zeta * R.mass * a1x;
        apy = cv * v1y - R.zeta * R.mass * a1y;
      }
      a.apart[g] = make_float2(apx, apy);
      a.uv[g] = sqrtf(wux * wux + wuy * wuy) * s_V[p];
      if constexpr (EL == 1) {
        const float QH = 2.0f * (qa * Ha + qb * Hb);
        a.pi[g] = make_float2(R.lam * (2.0f * QH * qa - Ha), R.lam * (2.0f * QH * qb - Hb));
      }
    }
  }
}

// ------------------------------------------------------------------ pass C
template <int T, int LPP, int COMP>
__global__ __launch_bounds__(WG) void k_pass_c(const StepArgs a) {
  __shared__ TileLDS<T> L;
  constexpr int MP = TileCfg<T>::MAXP;
  __shared__ float2 s_off[MP];
  __shared__ float s_dh[MP];
  RepDev R;
  int rep;
  if (!tile_begin<T>(a, L, R, rep)) return;
  const int ni = L.hdr[0], nint = L.hdr[2], nreg = L.hdr[3];
  const int S = L.cstart[nreg];
  for (int t = threadIdx.x; t < S; t += WG) {
    const int g = staged_global<T>(a, L, t);
    s_off[t] = a.off_cur[g];
    s_dh[t] = a.dh[g];
  }
  __syncthreads();
  const float umax = __uint_as_float(a.umax_cur[rep]);
  const float c0 = R.c0_factor * umax;
  const float pc = R.rho0 * c0 * c0 / R.gamma_eos;
  const int nin = L.cstart[nint];
  const int sub = threadIdx.x % LPP;
  for (int base = 0; base < nin; base += WG / LPP) {
    const int p = base + threadIdx.x / LPP;
    const bool act = p < nin;
    int st = 0;
    Acc<COMP> sd;
    sd.init();
    if (act) {
      st = find_cell(L.cstart, nint, p);
      const int li = st % ni, lj = st / ni;
      const float2 oi = s_off[p];
#pragma unroll 1
      for (int cidx = 0; cidx < 9; ++cidx) {
          const int dy = cidx / 3 - 1, dx = cidx % 3 - 1;
          const int sc = L.slot[(lj + dy + 1) * (ni + 2) + (li + dx + 1)];
          const int j1 = L.cstart[sc + 1];
          const float sx = (float)(-dx) * R.cs, sy = (float)(-dy) * R.cs;
          for (int j = L.cstart[sc] + sub; j < j1; j += LPP) {
            const float2 oj = s_off[j];
            float rx, ry, r2;
            if (pair_accept(oi.x, oi.y, oj.x, oj.y, sx, sy, R.R2, rx, ry, r2))
              sd.fma(s_dh[j], quintic_W(R, r2));
          }
          sd.end_cell();
        }
    }
    const float tot = sd.template total<LPP>();
    if (act && sub == 0) {
      const int g = L.gstart[st] + (p - L.cstart[st]);
      if (g < 0 || g >= a.ntot) { flag(a.flags, ERR_RANGE); continue; }
      const float Vi = a.V[g];
      const float dhi = s_dh[p];
      // Shepard filter with the self term, written for rho - rho0
      const float shep = Vi * fmaf(R.W0, dhi, tot);
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
    }
  }
}

// ------------------------------------------------------------------ pass D
template <int T, int LPP, int COMP, int FORM, int EL>
__global__ __launch_bounds__(WG) void k_pass_d(const StepArgs a) {
  __shared__ TileLDS<T> L;
  constexpr int MP = TileCfg<T>::MAXP;
  __shared__ float2 s_off[MP];
  __shared__ float s_V[MP];
  __shared__ float s_P[MP];
  __shared__ float2 s_pi[EL == 1 ? MP : 1];
  RepDev R;
  int rep;
  if (!tile_begin<T>(a, L, R, rep)) return;
  const int ni = L.hdr[0], nint = L.hdr[2], nreg = L.hdr[3];
  const int S = L.cstart[nreg];
  for (int t = threadIdx.x; t < S; t += WG) {
    const int g = staged_global<T>(a, L, t);
    s_off[t] = a.off_cur[g];
    s_V[t] = a.V[g];
    s_P[t] = a.P[g];
    if constexpr (EL == 1) s_pi[t] = a.pi[g];
  }
  __syncthreads();
  const int nin = L.cstart[nint];
  const int sub = threadIdx.x % LPP;
  float umax_w = 0.0f;
  bool rebin = false, bad = false;
  for (int base = 0; base < nin; base += WG / LPP) {
    const int p = base + threadIdx.x / LPP;
    const bool act = p < nin;
    int st = 0;
    Acc<COMP> Px, Py, Rx3, Ry3, Rs, Exx, Exy, Eyx, Eyy;
    Px.init(); Py.init(); Rx3.init(); Ry3.init(); Rs.init();
    Exx.init(); Exy.init(); Eyx.init(); Eyy.init();
    int cnt = 0;
    float2 oi = {0.f, 0.f};
    if (act) {
      st = find_cell(L.cstart, nint, p);
      const int li = st % ni, lj = st / ni;
      oi = s_off[p];
      const float Pi = s_P[p];
      float2 pii = {0.f, 0.f};
      if constexpr (EL == 1) pii = s_pi[p];
#pragma unroll 1
      for (int cidx = 0; cidx < 9; ++cidx) {
          const int dy = cidx / 3 - 1, dx = cidx % 3 - 1;
          const int sc = L.slot[(lj + dy + 1) * (ni + 2) + (li + dx + 1)];
          const int j1 = L.cstart[sc + 1];
          const float sx = (float)(-dx) * R.cs, sy = (float)(-dy) * R.cs;
          for (int j = L.cstart[sc] + sub; j < j1; j += LPP) {
            const float2 oj = s_off[j];
            float rx, ry, r2;
            if (!pair_accept(oi.x, oi.y, oj.x, oj.y, sx, sy, R.R2, rx, ry, r2)) continue;
            const KW k = quintic(R, r2);
            const float c = (FORM == 0) ? s_V[j] * k.F : k.F;
            const float f = (Pi + s_P[j]) * c;
            Px.fma(f, rx); Py.fma(f, ry);
            if constexpr (EL == 1) {
              const float2 pj = s_pi[j];
              const float cx = c * rx, cy = c * ry;
              const float dpa = pj.x - pii.x, dpb = pj.y - pii.y;
              Exx.fma(dpa, cx); Exy.fma(dpa, cy); Eyx.fma(dpb, cx); Eyy.fma(dpb, cy);
            }
            const float r3 = k.rinv * k.rinv * k.rinv;
            Rx3.fma(rx, r3); Ry3.fma(ry, r3); Rs.add(k.r);
            ++cnt;
          }
          Px.end_cell(); Py.end_cell(); Rx3.end_cell(); Ry3.end_cell(); Rs.end_cell();
          if constexpr (EL == 1) { Exx.end_cell(); Exy.end_cell(); Eyx.end_cell(); Eyy.end_cell(); }
        }
    }
    const float prx = Px.template total<LPP>(), pry = Py.template total<LPP>();
    const float srx = Rx3.template total<LPP>(), sry = Ry3.template total<LPP>(), sr = Rs.template total<LPP>();
    float exx = 0.f, exy = 0.f, eyx = 0.f, eyy = 0.f;
    if constexpr (EL == 1) {
      exx = Exx.template total<LPP>(); exy = Exy.template total<LPP>();
      eyx = Eyx.template total<LPP>(); eyy = Eyy.template total<LPP>();
    }
#pragma unroll
    for (int o = 1; o < LPP; o <<= 1) cnt += __shfl_xor(cnt, o, 64);
    if (act && sub == 0) {
      const int g = L.gstart[st] + (p - L.cstart[st]);
      if (g < 0 || g >= a.ntot) { flag(a.flags, ERR_RANGE); continue; }
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
      const float u1x = uh.x + hdt * ax, u1y = uh.y + hdt * ay;   // u^{n+1}
      float drx = 0.f, dry = 0.f;
      if (R.apd && cnt > 0) {
        const float r0 = sr / (float)cnt;
        const float f = r0 * r0 * a.uv[g] * R.dt;
        drx = f * srx; dry = f * sry;
      }
      const float unx = u1x + hdt * ax, uny = u1y + hdt * ay;      // u^{n+3/2}
      const float dispx = hdt * u1x + drx + hdt * unx;
      const float dispy = hdt * u1y + dry + hdt * uny;
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
      a.off_nxt[g] = nh;
      a.offlo[g] = nl;
      a.u[g] = make_float2(unx, uny);
      a.acc[g] = make_float2(ax, ay);
      a.drho[g] = drh + hdt * bk.w;
      umax_w = fmaxf(umax_w, sqrtf(unx * unx + uny * uny));
      if (nh.x < -R.skin_half || nh.x > R.cs + R.skin_half || nh.y < -R.skin_half || nh.y > R.cs + R.skin_half)
        rebin = true;
      if (!(isfinite(unx) && isfinite(uny) && isfinite(nh.x) && isfinite(nh.y) && isfinite(a.drho[g])))
        bad = true;
    }
  }
  // one atomic per wave for the max speed; NaN speeds are reported as errors
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) umax_w = fmaxf(umax_w, __shfl_xor(umax_w, o, 64));
  if ((threadIdx.x & 63) == 0 && umax_w > 0.0f) atomicMax(&a.umax_nxt[rep], __float_as_uint(umax_w));
  if (rebin) atomicOr(&a.flags[1], 1u);
  if (bad) flag(a.flags, ERR_NUMERIC);
}

// ---------------------------------------------------------- neighbour export
// mode 0: count neighbours of each particle into cnt[id]; mode 1: write ids.
template <int T>
__global__ __launch_bounds__(WG) void k_neighbors(const StepArgs a, const int* sid, int rep_only, int mode,
                                                  int* cnt, const int64_t* row_ptr, int32_t* col,
                                                  int64_t cap) {
  __shared__ TileLDS<T> L;
  constexpr int MP = TileCfg<T>::MAXP;
  __shared__ float2 s_off[MP];
  __shared__ int s_id[MP];
  RepDev R;
  int rep;
  if (!tile_begin<T>(a, L, R, rep)) return;
  if (rep != rep_only) return;
  const int ni = L.hdr[0], nint = L.hdr[2], nreg = L.hdr[3];
  const int S = L.cstart[nreg];
  for (int t = threadIdx.x; t < S; t += WG) {
    const int g = staged_global<T>(a, L, t);
    s_off[t] = a.off_cur[g];
    s_id[t] = sid[g];
  }
  __syncthreads();
  const int nin = L.cstart[nint];
  for (int p = threadIdx.x; p < nin; p += WG) {
    const int st = find_cell(L.cstart, nint, p);
    const int li = st % ni, lj = st / ni;
    const float2 oi = s_off[p];
    const int idi = s_id[p];
    if (idi < 0 || idi >= R.n) { flag(a.flags, ERR_RANGE); continue; }
    int c = 0;
    int64_t base = (mode == 1) ? row_ptr[idi] : 0;
#pragma unroll 1
    for (int cidx = 0; cidx < 9; ++cidx) {
        const int dy = cidx / 3 - 1, dx = cidx % 3 - 1;
        const int sc = L.slot[(lj + dy + 1) * (ni + 2) + (li + dx + 1)];
        const float sx = (float)(-dx) * R.cs, sy = (float)(-dy) * R.cs;
        for (int j = L.cstart[sc]; j < L.cstart[sc + 1]; ++j) {
          const float2 oj = s_off[j];
          float rx, ry, r2;
          if (pair_accept(oi.x, oi.y, oj.x, oj.y, sx, sy, R.R2, rx, ry, r2)) {
            if (mode == 1) {
              if (base + c < cap) col[base + c] = s_id[j];
              else flag(a.flags, ERR_RANGE);
            }
            ++c;
          }
        }
      }
    if (mode == 0) cnt[idi] = c;
  }
}

// ------------------------------------------------------------- dispatch
template <int T, int LPP, int COMP, int FORM, int EL>
static void launch4(int pass, const StepArgs& a, hipStream_t s) {
  const dim3 grid(a.nwork), block(WG);
  switch (pass) {
    case 1: hipLaunchKernelGGL((k_pass_a<T, LPP, COMP>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_pass_b<T, LPP, COMP, FORM, EL>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_pass_c<T, LPP, COMP>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_pass_d<T, LPP, COMP, FORM, EL>), grid, block, 0, s, a); break;
  }
}

// Supported combinations: the default physics (form 0, reduced stress) for
// tiles of 4 or 8 cells and 1, 2 or 4 lanes per particle with per-cell
// compensation; every compensation mode at T = 4, LPP = 1; the conservative
// form and the elastic lambda terms at T = 4, LPP = 1.
bool launch_pass(int pass, const PassCfg& c, const StepArgs& a, hipStream_t s) {
  if (c.FORM == 0 && c.EL == 0) {
    if (c.COMP == 1) {
      if (c.T == 4 && c.LPP == 1) { launch4<4, 1, 1, 0, 0>(pass, a, s); return true; }
      if (c.T == 4 && c.LPP == 2) { launch4<4, 2, 1, 0, 0>(pass, a, s); return true; }
      if (c.T == 4 && c.LPP == 4) { launch4<4, 4, 1, 0, 0>(pass, a, s); return true; }
      if (c.T == 8 && c.LPP == 1) { launch4<8, 1, 1, 0, 0>(pass, a, s); return true; }
      if (c.T == 8 && c.LPP == 2) { launch4<8, 2, 1, 0, 0>(pass, a, s); return true; }
      if (c.T == 8 && c.LPP == 4) { launch4<8, 4, 1, 0, 0>(pass, a, s); return true; }
    }
    if (c.T == 4 && c.LPP == 1 && c.COMP == 0) { launch4<4, 1, 0, 0, 0>(pass, a, s); return true; }
    if (c.T == 4 && c.LPP == 1 && c.COMP == 2) { launch4<4, 1, 2, 0, 0>(pass, a, s); return true; }
    return false;
  }
  if (c.T != 4 || c.LPP != 1 || c.COMP != 1) return false;
  if (c.FORM == 1 && c.EL == 0) { launch4<4, 1, 1, 1, 0>(pass, a, s); return true; }
  if (c.FORM == 0 && c.EL == 1) { launch4<4, 1, 1, 0, 1>(pass, a, s); return true; }
  return false;
}

void launch_neighbors(int T, const StepArgs& a, const int* sid, int rep, int mode, int* cnt,
                      const int64_t* row_ptr, int32_t* col, int64_t cap, hipStream_t s) {
  const dim3 grid(a.nwork), block(WG);
  if (T == 8)
    hipLaunchKernelGGL((k_neighbors<8>), grid, block, 0, s, a, sid, rep, mode, cnt, row_ptr, col, cap);
  else
    hipLaunchKernelGGL((k_neighbors<4>), grid, block, 0, s, a, sid, rep, mode, cnt, row_ptr, col, cap);
}

}  // namespace nem
