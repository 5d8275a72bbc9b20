// nem_mlp.hip -- the learned corrector's network on gfx950 matrix cores.
//
// A 12 -> 64 -> 64 -> 5 perceptron (tanh hidden layers, linear output) on
// z-scored inputs and targets. Every product runs on v_mfma_f32_16x16x32_bf16
// (BF16 operands, FP32 accumulation); master weights, Adam moments and all
// element-wise work stay in FP32. A wave owns 32 samples (two 16-row tiles) at
// a time and keeps its activations in LDS as BF16.
//
// MFMA 16x16x32 operand layout (wave64, lane l, i = 0..7 / 0..3):
//   A (16 x 32): A[l % 16][8 (l / 16) + i]      B (32 x 16): B[8 (l / 16) + i][l % 16]
//   D (16 x 16): D[4 (l / 16) + i][l % 16]
//
// Flat parameter vector (FP32): W1 (12 x 64, input-major), b1 (64), W2 (64 x 64),
// b2 (64), W3 (64 x 5), b3 (5).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace nem {

typedef __bf16 bf16;
typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NI = 12, NH = 64, NO = 5;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NI * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NO, NPARAM = OFF_B3 + NO;
constexpr int ROWS = 32;  // samples per wave iteration

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Fragment loads from row-major BF16 tiles in LDS.
// A block rows r0.., cols k0..: lane -> S[r0 + l%16][k0 + 8(l/16) + i]
__device__ __forceinline__ bf16x8 frag_a(const bf16* S, int ld, int r0, int k0, int l) {
  const bf16* p = S + (r0 + (l & 15)) * ld + k0 + (l >> 4) * 8;
  bf16x8 v;
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = p[i];
  return v;
}
// A = S^T: A[m][k] = S[k][m]; lane -> S[k0 + 8(l/16) + i][m0 + l%16]
__device__ __forceinline__ bf16x8 frag_at(const bf16* S, int ld, int m0, int k0, int l) {
  const bf16* p = S + (k0 + (l >> 4) * 8) * ld + m0 + (l & 15);
  bf16x8 v;
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = p[i * ld];
  return v;
}
// B block rows k0.., cols n0..: lane -> S[k0 + 8(l/16) + i][n0 + l%16]
__device__ __forceinline__ bf16x8 frag_b(const bf16* S, int ld, int k0, int n0, int l) {
  return frag_at(S, ld, n0, k0, l);
}
// B = S^T: B[k][n] = S[n][k]; lane -> S[n0 + l%16][k0 + 8(l/16) + i]
__device__ __forceinline__ bf16x8 frag_bt(const bf16* S, int ld, int k0, int n0, int l) {
  return frag_a(S, ld, n0, k0, l);
}

struct MlpNorm { float xm[NI], xs[NI], xr[NI], ym[NO], ys[NO]; };  // xr = 1 / xs

// tanh(x) = 1 - 2 / (exp(2x) + 1) on the hardware exp2 and reciprocal (about
// 1e-7 absolute error, far below the BF16 rounding of the activations it
// feeds); exp overflow gives +1, underflow -1.
__device__ __forceinline__ float fast_tanh(float x) {
  const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * x);  // 2 log2(e) x
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

// BF16 copies of the weights in LDS, zero-padded to MFMA shapes.
struct WLds {
  bf16 w1[32 * NH];   // rows 12..31 zero (K padding)
  bf16 w2[NH * NH];
  bf16 w3[NH * 16];   // cols 5..15 zero (N padding)
  bf16 w3t[32 * NH];  // W3^T, rows 5..31 zero
  float b1[NH], b2[NH], b3[16];
};

__device__ void load_weights(const float* P, WLds& W, bool need_t) {
  for (int t = threadIdx.x; t < 32 * NH; t += blockDim.x) {
    const int k = t / NH, n = t % NH;
    W.w1[t] = (bf16)(k < NI ? P[OFF_W1 + k * NH + n] : 0.0f);
  }
  for (int t = threadIdx.x; t < NH * NH; t += blockDim.x) W.w2[t] = (bf16)P[OFF_W2 + t];
  for (int t = threadIdx.x; t < NH * 16; t += blockDim.x) {
    const int k = t / 16, n = t % 16;
    W.w3[t] = (bf16)(n < NO ? P[OFF_W3 + k * NO + n] : 0.0f);
  }
  if (need_t)
    for (int t = threadIdx.x; t < 32 * NH; t += blockDim.x) {
      const int o = t / NH, k = t % NH;
      W.w3t[t] = (bf16)(o < NO ? P[OFF_W3 + k * NO + o] : 0.0f);
    }
  for (int t = threadIdx.x; t < NH; t += blockDim.x) { W.b1[t] = P[OFF_B1 + t]; W.b2[t] = P[OFF_B2 + t]; }
  for (int t = threadIdx.x; t < 16; t += blockDim.x) W.b3[t] = t < NO ? P[OFF_B3 + t] : 0.0f;
}

// Per-wave activation tiles (forward) and the extra tiles of the backward pass.
struct ActF {
  bf16 x[ROWS * 32];   // normalised inputs, cols 12..31 zero
  bf16 h1[ROWS * NH];
  bf16 h2[ROWS * NH];  // reused for dA1 in the backward pass
};
struct Act : ActF {
  bf16 dy[ROWS * 32];  // dL/dy (cols 5..31 zero)
  bf16 da2[ROWS * NH];
};

// Load 32 samples (rows base..base+31 of the index map) normalised into a.x.
__device__ __forceinline__ void load_x(const float* X, int64_t n, int64_t base, const MlpNorm& nm,
                                       const int64_t* idx, ActF& a, int l) {
  for (int t = l; t < ROWS * 32; t += 64) {
    const int r = t / 32, c = t % 32;
    float v = 0.0f;
    const int64_t s = base + r;
    if (c < NI && s < n) {
      const int64_t src = idx ? idx[s] : s;
      v = (X[src * NI + c] - nm.xm[c]) * nm.xr[c];
    }
    a.x[t] = (bf16)v;
  }
}

// Forward of 32 samples; y (FP32, normalised units) for lane l: rows
// rt*16 + 4(l/16) + i, col l%16 < 5.
__device__ __forceinline__ void forward32(const WLds& W, ActF& a, int l, f32x4 y[2]) {
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma(frag_a(a.x, 32, rt * 16, 0, l), frag_b(W.w1, NH, 0, nt * 16, l), acc);
      const int col = nt * 16 + (l & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) a.h1[(rt * 16 + (l >> 4) * 4 + i) * NH + col] = (bf16)fast_tanh(acc[i] + W.b1[col]);
    }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kc = 0; kc < 2; ++kc)
        acc = mfma(frag_a(a.h1, NH, rt * 16, kc * 32, l), frag_b(W.w2, NH, kc * 32, nt * 16, l), acc);
      const int col = nt * 16 + (l & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) a.h2[(rt * 16 + (l >> 4) * 4 + i) * NH + col] = (bf16)fast_tanh(acc[i] + W.b2[col]);
    }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < 2; ++kc)
      acc = mfma(frag_a(a.h2, NH, rt * 16, kc * 32, l), frag_b(W.w3, 16, kc * 32, 0, l), acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += W.b3[l & 15];
    y[rt] = acc;
  }
}

// ---------------------------------------------------------------- forward
// Y (n x 5): corrections in physical units (denormalised). maxnorm (may be
// NULL): max over samples of the Euclidean norm of the normalised output,
// as float bits.
//
// Inference keeps the activations in registers by computing each layer
// transposed, H^T = W^T X^T: the weights are the A operand (fragments in LDS,
// see FwdLds), the 16 samples of an iteration are the N dimension, and the
// output tile D[4g + i][c] (g = l / 16, c = l % 16) holds hidden units
// 16 mt + 4g + i of sample c. The next layer's B operand needs, in lane l,
// K slots 8g..8g+7 of sample c; numbering the hidden units so that K slot
// 8g + i of K tile kc is unit 16 (2 kc + i / 4) + 4g + i % 4 makes that
// operand exactly the lane's own D registers of tiles 2kc and 2kc+1 (the
// weights' K index uses the same numbering), so no data moves between lanes.
__device__ __forceinline__ int unit_of(int kc, int g, int i) { return 16 * (2 * kc + (i >> 2)) + 4 * g + (i & 3); }

// Weight fragments of the inference kernel in LDS, shared by the workgroup's
// four waves (per-wave register copies of all 5184 weights limited the kernel
// to one or two waves per SIMD): fragment f of lane l at frag[f * 64 + l],
// f = 0..3 layer 1 (m tile), 4..11 layer 2 (4 m tiles x 2 K tiles), 12..13
// layer 3 (K tiles). Biases per lane as the four rows it holds, layers 1 and 2
// pre-scaled by 2 log2(e) for the tanh below.
struct FwdLds {
  bf16x8 frag[14 * 64];
  f32x4 b1[4 * 64], b2[4 * 64], b3[64];
};
constexpr float TANH_K = 2.8853900817779268f;   // 2 log2(e)

// tanh(x) with x = d + bias and kb = TANH_K * bias (see fast_tanh)
__device__ __forceinline__ float tanh_kb(float d, float kb) {
  const float e = __builtin_amdgcn_exp2f(fmaf(TANH_K, d, kb));
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

// X rows are 48 bytes; VEC reads them as float4 (X 16-byte aligned).
template <bool VEC>
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ P, MlpNorm nm,
                                                     const float* __restrict__ X, int64_t n, float* Y,
                                                     unsigned* maxnorm) {
  constexpr int NB = 2;  // independent 16-sample blocks per iteration (instruction-level parallelism)
  __shared__ FwdLds W;
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, g = l >> 4, c = l & 15;
  // fill the fragments: A[m][k] = W^T, lane (gl, cl) holds k = 8 gl + i (in the
  // unit numbering of unit_of for layers 2 and 3) of row m = 16 mt + cl
  for (int t = threadIdx.x; t < 14 * 64; t += blockDim.x) {
    const int f = t >> 6, ln = t & 63, gl = ln >> 4, cl = ln & 15;
    bf16x8 v;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      float w;
      if (f < 4) {
        const int k = 8 * gl + i;
        w = k < NI ? P[OFF_W1 + k * NH + 16 * f + cl] : 0.0f;
      } else if (f < 12) {
        const int mt = (f - 4) >> 1, kc = (f - 4) & 1;
        w = P[OFF_W2 + unit_of(kc, gl, i) * NH + 16 * mt + cl];
      } else {
        w = cl < NO ? P[OFF_W3 + unit_of(f - 12, gl, i) * NO + cl] : 0.0f;
      }
      v[i] = (bf16)w;
    }
    W.frag[t] = v;
  }
  for (int t = threadIdx.x; t < 4 * 64; t += blockDim.x) {
    const int mt = t >> 6, gl = (t & 63) >> 4;
    f32x4 v1, v2;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v1[i] = TANH_K * P[OFF_B1 + 16 * mt + 4 * gl + i];
      v2[i] = TANH_K * P[OFF_B2 + 16 * mt + 4 * gl + i];
    }
    W.b1[t] = v1; W.b2[t] = v2;
  }
  for (int t = threadIdx.x; t < 64; t += blockDim.x) {
    f32x4 v3;
#pragma unroll
    for (int i = 0; i < 4; ++i) v3[i] = (4 * (t >> 4) + i < NO) ? P[OFF_B3 + 4 * (t >> 4) + i] : 0.0f;
    W.b3[t] = v3;
  }
  __syncthreads();
  // this lane's input features 8g + i (i < nf) and their normalisation
  const int nf = g == 0 ? 8 : (g == 1 ? NI - 8 : 0);
  float xm8[8], xr8[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    xm8[i] = i < nf ? nm.xm[8 * g + i] : 0.0f;
    xr8[i] = i < nf ? nm.xr[8 * g + i] : 0.0f;
  }
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  float mx = 0.0f;
  const int64_t nblk = (n + 15) / 16;
  for (int64_t b0 = ((int64_t)blockIdx.x * 4 + wv) * NB; b0 < nblk; b0 += (int64_t)gridDim.x * 4 * NB) {
    int64_t s[NB];
    bf16x8 xb[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      s[q] = (b0 + q) * 16 + c;
      const float* xrow = X + (s[q] < n ? s[q] : n - 1) * NI + 8 * g;  // clamped: in bounds for every lane
      float xv[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (VEC) {
        if (nf > 0) {
          const float4 v0 = *reinterpret_cast<const float4*>(xrow);
          xv[0] = v0.x; xv[1] = v0.y; xv[2] = v0.z; xv[3] = v0.w;
        }
        if (nf > 4) {
          const float4 v1 = *reinterpret_cast<const float4*>(xrow + 4);
          xv[4] = v1.x; xv[5] = v1.y; xv[6] = v1.z; xv[7] = v1.w;
        }
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (i < nf) xv[i] = xrow[i];
      }
      const float keep = s[q] < n ? 1.0f : 0.0f;
#pragma unroll
      for (int i = 0; i < 8; ++i) xb[q][i] = (bf16)(keep * ((xv[i] - xm8[i]) * xr8[i]));
    }
    // The fragment and bias reads below are the same every iteration; an
    // empty asm statement on the lane index keeps the compiler from hoisting
    // them out of the loop into registers (which would cost the occupancy the
    // LDS copy is for).
    int l_ = l;
    asm volatile("" : "+v"(l_));
    f32x4 d[NB][4];
    bf16x8 hb[NB][2];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const bf16x8 a = W.frag[mt * 64 + l_];
#pragma unroll
      for (int q = 0; q < NB; ++q) d[q][mt] = mfma(a, xb[q], zero);
    }
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      const f32x4 k0 = W.b1[(2 * kc) * 64 + l_], k1 = W.b1[(2 * kc + 1) * 64 + l_];
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          hb[q][kc][i] = (bf16)tanh_kb(d[q][2 * kc][i], k0[i]);
          hb[q][kc][4 + i] = (bf16)tanh_kb(d[q][2 * kc + 1][i], k1[i]);
        }
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const bf16x8 a0 = W.frag[(4 + 2 * mt) * 64 + l_], a1 = W.frag[(5 + 2 * mt) * 64 + l_];
#pragma unroll
      for (int q = 0; q < NB; ++q) d[q][mt] = mfma(a1, hb[q][1], mfma(a0, hb[q][0], zero));
    }
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      const f32x4 k0 = W.b2[(2 * kc) * 64 + l_], k1 = W.b2[(2 * kc + 1) * 64 + l_];
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          hb[q][kc][i] = (bf16)tanh_kb(d[q][2 * kc][i], k0[i]);
          hb[q][kc][4 + i] = (bf16)tanh_kb(d[q][2 * kc + 1][i], k1[i]);
        }
    }
    const bf16x8 a30 = W.frag[12 * 64 + l_], a31 = W.frag[13 * 64 + l_];
    const f32x4 b3 = W.b3[l_];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const f32x4 y = mfma(a31, hb[q][1], mfma(a30, hb[q][0], b3));
      // lane (g, c) holds outputs 4g + i of sample s: g = 0 -> 0..3, g = 1 -> 4
      float sq = 0.0f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int o = 4 * g + i;
        if (o < NO) {
          sq += y[i] * y[i];
          if (s[q] < n) Y[s[q] * NO + o] = y[i] * nm.ys[o] + nm.ym[o];
        }
      }
      sq += __shfl_xor(sq, 16, 64);
      sq += __shfl_xor(sq, 32, 64);
      if (s[q] < n) mx = fmaxf(mx, sqrtf(sq));
    }
  }
  if (maxnorm) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if (l == 0 && mx > 0.0f) atomicMax(maxnorm, __float_as_uint(mx));
  }
}

// --------------------------------------------------------------- backward
// Gradient of L = (1/2B) sum_s |y_s - t_s|^2 (normalised units) over the
// minibatch idx[0..B) of (X, T). Each wave accumulates its samples into
// registers and writes one partial gradient vector (partial[wave][NPARAM]) and
// its partial loss (lossp[wave]).
__global__ __launch_bounds__(128) void k_mlp_backward(const float* __restrict__ P, MlpNorm nm,
                                                      const float* __restrict__ X, const float* __restrict__ Tg,
                                                      const int64_t* __restrict__ idx, int64_t B, float* partial,
                                                      float* lossp) {
  __shared__ WLds W;
  __shared__ Act act[2];
  load_weights(P, W, true);
  __syncthreads();
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int gw = blockIdx.x * 2 + wv;
  Act& a = act[wv];
  f32x4 g1[2][4], g2[4][4], g3[4];
  float gb1[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0}, gb3 = 0.0f, ls = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    g3[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    g1[0][i] = g3[i]; g1[1][i] = g3[i];
#pragma unroll
    for (int j = 0; j < 4; ++j) g2[i][j] = g3[i];
  }
  const float invB = 1.0f / (float)B;
  const int64_t nblk = (B + ROWS - 1) / ROWS;
  for (int64_t b = gw; b < nblk; b += (int64_t)gridDim.x * 2) {
    const int64_t base = b * ROWS;
    load_x(X, B, base, nm, idx, a, l);
    __builtin_amdgcn_wave_barrier();
    f32x4 y[2];
    forward32(W, a, l, y);
    // dL/dy = (y - t) / B in normalised units; padded columns and rows are zero
    const int col = l & 15;
    for (int t = l; t < ROWS * 32; t += 64) a.dy[t] = (bf16)0.0f;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = rt * 16 + (l >> 4) * 4 + i;
        const int64_t s = base + r;
        float d = 0.0f;
        if (col < NO && s < B) {
          const float t = (Tg[idx[s] * NO + col] - nm.ym[col]) / nm.ys[col];
          d = y[rt][i] - t;
          ls += d * d;
        }
        d *= invB;
        gb3 += d;
        a.dy[r * 32 + col] = (bf16)d;
      }
    __builtin_amdgcn_wave_barrier();
    // gW3 (64 x 16) += H2^T dY
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) g3[mt] = mfma(frag_at(a.h2, NH, mt * 16, 0, l), frag_b(a.dy, 32, 0, 0, l), g3[mt]);
    // dA2 = (dY W3^T) * (1 - h2^2)
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(frag_a(a.dy, 32, rt * 16, 0, l), frag_b(W.w3t, NH, 0, nt * 16, l), acc);
        const int c = nt * 16 + (l & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = rt * 16 + (l >> 4) * 4 + i;
          const float h = (float)a.h2[r * NH + c];
          const float d = acc[i] * (1.0f - h * h);
          gb2[nt] += d;
          a.da2[r * NH + c] = (bf16)d;
        }
      }
    __builtin_amdgcn_wave_barrier();
    // gW2 (64 x 64) += H1^T dA2
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        g2[mt][nt] = mfma(frag_at(a.h1, NH, mt * 16, 0, l), frag_b(a.da2, NH, 0, nt * 16, l), g2[mt][nt]);
    // dA1 = (dA2 W2^T) * (1 - h1^2), stored over h2
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < 2; ++kc)
          acc = mfma(frag_a(a.da2, NH, rt * 16, kc * 32, l), frag_bt(W.w2, NH, kc * 32, nt * 16, l), acc);
        const int c = nt * 16 + (l & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = rt * 16 + (l >> 4) * 4 + i;
          const float h = (float)a.h1[r * NH + c];
          const float d = acc[i] * (1.0f - h * h);
          gb1[nt] += d;
          a.h2[r * NH + c] = (bf16)d;
        }
      }
    __builtin_amdgcn_wave_barrier();
    // gW1 (32 x 64, rows >= 12 unused) += X^T dA1
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        g1[mt][nt] = mfma(frag_at(a.x, 32, mt * 16, 0, l), frag_b(a.h2, NH, 0, nt * 16, l), g1[mt][nt]);
    __builtin_amdgcn_wave_barrier();
  }
  // bias sums: lanes with the same l%16 hold the same column
#pragma unroll
  for (int o = 16; o < 64; o <<= 1) {
    gb3 += __shfl_xor(gb3, o, 64);
#pragma unroll
    for (int k = 0; k < 4; ++k) { gb1[k] += __shfl_xor(gb1[k], o, 64); gb2[k] += __shfl_xor(gb2[k], o, 64); }
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) ls += __shfl_xor(ls, o, 64);
  float* out = partial + (size_t)gw * NPARAM;
  const int col = l & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int rr = (l >> 4) * 4 + i;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const int k = mt * 16 + rr;
      if (k < NI)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) out[OFF_W1 + k * NH + nt * 16 + col] = g1[mt][nt][i];
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const int k = mt * 16 + rr;
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) out[OFF_W2 + k * NH + nt * 16 + col] = g2[mt][nt][i];
      if (col < NO) out[OFF_W3 + k * NO + col] = g3[mt][i];
    }
  }
  if (l < 16) {
#pragma unroll
    for (int k = 0; k < 4; ++k) { out[OFF_B1 + k * 16 + l] = gb1[k]; out[OFF_B2 + k * 16 + l] = gb2[k]; }
    if (l < NO) out[OFF_B3 + l] = gb3;
  }
  if (l == 0) lossp[gw] = 0.5f * ls * invB;
}

// grads[p] = sum over waves of partial[w][p], in wave order.
__global__ void k_mlp_reduce(const float* partial, int nw, float* grads, const float* lossp, float* loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NPARAM) {
    float s = 0.0f;
    for (int w = 0; w < nw; ++w) s += partial[(size_t)w * NPARAM + p];
    grads[p] = s;
  }
  if (p == 0 && loss) {
    float s = 0.0f;
    for (int w = 0; w < nw; ++w) s += lossp[w];
    *loss = s;
  }
}

// One Adam step on the FP32 master weights.
__global__ void k_mlp_adam(float* P, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                           float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float gg = g[p];
  const float mm = b1 * m[p] + (1.0f - b1) * gg;
  const float vv = b2 * v[p] + (1.0f - b2) * gg * gg;
  m[p] = mm;
  v[p] = vv;
  P[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// Minibatch indices: a deterministic shuffle of [0, n) per epoch,
// idx[i] = (i * stride + offset) mod n with stride coprime to n.
__global__ void k_mlp_batch(int64_t* idx, int64_t first, int64_t B, int64_t n, int64_t stride, int64_t offset) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= B) return;
  const int64_t k = first + i;
  idx[i] = (int64_t)(((uint64_t)k * (uint64_t)stride + (uint64_t)offset) % (uint64_t)n);  // n, stride < 2^31
}

// Column means and standard deviations of X (n x NI) and T (n x NO) in FP64,
// two fixed-order passes (one block per column).
__global__ __launch_bounds__(256) void k_mlp_stats(const float* X, const float* T, int64_t n, double* out) {
  const int c = blockIdx.x;  // 0..NI-1 features, NI..NI+NO-1 targets
  const float* A = c < NI ? X : T;
  const int ld = c < NI ? NI : NO, cc = c < NI ? c : c - NI;
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += (double)A[i * ld + cc];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) { if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d]; __syncthreads(); }
  const double mean = sh[0] / (double)n;
  __syncthreads();
  double q = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) { const double d = (double)A[i * ld + cc] - mean; q += d * d; }
  sh[threadIdx.x] = q;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) { if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d]; __syncthreads(); }
  if (threadIdx.x == 0) { out[2 * c] = mean; out[2 * c + 1] = sqrt(sh[0] / (double)n); }
}

// ---------------------------------------------------------------- launchers
int mlp_nparam() { return NPARAM; }
int mlp_backward_waves(int64_t B) {
  const int64_t nblk = (B + ROWS - 1) / ROWS;
  return (int)std::min<int64_t>(std::max<int64_t>(nblk, 2), 1024) / 2 * 2;
}

void launch_mlp_forward(const float* P, const float* norm, const float* X, int64_t n, float* Y, unsigned* maxnorm,
                        hipStream_t s) {
  MlpNorm nm;
  for (int i = 0; i < NI; ++i) { nm.xm[i] = norm[i]; nm.xs[i] = norm[NI + i]; nm.xr[i] = 1.0f / norm[NI + i]; }
  for (int i = 0; i < NO; ++i) { nm.ym[i] = norm[2 * NI + i]; nm.ys[i] = norm[2 * NI + NO + i]; }
  const int64_t nblk = (n + 31) / 32;  // pairs of 16-sample blocks
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((nblk + 3) / 4, 1024));
  if (((uintptr_t)X & 15u) == 0)
    hipLaunchKernelGGL(k_mlp_forward<true>, dim3(grid), dim3(256), 0, s, P, nm, X, n, Y, maxnorm);
  else
    hipLaunchKernelGGL(k_mlp_forward<false>, dim3(grid), dim3(256), 0, s, P, nm, X, n, Y, maxnorm);
}

void launch_mlp_backward(const float* P, const float* norm, const float* X, const float* T, const int64_t* idx,
                         int64_t B, float* partial, float* lossp, int nwaves, hipStream_t s) {
  MlpNorm nm;
  for (int i = 0; i < NI; ++i) { nm.xm[i] = norm[i]; nm.xs[i] = norm[NI + i]; nm.xr[i] = 1.0f / norm[NI + i]; }
  for (int i = 0; i < NO; ++i) { nm.ym[i] = norm[2 * NI + i]; nm.ys[i] = norm[2 * NI + NO + i]; }
  hipLaunchKernelGGL(k_mlp_backward, dim3(nwaves / 2), dim3(128), 0, s, P, nm, X, T, idx, B, partial, lossp);
}

void launch_mlp_reduce(const float* partial, int nw, float* grads, const float* lossp, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_reduce, dim3((NPARAM + 255) / 256), dim3(256), 0, s, partial, nw, grads, lossp, loss);
}

void launch_mlp_adam(float* P, const float* g, float* m, float* v, float lr, int t, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, P, g, m, v, lr, b1, b2, 1e-8f, c1, c2);
}

void launch_mlp_batch(int64_t* idx, int64_t first, int64_t B, int64_t n, int64_t stride, int64_t offset,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_batch, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, idx, first, B, n, stride, offset);
}

void launch_mlp_stats(const float* X, const float* T, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_stats, dim3(NI + NO), dim3(256), 0, s, X, T, n, out);
}

}  // namespace nem
