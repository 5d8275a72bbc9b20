// nem_learn.hip -- the learned corrector: training samples drawn from the
// solver itself, the network's training loop, and macro steps of mult*dt whose
// Q and u are corrected by the network, with fine steps as the fallback.
//
// A macro step: take one step with time step mult*dt from the current state
// while pass B writes each particle's 12 inputs (Q, grad u, H, density,
// activity), run the network on them, and add the predicted corrections
// (dQxx, dQxy, dQyy, dux, duy) to Q and u. If the largest correction (in the
// network's normalised units) exceeds tau, the macro step is discarded and
// replayed from a device snapshot as mult steps of dt. Training targets are the
// difference between mult steps of dt and one step of mult*dt from the same
// state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "nem_dev.h"
#include "nem_sim.h"

namespace nem {

int mlp_nparam();
int mlp_backward_waves(int64_t B);
void launch_mlp_forward(const float* P, const float* norm, const float* X, int64_t n, float* Y, unsigned* maxnorm,
                        hipStream_t s);
void launch_mlp_backward(const float* P, const float* norm, const float* X, const float* T, const int64_t* idx,
                         int64_t B, float* partial, float* lossp, int nwaves, hipStream_t s);
void launch_mlp_reduce(const float* partial, int nw, float* grads, const float* lossp, float* loss, hipStream_t s);
void launch_mlp_adam(float* P, const float* g, float* m, float* v, float lr, int t, hipStream_t s);
void launch_mlp_batch(int64_t* idx, int64_t first, int64_t B, int64_t n, int64_t stride, int64_t offset,
                      hipStream_t s);
void launch_mlp_stats(const float* X, const float* T, int64_t n, double* out, hipStream_t s);

__device__ inline int rep_of(const RepDev* reps, int R, int k) {
  int lo = 0, hi = R;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (reps[mid].part_base <= k) lo = mid; else hi = mid;
  }
  return lo;
}

// Max of v over the workgroup (all threads call it; v >= 0), then one atomic
// into this workgroup's max-speed slot of replica r; any thread's relist
// request becomes one atomic on the Verlet rebuild flag.
__device__ __forceinline__ void block_speed_max(const SortArgs& s, unsigned* umax_cur, int r, float v, bool relist) {
  __shared__ float red[4];
  __shared__ int any_relist;
  if (threadIdx.x == 0) any_relist = 0;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (relist) any_relist = 1;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    if (m > 0.0f) atomicMax(&umax_cur[r * UMAX_SLOTS + (blockIdx.x & (UMAX_SLOTS - 1))], __float_as_uint(m));
    if (any_relist) atomicOr(&s.flags[2], 1u);
  }
}

// Offset moved further from its value at the last Verlet build than allowed.
__device__ __forceinline__ bool moved_too_far(const SortArgs& s, const RepDev& R, int k, float2 nh) {
  const float2 ob = s.off_build[k];
  const float bx = nh.x - ob.x, by = nh.y - ob.y;
  return bx * bx + by * by > R.disp2;
}

// Change every replica's time step by `factor`: recover r^n, u^n from the
// stored prediction (made with the old dt) and predict again with the new dt.
// Positions move by a few rounding units at most; the max-speed slots of the
// current parity are refilled (cleared by the caller). Grid: (chunks, R) of
// 256 threads; blockIdx.y is the replica.
__global__ __launch_bounds__(256) void k_repredict(SortArgs s, float factor, unsigned* umax_cur) {
  const int r = blockIdx.y;
  const RepDev& R = s.reps[r];
  const float dto = R.dt, dtn = dto * factor;
  float vmax = 0.0f;
  bool relist = false;
  for (int k = R.part_base + blockIdx.x * blockDim.x + threadIdx.x; k < R.part_base + R.n;
       k += gridDim.x * blockDim.x) {
    const float2 u = s.u[k], ac = s.acc[k], o = s.off[k], lo = s.offlo[k];
    const float unx = (u.x - 0.5f * dto * ac.x) + 0.5f * dtn * ac.x;
    const float uny = (u.y - 0.5f * dto * ac.y) + 0.5f * dtn * ac.y;
    const float dx = 0.5f * dtn * unx - 0.5f * dto * u.x, dy = 0.5f * dtn * uny - 0.5f * dto * u.y;
    float2 nh, nl;
    {
#pragma clang fp contract(off)
      float t = o.x + dx, bp = t - o.x, e = (o.x - (t - bp)) + (dx - bp), l2 = lo.x + e;
      nh.x = t + l2; nl.x = l2 - (nh.x - t);
      t = o.y + dy; bp = t - o.y; e = (o.y - (t - bp)) + (dy - bp); l2 = lo.y + e;
      nh.y = t + l2; nl.y = l2 - (nh.y - t);
    }
    s.off[k] = nh;
    s.offlo[k] = nl;
    s.u[k] = make_float2(unx, uny);
    vmax = fmaxf(vmax, sqrtf(unx * unx + uny * uny));
    relist |= moved_too_far(s, R, k, nh);
  }
  block_speed_max(s, umax_cur, r, vmax, relist);
}

// (Qxx, Qxy, Qyy, ux, uy) at the integer level into out[(part_base + id) * 5].
__global__ void k_export_qu(SortArgs s, float* out) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < s.ntot; k += gridDim.x * blockDim.x) {
    const int r = rep_of(s.reps, s.R, k);
    const RepDev& R = s.reps[r];
    const int id = s.id[k];
    if (id < 0 || id >= R.n) { atomicOr(s.flags, ERR_RANGE); continue; }
    const float2 q = s.q[k], u = s.u[k], ac = s.acc[k];
    float* o = out + (size_t)(R.part_base + id) * 5;
    o[0] = q.x; o[1] = q.y; o[2] = -q.x;
    o[3] = u.x - 0.5f * R.dt * ac.x;
    o[4] = u.y - 0.5f * R.dt * ac.y;
  }
}

__global__ void k_sub(float* T, const float* C, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    T[k] -= C[k];
}

// Add the network's corrections Y[k * 5] (storage order) to Q (projected on
// traceless tensors) and u; refill the max-speed slots (cleared by the
// caller). Grid as k_repredict. Skipped when the largest predicted correction
// norm (maxnorm, float bits) exceeds tau (bits of a positive float, so the
// unsigned comparison orders them as floats).
__global__ __launch_bounds__(256) void k_correct(SortArgs s, const float* Y, unsigned* umax_cur,
                                                 const unsigned* maxnorm, unsigned tau_bits, unsigned* host_norm) {
  // the norm for the host's fallback decision, stored straight into pinned
  // host memory (a plain vector store, visible once the kernel has completed)
  if (host_norm && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *host_norm = maxnorm ? *maxnorm : 0u;
  if (maxnorm && *maxnorm > tau_bits) return;  // the macro step will be replayed as fine steps
  const int r = blockIdx.y;
  const RepDev& R = s.reps[r];
  float vmax = 0.0f;
  bool relist = false;
  for (int k = R.part_base + blockIdx.x * blockDim.x + threadIdx.x; k < R.part_base + R.n;
       k += gridDim.x * blockDim.x) {
    const float* y = Y + (size_t)k * 5;
    float2 q = s.q[k], u = s.u[k];
    q.x += 0.5f * (y[0] - y[2]);
    q.y += y[1];
    u.x += y[3];
    u.y += y[4];
    s.q[k] = q;
    s.u[k] = u;
    // the stored position is r^{n+1} + u dt/2: move it with the corrected u
    const float dx = 0.5f * R.dt * y[3], dy = 0.5f * R.dt * y[4];
    const float2 o = s.off[k], lo = s.offlo[k];
    float2 nh, nl;
    {
#pragma clang fp contract(off)
      float t = o.x + dx, bp = t - o.x, e = (o.x - (t - bp)) + (dx - bp), l2 = lo.x + e;
      nh.x = t + l2; nl.x = l2 - (nh.x - t);
      t = o.y + dy; bp = t - o.y; e = (o.y - (t - bp)) + (dy - bp); l2 = lo.y + e;
      nh.y = t + l2; nl.y = l2 - (nh.y - t);
    }
    s.off[k] = nh;
    s.offlo[k] = nl;
    vmax = fmaxf(vmax, sqrtf(u.x * u.x + u.y * u.y));
    relist |= moved_too_far(s, R, k, nh);
  }
  block_speed_max(s, umax_cur, r, vmax, relist);
}

// Before the inference of a learned macro step: clear the largest-norm word
// and the max-speed slots that k_correct refills (one launch, no memset).
__global__ void k_learn_clear(unsigned* norm, unsigned* umax, int n_umax) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *norm = 0u;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_umax; i += gridDim.x * blockDim.x) umax[i] = 0u;
}

// dst[(part_base + id) * w + c] = src[k * w + c]: rows from storage order to
// original particle order.
__global__ void k_rows_by_id(SortArgs s, const float* src, float* dst, int w) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < s.ntot; k += gridDim.x * blockDim.x) {
    const int r = rep_of(s.reps, s.R, k);
    const RepDev& R = s.reps[r];
    const int id = s.id[k];
    if (id < 0 || id >= R.n) { atomicOr(s.flags, ERR_RANGE); continue; }
    const float* a = src + (size_t)k * w;
    float* b = dst + (size_t)(R.part_base + id) * w;
    for (int c = 0; c < w; ++c) b[c] = a[c];
  }
}

// Device-to-device copy of up to 12 buffers in one launch (16-byte chunks,
// then 4-byte words for the tail; every buffer is 4-byte sized and every
// buffer longer than 16 bytes starts 16-byte aligned).
struct CopySeg { const void* src; void* dst; int64_t bytes; };
struct CopyList { CopySeg seg[14]; int n; };
__global__ void k_copy_list(CopyList L) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int k = 0; k < L.n; ++k) {
    const CopySeg sg = L.seg[k];
    const int64_t n16 = sg.bytes / 16;
    const uint4* s16 = (const uint4*)sg.src;
    uint4* d16 = (uint4*)sg.dst;
    for (int64_t i = t0; i < n16; i += stride) d16[i] = s16[i];
    const int64_t n4 = (sg.bytes - n16 * 16) / 4;
    const uint32_t* s4 = (const uint32_t*)((const char*)sg.src + n16 * 16);
    uint32_t* d4 = (uint32_t*)((char*)sg.dst + n16 * 16);
    for (int64_t i = t0; i < n4; i += stride) d4[i] = s4[i];
  }
}

// Per-output statistics of targets T and predictions Y (n x 5) in FP64, one
// workgroup per output, a fixed summation order (deterministic):
// out[3o] = mean of T_o, out[3o + 1] = variance of T_o, out[3o + 2] = mean of
// (T_o - Y_o)^2.
__global__ __launch_bounds__(256) void k_eval_stats(const float* T, const float* Y, int64_t n, double* out) {
  const int o = blockIdx.x;
  __shared__ double sh[2][256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += (double)T[i * 5 + o];
  sh[0][threadIdx.x] = s;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (threadIdx.x < d) sh[0][threadIdx.x] += sh[0][threadIdx.x + d];
    __syncthreads();
  }
  const double mean = sh[0][0] / (double)n;
  __syncthreads();
  double v = 0.0, e = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double t = (double)T[i * 5 + o];
    const double dv = t - mean, de = t - (double)Y[i * 5 + o];
    v += dv * dv;
    e += de * de;
  }
  sh[0][threadIdx.x] = v;
  sh[1][threadIdx.x] = e;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (threadIdx.x < d) { sh[0][threadIdx.x] += sh[0][threadIdx.x + d]; sh[1][threadIdx.x] += sh[1][threadIdx.x + d]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { out[3 * o] = mean; out[3 * o + 1] = sh[0][0] / (double)n; out[3 * o + 2] = sh[1][0] / (double)n; }
}

// dst[k * w + c] = src[rows[k] * w + c] for the selected rows.
__global__ void k_gather_rows(const float* src, const int64_t* rows, int64_t nrows, int w, int64_t nsrc, float* dst,
                              unsigned* flags) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nrows; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = rows[k];
    if (r < 0 || r >= nsrc) { atomicOr(flags, ERR_RANGE); continue; }
    for (int c = 0; c < w; ++c) dst[k * w + c] = src[r * w + c];
  }
}

static int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048)); }

// (chunks, replicas) grid for the per-replica kernels.
static dim3 rep_grid(const nem_sim* s) {
  int64_t nmax = 1;
  for (const auto& R : s->reps) nmax = std::max<int64_t>(nmax, R.n);
  return dim3((unsigned)std::min<int64_t>((nmax + 255) / 256, 1024), (unsigned)s->R);
}

}  // namespace nem

using namespace nem;
using namespace nem_host;

struct nem_mlp {
  hipStream_t stream = nullptr;
  float* P = nullptr;      // FP32 master weights
  float* m = nullptr;      // Adam moments
  float* v = nullptr;
  float* g = nullptr;      // gradient
  float* norm = nullptr;   // x mean[12], x std[12], y mean[5], y std[5] (device)
  float hnorm[34];
  float* partial = nullptr;
  float* lossp = nullptr;
  float* loss = nullptr;
  int64_t* idx = nullptr;
  int64_t idx_cap = 0;
  int part_waves = 0;
  double* stats = nullptr;
  int adam_t = 0;
  std::string err;
};

namespace nem_host {

void free_snapshot(nem_sim* s) {
  for (auto& S : s->snap) {
    for (void* p : {(void*)S.off, (void*)S.offlo, (void*)S.u, (void*)S.q, (void*)S.acc, (void*)S.drho, (void*)S.id,
                    (void*)S.cell, (void*)S.img, (void*)S.qyy, (void*)S.cell_start, (void*)S.umax})
      if (p) hipFree(p);
    S = nem_sim::Snap();
  }
}

int take_snapshot(nem_sim* s, int i) {
  auto& S = s->snap[i];
  const size_t N = (size_t)s->ntot, C = (size_t)s->ncells;
  if (!S.alloc) {
    HIPCHK(hipMalloc((void**)&S.off, sizeof(float2) * N));
    HIPCHK(hipMalloc((void**)&S.offlo, sizeof(float2) * N));
    HIPCHK(hipMalloc((void**)&S.u, sizeof(float2) * N));
    HIPCHK(hipMalloc((void**)&S.q, sizeof(float2) * N));
    HIPCHK(hipMalloc((void**)&S.acc, sizeof(float2) * N));
    HIPCHK(hipMalloc((void**)&S.drho, sizeof(float) * N));
    HIPCHK(hipMalloc((void**)&S.id, sizeof(int) * N));
    HIPCHK(hipMalloc((void**)&S.cell, sizeof(int) * N));
    HIPCHK(hipMalloc((void**)&S.img, sizeof(int2) * N));
    HIPCHK(hipMalloc((void**)&S.qyy, sizeof(float) * N));
    HIPCHK(hipMalloc((void**)&S.cell_start, sizeof(int) * (C + 1)));
    HIPCHK(hipMalloc((void**)&S.umax, sizeof(unsigned) * (s->R * UMAX_SLOTS + 1)));  // + rebin request
    S.alloc = true;
  }
  const int p = s->parity;
  CopyList cl;
  cl.n = 0;
  bool full = false;
  auto add = [&](const void* src, void* dst, size_t bytes) {
    if (cl.n < (int)(sizeof(cl.seg) / sizeof(cl.seg[0]))) cl.seg[cl.n++] = CopySeg{src, dst, (int64_t)bytes};
    else full = true;
  };
  add(s->off[p], S.off, sizeof(float2) * N);
  add(s->offlo, S.offlo, sizeof(float2) * N);
  add(s->u, S.u, sizeof(float2) * N);
  add(s->q[p], S.q, sizeof(float2) * N);
  add(s->qyy[p], S.qyy, sizeof(float) * N);
  add(s->acc, S.acc, sizeof(float2) * N);
  add(s->drho, S.drho, sizeof(float) * N);
  add(s->id, S.id, sizeof(int) * N);
  add(s->cell, S.cell, sizeof(int) * N);
  add(s->img, S.img, sizeof(int2) * N);
  add(s->cell_start, S.cell_start, sizeof(int) * (C + 1));
  add(s->umax + (size_t)p * s->R * UMAX_SLOTS, S.umax, sizeof(unsigned) * s->R * UMAX_SLOTS);
  add(s->flags + 1, S.umax + s->R * UMAX_SLOTS, sizeof(unsigned));  // rebin request
  if (full) { s->err = "snapshot copy list too long"; return NEM_E_INVAL; }
  hipLaunchKernelGGL(k_copy_list, dim3(1024), dim3(256), 0, s->stream, cl);
  HIPCHK(hipGetLastError());
  S.parity = p;
  S.dt.resize(s->R);
  for (int r = 0; r < s->R; ++r) S.dt[r] = s->reps[r].dt;
  S.valid = true;
  return NEM_OK;
}

int restore_snapshot(nem_sim* s, int i) {
  auto& S = s->snap[i];
  if (!S.valid) return NEM_E_STATE;
  const size_t N = (size_t)s->ntot, C = (size_t)s->ncells;
  const int p = S.parity;
  CopyList cl;
  cl.n = 0;
  bool full = false;
  auto add = [&](const void* src, void* dst, size_t bytes) {
    if (cl.n < (int)(sizeof(cl.seg) / sizeof(cl.seg[0]))) cl.seg[cl.n++] = CopySeg{src, dst, (int64_t)bytes};
    else full = true;
  };
  add(S.off, s->off[p], sizeof(float2) * N);
  add(S.offlo, s->offlo, sizeof(float2) * N);
  add(S.u, s->u, sizeof(float2) * N);
  add(S.q, s->q[p], sizeof(float2) * N);
  add(S.qyy, s->qyy[p], sizeof(float) * N);
  add(S.acc, s->acc, sizeof(float2) * N);
  add(S.drho, s->drho, sizeof(float) * N);
  add(S.id, s->id, sizeof(int) * N);
  add(S.cell, s->cell, sizeof(int) * N);
  add(S.img, s->img, sizeof(int2) * N);
  add(S.cell_start, s->cell_start, sizeof(int) * (C + 1));
  add(S.umax, s->umax + (size_t)p * s->R * UMAX_SLOTS, sizeof(unsigned) * s->R * UMAX_SLOTS);
  // keep the sticky error bits (flags[0]), restore the rebin request (flags[1]);
  // the Verlet list is not part of the snapshot: rebuild it
  add(S.umax + s->R * UMAX_SLOTS, s->flags + 1, sizeof(unsigned));
  if (full) { s->err = "snapshot copy list too long"; return NEM_E_INVAL; }
  hipLaunchKernelGGL(k_copy_list, dim3(1024), dim3(256), 0, s->stream, cl);
  HIPCHK(hipGetLastError());
  launch_request_relist(s->flags, s->stream);
  s->parity = p;
  for (int r = 0; r < s->R; ++r) s->reps[r].dt = S.dt[r];
  int rc = upload_reps(s);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(s->stream));
  return NEM_OK;
}

// Scale every replica's dt by `factor` and re-predict the stored state.
static int scale_dt(nem_sim* s, float factor) {
  unsigned* um = s->umax + (size_t)s->parity * s->R * UMAX_SLOTS;
  HIPCHK(hipMemsetAsync(um, 0, sizeof(unsigned) * s->R * UMAX_SLOTS, s->stream));
  SortArgs a = sort_args(s, nullptr);
  hipLaunchKernelGGL(k_repredict, rep_grid(s), dim3(256), 0, s->stream, a, factor, um);
  HIPCHK(hipGetLastError());
  for (auto& R : s->reps) R.dt *= factor;
  return upload_reps(s);
}

static int check_flags(nem_sim* s) {
  unsigned f[2];
  int rc = read_flags(s, f);
  if (rc) return rc;
  return status_from_flags(s, f[0]);
}

}  // namespace nem_host

static int mlp_fail(nem_mlp* m, hipError_t e, const char* what) {
  m->err = std::string(what) + ": " + hipGetErrorString(e);
  return NEM_E_HIP;
}
#define MLPCHK(expr)                                      \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return mlp_fail(m, e_, #expr);  \
  } while (0)

static int mlp_ensure_idx(nem_mlp* m, int64_t B) {
  if (m->idx_cap >= B) return NEM_OK;
  if (m->idx) hipFree(m->idx);
  m->idx = nullptr;
  MLPCHK(hipMalloc((void**)&m->idx, sizeof(int64_t) * B));
  m->idx_cap = B;
  return NEM_OK;
}

static int mlp_ensure_partial(nem_mlp* m, int nw) {
  if (m->part_waves >= nw) return NEM_OK;
  if (m->partial) hipFree(m->partial);
  if (m->lossp) hipFree(m->lossp);
  m->partial = nullptr; m->lossp = nullptr;
  MLPCHK(hipMalloc((void**)&m->partial, sizeof(float) * (size_t)nw * mlp_nparam()));
  MLPCHK(hipMalloc((void**)&m->lossp, sizeof(float) * nw));
  m->part_waves = nw;
  return NEM_OK;
}

// Gradient of the mean loss over the index map m->idx[0..B) into m->g.
static int mlp_grad_batch(nem_mlp* m, const float* X, const float* T, int64_t B) {
  const int nw = mlp_backward_waves(B);
  int rc = mlp_ensure_partial(m, nw);
  if (rc) return rc;
  launch_mlp_backward(m->P, m->hnorm, X, T, m->idx, B, m->partial, m->lossp, nw, m->stream);
  launch_mlp_reduce(m->partial, nw, m->g, m->lossp, m->loss, m->stream);
  MLPCHK(hipGetLastError());
  return NEM_OK;
}

extern "C" {

int nem_mlp_nparams(void) { return mlp_nparam(); }

int nem_mlp_create(void* hip_stream, nem_mlp** out) {
  if (!out) return NEM_E_INVAL;
  nem_mlp* m = new nem_mlp();
  m->stream = (hipStream_t)hip_stream;
  const int np = mlp_nparam();
  bool ok = hipMalloc((void**)&m->P, sizeof(float) * np) == hipSuccess &&
            hipMalloc((void**)&m->m, sizeof(float) * np) == hipSuccess &&
            hipMalloc((void**)&m->v, sizeof(float) * np) == hipSuccess &&
            hipMalloc((void**)&m->g, sizeof(float) * np) == hipSuccess &&
            hipMalloc((void**)&m->norm, sizeof(float) * 34) == hipSuccess &&
            hipMalloc((void**)&m->loss, sizeof(float)) == hipSuccess &&
            hipMalloc((void**)&m->stats, sizeof(double) * 34) == hipSuccess;
  if (!ok) { nem_mlp_destroy(m); return NEM_E_NOMEM; }
  for (int i = 0; i < 12; ++i) { m->hnorm[i] = 0.0f; m->hnorm[12 + i] = 1.0f; }
  for (int i = 0; i < 5; ++i) { m->hnorm[24 + i] = 0.0f; m->hnorm[29 + i] = 1.0f; }
  hipMemsetAsync(m->P, 0, sizeof(float) * np, m->stream);
  hipMemsetAsync(m->m, 0, sizeof(float) * np, m->stream);
  hipMemsetAsync(m->v, 0, sizeof(float) * np, m->stream);
  hipMemcpyAsync(m->norm, m->hnorm, sizeof(m->hnorm), hipMemcpyHostToDevice, m->stream);
  if (hipStreamSynchronize(m->stream) != hipSuccess) { nem_mlp_destroy(m); return NEM_E_HIP; }
  *out = m;
  return NEM_OK;
}

int nem_mlp_set_weights(nem_mlp* m, const float* w) {
  if (!m || !w) return NEM_E_INVAL;
  const int np = mlp_nparam();
  MLPCHK(hipMemcpyAsync(m->P, w, sizeof(float) * np, hipMemcpyHostToDevice, m->stream));
  MLPCHK(hipMemsetAsync(m->m, 0, sizeof(float) * np, m->stream));
  MLPCHK(hipMemsetAsync(m->v, 0, sizeof(float) * np, m->stream));
  MLPCHK(hipStreamSynchronize(m->stream));
  m->adam_t = 0;
  return NEM_OK;
}

int nem_mlp_get_weights(nem_mlp* m, float* w) {
  if (!m || !w) return NEM_E_INVAL;
  MLPCHK(hipMemcpyAsync(w, m->P, sizeof(float) * mlp_nparam(), hipMemcpyDeviceToHost, m->stream));
  MLPCHK(hipStreamSynchronize(m->stream));
  return NEM_OK;
}

int nem_mlp_set_norm(nem_mlp* m, const float* norm) {
  if (!m || !norm) return NEM_E_INVAL;
  for (int i = 0; i < 34; ++i) m->hnorm[i] = norm[i];
  for (int i = 12; i < 24; ++i) if (!(m->hnorm[i] > 0)) m->hnorm[i] = 1.0f;
  for (int i = 29; i < 34; ++i) if (!(m->hnorm[i] > 0)) m->hnorm[i] = 1.0f;
  MLPCHK(hipMemcpyAsync(m->norm, m->hnorm, sizeof(m->hnorm), hipMemcpyHostToDevice, m->stream));
  MLPCHK(hipStreamSynchronize(m->stream));
  return NEM_OK;
}

int nem_mlp_get_norm(nem_mlp* m, float* norm) {
  if (!m || !norm) return NEM_E_INVAL;
  std::memcpy(norm, m->hnorm, sizeof(m->hnorm));
  return NEM_OK;
}

int nem_mlp_fit_norm(nem_mlp* m, const float* X, const float* T, int64_t n) {
  if (!m || !X || !T || n < 2) return NEM_E_INVAL;
  launch_mlp_stats(X, T, n, m->stats, m->stream);
  MLPCHK(hipGetLastError());
  double st[34];
  MLPCHK(hipMemcpyAsync(st, m->stats, sizeof(st), hipMemcpyDeviceToHost, m->stream));
  MLPCHK(hipStreamSynchronize(m->stream));
  float nm[34];
  for (int c = 0; c < 12; ++c) { nm[c] = (float)st[2 * c]; nm[12 + c] = (float)st[2 * c + 1]; }
  for (int c = 0; c < 5; ++c) { nm[24 + c] = (float)st[2 * (12 + c)]; nm[29 + c] = (float)st[2 * (12 + c) + 1]; }
  // constant inputs (zero spread) are passed through unscaled
  for (int i = 12; i < 24; ++i) if (!(nm[i] > 1e-30f)) nm[i] = 1.0f;
  for (int i = 29; i < 34; ++i) if (!(nm[i] > 1e-30f)) nm[i] = 1.0f;
  return nem_mlp_set_norm(m, nm);
}

int nem_mlp_forward(nem_mlp* m, const float* X, int64_t n, float* Y) {
  if (!m || !X || !Y || n < 1) return NEM_E_INVAL;
  launch_mlp_forward(m->P, m->hnorm, X, n, Y, nullptr, m->stream);
  MLPCHK(hipGetLastError());
  MLPCHK(hipStreamSynchronize(m->stream));
  return NEM_OK;
}

int nem_mlp_grad(nem_mlp* m, const float* X, const float* T, int64_t n, float* grad, double* loss) {
  if (!m || !X || !T || !grad || n < 1) return NEM_E_INVAL;
  int rc = mlp_ensure_idx(m, n);
  if (rc) return rc;
  launch_mlp_batch(m->idx, 0, n, n, 1, 0, m->stream);
  rc = mlp_grad_batch(m, X, T, n);
  if (rc) return rc;
  float l = 0.f;
  MLPCHK(hipMemcpyAsync(grad, m->g, sizeof(float) * mlp_nparam(), hipMemcpyDeviceToHost, m->stream));
  MLPCHK(hipMemcpyAsync(&l, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
  MLPCHK(hipStreamSynchronize(m->stream));
  if (loss) *loss = l;
  return NEM_OK;
}

int nem_mlp_train(nem_mlp* m, const float* X, const float* T, int64_t n, int32_t epochs, int32_t batch, double lr,
                  double* final_loss) {
  if (!m || !X || !T || n < 1 || epochs < 1 || batch < 32) return NEM_E_INVAL;
  const int64_t B = std::min<int64_t>(batch, n);
  int rc = mlp_ensure_idx(m, B);
  if (rc) return rc;
  // per-epoch shuffle: idx = (k * stride + offset) mod n with stride coprime to n
  auto gcd = [](int64_t a, int64_t b) { while (b) { int64_t t = a % b; a = b; b = t; } return a; };
  int64_t stride = (int64_t)(0.6180339887 * (double)n) | 1;
  while (gcd(stride, n) != 1) stride += 2;
  double last = 0.0;
  for (int e = 0; e < epochs; ++e) {
    const int64_t offset = (int64_t)((uint64_t)(e + 1) * 2654435761ull % (uint64_t)n);
    for (int64_t first = 0; first + B <= n; first += B) {
      launch_mlp_batch(m->idx, first, B, n, stride % n, offset, m->stream);
      rc = mlp_grad_batch(m, X, T, B);
      if (rc) return rc;
      ++m->adam_t;
      launch_mlp_adam(m->P, m->g, m->m, m->v, (float)lr, m->adam_t, m->stream);
    }
    MLPCHK(hipGetLastError());
  }
  float l = 0.f;
  MLPCHK(hipMemcpyAsync(&l, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
  MLPCHK(hipStreamSynchronize(m->stream));
  last = l;
  if (final_loss) *final_loss = last;
  return NEM_OK;
}

void nem_mlp_destroy(nem_mlp* m) {
  if (!m) return;
  if (m->stream) hipStreamSynchronize(m->stream);
  for (void* p : {(void*)m->P, (void*)m->m, (void*)m->v, (void*)m->g, (void*)m->norm, (void*)m->partial,
                  (void*)m->lossp, (void*)m->loss, (void*)m->idx, (void*)m->stats})
    if (p) hipFree(p);
  delete m;
}

int nem_mlp_eval(nem_mlp* m, const float* X, const float* T, int64_t n, double* rel_mse, double* max_norm) {
  if (!m || !X || n < 1 || (rel_mse && !T)) return NEM_E_INVAL;
  float* Y = nullptr;
  unsigned* mx = nullptr;
  MLPCHK(hipMalloc((void**)&Y, sizeof(float) * 5 * (size_t)n));
  if (hipMalloc((void**)&mx, sizeof(unsigned)) != hipSuccess) { hipFree(Y); m->err = "hipMalloc (max norm)"; return NEM_E_HIP; }
  hipError_t e = hipMemsetAsync(mx, 0, sizeof(unsigned), m->stream);
  if (e == hipSuccess) {
    launch_mlp_forward(m->P, m->hnorm, X, n, Y, mx, m->stream);
    if (rel_mse) hipLaunchKernelGGL(k_eval_stats, dim3(5), dim3(256), 0, m->stream, T, (const float*)Y, n, m->stats);
    e = hipGetLastError();
  }
  double st[15];
  unsigned hm = 0;
  if (e == hipSuccess && rel_mse) e = hipMemcpyAsync(st, m->stats, sizeof(st), hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&hm, mx, sizeof(hm), hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  hipFree(Y);
  hipFree(mx);
  if (e != hipSuccess) return mlp_fail(m, e, "nem_mlp_eval");
  if (rel_mse)
    for (int o = 0; o < 5; ++o) rel_mse[o] = st[3 * o + 1] > 0.0 ? st[3 * o + 2] / st[3 * o + 1] : NAN;
  if (max_norm) {
    float f;
    std::memcpy(&f, &hm, sizeof(f));
    *max_norm = f;
  }
  return NEM_OK;
}

int nem_mlp_mask_outputs(nem_mlp* m, const int32_t* off) {
  if (!m || !off) return NEM_E_INVAL;
  const int np = mlp_nparam();
  std::vector<float> w(np);
  int rc = nem_mlp_get_weights(m, w.data());
  if (rc) return rc;
  // flat layout: W1 (12 x 64), b1, W2 (64 x 64), b2, W3 (64 x 5, input-major), b3
  const int off_w3 = 12 * 64 + 64 + 64 * 64 + 64, off_b3 = off_w3 + 64 * 5;
  float nm[34];
  std::memcpy(nm, m->hnorm, sizeof(nm));
  for (int o = 0; o < 5; ++o) {
    if (!off[o]) continue;
    for (int i = 0; i < 64; ++i) w[off_w3 + i * 5 + o] = 0.0f;
    w[off_b3 + o] = 0.0f;
    nm[24 + o] = 0.0f;   // output mean: the component is exactly zero
  }
  rc = nem_mlp_set_weights(m, w.data());
  if (rc) return rc;
  return nem_mlp_set_norm(m, nm);
}

// Training samples of all particles into X (ntot x 12) and T (ntot x 5).
static int samples_into(nem_sim* s, int32_t mult, float* X, float* T);

int nem_samples(nem_sim* s, int32_t mult, float* X, float* T) {
  if (!s || mult < 2 || !X || !T) return NEM_E_INVAL;
  return samples_into(s, mult, X, T);
}

int nem_samples_rows(nem_sim* s, int32_t mult, const int64_t* rows, int64_t nrows, float* X, float* T) {
  if (!s || mult < 2 || !rows || nrows < 1 || !X || !T) return NEM_E_INVAL;
  const size_t N = (size_t)s->ntot;
  float *xa = nullptr, *ta = nullptr;
  int64_t* dr = nullptr;
  int rc = NEM_OK;
  auto chk = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && rc == NEM_OK) rc = hip_fail(s, e, what);
  };
  chk(hipMalloc((void**)&xa, sizeof(float) * 12 * N), "hipMalloc (samples)");
  chk(hipMalloc((void**)&ta, sizeof(float) * 5 * N), "hipMalloc (samples)");
  chk(hipMalloc((void**)&dr, sizeof(int64_t) * (size_t)nrows), "hipMalloc (rows)");
  if (!rc) chk(hipMemcpyAsync(dr, rows, sizeof(int64_t) * (size_t)nrows, hipMemcpyHostToDevice, s->stream), "rows");
  if (!rc) rc = samples_into(s, mult, xa, ta);
  if (!rc) {
    hipLaunchKernelGGL(k_gather_rows, dim3(grid_for(nrows)), dim3(256), 0, s->stream, (const float*)xa,
                       (const int64_t*)dr, nrows, 12, (int64_t)N, X, s->flags);
    hipLaunchKernelGGL(k_gather_rows, dim3(grid_for(nrows)), dim3(256), 0, s->stream, (const float*)ta,
                       (const int64_t*)dr, nrows, 5, (int64_t)N, T, s->flags);
    chk(hipGetLastError(), "k_gather_rows");
  }
  hipStreamSynchronize(s->stream);
  hipFree(xa);
  hipFree(ta);
  hipFree(dr);
  if (rc) return rc;
  return check_flags(s);
}

static int samples_into(nem_sim* s, int32_t mult, float* X, float* T) {
  if (s->hp[0].q3d) { s->err = "the learned corrector covers the 2x2 Q only"; return NEM_E_INVAL; }
  for (int r = 0; r < s->R; ++r)
    if (!s->has_state[r]) return NEM_E_STATE;
  int rc = take_snapshot(s);
  if (rc) return rc;
  float *coarse = nullptr, *xs = nullptr;
  const hipError_t e1 = hipMalloc((void**)&coarse, sizeof(float) * 5 * (size_t)s->ntot);
  const hipError_t e2 = hipMalloc((void**)&xs, sizeof(float) * 12 * (size_t)s->ntot);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    hipFree(coarse);
    hipFree(xs);
    return hip_fail(s, e1 != hipSuccess ? e1 : e2, "hipMalloc (sample buffers)");
  }
  // one step of mult*dt with the inputs captured (storage order), then put
  // them in original particle order
  rc = scale_dt(s, (float)mult);
  if (!rc) {
    s->feat = xs;
    rc = run_steps(s, 1);
    s->feat = nullptr;
  }
  if (!rc) {
    SortArgs a = sort_args(s, nullptr);
    hipLaunchKernelGGL(k_rows_by_id, dim3(grid_for(s->ntot)), dim3(256), 0, s->stream, a, (const float*)xs, X, 12);
    hipLaunchKernelGGL(k_export_qu, dim3(grid_for(s->ntot)), dim3(256), 0, s->stream, a, coarse);
  }
  // mult steps of dt from the same state
  if (!rc) rc = restore_snapshot(s);
  if (!rc) rc = run_steps(s, mult);
  if (!rc) {
    SortArgs a = sort_args(s, nullptr);
    hipLaunchKernelGGL(k_export_qu, dim3(grid_for(s->ntot)), dim3(256), 0, s->stream, a, T);
    hipLaunchKernelGGL(k_sub, dim3(grid_for(5 * (int64_t)s->ntot)), dim3(256), 0, s->stream, T, coarse,
                       5 * (int64_t)s->ntot);
  }
  if (!rc) rc = restore_snapshot(s);
  hipStreamSynchronize(s->stream);
  hipFree(coarse);
  hipFree(xs);
  if (rc) return rc;
  return check_flags(s);
}

int nem_step_learned(nem_sim* s, nem_mlp* m, int64_t n_macro, int32_t mult, double tau, int64_t* n_fallback,
                     double* max_norm) {
  if (!s || !m || n_macro < 0 || mult < 2 || !(tau > 0)) return NEM_E_INVAL;
  if (s->hp[0].q3d) { s->err = "the learned corrector covers the 2x2 Q only"; return NEM_E_INVAL; }
  for (int r = 0; r < s->R; ++r)
    if (!s->has_state[r]) return NEM_E_STATE;
  const size_t N = (size_t)s->ntot;
  const float tauf = (float)tau;
  unsigned tau_bits;
  std::memcpy(&tau_bits, &tauf, sizeof(tau_bits));
  float *X = nullptr, *Y = nullptr;
  unsigned *mx = nullptr, *hmx = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  int rc = NEM_OK;
  auto chk = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && rc == NEM_OK) rc = hip_fail(s, e, what);
    return e == hipSuccess;
  };
  chk(hipMalloc((void**)&X, sizeof(float) * 12 * N), "hipMalloc (inputs)");
  chk(hipMalloc((void**)&Y, sizeof(float) * 5 * N), "hipMalloc (corrections)");
  chk(hipMalloc((void**)&mx, sizeof(unsigned) * 2), "hipMalloc (max norm)");
  chk(hipHostMalloc((void**)&hmx, sizeof(unsigned) * 2, hipHostMallocMapped | hipHostMallocCoherent),
      "hipHostMalloc (max norm)");
  unsigned* dmx = nullptr;   // the device's address of hmx
  if (hmx) chk(hipHostGetDevicePointer((void**)&dmx, hmx, 0), "hipHostGetDevicePointer");
  for (auto& e : ev) chk(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
  // One macro step, enqueued without waiting: snapshot, a step of mult*dt with
  // the inputs captured, inference, and the correction (skipped on the device
  // when the largest correction norm exceeds tau), which also stores that norm
  // in pinned host memory for the host's fallback decision.
  auto enqueue = [&](int64_t k) -> int {
    const int b = (int)(k & 1);
    int e = take_snapshot(s, b);
    if (e) return e;
    s->feat = X;
    e = run_steps(s, 1);
    s->feat = nullptr;
    if (e) return e;
    unsigned* um = s->umax + (size_t)s->parity * s->R * UMAX_SLOTS;
    hipLaunchKernelGGL(k_learn_clear, dim3(1), dim3(256), 0, s->stream, mx + b, um, s->R * UMAX_SLOTS);
    launch_mlp_forward(m->P, m->hnorm, X, (int64_t)N, Y, mx + b, s->stream);
    SortArgs a = sort_args(s, nullptr);
    hipLaunchKernelGGL(k_correct, rep_grid(s), dim3(256), 0, s->stream, a, (const float*)Y, um,
                       (const unsigned*)(mx + b), tau_bits, dmx + b);
    if (!chk(hipGetLastError(), "k_correct")) return rc;
    if (!chk(hipEventRecord(ev[b], s->stream), "hipEventRecord")) return rc;
    return rc;
  };
  int64_t nfb = 0;
  float worst = 0.0f;
  if (!rc) rc = scale_dt(s, (float)mult);
  // Macro step k+1 is enqueued before the host looks at step k's norm, so the
  // device never waits for the host. If step k needs the fallback, step k+1
  // (speculative) is discarded with it: restore the state before step k,
  // replay it as mult steps of dt, and enqueue step k+1 again.
  if (!rc && n_macro > 0) rc = enqueue(0);
  for (int64_t k = 0; k < n_macro && !rc; ++k) {
    if (k + 1 < n_macro) rc = enqueue(k + 1);
    if (rc) break;
    if (!chk(hipEventSynchronize(ev[k & 1]), "hipEventSynchronize")) break;
    float fm;
    std::memcpy(&fm, &hmx[k & 1], sizeof(fm));
    worst = std::max(worst, fm);
    if (!(fm <= tauf)) {
      ++nfb;
      if (!chk(hipStreamSynchronize(s->stream), "hipStreamSynchronize")) break;
      rc = restore_snapshot(s, (int)(k & 1));
      if (!rc) rc = scale_dt(s, 1.0f / (float)mult);
      if (!rc) rc = run_steps(s, mult);
      if (!rc) rc = scale_dt(s, (float)mult);
      if (!rc && k + 1 < n_macro) rc = enqueue(k + 1);
    }
  }
  if (!rc) rc = scale_dt(s, 1.0f / (float)mult);
  hipStreamSynchronize(s->stream);
  for (auto& e : ev)
    if (e) hipEventDestroy(e);
  hipFree(X); hipFree(Y); hipFree(mx);
  if (hmx) hipHostFree(hmx);
  if (n_fallback) *n_fallback = nfb;
  if (max_norm) *max_norm = worst;
  if (rc) return rc;
  return check_flags(s);
}

}  // extern "C"
