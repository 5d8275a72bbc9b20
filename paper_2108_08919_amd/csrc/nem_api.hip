// nem_api.hip -- host runtime and C ABI of the nematic SPH library.
//
// The runtime validates parameters, lays out one device arena (caller-owned or
// allocated here), builds the per-replica tables and the tile work list, and
// enqueues the per-step kernel sequence on the caller's stream:
//   rebin (5 kernels, each returns at once unless a rebin was requested),
//   step-begin, pass A, pass B, pass C, pass D.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/nematic_sph.h"
#include "nem_dev.h"
#include "nem_sim.h"


using namespace nem;
using namespace nem_host;


// Scratch of the entry points that allocate nothing (nem_defects_noalloc): the
// M x M deposit grid (4 fields, FP64) for M <= NEM_NOALLOC_MAX_GRID, then two
// 64-bit defect counters. One copy per GPU for the life of the process; every
// call on a GPU shares it, so calls that overlap on one GPU race.
constexpr size_t NOALLOC_GRID_BYTES = sizeof(double) * 4 * (size_t)NEM_NOALLOC_MAX_GRID * NEM_NOALLOC_MAX_GRID;
constexpr size_t NOALLOC_BYTES = NOALLOC_GRID_BYTES + 256;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// Clears n 64-bit counters (a kernel, so that the call holds no memset node if
// a caller captures it).
__global__ void k_clear_u64(unsigned long long* p, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0ull;
}

namespace nem_host {

constexpr size_t ALIGN = 256;

// Device address of `scratch` on device dev, looked up once per device with
// that device current (each GPU holds its own copy at its own address).
// Returns nullptr when the lookup fails.
void* scratch_address(int dev, hipError_t* err) {
  static std::mutex mu;
  static void* addr[256] = {nullptr};
  std::lock_guard<std::mutex> lock(mu);
  *err = hipSuccess;
  if (dev < 0 || dev >= 256) { *err = hipErrorInvalidDevice; return nullptr; }
  if (!addr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) { *err = e; return nullptr; }
    addr[dev] = ptr;
  }
  return addr[dev];
}

struct Layout {
  size_t total = 0;
  size_t put(size_t bytes) {
    size_t o = (total + ALIGN - 1) / ALIGN * ALIGN;
    total = o + bytes;
    return o;
  }
};

// support radius of the smoothing kernel in units of h
double kappa(const nem_params& p) { return p.kernel == 1 ? 2.0 : 3.0; }

int cells_per_side(const nem_params& p) { return (int)std::floor(p.L / (kappa(p) * p.h + p.skin)); }

int check_params(const nem_params& p, int64_t n, std::string& why) {
  auto bad = [&](const char* m) { why = m; return NEM_E_INVAL; };
  if (!(p.L > 0) || !(p.h > 0) || !(p.dx > 0) || !(p.rho0 > 0) || !(p.dt > 0)) return bad("L, h, dx, rho0 and dt must be positive");
  if (!(p.skin >= 0)) return bad("skin must be >= 0");
  if (!(p.gamma_eos > 0)) return bad("gamma_eos must be positive");
  if (n < 1 || n > (int64_t)1 << 30) return bad("particle count out of range");
  if (p.kernel != 0 && p.kernel != 1) return bad("kernel must be 0 (quintic spline) or 1 (Wendland C2)");
  if (p.integrator != 0 && p.integrator != 1) return bad("integrator must be 0 (kick-drift-kick) or 1 (midpoint)");
  if (p.q3d != 0 && p.q3d != 1) return bad("q3d must be 0 (2x2 Q) or 1 (quasi-2D 3x3 Q)");
  if (p.q3d == 1 && (p.form != 0 || p.elastic != 0)) return bad("the quasi-2D Q needs form 0 and elastic 0");
  if (cells_per_side(p) < 3) return bad("box side must hold three cells of side >= kappa h + skin");
  if (p.form != 0 && p.form != 1) return bad("form must be 0 or 1");
  if (p.elastic != 0 && p.elastic != 1) return bad("elastic must be 0 or 1");
  if (p.form == 1 && p.elastic == 1) return bad("the conservative form has no elastic lambda terms on the GPU");
  for (double v : {p.eta, p.Gamma, p.lam, p.A, p.B, p.C, p.K, p.zeta, p.beta, p.c0_factor})
    if (!std::isfinite(v)) return bad("non-finite parameter");
  return NEM_OK;
}

int tiles_for(int nc, int T) { return (nc + T - 1) / T; }

RepDev make_rep(const nem_params& p, int nc, int cell_base, int part_base, int n, int T, int tile_base) {
  RepDev R;
  std::memset(&R, 0, sizeof(R));
  R.nc = nc; R.cell_base = cell_base; R.part_base = part_base; R.n = n;
  R.tiles_x = tiles_for(nc, T); R.tiles_y = tiles_for(nc, T); R.tile_base = tile_base; R.form = p.form;
  const double csd = p.L / nc;
  R.csd = csd; R.Ld = p.L;
  R.cs = (float)csd; R.cs_lo = (float)(csd - (double)R.cs);
  R.h = (float)p.h; R.hinv = (float)(1.0 / p.h);
  const double rs = kappa(p) * p.h;  // support radius
  R.R2 = (float)(rs * rs);
  R.kern = p.kernel;
  R.integ = p.integrator;
  R.q3d = p.q3d;
  if (p.kernel == 1) {
    const double a2 = 7.0 / (4.0 * M_PI * p.h * p.h);
    R.a2 = (float)a2; R.W0 = (float)a2; R.dWc = (float)(-5.0 * a2 / (p.h * p.h));
  } else {
    const double a2 = 7.0 / (478.0 * M_PI * p.h * p.h);
    R.a2 = (float)a2; R.W0 = (float)(66.0 * a2); R.dWc = (float)(-5.0 * a2 / p.h);
  }
  R.skin_half = (float)(0.5 * p.skin);
  R.rho0 = (float)p.rho0; R.eta = (float)p.eta; R.Gamma = (float)p.Gamma; R.lam = (float)p.lam;
  R.A = (float)p.A; R.B = (float)p.B; R.C = (float)p.C; R.K = (float)p.K; R.zeta = (float)p.zeta;
  R.dt = (float)p.dt; R.gamma_eos = (float)p.gamma_eos; R.beta = (float)p.beta;
  R.c0_factor = (float)p.c0_factor; R.mass = (float)(p.rho0 * p.dx * p.dx); R.inv_rho0 = (float)(1.0 / p.rho0);
  R.elastic = p.elastic; R.apd = p.apd;
  // Verlet skin: 3h + delta stays below 4 dx for h = 1.3 dx, so the list leaves
  // out the lattice's ring at 4 dx that a wider skin would carry every step
  const double delta = 0.075 * p.h;
  R.R2v = (float)((rs + delta) * (rs + delta));
  R.disp2 = (float)((0.45 * delta) * (0.45 * delta));
  return R;
}

// Offsets of every buffer for given sizes (shared by nem_arena_bytes and carve()).
struct Offs {
  size_t reps, work, cell_start, count, cursor, perm;
  size_t t_key, t_off, t_lo, t_u, t_q, t_drho, t_acc, t_id, t_img, t_qyy;
  size_t off0, off1, offlo, u, q0, q1, drho, acc, id, cell, img, qyy0, qyy1;
  size_t V, bk, dh, apart, uv, pi, P, drhat, flags, umax, stage, red, nl, ncnt, fe, vl, vcnt, off_build;
  size_t total;
};

Offs layout(int R, int64_t ntot, int64_t ncells, int64_t work_cap, int64_t stage_n) {
  Layout L;
  Offs o;
  const size_t N = (size_t)ntot, C = (size_t)ncells;
  o.reps = L.put(sizeof(RepDev) * R);
  o.work = L.put(sizeof(int) * 2 * (size_t)work_cap);
  o.cell_start = L.put(sizeof(int) * (C + 1));
  o.count = L.put(sizeof(int) * C);
  o.cursor = L.put(sizeof(int) * C);
  o.perm = L.put(sizeof(int) * N);
  o.t_key = L.put(sizeof(int) * N);
  o.t_off = L.put(sizeof(float2) * N);
  o.t_lo = L.put(sizeof(float2) * N);
  o.t_u = L.put(sizeof(float2) * N);
  o.t_q = L.put(sizeof(float2) * N);
  o.t_drho = L.put(sizeof(float) * N);
  o.t_acc = L.put(sizeof(float2) * N);
  o.t_id = L.put(sizeof(int) * N);
  o.t_img = L.put(sizeof(int2) * N);
  o.t_qyy = L.put(sizeof(float) * N);
  o.off0 = L.put(sizeof(float2) * N);
  o.off1 = L.put(sizeof(float2) * N);
  o.offlo = L.put(sizeof(float2) * N);
  o.u = L.put(sizeof(float2) * N);
  o.q0 = L.put(sizeof(float2) * N);
  o.q1 = L.put(sizeof(float2) * N);
  o.drho = L.put(sizeof(float) * N);
  o.acc = L.put(sizeof(float2) * N);
  o.id = L.put(sizeof(int) * N);
  o.cell = L.put(sizeof(int) * N);
  o.img = L.put(sizeof(int2) * N);
  o.qyy0 = L.put(sizeof(float) * N);
  o.qyy1 = L.put(sizeof(float) * N);
  o.V = L.put(sizeof(float) * N);
  o.bk = L.put(sizeof(float4) * N);
  o.dh = L.put(sizeof(float) * N);
  o.apart = L.put(sizeof(float2) * N);
  o.uv = L.put(sizeof(float) * N);
  o.pi = L.put(sizeof(float2) * N);
  o.P = L.put(sizeof(float) * N);
  o.drhat = L.put(sizeof(float) * N);
  o.flags = L.put(sizeof(unsigned) * 4);
  o.umax = L.put(sizeof(unsigned) * 2 * R * UMAX_SLOTS);
  o.nl = L.put(sizeof(uint32_t) * (KMAX / 2) * N);
  o.ncnt = L.put(sizeof(int) * N);
  o.fe = L.put(sizeof(double) * 2 * N);
  o.vl = L.put(sizeof(uint32_t) * (KMAX / 2) * N);
  o.vcnt = L.put(sizeof(int) * N);
  o.off_build = L.put(sizeof(float2) * N);
  o.stage = L.put(sizeof(double) * 9 * (size_t)stage_n);
  o.red = L.put(sizeof(double) * 64 * 1024);
  o.total = L.total + ALIGN;
  return o;
}

struct Sizes { int64_t ntot = 0, ncells = 0, work_cap = 0, stage_n = 0; };

int sizes_for(const nem_params* p, const int64_t* n, int R, Sizes& s, std::string& why) {
  if (R < 1 || R > 4096) { why = "replica count out of range"; return NEM_E_INVAL; }
  for (int r = 0; r < R; ++r) {
    int rc = check_params(p[r], n[r], why);
    if (rc) return rc;
    // one launch per pass serves every replica: the compiled variant is shared
    if (p[r].form != p[0].form || p[r].elastic != p[0].elastic || p[r].kernel != p[0].kernel ||
        p[r].q3d != p[0].q3d || p[r].integrator != p[0].integrator) {
      why = "replicas of one simulation must share form, elastic, kernel, q3d and integrator";
      return NEM_E_INVAL;
    }
    const int nc = cells_per_side(p[r]);
    s.ntot += n[r];
    s.ncells += (int64_t)nc * nc;
    const int64_t t4 = (int64_t)tiles_for(nc, 4);
    s.work_cap += t4 * t4;
    s.stage_n = std::max<int64_t>(s.stage_n, n[r]);
  }
  if (s.ntot >= ((int64_t)1 << 31) - 1 || s.ncells >= ((int64_t)1 << 31) - 2) {
    why = "more than 2^31 particles or cells";
    return NEM_E_INVAL;
  }
  return NEM_OK;
}

SortArgs sort_args(nem_sim* s, const unsigned* gate) {
  SortArgs a;
  a.reps = s->d_reps; a.R = s->R; a.ncells = s->ncells; a.ntot = s->ntot;
  a.cell_start = s->cell_start; a.count = s->count; a.cursor = s->cursor; a.perm = s->perm;
  a.t_key = s->t_key; a.t_off = s->t_off; a.t_lo = s->t_lo; a.t_u = s->t_u; a.t_q = s->t_q;
  a.t_drho = s->t_drho; a.t_acc = s->t_acc; a.t_id = s->t_id; a.t_img = s->t_img; a.t_qyy = s->t_qyy;
  a.off = s->off[s->parity]; a.offlo = s->offlo; a.u = s->u; a.q = s->q[s->parity];
  a.drho = s->drho; a.acc = s->acc; a.id = s->id; a.cell = s->cell; a.img = s->img;
  a.qyy = s->qyy[s->parity];
  a.flags = s->flags; a.gate = gate; a.off_build = s->off_build;
  return a;
}

StepArgs step_args(nem_sim* s) {
  StepArgs a;
  const int c = s->parity, x = 1 - s->parity;
  a.reps = s->d_reps; a.work = s->d_work; a.nwork = s->nwork; a.T = s->T; a.lpp = s->LPP; a.grid = s->persist;
  a.cell_start = s->cell_start; a.ncells = s->ncells; a.ntot = s->ntot;
  a.off_cur = s->off[c]; a.off_nxt = s->off[x]; a.offlo = s->offlo; a.u = s->u;
  a.q_cur = s->q[c]; a.q_nxt = s->q[x]; a.acc = s->acc; a.drho = s->drho; a.cell = s->cell;
  a.qyy_cur = s->qyy[c]; a.qyy_nxt = s->qyy[x];
  a.V = s->V; a.bk = s->bk; a.dh = s->dh; a.apart = s->apart; a.uv = s->uv; a.pi = s->pi;
  a.P = s->P; a.drhat = s->drhat; a.flags = s->flags;
  a.umax_cur = s->umax + (size_t)c * s->R * UMAX_SLOTS; a.umax_nxt = s->umax + (size_t)x * s->R * UMAX_SLOTS;
  a.nl = s->nl; a.ncnt = s->ncnt;
  a.feat = s->feat; a.id = s->id;
  a.vl = s->vl; a.vcnt = s->vcnt; a.off_build = s->off_build;
  return a;
}

int build_work(nem_sim* s) {
  std::vector<int> w;
  int tile_base = 0;
  for (int r = 0; r < s->R; ++r) {
    RepDev& R = s->reps[r];
    R.tiles_x = tiles_for(R.nc, s->T);
    R.tiles_y = tiles_for(R.nc, s->T);
    R.tile_base = tile_base;
    for (int t = 0; t < R.tiles_x * R.tiles_y; ++t) { w.push_back(r); w.push_back(t); }
    tile_base += R.tiles_x * R.tiles_y;
  }
  if ((int)(w.size() / 2) > s->work_cap) { s->err = "work list larger than its buffer"; return NEM_E_INVAL; }
  s->nwork = (int)(w.size() / 2);
  {
    // Full tiles first, the ragged edge tiles of boxes whose cell count is not
    // a multiple of T (fewer cells, less work) last, so that the end of each
    // launch runs the short work items (1% on the 32-replica ensemble). A
    // stable sort: an even box keeps its row-major order. The order of work
    // items does not change any result.
    std::vector<int> idx(s->nwork), cells(s->nwork);
    for (int k = 0; k < s->nwork; ++k) {
      const RepDev& R = s->reps[w[2 * k]];
      const int t = w[2 * k + 1], tx = t % R.tiles_x, ty = t / R.tiles_x;
      cells[k] = std::min(s->T, R.nc - tx * s->T) * std::min(s->T, R.nc - ty * s->T);
      idx[k] = k;
    }
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return cells[a] > cells[b]; });
    std::vector<int> v(w.size());
    for (int k = 0; k < s->nwork; ++k) { v[2 * k] = w[2 * idx[k]]; v[2 * k + 1] = w[2 * idx[k] + 1]; }
    w.swap(v);
  }
  HIPCHK(hipMemcpyAsync(s->d_work, w.data(), w.size() * sizeof(int), hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipMemcpyAsync(s->d_reps, s->reps.data(), sizeof(RepDev) * s->R, hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  return NEM_OK;
}

int read_flags(nem_sim* s, unsigned* f) {
  HIPCHK(hipMemcpyAsync(f, s->flags, sizeof(unsigned) * 2, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  return NEM_OK;
}

int status_from_flags(nem_sim* s, unsigned f) {
  if (f & ERR_RANGE) { s->err = "device index outside its buffer (access skipped)"; return NEM_E_RANGE; }
  if (f & ERR_OVERFLOW) {
    s->err = "a tile or cell holds more particles than the LDS staging capacity, or a particle has more than 96 entries in its neighbour list";
    return NEM_E_OVERFLOW;
  }
  if (f & ERR_NUMERIC) { s->err = "non-finite value in the state"; return NEM_E_NUMERIC; }
  if (f & ERR_SINGULAR) { s->err = "singular correction tensor (B = I used)"; return NEM_E_SINGULAR; }
  return NEM_OK;
}

hipEvent_t take_event(nem_sim* s) {
  if (!s->ev_free.empty()) { hipEvent_t e = s->ev_free.back(); s->ev_free.pop_back(); return e; }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Accumulate the durations of all recorded launches (synchronises the stream).
void collect_times(nem_sim* s) {
  if (s->ev_pend.empty()) return;
  hipStreamSynchronize(s->stream);
  for (auto& r : s->ev_pend) {
    float ms = 0.f;
    if (r.a && r.b && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      s->pass_ms[r.pass] += ms;
      s->pass_n[r.pass] += 1;
    }
    if (r.a) s->ev_free.push_back(r.a);
    if (r.b) s->ev_free.push_back(r.b);
  }
  s->ev_pend.clear();
}

// HIP events around one launch group on the library's stream (timing mode).
struct Timed {
  nem_sim* s;
  nem_sim::EvRec rec{0, nullptr, nullptr};
  Timed(nem_sim* s_, int p) : s(s_) {
    if (!s->timing) return;
    rec.pass = p;
    rec.a = take_event(s);
    if (rec.a) hipEventRecord(rec.a, s->stream);
  }
  ~Timed() {
    if (!s->timing) return;
    rec.b = take_event(s);
    if (rec.b) hipEventRecord(rec.b, s->stream);
    s->ev_pend.push_back(rec);
    if (s->ev_pend.size() > 8192) collect_times(s);
  }
};

PassCfg pass_cfg(const nem_sim* s) {
  return PassCfg{s->T, s->LPP, s->COMP, s->hp[0].form, s->hp[0].elastic, s->hp[0].kernel, s->hp[0].q3d,
                 s->hp[0].integrator};
}

// The start of a step on stream st: the rebin kernels (they return at once
// unless a rebin was requested), step-begin (decides whether pass A rebuilds
// the Verlet list) and pass A (Verlet build or walk: the list every pass walks,
// and the volumes).
int enqueue_prologue(nem_sim* s, hipStream_t st) {
  {
    Timed t(s, 0);
    SortArgs a = sort_args(s, s->flags + 1);
    launch_rebin_key(a, st);
    launch_sort_tail(a, 0, s->ntot, 0, s->ncells, 0, st);
  }
  StepArgs a = step_args(s);
  launch_step_begin(s->flags, a.umax_nxt, s->R, st);
  Timed t(s, 1);
  if (!launch_pass_a_verlet(pass_cfg(s), a, st)) { s->err = "unsupported kernel configuration"; return NEM_E_INVAL; }
  return NEM_OK;
}

// Enqueue one step (prologue, then passes B-D) on stream st for the current
// parity.
int enqueue_step(nem_sim* s, hipStream_t st) {
  int rc = enqueue_prologue(s, st);
  if (rc) return rc;
  const PassCfg cfg = pass_cfg(s);
  StepArgs a = step_args(s);
  for (int pass = 2; pass <= 4; ++pass) {
    Timed t(s, pass);
    if (!launch_pass(pass, cfg, a, st)) { s->err = "unsupported kernel configuration"; return NEM_E_INVAL; }
  }
  HIPCHK(hipGetLastError());
  return NEM_OK;
}

void drop_graphs(nem_sim* s) {
  for (auto& g : s->graph)
    if (g) { hipGraphExecDestroy(g); g = nullptr; }
}

// Capture graph_steps consecutive steps starting at each parity into a graph
// (once per configuration). No memset nodes: every clear is a kernel.
int capture_graphs(nem_sim* s) {
  if (!s->cap_stream) HIPCHK(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
  const int saved = s->parity;
  for (int par = 0; par < 2; ++par) {
    s->parity = par;
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    const int timing = s->timing;
    s->timing = 0;
    int rc = NEM_OK;
    for (int k = 0; k < s->graph_steps && !rc; ++k) {
      rc = enqueue_step(s, s->cap_stream);
      s->parity ^= 1;
    }
    s->timing = timing;
    hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
    if (rc) { if (g) hipGraphDestroy(g); s->parity = saved; return rc; }
    if (e != hipSuccess) { s->parity = saved; return hip_fail(s, e, "hipStreamEndCapture"); }
    e = hipGraphInstantiate(&s->graph[par], g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) { s->parity = saved; return hip_fail(s, e, "hipGraphInstantiate"); }
  }
  s->parity = saved;
  return NEM_OK;
}

void free_grid(nem_sim* s) {
  for (void* p : {(void*)s->g_grid, (void*)s->g_z, (void*)s->g_w, (void*)s->g_part, (void*)s->g_E, (void*)s->g_cnt})
    if (p) hipFree(p);
  s->g_grid = nullptr; s->g_z = nullptr; s->g_w = nullptr; s->g_part = nullptr; s->g_E = nullptr;
  s->g_cnt = nullptr; s->gM = 0; s->gbins = 0;
}

int shell_count(int M) { return (int)std::floor(std::sqrt(2.0) * (M / 2) + 0.5) + 1; }

int ensure_grid(nem_sim* s, int M) {
  if (s->gM == M) return NEM_OK;
  free_grid(s);
  const size_t MM = (size_t)M * M;
  const int nb = shell_count(M);
  HIPCHK(hipMalloc((void**)&s->g_grid, sizeof(double) * 4 * MM));
  HIPCHK(hipMalloc((void**)&s->g_z, sizeof(double2) * MM));
  HIPCHK(hipMalloc((void**)&s->g_w, sizeof(double2) * MM));
  HIPCHK(hipMalloc((void**)&s->g_part, sizeof(double) * (size_t)M * nb));
  HIPCHK(hipMalloc((void**)&s->g_E, sizeof(double) * nb));
  HIPCHK(hipMalloc((void**)&s->g_cnt, sizeof(unsigned long long) * 2));
  s->gM = M;
  s->gbins = nb;
  return NEM_OK;
}

// Shepard deposit of replica r onto the M x M grid buffer (device).
int deposit_grid(nem_sim* s, int r, int M) {
  if (r < 0 || r >= s->R || M < 8 || M > 2048 || (M & (M - 1))) { s->err = "grid side must be a power of two in [8, 2048]"; return NEM_E_INVAL; }
  if (!s->has_state[r]) return NEM_E_STATE;
  int rc = ensure_grid(s, M);
  if (rc) return rc;
  SortArgs a = sort_args(s, nullptr);
  launch_int_offsets(a, s->t_off, s->stream);
  StepArgs sa = step_args(s);
  sa.off_cur = s->t_off;
  launch_deposit(s->T, s->hp[r].kernel, sa, r, M, s->g_grid, s->stream);
  HIPCHK(hipGetLastError());
  return NEM_OK;
}

int run_steps(nem_sim* s, int64_t nsteps) {
  const bool graph = s->use_graph && !s->timing && !s->feat;
  if (graph && !s->graph[0]) {
    int rc = capture_graphs(s);
    if (rc) { drop_graphs(s); return rc; }
  }
  int64_t it = 0;
  if (graph) {
    // whole chunks of graph_steps steps; the parity after a chunk flips only
    // when the chunk length is odd
    for (; it + s->graph_steps <= nsteps; it += s->graph_steps) {
      HIPCHK(hipGraphLaunch(s->graph[s->parity], s->stream));
      if (s->graph_steps & 1) s->parity ^= 1;
    }
  }
  for (; it < nsteps; ++it) {
    int rc = enqueue_step(s, s->stream);
    if (rc) return rc;
    s->parity ^= 1;
  }
  return NEM_OK;
}

int upload_reps(nem_sim* s) {
  HIPCHK(hipMemcpyAsync(s->d_reps, s->reps.data(), sizeof(RepDev) * s->R, hipMemcpyHostToDevice, s->stream));
  return NEM_OK;
}

}  // namespace nem_host

extern "C" {

int nem_version(void) { return 200; }

const char* nem_strerror(int code) {
  switch (code) {
    case NEM_OK: return "ok";
    case NEM_E_INVAL: return "invalid argument";
    case NEM_E_NOMEM: return "not enough memory";
    case NEM_E_HIP: return "HIP runtime error";
    case NEM_E_NUMERIC: return "non-finite value in the state";
    case NEM_E_OVERFLOW: return "cell tile, cell or neighbour list over capacity";
    case NEM_E_SINGULAR: return "singular correction tensor";
    case NEM_E_STATE: return "wrong call order";
    case NEM_E_RANGE: return "device index out of range";
    default: return "unknown error";
  }
}

const char* nem_last_error(const nem_sim* s) { return s ? s->err.c_str() : "null solver"; }

int nem_arena_bytes(const nem_params* p, const int64_t* n, int32_t R, uint64_t* bytes) {
  if (!p || !n || !bytes) return NEM_E_INVAL;
  Sizes z;
  std::string why;
  int rc = sizes_for(p, n, R, z, why);
  if (rc) return rc;
  *bytes = layout(R, z.ntot, z.ncells, z.work_cap, z.stage_n).total;
  return NEM_OK;
}

int nem_create(const nem_params* p, const int64_t* n, int32_t R, void* dev_arena, uint64_t arena_bytes,
               void* hip_stream, nem_sim** out) {
  if (!p || !n || !out) return NEM_E_INVAL;
  *out = nullptr;
  Sizes z;
  std::string why;
  int rc = sizes_for(p, n, R, z, why);
  if (rc) return rc;
  nem_sim* s = new nem_sim();
  s->R = R;
  s->hp.assign(p, p + R);
  s->n.assign(n, n + R);
  s->ntot = (int)z.ntot;
  s->ncells = (int)z.ncells;
  s->work_cap = (int)z.work_cap;
  s->stage_n = z.stage_n;
  s->stream = (hipStream_t)hip_stream;
  const Offs o = layout(R, z.ntot, z.ncells, z.work_cap, z.stage_n);
  if (dev_arena) {
    if (arena_bytes < o.total) { delete s; return NEM_E_NOMEM; }
    s->arena = (char*)dev_arena;
    s->arena_bytes = arena_bytes;
  } else {
    void* m = nullptr;
    if (hipMalloc(&m, o.total) != hipSuccess) { delete s; return NEM_E_NOMEM; }
    s->arena = (char*)m;
    s->arena_bytes = o.total;
    s->own = true;
  }
  char* b = (char*)(((uintptr_t)s->arena + ALIGN - 1) / ALIGN * ALIGN);
  s->d_reps = (RepDev*)(b + o.reps); s->d_work = (int*)(b + o.work);
  s->cell_start = (int*)(b + o.cell_start); s->count = (int*)(b + o.count);
  s->cursor = (int*)(b + o.cursor); s->perm = (int*)(b + o.perm);
  s->t_key = (int*)(b + o.t_key); s->t_off = (float2*)(b + o.t_off); s->t_lo = (float2*)(b + o.t_lo);
  s->t_u = (float2*)(b + o.t_u); s->t_q = (float2*)(b + o.t_q); s->t_drho = (float*)(b + o.t_drho);
  s->t_acc = (float2*)(b + o.t_acc); s->t_id = (int*)(b + o.t_id); s->t_img = (int2*)(b + o.t_img);
  s->t_qyy = (float*)(b + o.t_qyy);
  s->off[0] = (float2*)(b + o.off0); s->off[1] = (float2*)(b + o.off1); s->offlo = (float2*)(b + o.offlo);
  s->u = (float2*)(b + o.u); s->q[0] = (float2*)(b + o.q0); s->q[1] = (float2*)(b + o.q1);
  s->drho = (float*)(b + o.drho); s->acc = (float2*)(b + o.acc); s->id = (int*)(b + o.id);
  s->cell = (int*)(b + o.cell); s->img = (int2*)(b + o.img);
  s->qyy[0] = (float*)(b + o.qyy0); s->qyy[1] = (float*)(b + o.qyy1);
  s->V = (float*)(b + o.V); s->bk = (float4*)(b + o.bk); s->dh = (float*)(b + o.dh);
  s->apart = (float2*)(b + o.apart); s->uv = (float*)(b + o.uv); s->pi = (float2*)(b + o.pi);
  s->P = (float*)(b + o.P); s->drhat = (float*)(b + o.drhat);
  s->flags = (unsigned*)(b + o.flags); s->umax = (unsigned*)(b + o.umax);
  s->stage = (double*)(b + o.stage); s->red = (double*)(b + o.red);
  s->nl = (uint32_t*)(b + o.nl); s->ncnt = (int*)(b + o.ncnt);
  s->fe = (double*)(b + o.fe);
  s->vl = (uint32_t*)(b + o.vl); s->vcnt = (int*)(b + o.vcnt); s->off_build = (float2*)(b + o.off_build);

  int cell_base = 0, part_base = 0;
  for (int r = 0; r < R; ++r) {
    const int nc = cells_per_side(p[r]);
    s->reps.push_back(make_rep(p[r], nc, cell_base, part_base, (int)n[r], s->T, 0));
    cell_base += nc * nc;
    part_base += (int)n[r];
  }
  s->has_state.assign(R, 0);
  hipError_t e = hipSuccess;
  // the no-allocation entry points' scratch on the current device
  e = hipGetDevice(&s->device);
  if (e == hipSuccess) s->scratch = scratch_address(s->device, &e);
  if (e != hipSuccess) { hip_fail(s, e, "scratch lookup (hipGetSymbolAddress)"); nem_destroy(s); return NEM_E_HIP; }
  // zero the whole arena once: counts and cursors must start at zero, and
  // replicas without a state keep empty cells
  if (e == hipSuccess) e = hipMemsetAsync(b, 0, o.total - ALIGN, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) { hip_fail(s, e, "arena init"); nem_destroy(s); return NEM_E_HIP; }
  rc = build_work(s);
  if (rc) { nem_destroy(s); return rc; }
  *out = s;
  return NEM_OK;
}

int nem_set_state(nem_sim* s, int32_t r, const double* x, const double* y, const double* ux, const double* uy,
                  const double* qxx, const double* qxy, const double* rho, const double* ax, const double* ay) {
  if (!s || r < 0 || r >= s->R || !x || !y || !ux || !uy || !qxx || !qxy || !rho) return NEM_E_INVAL;
  const int n = (int)s->n[r];
  const RepDev& R = s->reps[r];
  const double* src[9] = {x, y, ux, uy, qxx, qxy, rho, ax, ay};
  for (int f = 0; f < 9; ++f) {
    double* dst = s->stage + (size_t)f * n;
    if (src[f]) HIPCHK(hipMemcpyAsync(dst, src[f], sizeof(double) * n, hipMemcpyHostToDevice, s->stream));
    else HIPCHK(hipMemsetAsync(dst, 0, sizeof(double) * n, s->stream));
  }
  unsigned* um = s->umax + ((size_t)s->parity * s->R + r) * UMAX_SLOTS;
  HIPCHK(hipMemsetAsync(um, 0, sizeof(unsigned) * UMAX_SLOTS, s->stream));
  SortArgs a = sort_args(s, nullptr);
  launch_ingest(a, r, s->stage, n, s->umax + (size_t)s->parity * s->R * UMAX_SLOTS, s->stream);
  launch_sort_tail(a, R.part_base, n, R.cell_base, R.nc * R.nc, R.part_base, s->stream);
  launch_request_relist(s->flags, s->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s->stream));
  s->has_state[r] = 1;
  unsigned f[2];
  int rc = read_flags(s, f);
  if (rc) return rc;
  return status_from_flags(s, f[0]);
}

int nem_set_qyy(nem_sim* s, int32_t r, const double* qyy) {
  if (!s || r < 0 || r >= s->R || !qyy) return NEM_E_INVAL;
  if (!s->has_state[r]) { s->err = "set the state before Qyy"; return NEM_E_STATE; }
  if (!s->hp[r].q3d) { s->err = "Qyy is a state variable of the quasi-2D variant (q3d = 1) only"; return NEM_E_INVAL; }
  const int n = (int)s->n[r];
  HIPCHK(hipMemcpyAsync(s->stage, qyy, sizeof(double) * n, hipMemcpyHostToDevice, s->stream));
  SortArgs a = sort_args(s, nullptr);
  launch_qyy_io(a, r, n, s->stage, 1, s->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s->stream));
  unsigned f[2];
  int rc = read_flags(s, f);
  if (rc) return rc;
  return status_from_flags(s, f[0]);
}

int nem_get_qyy(nem_sim* s, int32_t r, double* qyy) {
  if (!s || r < 0 || r >= s->R || !qyy) return NEM_E_INVAL;
  if (!s->has_state[r]) { s->err = "state of this replica was never set"; return NEM_E_STATE; }
  if (!s->hp[r].q3d) { s->err = "Qyy is a state variable of the quasi-2D variant (q3d = 1) only"; return NEM_E_INVAL; }
  const int n = (int)s->n[r];
  SortArgs a = sort_args(s, nullptr);
  launch_qyy_io(a, r, n, s->stage, 0, s->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(qyy, s->stage, sizeof(double) * n, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  unsigned f[2];
  int rc = read_flags(s, f);
  if (rc) return rc;
  return status_from_flags(s, f[0]);
}

int nem_get_state(nem_sim* s, int32_t r, double* x, double* y, double* ux, double* uy, double* qxx, double* qxy,
                  double* rho, double* ax, double* ay) {
  if (!s || r < 0 || r >= s->R) return NEM_E_INVAL;
  if (!s->has_state[r]) { s->err = "state of this replica was never set"; return NEM_E_STATE; }
  const int n = (int)s->n[r];
  SortArgs a = sort_args(s, nullptr);
  launch_export(a, r, s->stage, n, s->stream);
  HIPCHK(hipGetLastError());
  double* dst[9] = {x, y, ux, uy, qxx, qxy, rho, ax, ay};
  for (int f = 0; f < 9; ++f)
    if (dst[f]) HIPCHK(hipMemcpyAsync(dst[f], s->stage + (size_t)f * n, sizeof(double) * n, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  unsigned f[2];
  int rc = read_flags(s, f);
  if (rc) return rc;
  return status_from_flags(s, f[0]);
}

int nem_step(nem_sim* s, int64_t nsteps) {
  if (!s || nsteps < 0) return NEM_E_INVAL;
  for (int r = 0; r < s->R; ++r)
    if (!s->has_state[r]) { s->err = "nem_set_state was not called for every replica"; return NEM_E_STATE; }
  return run_steps(s, nsteps);
}

int nem_sync(nem_sim* s) {
  if (!s) return NEM_E_INVAL;
  HIPCHK(hipStreamSynchronize(s->stream));
  collect_times(s);
  unsigned f[2];
  int rc = read_flags(s, f);
  if (rc) return rc;
  return status_from_flags(s, f[0]);
}

// ------------------------------------------------------------ checkpoints
// Whole-simulation checkpoint: a header (sizes, launch options, step parity and
// every replica's particle count and parameters, field by field), then the
// device state between steps in a fixed order: the current offsets, their low
// parts, u^{n+1/2}, the current Q (and Qyy), a^{n-1/2}, rho - rho0, ids, cells,
// image counters, cell starts, both parities' max-speed slots, the four flag
// words, and the Verlet list with its counts and build offsets. Everything a
// step reads before writing it is there, so a load continues bit for bit.
namespace {
constexpr char RAW_MAGIC[8] = {'N', 'E', 'M', 'R', 'A', 'W', '0', '1'};
constexpr int RAW_PD = 17, RAW_PI = 7;  // doubles and integers of nem_params

struct RawSeg { void* dev; size_t bytes; };

std::vector<RawSeg> raw_segments(nem_sim* s) {
  const size_t N = (size_t)s->ntot, C = (size_t)s->ncells;
  const int p = s->parity;
  return {{s->off[p], sizeof(float2) * N}, {s->offlo, sizeof(float2) * N}, {s->u, sizeof(float2) * N},
          {s->q[p], sizeof(float2) * N}, {s->qyy[p], sizeof(float) * N}, {s->acc, sizeof(float2) * N},
          {s->drho, sizeof(float) * N}, {s->id, sizeof(int) * N}, {s->cell, sizeof(int) * N},
          {s->img, sizeof(int2) * N}, {s->cell_start, sizeof(int) * (C + 1)},
          {s->umax, sizeof(unsigned) * 2 * (size_t)s->R * UMAX_SLOTS}, {s->flags, sizeof(unsigned) * 4},
          {s->vl, sizeof(uint32_t) * (KMAX / 2) * N}, {s->vcnt, sizeof(int) * N},
          {s->off_build, sizeof(float2) * N}};
}

void params_fields(const nem_params& q, double* d, int64_t* i) {
  const double dv[RAW_PD] = {q.L, q.dx, q.h, q.rho0, q.eta, q.Gamma, q.lam, q.A, q.B, q.C,
                             q.K, q.zeta, q.dt, q.gamma_eos, q.beta, q.c0_factor, q.skin};
  const int64_t iv[RAW_PI] = {q.form, q.elastic, q.apd, q.kernel, q.integrator, q.q3d, 0};
  std::memcpy(d, dv, sizeof(dv));
  std::memcpy(i, iv, sizeof(iv));
}

// Header: magic, then int64 words {version, R, ntot, ncells, parity, T, LPP,
// COMP}, then per replica {n, 17 doubles, 7 int64}.
size_t raw_header_bytes(int R) { return 8 + 8 * 8 + (size_t)R * (8 + 8 * RAW_PD + 8 * RAW_PI); }

size_t raw_total(nem_sim* s) {
  size_t t = raw_header_bytes(s->R);
  for (const RawSeg& g : raw_segments(s)) t += g.bytes;
  return t;
}
}  // namespace

int nem_raw_bytes(nem_sim* s, uint64_t* bytes) {
  if (!s || !bytes) return NEM_E_INVAL;
  *bytes = raw_total(s);
  return NEM_OK;
}

int nem_save_raw(nem_sim* s, void* host, uint64_t bytes) {
  if (!s || !host) return NEM_E_INVAL;
  for (int r = 0; r < s->R; ++r)
    if (!s->has_state[r]) { s->err = "nem_set_state was not called for every replica"; return NEM_E_STATE; }
  if (bytes < raw_total(s)) { s->err = "checkpoint buffer smaller than nem_raw_bytes"; return NEM_E_NOMEM; }
  char* b = (char*)host;
  std::memcpy(b, RAW_MAGIC, 8);
  const int64_t hw[8] = {1, s->R, s->ntot, s->ncells, s->parity, s->T, s->LPP, s->COMP};
  std::memcpy(b + 8, hw, sizeof(hw));
  char* w = b + 8 + sizeof(hw);
  for (int r = 0; r < s->R; ++r) {
    const int64_t n = s->n[r];
    std::memcpy(w, &n, 8);
    params_fields(s->hp[r], (double*)(w + 8), (int64_t*)(w + 8 + 8 * RAW_PD));
    w += 8 + 8 * RAW_PD + 8 * RAW_PI;
  }
  HIPCHK(hipStreamSynchronize(s->stream));
  for (const RawSeg& g : raw_segments(s)) {
    HIPCHK(hipMemcpyAsync(w, g.dev, g.bytes, hipMemcpyDeviceToHost, s->stream));
    w += g.bytes;
  }
  HIPCHK(hipStreamSynchronize(s->stream));
  unsigned f[2];
  int rc = read_flags(s, f);
  if (rc) return rc;
  return status_from_flags(s, f[0]);
}

int nem_load_raw(nem_sim* s, const void* host, uint64_t bytes) {
  if (!s || !host) return NEM_E_INVAL;
  const char* b = (const char*)host;
  auto bad = [&](const char* why) { s->err = std::string("nem_load_raw: ") + why; return NEM_E_INVAL; };
  if (bytes < raw_header_bytes(s->R) || std::memcmp(b, RAW_MAGIC, 8) != 0) return bad("not a checkpoint of this library");
  int64_t hw[8];
  std::memcpy(hw, b + 8, sizeof(hw));
  if (hw[0] != 1) return bad("unknown checkpoint version");
  if (hw[1] != s->R || hw[2] != s->ntot || hw[3] != s->ncells) return bad("replica count or sizes differ");
  if (!(hw[4] == 0 || hw[4] == 1) || !(hw[5] == 4 || hw[5] == 8) || !(hw[6] == 1 || hw[6] == 2 || hw[6] == 4) ||
      hw[7] < 0 || hw[7] > 2)
    return bad("corrupt header");
  const char* w = b + 8 + sizeof(hw);
  for (int r = 0; r < s->R; ++r) {
    int64_t n;
    std::memcpy(&n, w, 8);
    double d[RAW_PD], dh[RAW_PD];
    int64_t i[RAW_PI], ih[RAW_PI];
    std::memcpy(dh, w + 8, sizeof(dh));
    std::memcpy(ih, w + 8 + 8 * RAW_PD, sizeof(ih));
    params_fields(s->hp[r], d, i);
    if (n != s->n[r]) return bad("particle count of a replica differs");
    for (int k = 0; k < RAW_PD; ++k)
      if (std::memcmp(&d[k], &dh[k], sizeof(double)) != 0) return bad("parameters of a replica differ");
    for (int k = 0; k < RAW_PI; ++k)
      if (i[k] != ih[k]) return bad("parameters of a replica differ");
    w += 8 + 8 * RAW_PD + 8 * RAW_PI;
  }
  // segment sizes depend on the sizes only, so the length is checked before anything changes
  if (bytes < raw_total(s)) { s->err = "nem_load_raw: buffer shorter than the checkpoint"; return NEM_E_NOMEM; }
  // the saved launch options and parity (the Verlet list's LDS slots follow the tile)
  drop_graphs(s);
  const int T = (int)hw[5];
  s->LPP = (int)hw[6];
  s->COMP = (int)hw[7];
  if (T != s->T) {
    s->T = T;
    int rc = build_work(s);
    if (rc) return rc;
  }
  s->parity = (int)hw[4];
  for (const RawSeg& g : raw_segments(s)) {
    HIPCHK(hipMemcpyAsync(g.dev, w, g.bytes, hipMemcpyHostToDevice, s->stream));
    w += g.bytes;
  }
  HIPCHK(hipStreamSynchronize(s->stream));
  for (int r = 0; r < s->R; ++r) s->has_state[r] = 1;
  for (auto& sn : s->snap) sn.valid = false;
  unsigned f[2];
  int rc = read_flags(s, f);
  if (rc) return rc;
  return status_from_flags(s, f[0]);
}

int nem_neighbor_list(nem_sim* s, int32_t r, int32_t which, int64_t* row_ptr, int32_t* col, int64_t cap,
                      int64_t* nnz, int32_t* cell_xy, float* off_xy) {
  if (!s || r < 0 || r >= s->R || !row_ptr || !nnz || (which != 0 && which != 1)) return NEM_E_INVAL;
  if (!s->has_state[r]) return NEM_E_STATE;
  const int n = (int)s->n[r];
  // the next step's own start: rebin if requested, then the Verlet build or walk
  const int timing = s->timing;
  s->timing = 0;
  int rc = enqueue_prologue(s, s->stream);
  s->timing = timing;
  if (rc) return rc;
  // counts, row pointers and offsets in the staging area (9 * max n doubles)
  char* st = (char*)s->stage;
  int* d_cnt = (int*)st;
  int64_t* d_rp = (int64_t*)(st + ((sizeof(int) * (size_t)n + 7) / 8) * 8);
  int* d_cxy = (int*)(d_rp + n + 1);
  float* d_oxy = (float*)(d_cxy + 2 * (size_t)n);
  StepArgs a = step_args(s);
  const int kern = s->hp[0].kernel;
  launch_list_export(s->T, kern, a, r, which, 0, d_cnt, nullptr, nullptr, 0, s->stream);
  HIPCHK(hipGetLastError());
  std::vector<int> cnt(n);
  HIPCHK(hipMemcpyAsync(cnt.data(), d_cnt, sizeof(int) * n, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  {
    // a tile over capacity skips its particles: the counts are valid only without errors
    unsigned f[2];
    rc = read_flags(s, f);
    if (rc) return rc;
    rc = status_from_flags(s, f[0]);
    if (rc && rc != NEM_E_SINGULAR) return rc;
    rc = NEM_OK;
  }
  row_ptr[0] = 0;
  for (int i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i];
  *nnz = row_ptr[n];
  if (*nnz > cap || !col) {
    rc = NEM_E_NOMEM;
  } else {
    int32_t* d_col = nullptr;
    HIPCHK(hipMalloc(&d_col, sizeof(int32_t) * std::max<int64_t>(*nnz, 1)));
    hipError_t e = hipMemcpyAsync(d_rp, row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) {
      launch_list_export(s->T, kern, a, r, which, 1, d_cnt, d_rp, d_col, *nnz, s->stream);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(col, d_col, sizeof(int32_t) * *nnz, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    hipFree(d_col);
    if (e != hipSuccess) return hip_fail(s, e, "neighbour list export");
    for (int i = 0; i < n; ++i) std::sort(col + row_ptr[i], col + row_ptr[i + 1]);
  }
  if (cell_xy || off_xy) {
    SortArgs sa = sort_args(s, nullptr);
    launch_export_offsets(sa, r, n, d_cxy, d_oxy, s->stream);
    HIPCHK(hipGetLastError());
    if (cell_xy) HIPCHK(hipMemcpyAsync(cell_xy, d_cxy, sizeof(int32_t) * 2 * n, hipMemcpyDeviceToHost, s->stream));
    if (off_xy) HIPCHK(hipMemcpyAsync(off_xy, d_oxy, sizeof(float) * 2 * n, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
  }
  if (rc) return rc;
  unsigned f[2];
  rc = read_flags(s, f);
  if (rc) return rc;
  return status_from_flags(s, f[0]);
}

int nem_neighbors(nem_sim* s, int32_t r, int64_t* row_ptr, int32_t* col, int64_t cap, int64_t* nnz) {
  return nem_neighbor_list(s, r, 0, row_ptr, col, cap, nnz, nullptr, nullptr);
}

int nem_diagnostics(nem_sim* s, int32_t r, nem_diag* out) {
  if (!s || r < 0 || r >= s->R || !out) return NEM_E_INVAL;
  if (!s->has_state[r]) return NEM_E_STATE;
  SortArgs a = sort_args(s, nullptr);
  // pair sums at the integer time level: integer-level offsets into the
  // staging array, then pass A (volumes, neighbour list) and the free-energy
  // kernel on them; the per-step temporaries are rebuilt by the next step
  launch_int_offsets(a, s->t_off, s->stream);
  StepArgs sa = step_args(s);
  sa.off_cur = s->t_off;
  const PassCfg cfg{s->T, 1, 1, 0, 0, s->hp[0].kernel, 0, 0};
  if (!launch_pass(1, cfg, sa, s->stream)) return NEM_E_INVAL;
  launch_free_energy(s->T, s->hp[0].kernel, sa, s->fe, s->stream);
  launch_reduce(a, r, (int)s->n[r], s->fe, s->red, s->stream);
  HIPCHK(hipGetLastError());
  double h[8];
  unsigned ums[UMAX_SLOTS];
  HIPCHK(hipMemcpyAsync(h, s->red, sizeof(double) * 8, hipMemcpyDeviceToHost, s->stream));
  // c0 of the last step: its pass C read the slots of the parity before the flip
  const int last = 1 - s->parity;
  HIPCHK(hipMemcpyAsync(ums, s->umax + ((size_t)last * s->R + r) * UMAX_SLOTS, sizeof(ums),
                        hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  unsigned um = 0;
  for (unsigned v : ums) um = std::max(um, v);
  const double m = s->hp[r].rho0 * s->hp[r].dx * s->hp[r].dx;
  float umf;
  std::memcpy(&umf, &um, sizeof(umf));
  out->px = m * h[0];
  out->py = m * h[1];
  out->ke = h[2] / (double)s->n[r];
  out->umax = h[3];
  out->qmax = h[4];
  out->F = h[5];
  out->F_grad = h[6];
  out->c0 = s->hp[r].c0_factor * (double)umf;
  unsigned f[2];
  int rc = read_flags(s, f);
  if (rc) return rc;
  return status_from_flags(s, f[0]);
}

int nem_deposit(nem_sim* s, int32_t r, int32_t M, double* out) {
  if (!s || !out) return NEM_E_INVAL;
  int rc = deposit_grid(s, r, M);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(out, s->g_grid, sizeof(double) * 4 * (size_t)M * M, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  unsigned f[2];
  rc = read_flags(s, f);
  if (rc) return rc;
  return status_from_flags(s, f[0]);
}

int nem_spectrum(nem_sim* s, int32_t r, int32_t M, double* E, int32_t nbins, int32_t k_lo, int32_t k_hi,
                 double* slope) {
  if (!s || !E || nbins < 1) return NEM_E_INVAL;
  int rc = deposit_grid(s, r, M);
  if (rc) return rc;
  int logM = 0;
  while ((1 << logM) < M) ++logM;
  launch_fft2(s->g_grid, s->g_z, s->g_w, M, logM, s->stream);
  launch_shells(s->g_w, M, s->gbins, s->g_part, s->g_E, s->stream);
  HIPCHK(hipGetLastError());
  std::vector<double> h(s->gbins);
  HIPCHK(hipMemcpyAsync(h.data(), s->g_E, sizeof(double) * s->gbins, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  for (int n = 0; n < nbins; ++n) E[n] = n < s->gbins ? h[n] : 0.0;
  if (slope) {
    // least-squares slope of ln E against ln n over [k_lo, k_hi] (defaults 4, M/8)
    const int lo = k_lo > 0 ? k_lo : 4, hi = k_hi > 0 ? k_hi : M / 8;
    double sx = 0, sy = 0, sxx = 0, sxy = 0;
    int m = 0;
    for (int n = lo; n <= hi && n < s->gbins; ++n) {
      if (!(h[n] > 0)) continue;
      const double x = std::log((double)n), y = std::log(h[n]);
      sx += x; sy += y; sxx += x * x; sxy += x * y; ++m;
    }
    *slope = (m >= 2) ? (m * sxy - sx * sy) / (m * sxx - sx * sx) : NAN;
  }
  unsigned f[2];
  rc = read_flags(s, f);
  if (rc) return rc;
  return status_from_flags(s, f[0]);
}

int nem_vorticity_correlation(nem_sim* s, int32_t r, int32_t M, double* c_x, double* c_y, double* l_x,
                              double* l_y) {
  if (!s || !c_x || !c_y) return NEM_E_INVAL;
  int rc = deposit_grid(s, r, M);
  if (rc) return rc;
  int logM = 0;
  while ((1 << logM) < M) ++logM;
  launch_fft2(s->g_grid, s->g_z, s->g_w, M, logM, s->stream);
  launch_vort_correlation(s->g_w, M, logM, s->hp[r].L, s->g_z, s->g_w, s->g_part, s->stream);
  HIPCHK(hipGetLastError());
  std::vector<double> h(M + 2);
  HIPCHK(hipMemcpyAsync(h.data(), s->g_part, sizeof(double) * (M + 2), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  const int H = M / 2;
  const double a0 = h[0];
  const double dl = s->hp[r].L / M;
  // first zero crossing, linearly interpolated; -1 when the curve stays positive
  auto crossing = [&](const double* c) {
    for (int n = 1; n <= H; ++n)
      if (c[n] <= 0.0) return (n - 1 + c[n - 1] / (c[n - 1] - c[n])) * dl;
    return -1.0;
  };
  for (int n = 0; n <= H; ++n) {
    c_x[n] = a0 > 0.0 ? h[n] / a0 : NAN;
    c_y[n] = a0 > 0.0 ? h[H + 1 + n] / a0 : NAN;
  }
  if (l_x) *l_x = a0 > 0.0 ? crossing(c_x) : NAN;
  if (l_y) *l_y = a0 > 0.0 ? crossing(c_y) : NAN;
  unsigned f[2];
  rc = read_flags(s, f);
  if (rc) return rc;
  return status_from_flags(s, f[0]);
}

int nem_track(nem_sim* s, int32_t r, const int32_t* ids, int32_t n_ids, double* x, double* y) {
  if (!s || r < 0 || r >= s->R || n_ids < 0 || (n_ids > 0 && (!ids || !x || !y))) return NEM_E_INVAL;
  if (!s->has_state[r]) { s->err = "state of this replica was never set"; return NEM_E_STATE; }
  const int n = (int)s->n[r];
  if (n_ids > n) { s->err = "more ids than particles"; return NEM_E_INVAL; }
  for (int t = 0; t < n_ids; ++t)
    if (ids[t] < 0 || ids[t] >= n) { s->err = "particle id out of range"; return NEM_E_INVAL; }
  if (n_ids == 0) return NEM_OK;
  // staging (9 n doubles): inv[n] ints at 0, ids at n doubles, output at 2n doubles
  int* inv = (int*)s->stage;
  int* d_ids = (int*)(s->stage + n);
  double* out = s->stage + 2 * (size_t)n;
  HIPCHK(hipMemcpyAsync(d_ids, ids, sizeof(int32_t) * n_ids, hipMemcpyHostToDevice, s->stream));
  SortArgs a = sort_args(s, nullptr);
  launch_track(a, r, n, inv, d_ids, n_ids, out, s->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(x, out, sizeof(double) * n_ids, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipMemcpyAsync(y, out + n_ids, sizeof(double) * n_ids, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  unsigned f[2];
  int rc = read_flags(s, f);
  if (rc) return rc;
  return status_from_flags(s, f[0]);
}

int nem_mixing(nem_sim* s, int32_t r, const uint8_t* colour, int32_t ncol, int32_t B, int64_t* counts,
               double* index) {
  if (!s || r < 0 || r >= s->R || !colour || ncol < 1 || ncol > 255 || B < 1 || B > 1024) return NEM_E_INVAL;
  if (!s->has_state[r]) { s->err = "state of this replica was never set"; return NEM_E_STATE; }
  const int n = (int)s->n[r];
  for (int i = 0; i < n; ++i)
    if (colour[i] >= ncol) { s->err = "colour out of range"; return NEM_E_INVAL; }
  const size_t nb = (size_t)B * B * ncol;
  if (nb > s->mix_cap) {
    if (s->g_mix) HIPCHK(hipFree(s->g_mix));
    s->g_mix = nullptr; s->mix_cap = 0;
    HIPCHK(hipMalloc((void**)&s->g_mix, sizeof(unsigned long long) * nb));
    s->mix_cap = nb;
  }
  uint8_t* d_col = (uint8_t*)s->stage;  // n bytes of the 9 n double staging area
  HIPCHK(hipMemcpyAsync(d_col, colour, (size_t)n, hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipMemsetAsync(s->g_mix, 0, sizeof(unsigned long long) * nb, s->stream));
  SortArgs a = sort_args(s, nullptr);
  launch_colour_counts(a, r, n, d_col, ncol, B, s->g_mix, s->stream);
  HIPCHK(hipGetLastError());
  std::vector<unsigned long long> h(nb);
  HIPCHK(hipMemcpyAsync(h.data(), s->g_mix, sizeof(unsigned long long) * nb, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  unsigned f[2];
  int rc = read_flags(s, f);
  if (rc) return rc;
  rc = status_from_flags(s, f[0]);
  if (counts)
    for (size_t k = 0; k < nb; ++k) counts[k] = (int64_t)h[k];
  if (index) {
    // intensity of segregation: sum over bins and colours of N_b (phi_cb - phi_c)^2,
    // over its value sum_c N phi_c (1 - phi_c) for fully segregated colours
    std::vector<double> Nc(ncol, 0.0);
    double N = 0.0;
    for (size_t b = 0; b < (size_t)B * B; ++b)
      for (int c = 0; c < ncol; ++c) { Nc[c] += (double)h[b * ncol + c]; N += (double)h[b * ncol + c]; }
    double num = 0.0, den = 0.0;
    for (int c = 0; c < ncol; ++c) den += Nc[c] * (1.0 - Nc[c] / N);
    for (size_t b = 0; b < (size_t)B * B; ++b) {
      double Nb = 0.0;
      for (int c = 0; c < ncol; ++c) Nb += (double)h[b * ncol + c];
      if (Nb <= 0.0) continue;
      for (int c = 0; c < ncol; ++c) {
        const double d = (double)h[b * ncol + c] - Nb * Nc[c] / N;
        num += d * d / Nb;
      }
    }
    *index = den > 0.0 ? 1.0 - num / den : NAN;
  }
  return rc;
}

int nem_defects(nem_sim* s, int32_t r, int32_t M, int64_t* n_plus, int64_t* n_minus) {
  if (!s || !n_plus || !n_minus) return NEM_E_INVAL;
  int rc = deposit_grid(s, r, M);
  if (rc) return rc;
  HIPCHK(hipMemsetAsync(s->g_cnt, 0, sizeof(unsigned long long) * 2, s->stream));
  launch_winding(s->g_grid, M, s->g_cnt, s->stream);
  HIPCHK(hipGetLastError());
  unsigned long long c[2];
  HIPCHK(hipMemcpyAsync(c, s->g_cnt, sizeof(c), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  *n_plus = (int64_t)c[0];
  *n_minus = (int64_t)c[1];
  unsigned f[2];
  rc = read_flags(s, f);
  if (rc) return rc;
  return status_from_flags(s, f[0]);
}

int nem_defects_noalloc(nem_sim* s, int32_t r, int32_t M, int64_t* n_plus, int64_t* n_minus) {
  if (!s || !n_plus || !n_minus) return NEM_E_INVAL;
  if (r < 0 || r >= s->R) { s->err = "replica index out of range"; return NEM_E_INVAL; }
  if (M < 8 || M > NEM_NOALLOC_MAX_GRID || (M & (M - 1))) {
    s->err = "nem_defects_noalloc: grid side must be a power of two in [8, " + std::to_string(NEM_NOALLOC_MAX_GRID) +
             "] (the size of its static scratch)";
    return NEM_E_INVAL;
  }
  if (!s->has_state[r]) { s->err = "state of this replica was never set"; return NEM_E_STATE; }
  if (!s->scratch) { s->err = "no scratch on this device"; return NEM_E_HIP; }
  double* grid = (double*)s->scratch;
  unsigned long long* cnt = (unsigned long long*)((char*)s->scratch + NOALLOC_GRID_BYTES);
  // the same kernels as nem_defects: integer-level offsets (arena), deposit
  // (writes every node of the M x M grid), counters cleared, winding
  SortArgs a = sort_args(s, nullptr);
  launch_int_offsets(a, s->t_off, s->stream);
  StepArgs sa = step_args(s);
  sa.off_cur = s->t_off;
  launch_deposit(s->T, s->hp[r].kernel, sa, r, M, grid, s->stream);
  hipLaunchKernelGGL(k_clear_u64, dim3(1), dim3(64), 0, s->stream, cnt, 2);
  launch_winding(grid, M, cnt, s->stream);
  HIPCHK(hipGetLastError());
  unsigned long long c[2];
  HIPCHK(hipMemcpyAsync(c, cnt, sizeof(c), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  *n_plus = (int64_t)c[0];
  *n_minus = (int64_t)c[1];
  unsigned f[2];
  int rc = read_flags(s, f);
  if (rc) return rc;
  return status_from_flags(s, f[0]);
}

int nem_set_option(nem_sim* s, int32_t key, int64_t value) {
  if (!s) return NEM_E_INVAL;
  switch (key) {
    case NEM_OPT_TILE: {
      if (value != 4 && value != 8) return NEM_E_INVAL;
      drop_graphs(s);
      s->T = (int)value;
      launch_request_relist(s->flags, s->stream);  // LDS slots of the Verlet list change with the tile
      return build_work(s);
    }
    case NEM_OPT_LPP:
      if (value != 1 && value != 2 && value != 4) return NEM_E_INVAL;
      drop_graphs(s);
      s->LPP = (int)value;
      return NEM_OK;
    case NEM_OPT_COMP:
      if (value < 0 || value > 2) return NEM_E_INVAL;
      drop_graphs(s);
      s->COMP = (int)value;
      return NEM_OK;
    case NEM_OPT_TIMING:
      collect_times(s);
      s->timing = value ? 1 : 0;
      return NEM_OK;
    case NEM_OPT_GRAPH:
      if (value < 0 || value > 4096) return NEM_E_INVAL;
      drop_graphs(s);
      s->use_graph = value ? 1 : 0;
      s->graph_steps = value ? (int)value : 1;
      return NEM_OK;
    case NEM_OPT_PERSIST:
      if (value < 0 || value > (1 << 20)) return NEM_E_INVAL;
      drop_graphs(s);
      s->persist = (int)value;
      return NEM_OK;
    default:
      return NEM_E_INVAL;
  }
}

int nem_get_option(nem_sim* s, int32_t key, int64_t* value) {
  if (!s || !value) return NEM_E_INVAL;
  switch (key) {
    case NEM_OPT_TILE: *value = s->T; return NEM_OK;
    case NEM_OPT_LPP: *value = s->LPP; return NEM_OK;
    case NEM_OPT_COMP: *value = s->COMP; return NEM_OK;
    case NEM_OPT_TIMING: *value = s->timing; return NEM_OK;
    case NEM_OPT_GRAPH: *value = s->use_graph ? s->graph_steps : 0; return NEM_OK;
    case NEM_OPT_PERSIST: *value = s->persist; return NEM_OK;
    default: return NEM_E_INVAL;
  }
}

int nem_pass_times(nem_sim* s, double* ms, int64_t* launches, int32_t reset) {
  if (!s) return NEM_E_INVAL;
  collect_times(s);
  for (int p = 0; p < NEM_NPASS; ++p) {
    if (ms) ms[p] = s->pass_ms[p];
    if (launches) launches[p] = s->pass_n[p];
    if (reset) { s->pass_ms[p] = 0; s->pass_n[p] = 0; }
  }
  return NEM_OK;
}

void nem_destroy(nem_sim* s) {
  if (!s) return;
  if (s->stream) hipStreamSynchronize(s->stream);
  else hipDeviceSynchronize();
  collect_times(s);
  for (auto& e : s->ev_free) hipEventDestroy(e);
  drop_graphs(s);
  if (s->cap_stream) hipStreamDestroy(s->cap_stream);
  free_grid(s);
  if (s->g_mix) hipFree(s->g_mix);
  free_snapshot(s);
  if (s->own && s->arena) hipFree(s->arena);
  delete s;
}

}  // extern "C"
