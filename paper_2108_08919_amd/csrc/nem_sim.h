// nem_sim.h -- host-side state of one solver (private to the library).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/nematic_sph.h"
#include "nem_dev.h"

struct nem_sim {
  using RepDev = nem::RepDev;
  int R = 0;
  std::vector<nem_params> hp;
  std::vector<int64_t> n;
  int ntot = 0, ncells = 0;
  std::vector<RepDev> reps;
  hipStream_t stream = nullptr;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  bool own = false;
  RepDev* d_reps = nullptr;
  int* d_work = nullptr;
  int nwork = 0, work_cap = 0;
  int *cell_start = nullptr, *count = nullptr, *cursor = nullptr, *perm = nullptr;
  int* t_key = nullptr; float2 *t_off = nullptr, *t_lo = nullptr, *t_u = nullptr, *t_q = nullptr;
  float* t_drho = nullptr; float2* t_acc = nullptr; int* t_id = nullptr; int2* t_img = nullptr;
  float* t_qyy = nullptr;
  float2* off[2] = {nullptr, nullptr}; float2* offlo = nullptr; float2* u = nullptr;
  float2* q[2] = {nullptr, nullptr}; float* drho = nullptr; float2* acc = nullptr;
  float* qyy[2] = {nullptr, nullptr};  // quasi-2D variant: Qyy (ping-pong like q)
  int* id = nullptr; int* cell = nullptr;
  int2* img = nullptr;
  float* V = nullptr; float4* bk = nullptr; float* dh = nullptr; float2* apart = nullptr;
  float* uv = nullptr; float2* pi = nullptr; float* P = nullptr; float* drhat = nullptr;
  unsigned* flags = nullptr; unsigned* umax = nullptr;
  uint32_t* nl = nullptr; int* ncnt = nullptr; double* fe = nullptr;
  uint32_t* vl = nullptr; int* vcnt = nullptr; float2* off_build = nullptr;  // Verlet list
  double* stage = nullptr; int64_t stage_n = 0;
  double* red = nullptr;
  int parity = 0;
  std::vector<char> has_state;
  int T = 4, LPP = 1, COMP = 1;
  int persist = 0;        // > 0: persistent pass kernels with this many workgroups
  int graph_steps = 1;    // steps per captured graph
  int timing = 0;
  struct EvRec { int pass; hipEvent_t a, b; };
  std::vector<hipEvent_t> ev_free;
  std::vector<EvRec> ev_pend;
  int use_graph = 0;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  double pass_ms[NEM_NPASS] = {0};
  int64_t pass_n[NEM_NPASS] = {0};
  // grid-diagnostic buffers (allocated on first use, grown with M)
  int gM = 0, gbins = 0;
  double* g_grid = nullptr; double2* g_z = nullptr; double2* g_w = nullptr;
  double* g_part = nullptr; double* g_E = nullptr; unsigned long long* g_cnt = nullptr;
  // mixing histogram (B * B * ncol counters) and its capacity
  unsigned long long* g_mix = nullptr; size_t mix_cap = 0;
  // learned stepping: feature output of pass B (NULL when not capturing) and
  // the device snapshot used to restart a macro step with fine steps
  float* feat = nullptr;
  struct Snap {
    bool alloc = false, valid = false;
    float2 *off = nullptr, *offlo = nullptr, *u = nullptr, *q = nullptr, *acc = nullptr;
    float* drho = nullptr;
    int *id = nullptr, *cell = nullptr, *cell_start = nullptr;
    int2* img = nullptr;
    float* qyy = nullptr;
    unsigned* umax = nullptr;  // R * UMAX_SLOTS max-speed slots, then the rebin request
    int parity = 0;
    std::vector<float> dt;
  } snap[2];  // two, so that a learned macro step can run while the previous one is checked
  int device = 0;            // device current at nem_create
  void* scratch = nullptr;   // that device's copy of the no-allocation scratch
  std::string err;
};


namespace nem_host {

inline int hip_fail(nem_sim* s, hipError_t e, const char* what) {
  if (s) s->err = std::string(what) + ": " + hipGetErrorString(e);
  return NEM_E_HIP;
}
#define HIPCHK(expr)                                        \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) return nem_host::hip_fail(s, e_, #expr); \
  } while (0)

nem::SortArgs sort_args(nem_sim* s, const unsigned* gate);
nem::StepArgs step_args(nem_sim* s);
int read_flags(nem_sim* s, unsigned* f);
int status_from_flags(nem_sim* s, unsigned f);
int run_steps(nem_sim* s, int64_t nsteps);
int upload_reps(nem_sim* s);
void free_snapshot(nem_sim* s);
int take_snapshot(nem_sim* s, int i = 0);
int restore_snapshot(nem_sim* s, int i = 0);
int build_work(nem_sim* s);
void drop_graphs(nem_sim* s);

}  // namespace nem_host
