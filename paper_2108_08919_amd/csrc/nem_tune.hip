// nem_tune.hip -- autotuner of the pair-pass launch shape.
//
// Times every supported (tile side, lanes per particle, persistent grid size)
// combination on the solver's own state (all replicas, so uneven batches are
// tuned as a whole), restoring the state after each trial, and keeps the
// fastest. The search starts with a few untimed steps (the GPU's clocks ramp up
// under load, which otherwise penalises the first trials), and each trial
// takes the fastest of three timed repetitions after one warm-up step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "nem_dev.h"
#include "nem_sim.h"

using namespace nem;
using namespace nem_host;

extern "C" int nem_autotune(nem_sim* s, int32_t steps, int32_t* tile, int32_t* lpp, double* ms_per_step) {
  if (!s || steps < 1) return NEM_E_INVAL;
  for (int r = 0; r < s->R; ++r)
    if (!s->has_state[r]) return NEM_E_STATE;
  const int T0 = s->T, L0 = s->LPP, G0 = s->persist;
  int rc = take_snapshot(s);
  if (rc) return rc;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int timing = s->timing;
  s->timing = 0;
  // untimed steps on the current shape before the first trial
  rc = run_steps(s, 8);
  if (!rc) rc = (hipStreamSynchronize(s->stream) == hipSuccess) ? NEM_OK : NEM_E_HIP;
  {
    const int rr = restore_snapshot(s);
    if (!rc) rc = rr;
  }
  float best = 1e30f;
  int bT = T0, bL = L0, bG = G0;
  // persistent grids: 0 = one workgroup per tile (hardware dispatch), else
  // that many workgroups looping over the tile list (2, 4, 8 per CU)
  const int tiles[2] = {4, 8}, lanes[3] = {1, 2, 4}, grids[4] = {0, 512, 1024, 2048};
  for (int G : grids)
  for (int T : tiles)
    for (int L : lanes) {
      if (rc) break;
      drop_graphs(s);
      s->T = T;
      s->LPP = L;
      s->persist = G;
      rc = build_work(s);
      if (!rc) rc = run_steps(s, 1);  // warm-up (also rebins if requested)
      float ms = 1e30f;
      for (int k = 0; k < 3 && !rc; ++k) {
        if (!rc) rc = (hipEventRecord(e0, s->stream) == hipSuccess) ? NEM_OK : NEM_E_HIP;
        if (!rc) rc = run_steps(s, steps);
        if (!rc) rc = (hipEventRecord(e1, s->stream) == hipSuccess) ? NEM_OK : NEM_E_HIP;
        if (!rc) rc = (hipEventSynchronize(e1) == hipSuccess) ? NEM_OK : NEM_E_HIP;
        float t = 0.f;
        if (!rc && hipEventElapsedTime(&t, e0, e1) == hipSuccess) ms = std::min(ms, t);
      }
      if (!rc && ms / steps < best) {
        best = ms / steps;
        bT = T;
        bL = L;
        bG = G;
      }
      const int rr = restore_snapshot(s);
      if (!rc) rc = rr;
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  s->timing = timing;
  drop_graphs(s);
  s->T = rc ? T0 : bT;
  s->LPP = rc ? L0 : bL;
  s->persist = rc ? G0 : bG;
  const int rb = build_work(s);
  if (!rc) rc = rb;
  if (tile) *tile = s->T;
  if (lpp) *lpp = s->LPP;
  if (ms_per_step) *ms_per_step = best;
  return rc;
}
