// nem_tune.hip -- autotuner of the pair-pass launch shape.
//
// Times every supported (tile side, lanes per particle) pair on the solver's
// own state (all replicas, so uneven batches are tuned as a whole), restoring
// the state after each trial, and keeps the fastest.
#include <hip/hip_runtime.h>

#include <vector>

#include "nem_dev.h"
#include "nem_sim.h"

using namespace nem;
using namespace nem_host;

extern "C" int nem_autotune(nem_sim* s, int32_t steps, int32_t* tile, int32_t* lpp, double* ms_per_step) {
  if (!s || steps < 1) return NEM_E_INVAL;
  for (int r = 0; r < s->R; ++r)
    if (!s->has_state[r]) return NEM_E_STATE;
  const int T0 = s->T, L0 = s->LPP;
  int rc = take_snapshot(s);
  if (rc) return rc;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int timing = s->timing;
  s->timing = 0;
  float best = 1e30f;
  int bT = T0, bL = L0;
  const int tiles[2] = {4, 8}, lanes[3] = {1, 2, 4};
  for (int T : tiles)
    for (int L : lanes) {
      drop_graphs(s);
      s->T = T;
      s->LPP = L;
      rc = build_work(s);
      if (!rc) rc = run_steps(s, 1);  // warm-up (also rebins if requested)
      if (!rc) rc = (hipEventRecord(e0, s->stream) == hipSuccess) ? NEM_OK : NEM_E_HIP;
      if (!rc) rc = run_steps(s, steps);
      if (!rc) rc = (hipEventRecord(e1, s->stream) == hipSuccess) ? NEM_OK : NEM_E_HIP;
      if (!rc) rc = (hipEventSynchronize(e1) == hipSuccess) ? NEM_OK : NEM_E_HIP;
      float ms = 0.f;
      if (!rc && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms / steps < best) {
        best = ms / steps;
        bT = T;
        bL = L;
      }
      const int rr = restore_snapshot(s);
      if (!rc) rc = rr;
      if (rc) break;
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  s->timing = timing;
  drop_graphs(s);
  s->T = rc ? T0 : bT;
  s->LPP = rc ? L0 : bL;
  const int rb = build_work(s);
  if (!rc) rc = rb;
  if (tile) *tile = s->T;
  if (lpp) *lpp = s->LPP;
  if (ms_per_step) *ms_per_step = best;
  return rc;
}
