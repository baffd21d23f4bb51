// Batch lists against measured contraction time (Sec. V-B: the qubit batch sizes
// are a free parameter of the interface, and the paper measures contraction time
// against them).  Every candidate list gets its own plan; proportional NBS runs
// once untimed and once timed (HIP events on the caller's stream) over the
// caller's sample of trajectories and shots; the fastest list wins.  The error
// sets do not depend on the batch list, so one set of Kraus choices serves every
// candidate.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

extern "C" {

ptsbe_status_t ptsbe_tune_batches(const ptsbe_circuit_t* circuit, const ptsbe_plan_opts_t* base_opts,
                                  int32_t n_candidates, const int32_t* cand_offsets, const int32_t* cand_sizes,
                                  const uint8_t* d_kraus_idx, int64_t E, const int64_t* d_mult,
                                  const int64_t* d_shots_per_traj, uint64_t seed, uint64_t* d_shots,
                                  void* d_workspace, size_t workspace_bytes, void* stream, double* times_ms,
                                  int32_t* best) {
  if (!circuit || !base_opts || !cand_offsets || !cand_sizes || !times_ms || !best)
    return ptsbe::fail(PTSBE_ERR_INVALID_ARG, "null argument");
  if (n_candidates < 1) return ptsbe::fail(PTSBE_ERR_INVALID_ARG, "no candidate batch lists");
  if (base_opts->device < 0) return ptsbe::fail(PTSBE_ERR_INVALID_ARG, "tuning needs a device");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(base_opts->device));
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  HIP_TRY(hipEventCreate(&ev0));
  HIP_TRY(hipEventCreate(&ev1));
  *best = -1;
  double best_ms = 0.0;
  ptsbe_status_t st = PTSBE_OK;
  for (int32_t c = 0; c < n_candidates && st == PTSBE_OK; ++c) {
    times_ms[c] = -1.0;
    const int32_t lo = cand_offsets[c], hi = cand_offsets[c + 1];
    if (lo < 0 || hi <= lo) {
      st = ptsbe::fail(PTSBE_ERR_INVALID_ARG, "candidate offsets must increase");
      break;
    }
    ptsbe_plan_opts_t o = *base_opts;
    o.n_batches = hi - lo;
    o.batch_sizes = cand_sizes + lo;
    ptsbe_plan_t plan = nullptr;
    if (ptsbe_plan(circuit, &o, &plan) != PTSBE_OK) continue;   // unsupported list: time stays negative
    auto run = [&]() {
      return ptsbe_sample_shots(plan, d_kraus_idx, E, d_mult, d_shots_per_traj, PTSBE_MODE_PROPORTIONAL, seed, d_shots,
                                nullptr, nullptr, nullptr, nullptr, d_workspace, workspace_bytes, stream);
    };
    ptsbe_status_t r = run();
    if (r == PTSBE_OK) {
      hipError_t e = hipEventRecord(ev0, s);
      if (e == hipSuccess) r = run();
      if (e == hipSuccess && r == PTSBE_OK) e = hipEventRecord(ev1, s);
      if (e == hipSuccess && r == PTSBE_OK) e = hipEventSynchronize(ev1);
      float ms = 0.f;
      if (e == hipSuccess && r == PTSBE_OK) e = hipEventElapsedTime(&ms, ev0, ev1);
      if (e != hipSuccess) {
        st = ptsbe::fail(PTSBE_ERR_DEVICE, std::string("timing a candidate: ") + hipGetErrorString(e));
      } else if (r == PTSBE_OK) {
        times_ms[c] = ms;
        if (*best < 0 || ms < best_ms) {
          *best = c;
          best_ms = ms;
        }
      }
    }
    // a list the sampler rejects (batch wider than it draws, workspace too small)
    // keeps a negative time; a device error ends the call
    if (r == PTSBE_ERR_DEVICE) st = r;
    ptsbe_plan_destroy(plan);
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  if (st != PTSBE_OK) return st;
  if (*best < 0) return ptsbe::fail(PTSBE_ERR_UNSUPPORTED, "no candidate batch list could be planned and sampled");
  return PTSBE_OK;
}

}  // extern "C"
