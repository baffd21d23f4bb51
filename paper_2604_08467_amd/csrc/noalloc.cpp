// The allocation-free variant of ptsbe_contract_batch: the workspace of the
// batch-wise contraction (merged gates, per-trajectory tensors, per-element
// tensors, partial sums) is a fixed array in the library's device memory
// instead of a caller allocation, for callers that cannot allocate device
// memory.  Each GPU the library runs on holds its own copy of the array until
// the process ends.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

namespace {

constexpr size_t kScratchBytes = PTSBE_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The fixed workspace.  Host code never passes this name to a kernel or a copy:
// it stands for the device array only in hipGetSymbolAddress, whose result is
// the address on the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (looked up once per device, with the
// device current).
ptsbe_status_t scratch_on(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return ptsbe::fail(PTSBE_ERR_INVALID_ARG, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch_ptr[device]) {
    HIP_TRY(hipSetDevice(device));
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return ptsbe::fail(PTSBE_ERR_DEVICE, "hipGetSymbolAddress returned a null scratch address");
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return PTSBE_OK;
}

}  // namespace

extern "C" {

ptsbe_status_t ptsbe_contract_batch_noalloc(ptsbe_plan_t plan, int32_t j, const uint8_t* d_kraus_idx, int64_t E,
                                            const int32_t* d_elem_traj, const uint64_t* d_elem_prefix,
                                            int64_t n_elems, int32_t out_kind, void* d_out, double* d_elem_total,
                                            void* stream) {
  ptsbe::Plan* p = reinterpret_cast<ptsbe::Plan*>(plan);
  if (!p) return ptsbe::fail(PTSBE_ERR_INVALID_ARG, "null plan");
  if (p->device < 0) return ptsbe::fail(PTSBE_ERR_INVALID_ARG, "plan was built without a device");
  if (j < 0 || j >= (int)p->batches.size()) return ptsbe::fail(PTSBE_ERR_INVALID_ARG, "batch index out of range");
  if (E < 1 || n_elems < 0) return ptsbe::fail(PTSBE_ERR_INVALID_ARG, "bad counts");
  void* ws = nullptr;
  ptsbe_status_t st = scratch_on(p->device, &ws);
  if (st != PTSBE_OK) return st;
  // the call's persistent arrays must fit beside at least one trajectory chunk
  // and one element chunk (the executor sizes its chunks to the rest)
  size_t need = 0;
  st = ptsbe_contract_workspace_size(plan, j, 1, 1, &need);
  if (st != PTSBE_OK) return st;
  if (need > kScratchBytes)
    return ptsbe::fail(PTSBE_ERR_UNSUPPORTED,
                       "ptsbe_contract_batch_noalloc: one trajectory of batch " + std::to_string(j) + " needs " +
                           std::to_string(need) + " bytes, more than the " + std::to_string(kScratchBytes) +
                           "-byte static scratch; use ptsbe_contract_batch with a workspace");
  st = ptsbe_contract_batch(plan, j, d_kraus_idx, E, d_elem_traj, d_elem_prefix, n_elems, out_kind, d_out,
                            d_elem_total, ws, kScratchBytes, stream);
  if (st == PTSBE_ERR_OUT_OF_MEMORY)
    return ptsbe::fail(PTSBE_ERR_UNSUPPORTED,
                       "ptsbe_contract_batch_noalloc: E = " + std::to_string(E) + " trajectories and n_elems = " +
                           std::to_string(n_elems) + " elements need more than the " + std::to_string(kScratchBytes) +
                           "-byte static scratch (" + ptsbe_last_error() +
                           "); use ptsbe_contract_batch with a workspace");
  return st;
}

}  // extern "C"
