// Gate windows of the statevector method (the ket network of a trajectory
// contracted in circuit order, Sec. III-A: one schedule shared by every
// trajectory, each applying its own UPV-merged gates).  A window is a set of at
// most 12 qubits, qubit 0 among them; every 2^np-amplitude tile of a state whose
// other bits are fixed is read from HBM once, all of the window's gates are
// applied to it in LDS, and it is written back.
//
// The ops of a window are read through the scalar cache (uniform loads), the gate
// matrices of a trajectory and its gate-cluster matrices are staged in LDS when
// a workgroup reaches a new trajectory, and tiles move as 16-byte pairs of
// amplitudes (qubit 0 is tile bit 0).  With PIPE the next tile's loads are issued
// before the current tile's ops, so that they are in flight during its LDS work.
//
// A gate cluster (a 16 x 16 complex matrix on four tile positions, the product
// of several gates built once per trajectory) is a real 32 x 32 by 32 x 2^(np-4)
// product on MFMA: FP32 (v_mfma_f32_16x16x4f32), or with hi + lo 16-bit operands
// (v_mfma_f32_16x16x32_bf16 / _f16, three products hi*hi + hi*lo + lo*hi, FP32
// accumulation; fp16 scales every column by a power of two).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.h"
#include "internal.h"
#include "sv_tile.h"

namespace ptsbe {
namespace {

template <int PREC, int NP, bool PIPE>
__global__ void __launch_bounds__(kSvwThreads) sv_window_kernel(SvwArgs a, const SvOp* __restrict__ ops,
                                                               const float2* __restrict__ merged,
                                                               const float2* __restrict__ Ucl,
                                                               float2* __restrict__ psi) {
  extern __shared__ floatx4_t svw_lds[];
  float2* tile = reinterpret_cast<float2*>(svw_lds);
  floatx4_t* tile4 = svw_lds;
  constexpr int np = NP, PPT = 1 << (NP - 9);     // pairs per thread
  const int n = a.n;
  float2* Gs = tile + (1 << NP);                   // [n_plain][16]
  float2* Us = Gs + 16 * a.n_plain;                // [n_cl][256]
  const int tid = threadIdx.x;
  const int tb = n - np;
  const int64_t total = a.n_jobs << tb;
  const int64_t per = (total + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per, b1 = b0 + per < total ? b0 + per : total;
  if (b0 >= b1) return;
  // this thread's pair offset from its own bits (tile bits 1..8 = positions P[1..8])
  const uint32_t lo = pair_lo(a.P), pt2 = swz(2u * tid);
  auto tile_base = [&](int64_t bid) -> uint32_t {   // the tile's other bits, spread over the non-window positions
    return deposit_other((uint32_t)(bid & (((int64_t)1 << tb) - 1)), a.other);
  };
  floatx4_t v[PPT];
  load_pairs<NP>(psi + ((b0 >> tb) << n) + tile_base(b0), a.P, lo, v);
  int64_t last_job = -1;
  for (int64_t bid = b0; bid < b1; ++bid) {
    const int64_t job = bid >> tb;
    if (job != last_job) {
      // stage the trajectory's gate matrices and cluster matrices (the previous
      // tile's last barrier has passed: nobody reads Gs / Us any more)
      const int traj = a.traj_base + (int)job;
      for (int s = 0; s < a.n_ops; ++s) {
        const int kind = ops[s].kind;
        if (kind == kSvOpCluster) continue;
        const int d2 = kind == kSvOpGate1 ? 4 : 16;
        if (tid < d2) {
          float2 g = merged[((int64_t)traj * a.G + ops[s].gate) * 16 + ops[s].idx[tid]];
          if (ops[s].conj) g.y = -g.y;
          Gs[16 * ops[s].slot + tid] = g;
        }
      }
      for (int i = tid; i < 256 * a.n_cl; i += kSvwThreads)
        Us[i] = Ucl[((int64_t)job * a.n_cl_total + a.cl_first) * 256 + i];
      last_job = job;
    }
#pragma unroll
    for (int i = 0; i < PPT; ++i) lds_put_pair(tile4, pt2, i, v[i]);
    __syncthreads();   // the tile (and any staging) is complete before the first op
    if (PIPE && bid + 1 < b1) load_pairs<NP>(psi + (((bid + 1) >> tb) << n) + tile_base(bid + 1), a.P, lo, v);
    for (int s = 0; s < a.n_ops; ++s) {
      // the op's first four dwords as one uniform (scalar-cache) load: kind, p0, p1,
      // conj | cluster positions | gate | slot
      const uint4 w = reinterpret_cast<const uint4*>(ops)[2 * s];
      const int kind = (int)(w.x & 0xffu), slot = (int)w.w;
      if (kind == kSvOpGate1) {
        apply_gate1<NP>(Gs + 16 * slot, (int)((w.x >> 8) & 0xffu), tile);
      } else if (kind == kSvOpGate2) {
        apply_gate2<NP>(Gs + 16 * slot, (int)((w.x >> 8) & 0xffu), (int)((w.x >> 16) & 0xffu), tile);
      } else {
        const ClusterCols cc(w.y);
        if (PREC == PTSBE_C64)
          apply_cluster_f32(cc, Us + 256 * slot, np, tile);
        else
          apply_cluster_split<PREC == PTSBE_C64 ? PTSBE_SPLIT_BF16 : PREC>(cc, Us + 256 * slot, np, tile);
      }
    }
    {
      const uint32_t base = tile_base(bid);
      float2* A = psi + (job << n) + base;
#pragma unroll
      for (int i = 0; i < PPT; ++i) *reinterpret_cast<floatx4_t*>(A + (lo | pair_hi<NP>(a.P, i))) = lds_get_pair(tile4, pt2, i);
    }
    __syncthreads();   // every thread has read its part of the tile before it is refilled
    if (!PIPE && bid + 1 < b1) load_pairs<NP>(psi + (((bid + 1) >> tb) << n) + tile_base(bid + 1), a.P, lo, v);
  }
}

}  // namespace

size_t sv_window_lds_bytes(const SvWin& w) {
  if (w.np < 10 || w.np > kFuseMax || w.P[0] != 0) return 0;
  return ((size_t)1 << w.np) * sizeof(float2) + (size_t)w.n_plain * 16 * sizeof(float2) +
         (size_t)w.n_cl * 256 * sizeof(float2);
}

hipError_t launch_sv_window(const SvWin& w, const SvOp* d_ops, const float2* merged, int G, const float2* Ucl,
                            int n_cl_total, int64_t n_jobs, int32_t traj_base, float2* psi, int n, int precision,
                            hipStream_t stream) {
  if (n_jobs <= 0 || w.n_ops == 0) return hipSuccess;
  const size_t lds = sv_window_lds_bytes(w);
  if (lds == 0 || lds > 64 * 1024) return hipErrorInvalidValue;
  SvwArgs a{};
  a.n = n;
  a.np = w.np;
  a.n_ops = w.n_ops;
  a.n_plain = w.n_plain;
  a.n_cl = w.n_cl;
  a.cl_first = w.cl_first;
  a.n_cl_total = n_cl_total;
  a.G = G;
  for (int k = 0; k < kFuseMax; ++k) a.P[k] = w.P[k];
  a.other = w.other;
  a.n_jobs = n_jobs;
  a.traj_base = traj_base;
  const int64_t total = n_jobs << (n - w.np);
  const SvOp* ops = d_ops + w.op_off;
  auto go = [&](auto kernel) -> hipError_t {
    // one resident generation of workgroups, each walking a contiguous range of tiles
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kSvwThreads, lds);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int64_t resident = (int64_t)std::max(per_cu, 1) * std::max(cus, 1);
    const dim3 grid((unsigned)std::min<int64_t>(total, resident));
    hipLaunchKernelGGL(kernel, grid, dim3(kSvwThreads), lds, stream, a, ops, merged, Ucl, psi);
    return hipGetLastError();
  };
  auto by_np = [&](auto k10, auto k11, auto k12) { return w.np == 10 ? go(k10) : w.np == 11 ? go(k11) : go(k12); };
  if (precision == PTSBE_SPLIT_BF16)
    return by_np(sv_window_kernel<PTSBE_SPLIT_BF16, 10, true>, sv_window_kernel<PTSBE_SPLIT_BF16, 11, true>,
                 sv_window_kernel<PTSBE_SPLIT_BF16, 12, true>);
  if (precision == PTSBE_SPLIT_F16)
    return by_np(sv_window_kernel<PTSBE_SPLIT_F16, 10, true>, sv_window_kernel<PTSBE_SPLIT_F16, 11, true>,
                 sv_window_kernel<PTSBE_SPLIT_F16, 12, true>);
  return by_np(sv_window_kernel<PTSBE_C64, 10, true>, sv_window_kernel<PTSBE_C64, 11, true>,
               sv_window_kernel<PTSBE_C64, 12, true>);
}

}  // namespace ptsbe
