// Kernels of the statevector method: batch marginals as partial sums over each
// trajectory's statevector (Sec. II-B, the marginal of batch j given the prefix
// is a sum of |psi|^2 over the later qubits), the last batch's amplitudes, and
// per-chunk element initialisation.  All of them are HBM-bound streams over the
// state; the gate windows themselves run in fused_inplace_kernel.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace ptsbe {
namespace {

constexpr int kSvThreads = 256;

__device__ inline double norm2(float2 v) { return (double)v.x * v.x + (double)v.y * v.y; }

__device__ inline const float2* elem_state(const SvMargArgs& a, int64_t e, uint64_t& s) {
  s = a.start > 0 ? (a.elem_prefix[e * a.NW] & ((1ull << a.start) - 1ull)) : 0ull;
  return a.psi + ((int64_t)(a.elem_traj[e] - a.traj_base) << a.n);
}

// 2^b >= 256: thread t owns the batch values x = t + 256 i (i < NX).  For a
// fixed later-qubit value y the workgroup reads 2^b amplitudes with stride
// 2^start (contiguous at the first batch).
template <int NX>
__global__ void __launch_bounds__(kSvThreads) sv_marg_wide_kernel(SvMargArgs a) {
  for (int64_t bid = blockIdx.x; bid < (a.n_elems << a.log_split); bid += gridDim.x) {
  const int64_t e = bid >> a.log_split;
  const int64_t sl = bid & (((int64_t)1 << a.log_split) - 1);
  const int tid = threadIdx.x;
  const int ybits = a.n - a.start - a.b;
  const int64_t ys = (int64_t)1 << (ybits - a.log_split);
  const int64_t y0 = sl * ys;
  uint64_t s;
  const float2* P = elem_state(a, e, s);
  const int sb = a.start + a.b;
  double acc[NX];
#pragma unroll
  for (int i = 0; i < NX; ++i) acc[i] = 0.0;
#pragma unroll 2
  for (int64_t y = y0; y < y0 + ys; ++y) {
    const float2* row = P + (y << sb) + s;
#pragma unroll
    for (int i = 0; i < NX; ++i) acc[i] += norm2(row[(int64_t)(tid + kSvThreads * i) << a.start]);
  }
  double* out = a.part + ((e << a.log_split) + sl) * ((int64_t)NX * kSvThreads);
#pragma unroll
  for (int i = 0; i < NX; ++i) out[tid + kSvThreads * i] = acc[i];
  }
}

// 2^b < 256: R = 256 / 2^b threads share a batch value x, striding over y;
// their partial sums are combined in a fixed order.
__global__ void __launch_bounds__(kSvThreads) sv_marg_narrow_kernel(SvMargArgs a) {
  __shared__ double red[kSvThreads];
  for (int64_t bid = blockIdx.x; bid < (a.n_elems << a.log_split); bid += gridDim.x) {
  const int64_t e = bid >> a.log_split;
  const int64_t sl = bid & (((int64_t)1 << a.log_split) - 1);
  const int tid = threadIdx.x;
  const int X = 1 << a.b, R = kSvThreads >> a.b;
  const int x = tid & (X - 1), r = tid >> a.b;
  const int ybits = a.n - a.start - a.b;
  const int64_t ys = (int64_t)1 << (ybits - a.log_split);
  const int64_t y0 = sl * ys;
  uint64_t s;
  const float2* P = elem_state(a, e, s);
  const int sb = a.start + a.b;
  double acc = 0.0;
  for (int64_t y = y0 + r; y < y0 + ys; y += R) acc += norm2(P[(y << sb) + ((int64_t)x << a.start) + s]);
  red[tid] = acc;
  __syncthreads();
  if (tid < X) {
    double t = 0.0;
    for (int k = 0; k < R; ++k) t += red[k * X + tid];
    a.part[((e << a.log_split) + sl) * X + tid] = t;
  }
  __syncthreads();
  }
}

__global__ void sv_pop_reduce_kernel(SvMargArgs a) {
  const int64_t X = (int64_t)1 << a.b;
  const int64_t ns = (int64_t)1 << a.log_split;
  for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < a.n_elems * X;
       id += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = id >> a.b, x = id & (X - 1);
    double t = 0.0;
    for (int64_t sl = 0; sl < ns; ++sl) t += a.part[((e << a.log_split) + sl) * X + x];
    a.pop[id] = (float)t;
  }
}

__global__ void sv_amp_kernel(SvMargArgs a, float2* amp) {
  const int64_t X = (int64_t)1 << a.b;
  for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < a.n_elems * X;
       id += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = id >> a.b, x = id & (X - 1);
    uint64_t s;
    const float2* P = elem_state(a, e, s);
    amp[id] = P[(x << a.start) + (int64_t)s];
  }
}

__global__ void init_traj_range_kernel(int64_t t0, int64_t count, const int64_t* m, const int64_t* base,
                                       int32_t* elem_traj, uint64_t* elem_prefix, int NW, int32_t* shot_off,
                                       int32_t* shot_cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t t = t0 + i;
  elem_traj[i] = (int32_t)t;
  for (int w = 0; w < NW; ++w) elem_prefix[i * NW + w] = 0ull;
  shot_off[i] = (int32_t)base[t];
  shot_cnt[i] = (int32_t)m[t];
}

}  // namespace

hipError_t launch_sv_marginal(const SvMargArgs& a, hipStream_t stream) {
  if (a.n_elems <= 0) return hipSuccess;
  if (a.b < 1 || a.b > 12 || a.start < 0 || a.start + a.b > a.n || a.log_split < 0 ||
      a.log_split > a.n - a.start - a.b || (a.n_elems << a.log_split) > a.part_rows)
    return hipErrorInvalidValue;
  const dim3 grid(grid_blocks(a.n_elems << a.log_split));
  switch (a.b) {
    case 8: hipLaunchKernelGGL(sv_marg_wide_kernel<1>, grid, dim3(kSvThreads), 0, stream, a); break;
    case 9: hipLaunchKernelGGL(sv_marg_wide_kernel<2>, grid, dim3(kSvThreads), 0, stream, a); break;
    case 10: hipLaunchKernelGGL(sv_marg_wide_kernel<4>, grid, dim3(kSvThreads), 0, stream, a); break;
    case 11: hipLaunchKernelGGL(sv_marg_wide_kernel<8>, grid, dim3(kSvThreads), 0, stream, a); break;
    case 12: hipLaunchKernelGGL(sv_marg_wide_kernel<16>, grid, dim3(kSvThreads), 0, stream, a); break;
    default: hipLaunchKernelGGL(sv_marg_narrow_kernel, grid, dim3(kSvThreads), 0, stream, a); break;
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int64_t total = a.n_elems << a.b;
  hipLaunchKernelGGL(sv_pop_reduce_kernel, dim3(grid_blocks((total + 255) / 256)), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_sv_amplitudes(const SvMargArgs& a, float2* amp, hipStream_t stream) {
  if (a.n_elems <= 0) return hipSuccess;
  if (a.start + a.b != a.n) return hipErrorInvalidValue;
  const int64_t total = a.n_elems << a.b;
  hipLaunchKernelGGL(sv_amp_kernel, dim3(grid_blocks((total + 255) / 256)), dim3(256), 0, stream, a, amp);
  return hipGetLastError();
}

hipError_t launch_init_traj_range(int64_t t0, int64_t count, const int64_t* shots_per_traj,
                                  const int64_t* traj_shot_base, int32_t* elem_traj, uint64_t* elem_prefix,
                                  int NW, int32_t* shot_off, int32_t* shot_cnt, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(init_traj_range_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream, t0, count,
                     shots_per_traj, traj_shot_base, elem_traj, elem_prefix, NW, shot_off, shot_cnt);
  return hipGetLastError();
}

}  // namespace ptsbe
