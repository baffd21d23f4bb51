// Kernels of the windowed adjoint contraction (reverse-mode derivatives of
// trajectory-averaged quantities through each trajectory's statevector; an
// addition to the paper's method that reuses its unified gate schedule and UPV
// merge).  The forward pass applies the gate windows of the statevector
// schedule out of place, so that the state after every window stays as a
// checkpoint.  The backward pass walks the windows in reverse: per 2^np tile it
// loads the state after the window and the adjoint state lambda, and for every
// op of the window (last first) forms psi_{k-1} and lambda_{k-1} = A_k^dag
// lambda_k in LDS, accumulating
//   rotation exp(-i theta P / 2):  d f / d theta = Im <lambda_{k-1}| P |psi_{k-1}>
//   gate-tensor adjoint:           N_k = sum_rest lambda_{k-1} psi_{k-1}^dag
// (M_k = U_k N_k is the derivative with respect to the conjugate of the bare
// gate U_k; the host multiplies by U_k, shared by all trajectories).  When every
// inserted operator is unitary, psi_{k-1} = A_k^dag psi_k; otherwise the tile is
// recomputed from the window's starting checkpoint up to op k-1.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.h"
#include "internal.h"

namespace ptsbe {
namespace {

constexpr int kAdjThreads = 256;

__device__ inline bool adj_czero(float2 v) { return v.x == 0.f && v.y == 0.f; }

// Offset of tile entry l (bit b of l -> window position P[b]) within the state.
__device__ inline uint32_t adj_local_offset(const AdjArgs& a, uint32_t l) {
  uint32_t off = 0;
#pragma unroll
  for (int b = 0; b < kFuseMax; ++b)
    if (b < a.np) off |= ((l >> b) & 1u) << a.P[b];
  return off;
}

__device__ inline uint32_t adj_tile_base(const AdjArgs& a, uint32_t t) {
  uint32_t out = 0, mask = a.other;
  for (int bit = 0; mask; ++bit, mask &= mask - 1u) out |= ((t >> bit) & 1u) << __builtin_ctz(mask);
  return out;
}

// g (d x d, staged, row-major over the op's local index: bit 0 <-> p0, bit 1 <-> p1)
// applied in place to the tile.  Ends with a barrier.
__device__ inline void adj_apply(const float2* __restrict__ g, int kind, int p0, int p1, uint32_t nt, float2* T) {
  if (kind == kSvOpGate1) {
    const float2 g00 = g[0], g01 = g[1], g10 = g[2], g11 = g[3];
    const uint32_t o = 1u << p0, lm = o - 1u;
    for (uint32_t m = threadIdx.x; m < (nt >> 1); m += kAdjThreads) {
      const uint32_t lb = ((m & ~lm) << 1) | (m & lm);
      const float2 a0 = T[lb], a1 = T[lb + o];
      T[lb] = cfma(g01, a1, cmul(g00, a0));
      T[lb + o] = cfma(g11, a1, cmul(g10, a0));
    }
  } else {
    float2 gm[4][4];
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int k = 0; k < 4; ++k) gm[n][k] = g[n * 4 + k];
    const uint32_t o1 = 1u << p0, o2 = 1u << p1, o3 = o1 | o2;
    const int pa = p0 < p1 ? p0 : p1, pb = p0 < p1 ? p1 : p0;
    const uint32_t ma = (1u << pa) - 1u, mb = (1u << pb) - 1u;
    for (uint32_t m = threadIdx.x; m < (nt >> 2); m += kAdjThreads) {
      uint32_t lb = ((m & ~ma) << 1) | (m & ma);
      lb = ((lb & ~mb) << 1) | (lb & mb);
      const float2 a0 = T[lb], a1 = T[lb + o1], a2 = T[lb + o2], a3 = T[lb + o3];
      const uint32_t off[4] = {0u, o1, o2, o3};
#pragma unroll
      for (int n = 0; n < 4; ++n)
        T[lb + off[n]] = cfma(gm[n][3], a3, cfma(gm[n][2], a2, cfma(gm[n][1], a1, cmul(gm[n][0], a0))));
    }
  }
  __syncthreads();
}

// Sum of v over the workgroup's threads in FP64 (wavefront shuffles, then the
// four wavefronts in a fixed order).  Every thread gets the sum.
__device__ inline double adj_block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// The op's accumulations from the tile pair (Lt = lambda_{k-1}, Pt = psi_{k-1}):
// the rotation derivative Im <L|P|Psi> (axis >= 0) into acc_rot, and, when nacc
// holds a slot, N_ab = sum_rest L_a conj(Psi_b) into acc_n (2 d^2 doubles).
__device__ inline void adj_accumulate(const AdjOp& op, uint32_t nt, const float2* Lt, const float2* Pt, double* red,
                                      double* acc_rot, double* acc_n, bool want_n) {
  const int d = op.kind == kSvOpGate1 ? 2 : 4;
  if (op.axis >= 0) {
    // <L| P |Psi> over pairs (lb, lb + o) of the rotation qubit
    const uint32_t o = 1u << op.p0, lm = o - 1u;
    float im = 0.f;
    for (uint32_t m = threadIdx.x; m < (nt >> 1); m += kAdjThreads) {
      const uint32_t lb = ((m & ~lm) << 1) | (m & lm);
      const float2 l0 = Lt[lb], l1 = Lt[lb + o], s0 = Pt[lb], s1 = Pt[lb + o];
      // P s: X (s1, s0); Y (-i s1, i s0); Z (s0, -s1); Im(conj(l) . Ps)
      float2 q0, q1;
      if (op.axis == 0) { q0 = s1; q1 = s0; }
      else if (op.axis == 1) { q0 = make_float2(s1.y, -s1.x); q1 = make_float2(-s0.y, s0.x); }
      else { q0 = s0; q1 = make_float2(-s1.x, -s1.y); }
      im += l0.x * q0.y - l0.y * q0.x + l1.x * q1.y - l1.y * q1.x;
    }
    const double t = adj_block_sum((double)im, red);
    if (threadIdx.x == 0) *acc_rot += t;
  }
  if (want_n && op.nslot >= 0) {
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        float re = 0.f, imv = 0.f;
        if (d == 2) {
          const uint32_t o = 1u << op.p0, lm = o - 1u;
          for (uint32_t m = threadIdx.x; m < (nt >> 1); m += kAdjThreads) {
            const uint32_t lb = ((m & ~lm) << 1) | (m & lm);
            const float2 l = Lt[lb + (a ? o : 0u)], s = Pt[lb + (b ? o : 0u)];
            re += l.x * s.x + l.y * s.y;       // l conj(s)
            imv += l.y * s.x - l.x * s.y;
          }
        } else {
          const uint32_t o1 = 1u << op.p0, o2 = 1u << op.p1;
          const int pa = op.p0 < op.p1 ? op.p0 : op.p1, pb = op.p0 < op.p1 ? op.p1 : op.p0;
          const uint32_t ma = (1u << pa) - 1u, mb = (1u << pb) - 1u;
          const uint32_t oa = ((a & 1) ? o1 : 0u) | ((a & 2) ? o2 : 0u), ob = ((b & 1) ? o1 : 0u) | ((b & 2) ? o2 : 0u);
          for (uint32_t m = threadIdx.x; m < (nt >> 2); m += kAdjThreads) {
            uint32_t lb = ((m & ~ma) << 1) | (m & ma);
            lb = ((lb & ~mb) << 1) | (lb & mb);
            const float2 l = Lt[lb + oa], s = Pt[lb + ob];
            re += l.x * s.x + l.y * s.y;
            imv += l.y * s.x - l.x * s.y;
          }
        }
        const double tr = adj_block_sum((double)re, red);
        const double ti = adj_block_sum((double)imv, red);
        if (threadIdx.x == 0) {
          acc_n[2 * (a * d + b)] += tr;
          acc_n[2 * (a * d + b) + 1] += ti;
        }
      }
  }
  __syncthreads();
}

// MODE 0: forward window, psi_out = A_window psi_in (out of place).
// MODE 1: backward window with psi_{k-1} = A_k^dag psi_k (unitary inserted operators);
//         psi_in = state after the window, lam in place.
// MODE 2: backward window with psi_{k-1} recomputed from psi_in = state before the window.
template <int MODE>
__global__ void __launch_bounds__(kAdjThreads) adj_window_kernel(AdjArgs a, const AdjOp* __restrict__ ops) {
  extern __shared__ float2 adj_lds[];
  const uint32_t nt = 1u << a.np;
  float2* T0 = adj_lds;                                  // psi (MODE 0, 1), window start (MODE 2)
  float2* T1 = T0 + nt;                                  // lambda (MODE 1, 2)
  float2* T2 = T1 + nt;                                  // psi_{k-1} (MODE 2)
  float2* Gf = (MODE == 1 ? T2 : (MODE == 2 ? T2 + nt : T1));   // forward gates [n_ops][16] (MODE 0, 2)
  float2* Gb = Gf + (MODE == 1 ? 0 : 16 * a.n_ops);      // adjoint gates [n_ops][16] (MODE 1, 2)
  double* red = reinterpret_cast<double*>(Gb + (MODE == 0 ? 0 : 16 * a.n_ops));   // [4]
  double* acc_rot = red + 4;                             // [n_ops] rotation derivatives of this workgroup
  double* acc_n = acc_rot + a.n_ops;                     // [n_nslots][32] gate adjoints of this workgroup
  const int tid = threadIdx.x;
  const int tb = a.n - a.np;
  const int64_t total = a.n_jobs << tb;
  const int64_t per = (total + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per, b1 = b0 + per < total ? b0 + per : total;
  if (MODE != 0) {
    for (int i = tid; i < a.n_ops + 32 * a.n_nslots; i += kAdjThreads) acc_rot[i] = 0.0;
  }
  __syncthreads();
  const uint32_t off_t = adj_local_offset(a, tid & (nt - 1));
  int64_t last_job = -1;
  for (int64_t bid = b0; bid < b1; ++bid) {
    const int64_t job = bid >> tb;
    const uint32_t base = adj_tile_base(a, (uint32_t)(bid & (((int64_t)1 << tb) - 1)));
    if (job != last_job) {
      const int traj = a.traj_base + (int)job;
      for (int i = tid; i < 16 * a.n_ops; i += kAdjThreads) {
        const AdjOp& op = ops[i >> 4];
        const int e = i & 15;
        const int d2 = op.kind == kSvOpGate1 ? 4 : 16;
        const int64_t gi = ((int64_t)traj * a.G + op.gate) * 16;
        if (MODE != 1) Gf[i] = e < d2 ? a.A[gi + op.idx[e]] : make_float2(0.f, 0.f);
        if (MODE != 0) Gb[i] = e < d2 ? a.Ad[gi + op.idx[e]] : make_float2(0.f, 0.f);
      }
      last_job = job;
    }
    const float2* Pin = a.psi_in + (job << a.n) + base;
    float2* Lg = MODE != 0 ? a.lam + (job << a.n) + base : nullptr;
    // entry l = tid + 256 i: the thread's bits and the iteration's bits land on
    // disjoint window positions, so off(l) = off_t | off(256 i)
    for (uint32_t l = tid; l < nt; l += kAdjThreads) {
      const uint32_t off = off_t | adj_local_offset(a, l - tid);
      T0[l] = Pin[off];
      if (MODE != 0) T1[l] = Lg[off];
    }
    __syncthreads();
    if (MODE == 0) {
      for (int k = 0; k < a.n_ops; ++k) adj_apply(Gf + 16 * k, ops[k].kind, ops[k].p0, ops[k].p1, nt, T0);
      float2* Po = a.psi_out + (job << a.n) + base;
      for (uint32_t l = tid; l < nt; l += kAdjThreads) Po[off_t | adj_local_offset(a, l - tid)] = T0[l];
    } else {
      for (int k = a.n_ops - 1; k >= 0; --k) {
        const AdjOp op = ops[k];
        float2* Ps = T0;
        if (MODE == 1) {
          adj_apply(Gb + 16 * k, op.kind, op.p0, op.p1, nt, T0);         // psi_{k-1}
        } else {
          for (uint32_t l = tid; l < nt; l += kAdjThreads) T2[l] = T0[l];
          __syncthreads();
          for (int q = 0; q < k; ++q) adj_apply(Gf + 16 * q, ops[q].kind, ops[q].p0, ops[q].p1, nt, T2);
          Ps = T2;
        }
        adj_apply(Gb + 16 * k, op.kind, op.p0, op.p1, nt, T1);           // lambda_{k-1}
        if (op.axis >= 0 || (a.want_n && op.nslot >= 0))
          adj_accumulate(op, nt, T1, Ps, red, acc_rot + k, acc_n + 32 * (op.nslot < 0 ? 0 : op.nslot), a.want_n);
      }
      for (uint32_t l = tid; l < nt; l += kAdjThreads) Lg[off_t | adj_local_offset(a, l - tid)] = T1[l];
    }
    __syncthreads();
  }
  if (MODE != 0) {
    // this workgroup's sums (zero if it had no tiles), in workgroup order
    double* out = a.wg_acc + (int64_t)blockIdx.x * (a.n_ops + 32 * a.n_nslots);
    for (int i = tid; i < a.n_ops + 32 * a.n_nslots; i += kAdjThreads) out[i] = acc_rot[i];
  }
}

// The diagonal of O = sum_t c_t Z_a Z_b over the 2^n basis states (once per call).
__global__ void adj_zz_diag_kernel(int n, const int32_t* __restrict__ zq, const double* __restrict__ zc, int n_terms,
                                   double* __restrict__ diag) {
  const int64_t per = (int64_t)1 << n;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < per; x += (int64_t)gridDim.x * blockDim.x) {
    double o = 0.0;
    for (int t = 0; t < n_terms; ++t) {
      const int za = 1 - 2 * (int)((x >> zq[2 * t]) & 1);
      const int zb = 1 - 2 * (int)((x >> zq[2 * t + 1]) & 1);
      o += zc[t] * (double)(za * zb);
    }
    diag[x] = o;
  }
}

// Seed of the backward pass for each trajectory of a chunk: lambda = w O psi (O
// diagonal), or the caller's psi-bar; and partial sums of <psi|O|psi>: slice k of
// kAdjSeedSlices of each trajectory's state is one workgroup, whose FP64 sum goes
// to part[job][k] (summed in slice order by adj_seed_sum_kernel).
constexpr int kAdjSeedSlices = 64;
__global__ void __launch_bounds__(256) adj_seed_kernel(AdjSeedArgs s) {
  __shared__ double red[256];
  const int64_t job = blockIdx.x / kAdjSeedSlices;
  const int k = blockIdx.x % kAdjSeedSlices;
  const int64_t per = (int64_t)1 << s.n;
  const int64_t len = per >= kAdjSeedSlices ? per / kAdjSeedSlices : (k == 0 ? per : 0);
  const int64_t x0 = (int64_t)k * len;
  const int64_t traj = s.traj_base + job;
  const float2* p = s.psi + job * per;
  float2* l = s.lam ? s.lam + job * per : nullptr;
  const float w = (float)s.weights[traj];
  double acc = 0.0;
  for (int64_t x = x0 + threadIdx.x; x < x0 + len; x += 256) {
    const double o = s.obs_diag[x];
    const float2 v = p[x];
    if (l) l[x] = s.psi_bar ? s.psi_bar[traj * per + x] : make_float2(w * (float)o * v.x, w * (float)o * v.y);
    acc += o * ((double)v.x * v.x + (double)v.y * v.y);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) s.part[job * kAdjSeedSlices + k] = red[0];
}

__global__ void adj_seed_sum_kernel(const double* __restrict__ part, int64_t n_jobs, int32_t traj_base,
                                    double* __restrict__ values) {
  for (int64_t job = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; job < n_jobs; job += (int64_t)gridDim.x * blockDim.x) {
    double t = 0.0;
    for (int k = 0; k < kAdjSeedSlices; ++k) t += part[job * kAdjSeedSlices + k];
    values[traj_base + job] = t;
  }
}

// Sum of the workgroups' accumulators of one backward window into the call's
// per-op totals, tot[i] += sum_wg wg_acc[wg][i]: one workgroup per entry i,
// strided partial sums in a fixed order and a fixed tree (deterministic).
__global__ void __launch_bounds__(256) adj_reduce_kernel(const double* __restrict__ wg_acc, int n_wg, int width,
                                                        double* __restrict__ tot) {
  __shared__ double red[256];
  for (int i = blockIdx.x; i < width; i += gridDim.x) {
    double s = 0.0;
    for (int w = threadIdx.x; w < n_wg; w += 256) s += wg_acc[(int64_t)w * width + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) tot[i] += red[0];
    __syncthreads();
  }
}

}  // namespace

size_t adj_window_lds_bytes(int mode, int np, int n_ops, int n_nslots) {
  const size_t nt = (size_t)1 << np;
  const size_t tiles = mode == 0 ? 1 : (mode == 1 ? 2 : 3);
  const size_t gates = (mode == 0 || mode == 1) ? 1 : 2;
  return tiles * nt * sizeof(float2) + gates * 16 * (size_t)n_ops * sizeof(float2) +
         (mode == 0 ? 0 : (4 + (size_t)n_ops + 32 * (size_t)n_nslots) * sizeof(double));
}

int adj_window_grid(int mode, size_t lds, int64_t tiles) {
  int per_cu = 0, dev = 0, cus = 0;
  hipError_t e = hipSuccess;
  if (mode == 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, adj_window_kernel<0>, kAdjThreads, lds);
  else if (mode == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, adj_window_kernel<1>, kAdjThreads, lds);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, adj_window_kernel<2>, kAdjThreads, lds);
  if (e != hipSuccess || hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return (int)std::min<int64_t>(tiles, (int64_t)std::max(per_cu, 1) * std::max(cus, 1));
}

hipError_t launch_adj_window(int mode, const AdjArgs& a, const AdjOp* d_ops, int grid, hipStream_t stream) {
  const size_t lds = adj_window_lds_bytes(mode, a.np, a.n_ops, a.n_nslots);
  if (mode == 0)
    hipLaunchKernelGGL(adj_window_kernel<0>, dim3(grid), dim3(kAdjThreads), lds, stream, a, d_ops);
  else if (mode == 1)
    hipLaunchKernelGGL(adj_window_kernel<1>, dim3(grid), dim3(kAdjThreads), lds, stream, a, d_ops);
  else
    hipLaunchKernelGGL(adj_window_kernel<2>, dim3(grid), dim3(kAdjThreads), lds, stream, a, d_ops);
  return hipGetLastError();
}

hipError_t launch_adj_zz_diag(int n, const int32_t* zq, const double* zc, int n_terms, double* diag,
                              hipStream_t stream) {
  const int64_t per = (int64_t)1 << n;
  hipLaunchKernelGGL(adj_zz_diag_kernel, dim3((unsigned)std::min<int64_t>((per + 255) / 256, 4096)), dim3(256), 0,
                     stream, n, zq, zc, n_terms, diag);
  return hipGetLastError();
}

hipError_t launch_adj_seed(const AdjSeedArgs& s, int64_t n_jobs, hipStream_t stream) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(adj_seed_kernel, dim3((unsigned)(n_jobs * kAdjSeedSlices)), dim3(256), 0, stream, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !s.values) return e;
  hipLaunchKernelGGL(adj_seed_sum_kernel, dim3((unsigned)std::min<int64_t>((n_jobs + 63) / 64, 1024)), dim3(64), 0,
                     stream, s.part, n_jobs, s.traj_base, s.values);
  return hipGetLastError();
}

hipError_t launch_adj_reduce(const double* wg_acc, int n_wg, int width, double* tot, hipStream_t stream) {
  if (width <= 0) return hipSuccess;
  hipLaunchKernelGGL(adj_reduce_kernel, dim3((unsigned)std::min(width, 4096)), dim3(256), 0, stream, wg_acc, n_wg,
                     width, tot);
  return hipGetLastError();
}

}  // namespace ptsbe
