// Helper kernels of the adjoint contraction: the merged gates A = S U(theta)
// and their adjoints for every (trajectory, gate), state initialisation, copies
// and the weighted value sum (the window passes are in adj_kernels.hip).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace ptsbe {
namespace {

__device__ inline float2 cfma2(float2 a, float2 b, float2 c) {
  return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}

// M (d x d) = S . B where S is the product of the gate's inserted operators for
// trajectory traj (later sites on the left) and B a d x d matrix (row-major).
__device__ void site_product_times(const GateCtx& g, int gate, int traj, const float2* B, float2* out) {
  const DeviceGate* G = g.gates + gate;
  const int d = G->arity == 2 ? 4 : 2;
  float2 m[16], t[16];
  for (int i = 0; i < 16; ++i) m[i] = i < d * d ? B[i] : make_float2(0.f, 0.f);
  const uint8_t* kr = g.kraus + (int64_t)traj * g.S;
  for (int s = G->site_begin; s < G->site_end; ++s) {
    const int site = g.gate_site_list[s];
    const float2* op = g.site_ops + ((int64_t)site * g.max_kraus + kr[site]) * 16;
    for (int r = 0; r < d; ++r)
      for (int c = 0; c < d; ++c) {
        float2 acc = make_float2(0.f, 0.f);
        for (int x = 0; x < d; ++x) acc = cfma2(op[r * d + x], m[x * d + c], acc);
        t[r * d + c] = acc;
      }
    for (int i = 0; i < d * d; ++i) m[i] = t[i];
  }
  for (int i = 0; i < 16; ++i) out[i] = m[i];
}

// Rotation exp(-i theta P / 2) and its theta-derivative (2x2, row-major).
__device__ void rotation_pair(int axis, double theta, float2* U, float2* dU) {
  const double c = cos(0.5 * theta), s = sin(0.5 * theta);
  // U = c I - i s P ; dU = -(s/2) I - i (c/2) P
  double P[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // interleaved 2x2 complex
  if (axis == 0) { P[2] = 1; P[4] = 1; }
  else if (axis == 1) { P[3] = -1; P[5] = 1; }
  else { P[0] = 1; P[6] = -1; }
  for (int i = 0; i < 4; ++i) {
    const double id = (i == 0 || i == 3) ? 1.0 : 0.0;
    const double pr = P[2 * i], pi = P[2 * i + 1];
    // -i * (a + i b) = b - i a
    U[i] = make_float2((float)(c * id + s * pi), (float)(-s * pr));
    dU[i] = make_float2((float)(-0.5 * s * id + 0.5 * c * pi), (float)(-0.5 * c * pr));
  }
}

__global__ void grad_gates_kernel(GradGateArgs a) {
  for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < a.E * a.g.G; id += (int64_t)gridDim.x * blockDim.x) {
    const int traj = (int)(id / a.g.G), gate = (int)(id % a.g.G);
    const DeviceGate* G = a.g.gates + gate;
    const int d = G->arity == 2 ? 4 : 2;
    float2 base[16], m[16];
    const int prm = a.gate_param[gate];
    float2 dU[4];
    if (prm >= 0) {
      rotation_pair(a.gate_axis[gate], a.theta[prm], base, dU);
    } else {
      for (int i = 0; i < 16; ++i) base[i] = G->raw[i];
    }
    site_product_times(a.g, gate, traj, base, m);
    float2* o = a.merged + id * 16;
    float2* od = a.dagger + id * 16;
    for (int i = 0; i < 16; ++i) o[i] = m[i];
    for (int r = 0; r < 16; ++r) od[r] = make_float2(0.f, 0.f);
    for (int r = 0; r < d; ++r)
      for (int c = 0; c < d; ++c) {
        const float2 v = m[c * d + r];
        od[r * d + c] = make_float2(v.x, -v.y);
      }
    const int slot = a.gate_slot[gate];
    if (slot >= 0) {
      float2 dm[16];
      site_product_times(a.g, gate, traj, dU, dm);
      float2* odm = a.dmerged + ((int64_t)traj * a.n_slots + slot) * 16;
      for (int i = 0; i < 16; ++i) odm[i] = dm[i];
    }
  }
}

__global__ void state_init_kernel(float2* psi, int64_t n_jobs, int n) {
  const int64_t per = (int64_t)1 << n;
  for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < per * n_jobs; id += (int64_t)gridDim.x * blockDim.x) {
    psi[id] = make_float2((id % per) == 0 ? 1.f : 0.f, 0.f);
  }
}

__global__ void copy_kernel(const float2* __restrict__ src, float2* __restrict__ dst, int64_t n) {
  for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < n; id += (int64_t)gridDim.x * blockDim.x)
    dst[id] = src[id];
}

__global__ void value_sum_kernel(const double* __restrict__ vals, const double* __restrict__ w, int64_t E,
                                 double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < E; t += 256) acc += w[t] * vals[t];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int wd = 128; wd > 0; wd >>= 1) {
    if ((int)threadIdx.x < wd) red[threadIdx.x] += red[threadIdx.x + wd];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// dst[j] = src[idx[j]] for rows of `len` entries (len a power of two, 2^lb).
__global__ void gather_rows_kernel(const float2* __restrict__ src, const int32_t* __restrict__ idx,
                                   float2* __restrict__ dst, int64_t total, int lb) {
  const int64_t len = (int64_t)1 << lb;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[(int64_t)idx[i >> lb] * len + (i & (len - 1))];
}

}  // namespace

hipError_t launch_gather_rows(const float2* src, const int32_t* idx, float2* dst, int64_t n_rows, int row_bits,
                              hipStream_t stream) {
  const int64_t total = n_rows << row_bits;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_blocks((total + 255) / 256)), dim3(256), 0, stream, src, idx, dst,
                     total, row_bits);
  return hipGetLastError();
}

hipError_t launch_grad_gates(const GradGateArgs& a, hipStream_t stream) {
  const int64_t n = a.E * a.g.G;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(grad_gates_kernel, dim3(grid_blocks((n + 127) / 128)), dim3(128), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_state_init(float2* psi, int64_t n_jobs, int n, hipStream_t stream) {
  const int64_t total = n_jobs << n;
  hipLaunchKernelGGL(state_init_kernel, dim3(grid_blocks((total + 255) / 256)), dim3(256), 0, stream, psi, n_jobs, n);
  return hipGetLastError();
}

hipError_t launch_copy(const float2* src, float2* dst, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_kernel, dim3(grid_blocks((n + 255) / 256)), dim3(256), 0, stream, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_value_sum(const double* vals, const double* w, int64_t E, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(value_sum_kernel, dim3(1), dim3(256), 0, stream, vals, w, E, out);
  return hipGetLastError();
}

}  // namespace ptsbe
