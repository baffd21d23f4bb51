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
#include "sv_tile.h"

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

// ---------------------------------------------------------------------------
// Tile kernels for windows of 10..12 qubits with qubit 0 at tile bit 0 (the
// statevector window layout): 16-byte amplitude pairs between HBM and a swizzled
// LDS tile, ops read through the scalar cache.
//
__device__ inline float adj_wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Im(conj(l) . P s) summed over the pair (s0, s1), (l0, l1) of the rotation qubit,
// P = X, Y, Z by axis 0, 1, 2.
__device__ inline float adj_rot_term(int axis, float2 l0, float2 l1, float2 s0, float2 s1) {
  float2 q0, q1;
  if (axis == 0) { q0 = s1; q1 = s0; }
  else if (axis == 1) { q0 = make_float2(s1.y, -s1.x); q1 = make_float2(-s0.y, s0.x); }
  else { q0 = s0; q1 = make_float2(-s1.x, -s1.y); }
  return l0.x * q0.y - l0.y * q0.x + l1.x * q1.y - l1.y * q1.x;
}

// Backward window with psi_{k-1} = A_k^dag psi_k (every inserted operator
// unitary): per tile, psi (the state after the window) and lambda in LDS; for each
// op, last first, one pass applies A_k^dag to both at the op's pairs or quads and
// accumulates, in registers, the rotation derivative Im <lambda_{k-1}|P|psi_{k-1}>
// and (WN) the gate adjoint N_ab = sum lambda_{k-1,a} conj(psi_{k-1,b}) from the
// same amplitudes.  Per op the thread sums are reduced over each wavefront with
// shuffles, the four wavefronts' sums are added in a fixed order after the op's
// barrier (double-buffered by op parity) into FP64 workgroup accumulators.
template <int NP, bool WN>
__global__ void __launch_bounds__(kSvwThreads) adj_bwd_tile_kernel(AdjArgs a, const AdjOp* __restrict__ ops) {
  constexpr int PPT = 1 << (NP - 9);
  constexpr uint32_t nt = 1u << NP;
  extern __shared__ floatx4_t adj_lds4[];
  float2* T0 = reinterpret_cast<float2*>(adj_lds4);      // psi
  float2* T1 = T0 + nt;                                  // lambda
  float2* Gb = T1 + nt;                                  // [n_ops][16] adjoint matrices
  double* red = reinterpret_cast<double*>(Gb + 16 * a.n_ops);   // [2][4][33] wavefront sums
  double* acc = red + 2 * 4 * 33;                        // [n_ops + 32 n_nslots]
  floatx4_t* T04 = reinterpret_cast<floatx4_t*>(T0);
  floatx4_t* T14 = reinterpret_cast<floatx4_t*>(T1);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int width = a.n_ops + 32 * a.n_nslots;
  const int tb = a.n - NP;
  const int64_t total = a.n_jobs << tb;
  const int64_t per = (total + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per, b1 = b0 + per < total ? b0 + per : total;
  for (int i = tid; i < width; i += kSvwThreads) acc[i] = 0.0;
  const uint32_t lo = pair_lo(a.P), pt2 = swz(2u * tid);
  int64_t last_job = -1;
  for (int64_t bid = b0; bid < b1; ++bid) {
    const int64_t job = bid >> tb;
    if (job != last_job) {
      const int traj = a.traj_base + (int)job;
      for (int i = tid; i < 16 * a.n_ops; i += kSvwThreads) {
        const AdjOp& op = ops[i >> 4];
        const int e = i & 15, d2 = op.kind == kSvOpGate1 ? 4 : 16;
        Gb[i] = e < d2 ? a.Ad[((int64_t)traj * a.G + op.gate) * 16 + op.idx[e]] : make_float2(0.f, 0.f);
      }
      last_job = job;
    }
    const uint32_t base = deposit_other((uint32_t)(bid & (((int64_t)1 << tb) - 1)), a.other);
    const float2* Pin = a.psi_in + (job << a.n) + base;
    float2* Lg = a.lam + (job << a.n) + base;
    {
      floatx4_t v[PPT], w[PPT];
      load_pairs<NP>(Pin, a.P, lo, v);
      load_pairs<NP>(Lg, a.P, lo, w);
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        lds_put_pair(T04, pt2, i, v[i]);
        lds_put_pair(T14, pt2, i, w[i]);
      }
    }
    __syncthreads();
    for (int k = a.n_ops - 1; k >= 0; --k) {
      const uint4 wd = reinterpret_cast<const uint4*>(ops)[2 * k];
      const int kind = (int)(wd.x & 0xffu), p0 = (int)((wd.x >> 8) & 0xffu), p1 = (int)((wd.x >> 16) & 0xffu);
      const int axis = (int)(int8_t)((wd.x >> 24) & 0xffu), nslot = (int)wd.z;
      const bool take_n = WN && nslot >= 0;
      const float2* g = Gb + 16 * k;
      float rot = 0.f;
      float nac[32];
      if (WN) {
#pragma unroll
        for (int i = 0; i < 32; ++i) nac[i] = 0.f;
      }
      int cnt = 0;   // sums this op reduces: rotation first, then 2 d^2 entries of N
      if (kind == kSvOpGate1) {
        const float2 g00 = g[0], g01 = g[1], g10 = g[2], g11 = g[3];
        const uint32_t pt = swz(ins0(tid, p0)), so = swz(1u << p0);
#pragma unroll 2
        for (uint32_t i = 0; i < (nt >> 1) / kSvwThreads; ++i) {
          const uint32_t l0 = pt ^ swz(ins0(kSvwThreads * i, p0)), l1 = l0 ^ so;
          const float2 a0 = T0[l0], a1 = T0[l1], c0 = T1[l0], c1 = T1[l1];
          const float2 s0 = cfma(g01, a1, cmul(g00, a0)), s1 = cfma(g11, a1, cmul(g10, a0));
          const float2 m0 = cfma(g01, c1, cmul(g00, c0)), m1 = cfma(g11, c1, cmul(g10, c0));
          T0[l0] = s0;
          T0[l1] = s1;
          T1[l0] = m0;
          T1[l1] = m1;
          if (axis >= 0) rot += adj_rot_term(axis, m0, m1, s0, s1);
          if (take_n) {
            const float2 L[2] = {m0, m1}, S[2] = {s0, s1};
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
              for (int y = 0; y < 2; ++y) {
                nac[2 * (x * 2 + y)] += L[x].x * S[y].x + L[x].y * S[y].y;       // l conj(s)
                nac[2 * (x * 2 + y) + 1] += L[x].y * S[y].x - L[x].x * S[y].y;
              }
          }
        }
        cnt = take_n ? 9 : 1;
      } else {
        float2 gm[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) gm[x][y] = g[x * 4 + y];
        const int pa = p0 < p1 ? p0 : p1, pb = p0 < p1 ? p1 : p0;
        const uint32_t pt = swz(ins0(ins0(tid, pa), pb));
        const uint32_t s1 = swz(1u << p0), s2 = swz(1u << p1), s3 = s1 ^ s2;
#pragma unroll 2
        for (uint32_t i = 0; i < (nt >> 2) / kSvwThreads; ++i) {
          const uint32_t lb = pt ^ swz(ins0(ins0(kSvwThreads * i, pa), pb));
          const uint32_t off[4] = {lb, lb ^ s1, lb ^ s2, lb ^ s3};
          float2 A[4], C[4], S[4], L[4];
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            A[x] = T0[off[x]];
            C[x] = T1[off[x]];
          }
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            S[x] = cfma(gm[x][3], A[3], cfma(gm[x][2], A[2], cfma(gm[x][1], A[1], cmul(gm[x][0], A[0]))));
            L[x] = cfma(gm[x][3], C[3], cfma(gm[x][2], C[2], cfma(gm[x][1], C[1], cmul(gm[x][0], C[0]))));
          }
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            T0[off[x]] = S[x];
            T1[off[x]] = L[x];
          }
          if (take_n) {
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
              for (int y = 0; y < 4; ++y) {
                nac[2 * (x * 4 + y)] += L[x].x * S[y].x + L[x].y * S[y].y;
                nac[2 * (x * 4 + y) + 1] += L[x].y * S[y].x - L[x].x * S[y].y;
              }
          }
        }
        cnt = take_n ? 33 : 0;
      }
      // wavefront sums into this op's staging slot (parity k & 1)
      double* rs = red + (k & 1) * 4 * 33 + wave * 33;
      if (axis >= 0) {
        const float t = adj_wave_sum(rot);
        if (lane == 0) rs[0] = (double)t;
      }
      if (take_n) {
        const int m = kind == kSvOpGate1 ? 8 : 32;
#pragma unroll
        for (int i = 0; i < 32; ++i) {
          if (i < m) {
            const float t = adj_wave_sum(nac[i]);
            if (lane == 0) rs[1 + i] = (double)t;
          }
        }
      }
      __syncthreads();   // the op's tiles and wavefront sums are complete
      if (tid < cnt && (tid > 0 || axis >= 0)) {
        const double* r0 = red + (k & 1) * 4 * 33;
        const double t = r0[tid] + r0[33 + tid] + r0[66 + tid] + r0[99 + tid];
        if (tid == 0) acc[k] += t;
        else acc[a.n_ops + 32 * nslot + (tid - 1)] += t;
      }
    }
#pragma unroll
    for (int i = 0; i < PPT; ++i)
      *reinterpret_cast<floatx4_t*>(Lg + (lo | pair_hi<NP>(a.P, i))) = lds_get_pair(T14, pt2, i);
    __syncthreads();   // every thread has read its part of lambda, and acc is complete
  }
  __syncthreads();
  double* out = a.wg_acc + (int64_t)blockIdx.x * width;
  for (int i = tid; i < width; i += kSvwThreads) out[i] = acc[i];
}

// ---------------------------------------------------------------------------
// Group passes: the ops of one group (at most kAdjGroupMax consecutive ops on at
// most two tile positions, build_adj_groups) are applied in one pass over the
// tile, each thread holding its pairs (one position) or quads (two positions)
// in registers from one LDS read to one LDS write, with one barrier per group
// instead of one per op.

// 2 x 2 matrix (g00 g01; g10 g11) on the pair (x0, x1).
__device__ inline void adj_g2(float2 g00, float2 g01, float2 g10, float2 g11, float2& x0, float2& x1) {
  const float2 a0 = x0, a1 = x1;
  x0 = cfma(g01, a1, cmul(g00, a0));
  x1 = cfma(g11, a1, cmul(g10, a0));
}

// 4 x 4 matrix gm on a quad held in tile-position order (bit 0 <-> pa, bit 1 <->
// pb); sw: the op's local bit 0 is pb (its index bits are swapped).
__device__ inline void adj_g4(const float2 (&gm)[4][4], bool sw, float2 (&q)[4]) {
  const float2 x0 = q[0], x1 = sw ? q[2] : q[1], x2 = sw ? q[1] : q[2], x3 = q[3];
  float2 y[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) y[r] = cfma(gm[r][3], x3, cfma(gm[r][2], x2, cfma(gm[r][1], x1, cmul(gm[r][0], x0))));
  q[0] = y[0];
  q[1] = sw ? y[2] : y[1];
  q[2] = sw ? y[1] : y[2];
  q[3] = y[3];
}

// Forward window, one group pass per group: psi_out = A_window psi_in per tile.
template <int NP>
__global__ void __launch_bounds__(kSvwThreads) adj_fwd_group_kernel(AdjArgs a, const AdjOp* __restrict__ ops) {
  constexpr int PPT = 1 << (NP - 9);
  constexpr uint32_t nt = 1u << NP;
  constexpr int NPR = (nt >> 1) / kSvwThreads, NQD = (nt >> 2) / kSvwThreads;
  extern __shared__ floatx4_t adj_lds4[];
  float2* T0 = reinterpret_cast<float2*>(adj_lds4);
  float2* Gf = T0 + nt;                                  // [n_ops][16]
  floatx4_t* T04 = adj_lds4;
  const int tid = threadIdx.x;
  const int tb = a.n - NP;
  const int64_t total = a.n_jobs << tb;
  const int64_t per = (total + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per, b1 = b0 + per < total ? b0 + per : total;
  const uint32_t lo = pair_lo(a.P), pt2 = swz(2u * tid);
  int64_t last_job = -1;
  for (int64_t bid = b0; bid < b1; ++bid) {
    const int64_t job = bid >> tb;
    if (job != last_job) {
      // the previous tile ended with a barrier: nobody reads Gf any more
      const int traj = a.traj_base + (int)job;
      for (int i = tid; i < 16 * a.n_ops; i += kSvwThreads) {
        const AdjOp& op = ops[i >> 4];
        const int e = i & 15, d2 = op.kind == kSvOpGate1 ? 4 : 16;
        Gf[i] = e < d2 ? a.A[((int64_t)traj * a.G + op.gate) * 16 + op.idx[e]] : make_float2(0.f, 0.f);
      }
      last_job = job;
    }
    const uint32_t base = deposit_other((uint32_t)(bid & (((int64_t)1 << tb) - 1)), a.other);
    {
      floatx4_t v[PPT];
      load_pairs<NP>(a.psi_in + (job << a.n) + base, a.P, lo, v);
#pragma unroll
      for (int i = 0; i < PPT; ++i) lds_put_pair(T04, pt2, i, v[i]);
    }
    __syncthreads();
    for (int gi = 0; gi < a.n_groups; ++gi) {
      const uint4 gd = reinterpret_cast<const uint4*>(a.groups)[gi];
      const int nq = (int)(gd.x & 0xffu), pa = (int)((gd.x >> 8) & 0xffu), pb = (int)((gd.x >> 16) & 0xffu);
      const int cnt = (int)((gd.x >> 24) & 0xffu), first = (int)gd.y;
      if (nq == 1) {
        const uint32_t pt = swz(ins0(tid, pa)), so = swz(1u << pa);
        float2 X0[NPR], X1[NPR];
#pragma unroll
        for (int i = 0; i < NPR; ++i) {
          const uint32_t l0 = pt ^ swz(ins0(kSvwThreads * i, pa));
          X0[i] = T0[l0];
          X1[i] = T0[l0 ^ so];
        }
#pragma unroll 1
        for (int j = 0; j < cnt; ++j) {
          const float2* g = Gf + 16 * (first + j);
          const float2 g00 = g[0], g01 = g[1], g10 = g[2], g11 = g[3];
#pragma unroll
          for (int i = 0; i < NPR; ++i) adj_g2(g00, g01, g10, g11, X0[i], X1[i]);
        }
#pragma unroll
        for (int i = 0; i < NPR; ++i) {
          const uint32_t l0 = pt ^ swz(ins0(kSvwThreads * i, pa));
          T0[l0] = X0[i];
          T0[l0 ^ so] = X1[i];
        }
      } else {
        const uint32_t pt = swz(ins0(ins0(tid, pa), pb)), s1 = swz(1u << pa), s2 = swz(1u << pb);
        float2 X[NQD][4];
#pragma unroll
        for (int i = 0; i < NQD; ++i) {
          const uint32_t lb = pt ^ swz(ins0(ins0(kSvwThreads * i, pa), pb));
          X[i][0] = T0[lb];
          X[i][1] = T0[lb ^ s1];
          X[i][2] = T0[lb ^ s2];
          X[i][3] = T0[lb ^ s1 ^ s2];
        }
#pragma unroll 1
        for (int j = 0; j < cnt; ++j) {
          const int k = first + j;
          const uint4 w = reinterpret_cast<const uint4*>(ops)[2 * k];
          const int kind = (int)(w.x & 0xffu), p0 = (int)((w.x >> 8) & 0xffu);
          const float2* g = Gf + 16 * k;
          if (kind == kSvOpGate1) {
            const float2 g00 = g[0], g01 = g[1], g10 = g[2], g11 = g[3];
            const bool hi = p0 != pa;   // the op's qubit is quad bit 1
#pragma unroll
            for (int i = 0; i < NQD; ++i) {
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                const int e0 = hi ? h : 2 * h, e1 = hi ? h + 2 : 2 * h + 1;
                adj_g2(g00, g01, g10, g11, X[i][e0], X[i][e1]);
              }
            }
          } else {
            float2 gm[4][4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
              for (int c = 0; c < 4; ++c) gm[r][c] = g[r * 4 + c];
            const bool sw = p0 != pa;
#pragma unroll
            for (int i = 0; i < NQD; ++i) adj_g4(gm, sw, X[i]);
          }
        }
#pragma unroll
        for (int i = 0; i < NQD; ++i) {
          const uint32_t lb = pt ^ swz(ins0(ins0(kSvwThreads * i, pa), pb));
          T0[lb] = X[i][0];
          T0[lb ^ s1] = X[i][1];
          T0[lb ^ s2] = X[i][2];
          T0[lb ^ s1 ^ s2] = X[i][3];
        }
      }
      __syncthreads();
    }
    {
      float2* Po = a.psi_out + (job << a.n) + base;
#pragma unroll
      for (int i = 0; i < PPT; ++i)
        *reinterpret_cast<floatx4_t*>(Po + (lo | pair_hi<NP>(a.P, i))) = lds_get_pair(T04, pt2, i);
    }
    __syncthreads();
  }
}

// Backward window with unitary inserted operators, one group pass per group (in
// reverse): each thread holds psi and lambda at its pairs or quads, applies the
// group's A_k^dag last op first, and sums each rotation's
// Im <lambda_{k-1}|P|psi_{k-1}> over its amplitudes, then over the wavefront
// (shuffles, no barrier); after the group's barrier the four wavefronts' sums are
// added in a fixed order (staging double-buffered by group parity).
template <int NP>
__global__ void __launch_bounds__(kSvwThreads) adj_bwd_group_kernel(AdjArgs a, const AdjOp* __restrict__ ops) {
  constexpr int PPT = 1 << (NP - 9);
  constexpr uint32_t nt = 1u << NP;
  constexpr int NPR = (nt >> 1) / kSvwThreads, NQD = (nt >> 2) / kSvwThreads;
  extern __shared__ floatx4_t adj_lds4[];
  float2* T0 = reinterpret_cast<float2*>(adj_lds4);      // psi
  float2* T1 = T0 + nt;                                  // lambda
  float2* Gb = T1 + nt;                                  // [n_ops][16] adjoint matrices
  double* red = reinterpret_cast<double*>(Gb + 16 * a.n_ops);   // [2][4][kAdjGroupMax]
  double* acc = red + 2 * 4 * 33;                        // [n_ops] (the same layout bound as the per-op kernel)
  floatx4_t* T04 = reinterpret_cast<floatx4_t*>(T0);
  floatx4_t* T14 = reinterpret_cast<floatx4_t*>(T1);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tb = a.n - NP;
  const int64_t total = a.n_jobs << tb;
  const int64_t per = (total + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per, b1 = b0 + per < total ? b0 + per : total;
  for (int i = tid; i < a.n_ops; i += kSvwThreads) acc[i] = 0.0;
  const uint32_t lo = pair_lo(a.P), pt2 = swz(2u * tid);
  int64_t last_job = -1;
  for (int64_t bid = b0; bid < b1; ++bid) {
    const int64_t job = bid >> tb;
    if (job != last_job) {
      const int traj = a.traj_base + (int)job;
      for (int i = tid; i < 16 * a.n_ops; i += kSvwThreads) {
        const AdjOp& op = ops[i >> 4];
        const int e = i & 15, d2 = op.kind == kSvOpGate1 ? 4 : 16;
        Gb[i] = e < d2 ? a.Ad[((int64_t)traj * a.G + op.gate) * 16 + op.idx[e]] : make_float2(0.f, 0.f);
      }
      last_job = job;
    }
    const uint32_t base = deposit_other((uint32_t)(bid & (((int64_t)1 << tb) - 1)), a.other);
    float2* Lg = a.lam + (job << a.n) + base;
    {
      floatx4_t v[PPT], w[PPT];
      load_pairs<NP>(a.psi_in + (job << a.n) + base, a.P, lo, v);
      load_pairs<NP>(Lg, a.P, lo, w);
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        lds_put_pair(T04, pt2, i, v[i]);
        lds_put_pair(T14, pt2, i, w[i]);
      }
    }
    __syncthreads();
    for (int gi = a.n_groups - 1; gi >= 0; --gi) {
      const uint4 gd = reinterpret_cast<const uint4*>(a.groups)[gi];
      const int nq = (int)(gd.x & 0xffu), pa = (int)((gd.x >> 8) & 0xffu), pb = (int)((gd.x >> 16) & 0xffu);
      const int cnt = (int)((gd.x >> 24) & 0xffu), first = (int)gd.y;
      double* rs = red + (gi & 1) * 4 * kAdjGroupMax + wave * kAdjGroupMax;   // wavefront sums, by op
      if (nq == 1) {
        const uint32_t pt = swz(ins0(tid, pa)), so = swz(1u << pa);
        float2 S0[NPR], S1[NPR], L0[NPR], L1[NPR];
#pragma unroll
        for (int i = 0; i < NPR; ++i) {
          const uint32_t l0 = pt ^ swz(ins0(kSvwThreads * i, pa));
          S0[i] = T0[l0];
          S1[i] = T0[l0 ^ so];
          L0[i] = T1[l0];
          L1[i] = T1[l0 ^ so];
        }
#pragma unroll 1
        for (int j = cnt - 1; j >= 0; --j) {
          const int k = first + j;
          const uint4 w = reinterpret_cast<const uint4*>(ops)[2 * k];
          const int axis = (int)(int8_t)((w.x >> 24) & 0xffu);
          const float2* g = Gb + 16 * k;
          const float2 g00 = g[0], g01 = g[1], g10 = g[2], g11 = g[3];
          float rot = 0.f;
#pragma unroll
          for (int i = 0; i < NPR; ++i) {
            adj_g2(g00, g01, g10, g11, S0[i], S1[i]);
            adj_g2(g00, g01, g10, g11, L0[i], L1[i]);
            if (axis >= 0) rot += adj_rot_term(axis, L0[i], L1[i], S0[i], S1[i]);
          }
          if (axis >= 0) {
            const float t = adj_wave_sum(rot);
            if (lane == 0) rs[j] = (double)t;
          }
        }
#pragma unroll
        for (int i = 0; i < NPR; ++i) {
          const uint32_t l0 = pt ^ swz(ins0(kSvwThreads * i, pa));
          T0[l0] = S0[i];
          T0[l0 ^ so] = S1[i];
          T1[l0] = L0[i];
          T1[l0 ^ so] = L1[i];
        }
      } else {
        const uint32_t pt = swz(ins0(ins0(tid, pa), pb)), s1 = swz(1u << pa), s2 = swz(1u << pb);
        float2 S[NQD][4], L[NQD][4];
#pragma unroll
        for (int i = 0; i < NQD; ++i) {
          const uint32_t lb = pt ^ swz(ins0(ins0(kSvwThreads * i, pa), pb));
          const uint32_t off[4] = {lb, lb ^ s1, lb ^ s2, lb ^ s1 ^ s2};
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            S[i][x] = T0[off[x]];
            L[i][x] = T1[off[x]];
          }
        }
#pragma unroll 1
        for (int j = cnt - 1; j >= 0; --j) {
          const int k = first + j;
          const uint4 w = reinterpret_cast<const uint4*>(ops)[2 * k];
          const int kind = (int)(w.x & 0xffu), p0 = (int)((w.x >> 8) & 0xffu);
          const int axis = (int)(int8_t)((w.x >> 24) & 0xffu);
          const float2* g = Gb + 16 * k;
          if (kind == kSvOpGate1) {
            const float2 g00 = g[0], g01 = g[1], g10 = g[2], g11 = g[3];
            const bool hi = p0 != pa;   // the op's qubit is quad bit 1
            float rot = 0.f;
#pragma unroll
            for (int i = 0; i < NQD; ++i) {
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                // pair h: quad entries (2h, 2h + 1) on bit 0, (h, h + 2) on bit 1
                const int e0 = hi ? h : 2 * h, e1 = hi ? h + 2 : 2 * h + 1;
                adj_g2(g00, g01, g10, g11, S[i][e0], S[i][e1]);
                adj_g2(g00, g01, g10, g11, L[i][e0], L[i][e1]);
                if (axis >= 0) rot += adj_rot_term(axis, L[i][e0], L[i][e1], S[i][e0], S[i][e1]);
              }
            }
            if (axis >= 0) {
              const float t = adj_wave_sum(rot);
              if (lane == 0) rs[j] = (double)t;
            }
          } else {
            float2 gm[4][4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
              for (int c = 0; c < 4; ++c) gm[r][c] = g[r * 4 + c];
            const bool sw = p0 != pa;
#pragma unroll
            for (int i = 0; i < NQD; ++i) {
              adj_g4(gm, sw, S[i]);
              adj_g4(gm, sw, L[i]);
            }
          }
        }
#pragma unroll
        for (int i = 0; i < NQD; ++i) {
          const uint32_t lb = pt ^ swz(ins0(ins0(kSvwThreads * i, pa), pb));
          const uint32_t off[4] = {lb, lb ^ s1, lb ^ s2, lb ^ s1 ^ s2};
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            T0[off[x]] = S[i][x];
            T1[off[x]] = L[i][x];
          }
        }
      }
      __syncthreads();   // the group's tiles and wavefront sums are complete
      if (tid < cnt && ((gd.z >> tid) & 1u)) {
        const double* r0 = red + (gi & 1) * 4 * kAdjGroupMax;
        acc[first + tid] += r0[tid] + r0[kAdjGroupMax + tid] + r0[2 * kAdjGroupMax + tid] + r0[3 * kAdjGroupMax + tid];
      }
    }
#pragma unroll
    for (int i = 0; i < PPT; ++i)
      *reinterpret_cast<floatx4_t*>(Lg + (lo | pair_hi<NP>(a.P, i))) = lds_get_pair(T14, pt2, i);
    __syncthreads();   // every thread has read its part of lambda, and acc is complete
  }
  __syncthreads();
  double* out = a.wg_acc + (int64_t)blockIdx.x * a.n_ops;
  for (int i = tid; i < a.n_ops; i += kSvwThreads) out[i] = acc[i];
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
  // one layout bound for both kernel forms: the tile kernels' backward form adds
  // double-buffered wavefront sums [2][4][33] ahead of the accumulators
  const size_t nt = (size_t)1 << np;
  const size_t tiles = mode == 0 ? 1 : (mode == 1 ? 2 : 3);
  const size_t gates = (mode == 0 || mode == 1) ? 1 : 2;
  return tiles * nt * sizeof(float2) + gates * 16 * (size_t)n_ops * sizeof(float2) +
         (mode == 0 ? 0 : (2 * 4 * 33 + (size_t)n_ops + 32 * (size_t)n_nslots) * sizeof(double));
}

namespace {
using AdjKernel = void (*)(AdjArgs, const AdjOp*);
// The kernel a window runs: the tile kernels for windows of 10..12 qubits with
// qubit 0 at tile bit 0 (forward, and backward with unitary inserted operators);
// otherwise the general kernel.
AdjKernel adj_kernel(int mode, const AdjArgs& a) {
  const bool tile = mode != 2 && a.np >= 10 && a.np <= 12 && a.P[0] == 0;
  if (!tile) return mode == 0 ? adj_window_kernel<0> : (mode == 1 ? adj_window_kernel<1> : adj_window_kernel<2>);
  if (mode == 0)
    return a.np == 10 ? adj_fwd_group_kernel<10> : (a.np == 11 ? adj_fwd_group_kernel<11> : adj_fwd_group_kernel<12>);
  if (a.want_n)   // gate adjoints: one op per pass (the N sums need every op's own amplitudes)
    return a.np == 10 ? adj_bwd_tile_kernel<10, true>
                      : (a.np == 11 ? adj_bwd_tile_kernel<11, true> : adj_bwd_tile_kernel<12, true>);
  return a.np == 10 ? adj_bwd_group_kernel<10> : (a.np == 11 ? adj_bwd_group_kernel<11> : adj_bwd_group_kernel<12>);
}
}  // namespace

int adj_window_grid(int mode, const AdjArgs& a, size_t lds) {
  int per_cu = 0, dev = 0, cus = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, adj_kernel(mode, a), kAdjThreads, lds);
  if (e != hipSuccess || hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const int64_t tiles = a.n_jobs << (a.n - a.np);
  return (int)std::min<int64_t>(tiles, (int64_t)std::max(per_cu, 1) * std::max(cus, 1));
}

hipError_t launch_adj_window(int mode, const AdjArgs& a, const AdjOp* d_ops, int grid, hipStream_t stream) {
  const size_t lds = adj_window_lds_bytes(mode, a.np, a.n_ops, a.n_nslots);
  hipLaunchKernelGGL(adj_kernel(mode, a), dim3(grid), dim3(kAdjThreads), lds, stream, a, d_ops);
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
