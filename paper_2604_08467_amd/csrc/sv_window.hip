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

namespace ptsbe {
namespace {

constexpr int kSvwThreads = 256;

struct SvwArgs {
  int n, np, n_ops, n_plain, n_cl, cl_first, n_cl_total, G;
  uint32_t other;          // bit mask of the qubits outside the window
  int P[kFuseMax];
  int64_t n_jobs;
  int32_t traj_base;
};

typedef __bf16 svw_bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 svw_f16x8 __attribute__((ext_vector_type(8)));
template <int PREC> struct SvwSplit;
template <> struct SvwSplit<PTSBE_SPLIT_BF16> {
  typedef __bf16 E;
  typedef svw_bf16x8 V;
  static __device__ floatx4_t mfma(V a, V b, floatx4_t c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
template <> struct SvwSplit<PTSBE_SPLIT_F16> {
  typedef _Float16 E;
  typedef svw_f16x8 V;
  static __device__ floatx4_t mfma(V a, V b, floatx4_t c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};

// Column addressing of a cluster on tile positions cp[0..3]: cluster-local state
// v sits at offset soff(v); the other tile bits (the column) are deposited around
// the four positions (cs: cp ascending).
struct ClusterCols {
  int cp[4], cs[4];
  __device__ explicit ClusterCols(uint32_t pos) {    // byte i: position of cluster-local bit i
#pragma unroll
    for (int i = 0; i < 4; ++i) cp[i] = cs[i] = (int)((pos >> (8 * i)) & 0xffu);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (cs[k] > cs[k + 1]) { const int t = cs[k]; cs[k] = cs[k + 1]; cs[k + 1] = t; }
  }
  __device__ uint32_t soff(int v) const {
    return ((uint32_t)(v & 1) << cp[0]) | ((uint32_t)((v >> 1) & 1) << cp[1]) |
           ((uint32_t)((v >> 2) & 1) << cp[2]) | ((uint32_t)((v >> 3) & 1) << cp[3]);
  }
  __device__ uint32_t colbase(uint32_t col) const {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t lo = col & ((1u << cs[i]) - 1u);
      col = ((col >> cs[i]) << (cs[i] + 1)) | lo;
    }
    return col;
  }
};

// Split-precision cluster: [Yr; Yi] = [[Ur, -Ui], [Ui, Ur]] [Xr; Xi] with the inner
// index interleaved (k = 2 v + c: state v, c = 0 real / 1 imaginary part), so that
// lane 16 q + j holds states 4q .. 4q+3 of column j (B) or of output row j (A).
// One 16x16x32 MFMA covers the whole inner dimension: per 16 columns, 2 row tiles
// (real and imaginary outputs) x 3 products.  Each wavefront reads and then
// overwrites only its own columns.  Needs blockDim.x == 256 and np >= 10.
template <int PREC>
__device__ inline void apply_cluster_split(const ClusterCols& cc, const float2* __restrict__ U, int np, float2* tile) {
  typedef typename SvwSplit<PREC>::E E;
  typedef typename SvwSplit<PREC>::V V;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, q = lane >> 4, j = lane & 15;
  V ah[2], al[2];
  {
    float a[2][8];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float2 u = U[j * 16 + 4 * q + i];
      a[0][2 * i] = u.x;  a[0][2 * i + 1] = -u.y;    // real output row:  Ur Xr - Ui Xi
      a[1][2 * i] = u.y;  a[1][2 * i + 1] = u.x;     // imaginary output: Ui Xr + Ur Xi
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const E h = (E)a[rt][i];
        ah[rt][i] = h;
        al[rt][i] = (E)(a[rt][i] - (float)h);
      }
  }
  const int ncol = 1 << (np - 4), per_wave = ncol >> 2, nct = per_wave >> 4;
  for (int ct = 0; ct < nct; ++ct) {
    const uint32_t cb = cc.colbase((uint32_t)(wave * per_wave + 16 * ct + j));
    float x[8];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float2 v = tile[cb + cc.soff(4 * q + i)];
      x[2 * i] = v.x;
      x[2 * i + 1] = v.y;
    }
    float scale = 1.f, unscale = 1.f;
    if (PREC == PTSBE_SPLIT_F16) {
      // one power of two per column (its four lanes agree): largest |x| to [2^14, 2^15)
      float m = 0.f;
#pragma unroll
      for (int i = 0; i < 8; ++i) m = fmaxf(m, fabsf(x[i]));
      m = fmaxf(m, __shfl_xor(m, 16));
      m = fmaxf(m, __shfl_xor(m, 32));
      if (m > 0.f) {
        int e;
        (void)frexpf(m, &e);             // m = f 2^e, f in [1/2, 1)
        scale = ldexpf(1.f, 15 - e);
        unscale = ldexpf(1.f, e - 15);
      }
    }
    V bh, bl;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float xs = x[i] * scale;
      const E h = (E)xs;
      bh[i] = h;
      bl[i] = (E)(xs - (float)h);
    }
    floatx4_t acc[2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      acc[rt] = floatx4_t{0.f, 0.f, 0.f, 0.f};
      acc[rt] = SvwSplit<PREC>::mfma(ah[rt], bh, acc[rt]);
      acc[rt] = SvwSplit<PREC>::mfma(ah[rt], bl, acc[rt]);
      acc[rt] = SvwSplit<PREC>::mfma(al[rt], bh, acc[rt]);
    }
    // D[4 q + i][j]: output state 4 q + i of column j
#pragma unroll
    for (int i = 0; i < 4; ++i) tile[cb + cc.soff(4 * q + i)] = make_float2(acc[0][i] * unscale, acc[1][i] * unscale);
  }
  __syncthreads();
}

// FP32 cluster on v_mfma_f32_16x16x4f32 (inner index k < 16 real, >= 16 imaginary
// parts; lane 16 q + j takes states 4 s + q of column j), U in LDS.
__device__ inline void apply_cluster_f32(const ClusterCols& cc, const float2* __restrict__ U, int np, float2* tile) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, q = lane >> 4, j = lane & 15;
  float af[2][8];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float2 u = U[j * 16 + 4 * s + q];
    af[0][s] = u.x;  af[0][s + 4] = -u.y;
    af[1][s] = u.y;  af[1][s + 4] = u.x;
  }
  const int ncol = 1 << (np - 4), per_wave = ncol >> 2, nct = per_wave >> 4;
  for (int ct = 0; ct < nct; ++ct) {
    const uint32_t cb = cc.colbase((uint32_t)(wave * per_wave + 16 * ct + j));
    float2 x[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) x[s] = tile[cb + cc.soff(4 * s + q)];
    floatx4_t acc0 = floatx4_t{0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const float b = s < 4 ? x[s].x : x[s - 4].y;
      acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(af[0][s], b, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(af[1][s], b, acc1, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) tile[cb + cc.soff(4 * q + i)] = make_float2(acc0[i], acc1[i]);
  }
  __syncthreads();
}

__device__ inline bool czero(float2 v) { return v.x == 0.f && v.y == 0.f; }

// A one-qubit gate in place on tile position p (g: [n][k] row-major).
template <int NP>
__device__ inline void apply_gate1(const float2* __restrict__ G, int p, float2* tile) {
  constexpr uint32_t nt = 1u << NP;
  const float2 g00 = G[0], g01 = G[1], g10 = G[2], g11 = G[3];
  const uint32_t o = 1u << p, lo_mask = o - 1u;
  if ((czero(g00) || czero(g01)) && (czero(g10) || czero(g11))) {
    // monomial (diagonal or anti-diagonal): one product per amplitude
    const bool swap0 = czero(g00), swap1 = czero(g11);
    const float2 d0 = swap0 ? g01 : g00, d1 = swap1 ? g10 : g11;
#pragma unroll 2
    for (uint32_t m = threadIdx.x; m < (nt >> 1); m += kSvwThreads) {
      const uint32_t lb = ((m & ~lo_mask) << 1) | (m & lo_mask);
      const float2 a0 = tile[lb], a1 = tile[lb + o];
      tile[lb] = cmul(d0, swap0 ? a1 : a0);
      tile[lb + o] = cmul(d1, swap1 ? a0 : a1);
    }
  } else {
#pragma unroll 2
    for (uint32_t m = threadIdx.x; m < (nt >> 1); m += kSvwThreads) {
      const uint32_t lb = ((m & ~lo_mask) << 1) | (m & lo_mask);
      const float2 a0 = tile[lb], a1 = tile[lb + o];
      tile[lb] = cfma(g01, a1, cmul(g00, a0));
      tile[lb + o] = cfma(g11, a1, cmul(g10, a0));
    }
  }
  __syncthreads();
}

// A two-qubit gate in place on tile positions p0 (local bit 0) and p1 (local bit 1).
template <int NP>
__device__ inline void apply_gate2(const float2* __restrict__ Gm, int p0, int p1, float2* tile) {
  constexpr uint32_t nt = 1u << NP;
  float2 g[4][4];
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int k = 0; k < 4; ++k) g[n][k] = Gm[n * 4 + k];
  const uint32_t o1 = 1u << p0, o2 = 1u << p1, o3 = o1 | o2;
  const int pa = p0 < p1 ? p0 : p1, pb = p0 < p1 ? p1 : p0;   // zero bits inserted low one first
  const uint32_t ma = (1u << pa) - 1u, mb = (1u << pb) - 1u;
  int col[4];
  bool mono = true;
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    col[n] = -1;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (!czero(g[n][k])) {
        mono = mono && col[n] < 0;
        col[n] = k;
      }
  }
  if (mono) {
    // at most one nonzero per row (diagonal gates with diagonal Kraus factors,
    // CNOT, Pauli products): one product per amplitude
    float2 gd[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int c = col[n];
      gd[n] = c == 0 ? g[n][0] : c == 1 ? g[n][1] : c == 2 ? g[n][2] : c == 3 ? g[n][3] : make_float2(0.f, 0.f);
    }
#pragma unroll 2
    for (uint32_t m = threadIdx.x; m < (nt >> 2); m += kSvwThreads) {
      uint32_t lb = ((m & ~ma) << 1) | (m & ma);
      lb = ((lb & ~mb) << 1) | (lb & mb);
      const float2 a0 = tile[lb], a1 = tile[lb + o1], a2 = tile[lb + o2], a3 = tile[lb + o3];
      const uint32_t off[4] = {0u, o1, o2, o3};
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const int c = col[n];
        const float2 x = c == 0 ? a0 : c == 1 ? a1 : c == 2 ? a2 : a3;
        tile[lb + off[n]] = cmul(gd[n], x);
      }
    }
  } else {
#pragma unroll 2
    for (uint32_t m = threadIdx.x; m < (nt >> 2); m += kSvwThreads) {
      uint32_t lb = ((m & ~ma) << 1) | (m & ma);
      lb = ((lb & ~mb) << 1) | (lb & mb);
      const float2 a0 = tile[lb], a1 = tile[lb + o1], a2 = tile[lb + o2], a3 = tile[lb + o3];
      const uint32_t off[4] = {0u, o1, o2, o3};
#pragma unroll
      for (int n = 0; n < 4; ++n)
        tile[lb + off[n]] = cfma(g[n][3], a3, cfma(g[n][2], a2, cfma(g[n][1], a1, cmul(g[n][0], a0))));
    }
  }
  __syncthreads();
}

// Global offset of pair slot i of this thread within a tile (pair index
// tid + 256 i = tile bits 1..NP-1; tile bit 0 is qubit 0, the pair's two halves).
template <int NP>
__device__ inline uint32_t pair_hi(const SvwArgs& a, int i) {
  uint32_t off = 0;
#pragma unroll
  for (int b = 0; b < NP - 9; ++b) off |= (uint32_t)((i >> b) & 1) << a.P[9 + b];
  return off;
}

// The thread's pairs of one tile (A: the tile's first amplitude) into v.
template <int NP>
__device__ inline void load_pairs(const float2* __restrict__ A, const SvwArgs& a, uint32_t lo,
                                  floatx4_t (&v)[1 << (NP - 9)]) {
#pragma unroll
  for (int i = 0; i < (1 << (NP - 9)); ++i) v[i] = *reinterpret_cast<const floatx4_t*>(A + (lo | pair_hi<NP>(a, i)));
}

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
  uint32_t lo = 0;
#pragma unroll
  for (int b = 0; b < 8; ++b) lo |= (uint32_t)((tid >> b) & 1) << a.P[b + 1];
  auto tile_base = [&](int64_t bid) -> uint32_t {   // the tile's other bits, spread over the non-window positions
    const uint32_t t = (uint32_t)(bid & (((int64_t)1 << tb) - 1));
    uint32_t out = 0, mask = a.other;
    for (int bit = 0; mask; ++bit, mask &= mask - 1u) out |= ((t >> bit) & 1u) << __builtin_ctz(mask);
    return out;
  };
  floatx4_t v[PPT];
  load_pairs<NP>(psi + ((b0 >> tb) << n) + tile_base(b0), a, lo, v);
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
    for (int i = 0; i < PPT; ++i) tile4[tid + kSvwThreads * i] = v[i];
    __syncthreads();   // the tile (and any staging) is complete before the first op
    if (PIPE && bid + 1 < b1) load_pairs<NP>(psi + (((bid + 1) >> tb) << n) + tile_base(bid + 1), a, lo, v);
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
      for (int i = 0; i < PPT; ++i) *reinterpret_cast<floatx4_t*>(A + (lo | pair_hi<NP>(a, i))) = tile4[tid + kSvwThreads * i];
    }
    __syncthreads();   // every thread has read its part of the tile before it is refilled
    if (!PIPE && bid + 1 < b1) load_pairs<NP>(psi + (((bid + 1) >> tb) << n) + tile_base(bid + 1), a, lo, v);
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
  uint32_t win = 0;
  for (int k = 0; k < kFuseMax; ++k) {
    a.P[k] = w.P[k];
    if (k < w.np) win |= 1u << w.P[k];
  }
  a.other = (n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u)) & ~win;
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
