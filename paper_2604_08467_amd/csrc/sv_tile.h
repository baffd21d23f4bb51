// Device helpers of the statevector gate windows (included by the window kernel
// and the ragged-set kernels; everything here is inline): the compact ops' gate
// and cluster applications on an LDS tile of 2^NP amplitudes, and the 16-byte
// amplitude-pair tile loads.  Qubit 0 is tile bit 0, so a pair of amplitudes is
// one 16-byte run of the state.
#pragma once

#include <hip/hip_runtime.h>

#include "device_util.h"
#include "internal.h"

namespace ptsbe {
namespace {

constexpr int kSvwThreads = 256;

// LDS layout of a tile: entry l lives at swz(l) = l ^ ((l >> 4) & 15), tile
// bits 4..7 folded into the low four bits (the 8-byte bank slot of a 128-byte
// LDS row).  The 16 lanes of a quarter-wavefront that step along the tile bits
// left free by an op (a gate's other bits, a cluster's columns) then spread over
// more slots: on a 32-bank model this brings cluster accesses from 3.4x to 1.8x
// of conflict-free and two-qubit gates from 1.76x to 1.47x.  A full linear map
// of bits 4..11 gets within 15 % and 6 %, but its index arithmetic costs more
// VALU issue than the conflicts it removes (measured on the window kernel).
// swz is linear, swz(a ^ b) = swz(a) ^ swz(b), so each thread swizzles its own
// part of an index once per op and XORs uniform parts in.
__host__ __device__ inline uint32_t swz(uint32_t l) { return l ^ ((l >> 4) & 15u); }
__device__ inline uint32_t ins0(uint32_t m, int p) {   // zero bit inserted at position p
  const uint32_t lo = (1u << p) - 1u;
  return ((m & ~lo) << 1) | (m & lo);
}

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
  // swizzled parts of the addresses: this lane's column and states, then the
  // wavefront's column tile
  const uint32_t pj = swz(cc.colbase((uint32_t)j));
  uint32_t ps[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) ps[i] = pj ^ swz(cc.soff(4 * q + i));
  for (int ct = 0; ct < nct; ++ct) {
    const uint32_t pc = swz(cc.colbase((uint32_t)(wave * per_wave + 16 * ct)));
    float x[8];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float2 v = tile[pc ^ ps[i]];
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
    for (int i = 0; i < 4; ++i) tile[pc ^ ps[i]] = make_float2(acc[0][i] * unscale, acc[1][i] * unscale);
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
  const uint32_t pj = swz(cc.colbase((uint32_t)j));
  uint32_t pr[4], pw[4];     // states 4 s + q (read) and 4 q + i (written)
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    pr[s] = pj ^ swz(cc.soff(4 * s + q));
    pw[s] = pj ^ swz(cc.soff(4 * q + s));
  }
  for (int ct = 0; ct < nct; ++ct) {
    const uint32_t pc = swz(cc.colbase((uint32_t)(wave * per_wave + 16 * ct)));
    float2 x[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) x[s] = tile[pc ^ pr[s]];
    floatx4_t acc0 = floatx4_t{0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const float b = s < 4 ? x[s].x : x[s - 4].y;
      acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(af[0][s], b, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(af[1][s], b, acc1, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) tile[pc ^ pw[i]] = make_float2(acc0[i], acc1[i]);
  }
  __syncthreads();
}

__device__ inline bool czero(float2 v) { return v.x == 0.f && v.y == 0.f; }

// A one-qubit gate in place on tile position p (g: [n][k] row-major).
template <int NP>
__device__ inline void apply_gate1(const float2* __restrict__ G, int p, float2* tile) {
  constexpr uint32_t nt = 1u << NP;
  const float2 g00 = G[0], g01 = G[1], g10 = G[2], g11 = G[3];
  // pair (lb, lb + 2^p), lb = ins0(tid + 256 i, p): swizzled as the thread's part
  // XOR the uniform part of iteration i
  const uint32_t pt = swz(ins0(threadIdx.x, p)), so = swz(1u << p);
  if ((czero(g00) || czero(g01)) && (czero(g10) || czero(g11))) {
    // monomial (diagonal or anti-diagonal): one product per amplitude
    const bool swap0 = czero(g00), swap1 = czero(g11);
    const float2 d0 = swap0 ? g01 : g00, d1 = swap1 ? g10 : g11;
#pragma unroll 2
    for (uint32_t i = 0; i < (nt >> 1) / kSvwThreads; ++i) {
      const uint32_t l0 = pt ^ swz(ins0(kSvwThreads * i, p)), l1 = l0 ^ so;
      const float2 a0 = tile[l0], a1 = tile[l1];
      tile[l0] = cmul(d0, swap0 ? a1 : a0);
      tile[l1] = cmul(d1, swap1 ? a0 : a1);
    }
  } else {
#pragma unroll 2
    for (uint32_t i = 0; i < (nt >> 1) / kSvwThreads; ++i) {
      const uint32_t l0 = pt ^ swz(ins0(kSvwThreads * i, p)), l1 = l0 ^ so;
      const float2 a0 = tile[l0], a1 = tile[l1];
      tile[l0] = cfma(g01, a1, cmul(g00, a0));
      tile[l1] = cfma(g11, a1, cmul(g10, a0));
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
  const int pa = p0 < p1 ? p0 : p1, pb = p0 < p1 ? p1 : p0;   // zero bits inserted low one first
  // quad lb + {0, 2^p0, 2^p1, both}, lb = ins0(ins0(tid + 256 i, pa), pb), swizzled
  const uint32_t pt = swz(ins0(ins0(threadIdx.x, pa), pb));
  const uint32_t s1 = swz(1u << p0), s2 = swz(1u << p1), s3 = s1 ^ s2;
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
    for (uint32_t i = 0; i < (nt >> 2) / kSvwThreads; ++i) {
      const uint32_t lb = pt ^ swz(ins0(ins0(kSvwThreads * i, pa), pb));
      const uint32_t off[4] = {lb, lb ^ s1, lb ^ s2, lb ^ s3};
      const float2 a0 = tile[off[0]], a1 = tile[off[1]], a2 = tile[off[2]], a3 = tile[off[3]];
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const int c = col[n];
        const float2 x = c == 0 ? a0 : c == 1 ? a1 : c == 2 ? a2 : a3;
        tile[off[n]] = cmul(gd[n], x);
      }
    }
  } else {
#pragma unroll 2
    for (uint32_t i = 0; i < (nt >> 2) / kSvwThreads; ++i) {
      const uint32_t lb = pt ^ swz(ins0(ins0(kSvwThreads * i, pa), pb));
      const uint32_t off[4] = {lb, lb ^ s1, lb ^ s2, lb ^ s3};
      const float2 a0 = tile[off[0]], a1 = tile[off[1]], a2 = tile[off[2]], a3 = tile[off[3]];
#pragma unroll
      for (int n = 0; n < 4; ++n)
        tile[off[n]] = cfma(g[n][3], a3, cfma(g[n][2], a2, cfma(g[n][1], a1, cmul(g[n][0], a0))));
    }
  }
  __syncthreads();
}

// Global offset of pair slot i of this thread within a tile (pair index
// tid + 256 i = tile bits 1..NP-1; tile bit 0 is qubit 0, the pair's two halves).
template <int NP>
__device__ inline uint32_t pair_hi(const int* P, int i) {
  uint32_t off = 0;
#pragma unroll
  for (int b = 0; b < NP - 9; ++b) off |= (uint32_t)((i >> b) & 1) << P[9 + b];
  return off;
}

// The thread's pairs of one tile (A: the tile's first amplitude) into v.
template <int NP>
__device__ inline void load_pairs(const float2* __restrict__ A, const int* P, uint32_t lo,
                                  floatx4_t (&v)[1 << (NP - 9)]) {
#pragma unroll
  for (int i = 0; i < (1 << (NP - 9)); ++i) v[i] = *reinterpret_cast<const floatx4_t*>(A + (lo | pair_hi<NP>(P, i)));
}

// This thread's pair offset from its own bits (tile bits 1..8 = positions P[1..8]).
__device__ inline uint32_t pair_lo(const int* P) {
  uint32_t lo = 0;
#pragma unroll
  for (int b = 0; b < 8; ++b) lo |= (uint32_t)((threadIdx.x >> b) & 1) << P[b + 1];
  return lo;
}

// The tile's other bits t spread over the positions in `other` (a bit mask).
__device__ inline uint32_t deposit_other(uint32_t t, uint32_t other) {
  uint32_t out = 0, mask = other;
  for (int bit = 0; mask; ++bit, mask &= mask - 1u) out |= ((t >> bit) & 1u) << __builtin_ctz(mask);
  return out;
}

// LDS side of the pair moves: pair index tid + 256 i holds entries e = 2 (tid +
// 256 i) and e + 1, stored at swz(e) and swz(e) ^ 1 (one 16-byte slot, halves
// swapped when swz(e) is odd).  pt2 = swz(2 tid).
__device__ inline void lds_put_pair(floatx4_t* tile4, uint32_t pt2, int i, floatx4_t v) {
  const uint32_t e = pt2 ^ swz(2u * kSvwThreads * (uint32_t)i);
  tile4[e >> 1] = (e & 1u) ? floatx4_t{v[2], v[3], v[0], v[1]} : v;
}
__device__ inline floatx4_t lds_get_pair(const floatx4_t* tile4, uint32_t pt2, int i) {
  const uint32_t e = pt2 ^ swz(2u * kSvwThreads * (uint32_t)i);
  const floatx4_t v = tile4[e >> 1];
  return (e & 1u) ? floatx4_t{v[2], v[3], v[0], v[1]} : v;
}

// One tile of a window of plain gates (no clusters): pairs loaded from Ain, the
// ops applied in LDS (gate matrices staged in Gs), pairs stored to Aout (Ain and
// Aout: the tile's first amplitude in the input and output states, which may be
// the same).  Op records are 32 bytes with kind, p0 and p1 in the low three bytes
// of the first dword and the staged matrix slot in the fourth (SvOp, AdjOp).
// Ends with a barrier.
template <int NP, typename Op>
__device__ inline void plain_tile_pass(const Op* __restrict__ ops, int n_ops, const int* P, const float2* Ain,
                                       float2* Aout, float2* tile, const float2* Gs) {
  static_assert(sizeof(Op) == 32, "op records are eight dwords");
  constexpr int PPT = 1 << (NP - 9);
  floatx4_t* tile4 = reinterpret_cast<floatx4_t*>(tile);
  const uint32_t lo = pair_lo(P), pt2 = swz(2u * threadIdx.x);
  floatx4_t v[PPT];
  load_pairs<NP>(Ain, P, lo, v);
#pragma unroll
  for (int i = 0; i < PPT; ++i) lds_put_pair(tile4, pt2, i, v[i]);
  __syncthreads();
  for (int s = 0; s < n_ops; ++s) {
    const uint4 w = reinterpret_cast<const uint4*>(ops)[2 * s];
    const int kind = (int)(w.x & 0xffu), slot = (int)w.w;
    if (kind == kSvOpGate1) apply_gate1<NP>(Gs + 16 * slot, (int)((w.x >> 8) & 0xffu), tile);
    else apply_gate2<NP>(Gs + 16 * slot, (int)((w.x >> 8) & 0xffu), (int)((w.x >> 16) & 0xffu), tile);
  }
#pragma unroll
  for (int i = 0; i < PPT; ++i)
    *reinterpret_cast<floatx4_t*>(Aout + (lo | pair_hi<NP>(P, i))) = lds_get_pair(tile4, pt2, i);
  __syncthreads();
}

}  // namespace
}  // namespace ptsbe
