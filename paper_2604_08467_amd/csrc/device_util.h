// Device helpers shared by the sweep, statevector and ragged kernels (included
// by each kernel translation unit; everything here is inline).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace ptsbe {
namespace {

__device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 cfma(float2 a, float2 b, float2 c) {
  return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}

__device__ inline uint32_t bit_of_prefix(const uint64_t* pw, int q) {
  return (uint32_t)((pw[q >> 6] >> (q & 63)) & 1ull);
}

// Gate entry i (< 16) of (traj, gate), conjugated for bra tensors.
__device__ inline float2 gate_entry(const GateCtx& g, int gate, int traj, int conj, int i) {
  float2 v = g.merged[((int64_t)traj * g.G + gate) * 16 + i];
  if (conj) v.y = -v.y;
  return v;
}

__device__ inline uint32_t insert_zero_bits(uint32_t m, const int32_t* pos, int n) {
  for (int i = 0; i < n; ++i) {
    const int p = pos[i];
    const uint32_t lo = m & ((1u << p) - 1u);
    m = ((m >> p) << (p + 1)) | lo;
  }
  return m;
}

__device__ inline uint32_t deposit_tile(uint32_t t, const int* P, int np, int r) {
  // spread the bits of t over the positions not in P (ascending)
  uint32_t out = 0;
  int pi = 0, bit = 0;
  for (int q = 0; q < r; ++q) {
    if (pi < np && P[pi] == q) { ++pi; continue; }
    out |= ((t >> bit) & 1u) << q;
    ++bit;
  }
  return out;
}

// UPV merge of one (trajectory, gate) into out[16] (per thread, FP32 products).
__device__ void merge_gate(const GateCtx& g, int gate, int traj, float2* out) {
  const DeviceGate* G = g.gates + gate;
  const int sb = G->site_begin, se = G->site_end;
  const uint8_t* kr = g.kraus + (int64_t)traj * g.S;
  bool dev = false;
  for (int s = sb; s < se; ++s) dev |= kr[g.gate_site_list[s]] != 0;
  if (!dev) {
    for (int i = 0; i < 16; ++i) out[i] = G->def[i];
    return;
  }
  const int d = G->arity == 2 ? 4 : 2;
  float2 m[16], t[16];
  for (int i = 0; i < 16; ++i) m[i] = G->raw[i];
  for (int s = sb; s < se; ++s) {
    const int site = g.gate_site_list[s];
    const int k = kr[site];
    const float2* op = g.site_ops + ((int64_t)site * g.max_kraus + k) * 16;
    for (int r = 0; r < d; ++r)
      for (int c = 0; c < d; ++c) {
        float2 acc = make_float2(0.f, 0.f);
        for (int x = 0; x < d; ++x) acc = cfma(op[r * d + x], m[x * d + c], acc);
        t[r * d + c] = acc;
      }
    for (int i = 0; i < d * d; ++i) m[i] = t[i];
  }
  for (int i = 0; i < 16; ++i) out[i] = m[i];
}

// Gate matrices of a window are staged in LDS kGateChunk steps at a time (16
// entries each), so that every step reads its matrix with LDS broadcasts.
constexpr int kGateChunk = 32;

// One tile pass of a window of in-place steps (positions P, |P| = np, of a rank-r
// tensor A of one job): the 2^np entries whose other bits equal the tile index t
// are loaded into LDS, every step is applied there (gate operands of trajectory
// traj, staged in Gm[16 * kGateChunk]), and the tile is written back.  pw: the job's
// prefix words in LDS (for sliced legs).  Ends with a barrier, so the caller may
// reuse tile and Gm at once.
__device__ inline void window_tile_pass(const FusedStep* fs, int n_fs, const int* P, int np, int r, uint32_t t,
                                        float2* Aj, const GateCtx& g_, int traj, const uint64_t* pw,
                                        float2* tile, float2* Gm) {
  const uint32_t base = deposit_tile(t, P, np, r);
  const uint32_t nt = 1u << np;
  for (uint32_t l = threadIdx.x; l < nt; l += blockDim.x) {
    uint32_t off = base;
    for (int i = 0; i < np; ++i) off |= ((l >> i) & 1u) << P[i];
    tile[l] = Aj[off];
  }
  __syncthreads();   // the tile is complete before any step reads it
  for (int s = 0; s < n_fs; ++s) {
    const FusedStep& st = fs[s];
    if (s % kGateChunk == 0) {   // every thread is past step s - 1 (it ended with a barrier)
      const int cnt = (n_fs - s < kGateChunk ? n_fs - s : kGateChunk) * 16;
      for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        const FusedStep& sj = fs[s + i / 16];
        Gm[i] = gate_entry(g_, sj.gate, traj, sj.conj, i % 16);
      }
      __syncthreads();
    }
    const float2* G = Gm + 16 * (s % kGateChunk);
    // a plain gate applied in place: no hyper or sliced legs, outputs where the inputs were
    const bool plain = st.nH == 0 && st.nS == 0 && st.nK == st.nN && st.nK >= 1 && st.nK <= 2 &&
                       st.noff[1] == st.koff[1] && (st.nK == 1 || (st.noff[2] == st.koff[2] && st.noff[3] == st.koff[3]));
    if (plain && st.nK == 1) {
      // one-qubit gate in place: the 2x2 matrix in registers, pairs (lb, lb + o)
      float2 g[2][2];
#pragma unroll
      for (int n = 0; n < 2; ++n)
#pragma unroll
        for (int k = 0; k < 2; ++k) g[n][k] = G[st.nB[n] + st.kB[k]];
      const int p = st.kloc[0];
      const uint32_t o = st.koff[1], lo_mask = (1u << p) - 1u;
      const bool z00 = g[0][0].x == 0.f && g[0][0].y == 0.f, z01 = g[0][1].x == 0.f && g[0][1].y == 0.f;
      const bool z10 = g[1][0].x == 0.f && g[1][0].y == 0.f, z11 = g[1][1].x == 0.f && g[1][1].y == 0.f;
      if ((z00 || z01) && (z10 || z11)) {
        // monomial (diagonal or anti-diagonal): one product per amplitude
        // row 0 takes a0 unless g00 == 0 (then a1); row 1 takes a1 unless g11 == 0 (then a0)
        const bool swap0 = z00, swap1 = z11;
        const float2 d0 = swap0 ? g[0][1] : g[0][0], d1 = swap1 ? g[1][0] : g[1][1];
        for (uint32_t m = threadIdx.x; m < (nt >> 1); m += blockDim.x) {
          const uint32_t lb = ((m & ~lo_mask) << 1) | (m & lo_mask);
          const float2 a0 = tile[lb], a1 = tile[lb + o];
          tile[lb] = cmul(d0, swap0 ? a1 : a0);
          tile[lb + o] = cmul(d1, swap1 ? a0 : a1);
        }
      } else {
        for (uint32_t m = threadIdx.x; m < (nt >> 1); m += blockDim.x) {
          const uint32_t lb = ((m & ~lo_mask) << 1) | (m & lo_mask);
          const float2 a0 = tile[lb], a1 = tile[lb + o];
          tile[lb] = cfma(g[0][1], a1, cmul(g[0][0], a0));
          tile[lb + o] = cfma(g[1][1], a1, cmul(g[1][0], a0));
        }
      }
      __syncthreads();
      continue;
    }
    if (plain && st.nK == 2) {
      // two-qubit gate in place: the 4x4 matrix in registers, quads at lb + koff[k]
      float2 g[4][4];
#pragma unroll
      for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int k = 0; k < 4; ++k) g[n][k] = G[st.nB[n] + st.kB[k]];
      const int p0 = st.kloc[0], p1 = st.kloc[1];
      const uint32_t o1 = st.koff[1], o2 = st.koff[2], o3 = st.koff[3];
      const uint32_t m0 = (1u << p0) - 1u, m1 = (1u << p1) - 1u;
      const uint32_t off[4] = {0u, o1, o2, o3};
      // monomial matrix (at most one nonzero per row: diagonal gates such as CZ
      // with diagonal Kraus factors, CNOT and Pauli products): one product per amplitude
      int col[4];
      bool mono = true;
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        col[n] = -1;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (g[n][k].x != 0.f || g[n][k].y != 0.f) {
            mono = mono && col[n] < 0;
            col[n] = k;
          }
      }
      if (mono) {
        float2 gd[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          const int c = col[n];
          gd[n] = c == 0 ? g[n][0] : c == 1 ? g[n][1] : c == 2 ? g[n][2] : c == 3 ? g[n][3] : make_float2(0.f, 0.f);
        }
        for (uint32_t m = threadIdx.x; m < (nt >> 2); m += blockDim.x) {
          uint32_t lb = ((m & ~m0) << 1) | (m & m0);
          lb = ((lb & ~m1) << 1) | (lb & m1);
          const float2 a0 = tile[lb], a1 = tile[lb + o1], a2 = tile[lb + o2], a3 = tile[lb + o3];
#pragma unroll
          for (int n = 0; n < 4; ++n) {
            const int c = col[n];
            const float2 x = c == 0 ? a0 : c == 1 ? a1 : c == 2 ? a2 : a3;
            tile[lb + off[n]] = cmul(gd[n], x);
          }
        }
      } else {
        for (uint32_t m = threadIdx.x; m < (nt >> 2); m += blockDim.x) {
          uint32_t lb = ((m & ~m0) << 1) | (m & m0);
          lb = ((lb & ~m1) << 1) | (lb & m1);
          const float2 a0 = tile[lb], a1 = tile[lb + o1], a2 = tile[lb + o2], a3 = tile[lb + o3];
#pragma unroll
          for (int n = 0; n < 4; ++n)
            tile[lb + off[n]] = cfma(g[n][3], a3, cfma(g[n][2], a2, cfma(g[n][1], a1, cmul(g[n][0], a0))));
        }
      }
      __syncthreads();
      continue;
    }
    int sb = 0;
    for (int i = 0; i < st.nS; ++i) sb += (int)bit_of_prefix(pw, st.sq[i]) * st.sw[i];
    const uint32_t nm = nt >> st.nK;
    const int nk = 1 << st.nK, nn = 1 << st.nN;
    for (uint32_t m = threadIdx.x; m < nm; m += blockDim.x) {
      const uint32_t lb = insert_zero_bits(m, st.kloc, st.nK);
      float2 a[16];
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < nk) a[k] = tile[lb + st.koff[k]];
      int hidx = sb;
      for (int i = 0; i < st.nH; ++i) {
        const uint32_t bit = st.h_inP[i] ? (lb >> st.h_pos[i]) & 1u : (base >> st.h_pos[i]) & 1u;
        hidx += (int)bit * st.hw[i];
      }
      for (int n = 0; n < nn; ++n) {
        float2 acc = make_float2(0.f, 0.f);
        const int bn = hidx + st.nB[n];
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (k < nk) acc = cfma(a[k], G[bn + st.kB[k]], acc);
        tile[lb + st.noff[n]] = acc;
      }
    }
    __syncthreads();
  }
  for (uint32_t l = threadIdx.x; l < nt; l += blockDim.x) {
    uint32_t off = base;
    for (int i = 0; i < np; ++i) off |= ((l >> i) & 1u) << P[i];
    Aj[off] = tile[l];
  }
  __syncthreads();
}

}  // namespace
}  // namespace ptsbe
