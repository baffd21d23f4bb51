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
static_assert(kGateChunk == kGateChunkHost, "the planner splits gate clusters at the same chunk boundary");
typedef float floatx4_t __attribute__((ext_vector_type(4)));

// Product U = G_L ... G_1 of a gate cluster (L plain steps fs[0..L) on the 4
// tile positions cp = fs[0].cl_pos), a 16 x 16 matrix on the cluster's 4 bits
// (bit i of a cluster state = tile bit cp[i]; bits no member touches act as
// identity), built in LDS by 256 threads (one entry each) from the gate matrices
// G (16 per step).  Ua / Ub: 256 entries each.  Returns the buffer holding U.
__device__ inline float2* build_cluster(const FusedStep* fs, int L, const float2* G, float2* Ua, float2* Ub) {
  const int tid = threadIdx.x;
  int cp[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) cp[i] = fs[0].cl_pos[i];
  {
    const int r = tid >> 4, c = tid & 15;
    Ua[tid] = make_float2(r == c ? 1.f : 0.f, 0.f);
  }
  __syncthreads();
  for (int m = 0; m < L; ++m) {           // U <- G_m U
    const FusedStep& st = fs[m];
    const float2* Gm = G + 16 * m;
    int cb0 = 0, cb1 = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (cp[i] == st.kloc[0]) cb0 = i;
      if (st.nK == 2 && cp[i] == st.kloc[1]) cb1 = i;
    }
    const int r = tid >> 4, c = tid & 15;
    float2 acc = make_float2(0.f, 0.f);
    if (st.nK == 1) {
      const int n = (r >> cb0) & 1;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int rk = (r & ~(1 << cb0)) | (k << cb0);
        acc = cfma(Gm[st.nB[n] + st.kB[k]], Ua[rk * 16 + c], acc);
      }
    } else {
      const int n = ((r >> cb0) & 1) | (((r >> cb1) & 1) << 1);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int rk = (r & ~((1 << cb0) | (1 << cb1))) | ((k & 1) << cb0) | ((k >> 1) << cb1);
        acc = cfma(Gm[st.nB[n] + st.kB[k]], Ua[rk * 16 + c], acc);
      }
    }
    Ub[tid] = acc;
    __syncthreads();
    float2* t = Ua; Ua = Ub; Ub = t;
  }
  return Ua;
}

// Apply a gate cluster's matrix U (16 x 16, row-major, built beforehand; in
// global memory) to the tile: [Yr; Yi] = [[Ur, -Ui], [Ui, Ur]] [Xr; Xi] on
// v_mfma_f32_16x16x4f32, 32 x 32 times 32 x 2^(np-4) (tile columns = the other
// np - 4 bits), each wavefront on its own quarter of the columns, so that it
// reads and then overwrites only its own entries.  Needs blockDim.x == 256 and
// np >= 10.  Ends with a barrier.
__device__ inline void apply_cluster(const int* cl_pos, const float2* __restrict__ U, int np, float2* tile) {
  const int tid = threadIdx.x;
  int cp[4], cs[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) cp[i] = cs[i] = cl_pos[i];
#pragma unroll
  for (int i = 0; i < 4; ++i)              // ascending copy, for the column deposit
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (cs[k] > cs[k + 1]) { const int t = cs[k]; cs[k] = cs[k + 1]; cs[k + 1] = t; }
  // A fragments: lane holds A[16 rt + lane % 16][4 s + lane / 16]; columns 4s+q and 4(s-4)+q coincide
  const int lane = tid & 63, wave = tid >> 6, q = lane >> 4, j = lane & 15;
  float2 u4[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) u4[s] = U[j * 16 + 4 * s + q];
  float af[2][8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const float2 u = u4[s & 3];
    af[0][s] = s < 4 ? u.x : -u.y;        // [Ur, -Ui]
    af[1][s] = s < 4 ? u.y : u.x;         // [Ui,  Ur]
  }
  auto soff = [&](int v) -> uint32_t {
    return ((uint32_t)(v & 1) << cp[0]) | ((uint32_t)((v >> 1) & 1) << cp[1]) |
           ((uint32_t)((v >> 2) & 1) << cp[2]) | ((uint32_t)((v >> 3) & 1) << cp[3]);
  };
  auto colbase = [&](uint32_t col) -> uint32_t {   // insert zero bits at the cluster positions
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t lo = col & ((1u << cs[i]) - 1u);
      col = ((col >> cs[i]) << (cs[i] + 1)) | lo;
    }
    return col;
  };
  const int ncol = 1 << (np - 4), per_wave = ncol >> 2, nct = per_wave >> 4;
  floatx4_t acc[2][4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    acc[0][ct] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    acc[1][ct] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    if (ct < nct) {
      const uint32_t cb = colbase((uint32_t)(wave * per_wave + 16 * ct + j));
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const float2 x = tile[cb + soff((4 * s + q) & 15)];
        const float b = s < 4 ? x.x : x.y;
        acc[0][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[0][s], b, acc[0][ct], 0, 0, 0);
        acc[1][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[1][s], b, acc[1][ct], 0, 0, 0);
      }
    }
  }
  // D[16 rt + 4 q + i][col]: state 4 q + i, real part from rt = 0, imaginary from rt = 1
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
    if (ct < nct) {
      const uint32_t cb = colbase((uint32_t)(wave * per_wave + 16 * ct + j));
#pragma unroll
      for (int i = 0; i < 4; ++i) tile[cb + soff(4 * q + i)] = make_float2(acc[0][ct][i], acc[1][ct][i]);
    }
  __syncthreads();
}

// One tile pass of a window of in-place steps (positions P, |P| = np, of a rank-r
// tensor A of one job): the 2^np entries whose other bits equal the tile index t
// are loaded into LDS, every step is applied there (gate operands of trajectory
// traj, staged in Gm[16 * kGateChunk]), and the tile is written back.  pw: the job's
// prefix words in LDS (for sliced legs); Ucl: the job's gate-cluster matrices,
// used when CLUSTERS (else the steps of a cluster run one by one); gates_ready:
// Gm already holds the first kGateChunk gates of these steps for traj (the
// previous pass of this workgroup had the same steps and trajectory and at most
// kGateChunk of them).  blockDim.x == 256.  Ends with a barrier, so the caller may
// reuse tile and Gm at once.
// Offsets of a tile's entries l = threadIdx.x + 256 i (blockDim.x == 256): the
// tile-local bits 0..7 come from the thread, bits 8.. from i.
__device__ inline uint32_t tile_lo_offset(const int* P, int np) {
  uint32_t off = 0;
  const uint32_t l = threadIdx.x;
  for (int b = 0; b < np && b < 8; ++b) off |= ((l >> b) & 1u) << P[b];
  return off;
}
__device__ inline uint32_t tile_hi_offset(const int* P, int np, uint32_t i) {
  uint32_t off = 0;
  for (int b = 8; b < np; ++b) off |= ((i >> (b - 8)) & 1u) << P[b];
  return off;
}

template <bool CLUSTERS = false>
__device__ inline void window_tile_pass(const FusedStep* fs, int n_fs, const int* P, int np, int r, uint32_t t,
                                        float2* Aj, const GateCtx& g_, int traj, const uint64_t* pw,
                                        float2* tile, float2* Gm, const float2* Ucl, bool gates_ready = false) {
  const uint32_t base = deposit_tile(t, P, np, r);
  const uint32_t nt = 1u << np;
  constexpr int kPer = (1 << kFuseMax) / 256;      // entries per thread at most
  const uint32_t lo = base | tile_lo_offset(P, np);
  {
    // all of the thread's loads in flight before the first LDS write
    float2 v[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i)
      if (threadIdx.x + 256u * i < nt) v[i] = Aj[lo | tile_hi_offset(P, np, (uint32_t)i)];
#pragma unroll
    for (int i = 0; i < kPer; ++i)
      if (threadIdx.x + 256u * i < nt) tile[threadIdx.x + 256u * i] = v[i];
  }
  __syncthreads();   // the tile is complete before any step reads it
  for (int s = 0; s < n_fs; ++s) {
    const FusedStep& st = fs[s];
    if (s % kGateChunk == 0 && !(s == 0 && gates_ready)) {   // every thread is past step s - 1 (barrier)
      const int cnt = (n_fs - s < kGateChunk ? n_fs - s : kGateChunk) * 16;
      for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        const FusedStep& sj = fs[s + i / 16];
        Gm[i] = gate_entry(g_, sj.gate, traj, sj.conj, i % 16);
      }
      __syncthreads();
    }
    const float2* G = Gm + 16 * (s % kGateChunk);
    if (CLUSTERS && st.cl_len > 0) {   // a gate cluster on MFMA, matrix built beforehand (ends with a barrier)
      apply_cluster(st.cl_pos, Ucl + 256 * st.cl_id, np, tile);
      s += st.cl_len - 1;        // the cluster lies inside one staged chunk
      continue;
    }
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
#pragma unroll
  for (int i = 0; i < kPer; ++i)
    if (threadIdx.x + 256u * i < nt) Aj[lo | tile_hi_offset(P, np, (uint32_t)i)] = tile[threadIdx.x + 256u * i];
  __syncthreads();
}

}  // namespace
}  // namespace ptsbe
