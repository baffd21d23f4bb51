// HIP kernels of the PTSBE hot path for CDNA4 (gfx950, 64-wide wavefronts).
//
//  * gate operand load with the unified-path-variation merge fused in (Sec.
//    III-A): the default-branch merged tensor is shared; a (trajectory, gate)
//    whose sampled Kraus indices deviate gets (prod K/sqrt(q)) . d_l on the fly.
//  * part_vm_kernel: a whole sweep (a list of absorb steps) for one job with the
//    running tensor in LDS (small per-element / per-trajectory parts).
//  * absorb_global_kernel: one absorb step over all jobs in HBM (large parts).
//  * join kernels: the per-element contraction of the prefix part with the
//    per-trajectory part, giving marginals (doubled network) or amplitudes.
//  * sample_kernel: FP64 inclusive prefix sum of a marginal in LDS and
//    inverse-CDF draws for every shot routed through the element (Sec. II-B).
//  * children_kernel: non-degenerate batching (Sec. III-B): the distinct
//    (prefix, x) of an element's shots become the next batch's elements.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.h"
#include "internal.h"
#include "philox.h"

namespace ptsbe {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));



__global__ void upv_merge_kernel(GateCtx g, int64_t E, float2* __restrict__ merged) {
  for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < E * g.G; id += (int64_t)gridDim.x * blockDim.x) {
    const int traj = (int)(id / g.G), gate = (int)(id % g.G);
    float2 m[16];
    merge_gate(g, gate, traj, m);
    float4* o = reinterpret_cast<float4*>(merged + id * 16);
    for (int i = 0; i < 8; ++i) o[i] = make_float4(m[2 * i].x, m[2 * i].y, m[2 * i + 1].x, m[2 * i + 1].y);
  }
}



__device__ inline int slice_base(const AbsorbStep& st, const uint64_t* prefix) {
  int sb = 0;
  for (int i = 0; i < st.nS; ++i) sb += (int)bit_of_prefix(prefix, st.sq[i]) * st.sw[i];
  return sb;
}

// C entries of all n for one kept index m (tables precomputed by the planner)
__device__ inline void absorb_one(const AbsorbStep& st, int sbase, uint32_t m, const float2* A, float2* C,
                                  const float2* Gm) {
  // the 16 slots are unrolled with a predicate so that a[] stays in registers
  float2 a[16];
  const int nK = st.nK, nN = st.nN;
  const uint32_t abase = insert_zero_bits(m, st.kpos, nK);
  const int nk = 1 << nK;
  // A always holds the running tensor; before the first step it is the scalar 1
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (k < nk) a[k] = A[abase + st.koff[k]];
  int hidx = sbase;
  for (int i = 0; i < st.nH; ++i) hidx += (int)((m >> st.hm[i]) & 1u) * st.hw[i];
  const uint32_t cbase = insert_zero_bits(m, st.npos, nN);
  const int nn = 1 << nN;
  for (int n = 0; n < nn; ++n) {
    float2 acc = make_float2(0.f, 0.f);
    const int bn = hidx + st.nB[n];
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (k < nk) acc = cfma(a[k], Gm[bn + st.kB[k]], acc);
    C[cbase + st.noff[n]] = acc;
  }
}

// U kept indices m[u] at once (m[u] < nm for u < nu): every A load of the U
// indices is issued before the first product, so a thread keeps U * 2^nK loads
// in flight (the steps in HBM are bound by memory latency otherwise).  NK is an
// upper bound of 2^nK.
template <int NK, int U>
__device__ inline void absorb_multi(const AbsorbStep& st, int sbase, const uint32_t* m, int nu, const float2* A,
                                    float2* C, const float2* Gm) {
  float2 a[U][NK];
  const int nK = st.nK, nN = st.nN;
  const int nk = 1 << nK;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t abase = insert_zero_bits(m[u], st.kpos, nK);
#pragma unroll
    for (int k = 0; k < NK; ++k)
      if (u < nu && k < nk) a[u][k] = A[abase + st.koff[k]];
  }
  const int nn = 1 << nN;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (u >= nu) break;
    int hidx = sbase;
    for (int i = 0; i < st.nH; ++i) hidx += (int)((m[u] >> st.hm[i]) & 1u) * st.hw[i];
    const uint32_t cbase = insert_zero_bits(m[u], st.npos, nN);
    for (int n = 0; n < nn; ++n) {
      float2 acc = make_float2(0.f, 0.f);
      const int bn = hidx + st.nB[n];
#pragma unroll
      for (int k = 0; k < NK; ++k)
        if (k < nk) acc = cfma(a[u][k], Gm[bn + st.kB[k]], acc);
      C[cbase + st.noff[n]] = acc;
    }
  }
}

// ------------------------------------------------------------------ LDS sweep
// One absorb step over the (job, kept index) items of a workgroup's jobs, for a
// step with NK contracted and NN new legs (NK + NN <= 4: a gate tensor has at
// most four legs).  The step's tables are read once into registers before the
// item loop, and each item issues all of its LDS reads (2^NK entries of A,
// 2^(NK+NN) gate entries) before its first product, so that a step costs one
// round of scalar loads and one round of LDS latency instead of one per product.
// Products are accumulated in the order of absorb_one (k ascending from zero),
// so the results are the same bit for bit.
// PLAIN: no hyper or sliced legs; the staged gate is in (n, k) order, so the
// gate entries of a product are read at fixed offsets from the job's slot.
template <int NK, int NN, bool PLAIN>
// C rows are c_stride apart from Cb: the LDS buffer, or the output in HBM for a
// last step that raises the rank past every other tensor of the sweep.
__device__ __forceinline__ void vm_step(const AbsorbStep& st, int nj, int lnm, int buf_elems, const float2* bufA,
                                        float2* Cb, int64_t c_stride, const float2* G, const int* slot,
                                        const uint64_t* pw, int NW) {
  constexpr int nk = 1 << NK, nn = 1 << NN;
  const int items = nj << lnm;
  if ((int)threadIdx.x >= items) return;   // waves without items skip the step's table reads
  int kpos[NK > 0 ? NK : 1], npos[NN > 0 ? NN : 1], hm[4], hw[4], sq[kMaxSlices], sw[kMaxSlices];
  uint32_t koff[nk], noff[nn];
  int kB[nk], nB[nn];
#pragma unroll
  for (int i = 0; i < NK; ++i) kpos[i] = st.kpos[i];
#pragma unroll
  for (int i = 0; i < NN; ++i) npos[i] = st.npos[i];
#pragma unroll
  for (int k = 0; k < nk; ++k) { koff[k] = st.koff[k]; kB[k] = st.kB[k]; }
#pragma unroll
  for (int n = 0; n < nn; ++n) { noff[n] = st.noff[n]; nB[n] = st.nB[n]; }
#pragma unroll
  for (int i = 0; i < 4; ++i) { hm[i] = st.hm[i]; hw[i] = st.hw[i]; }
#pragma unroll
  for (int i = 0; i < kMaxSlices; ++i) { sq[i] = st.sq[i]; sw[i] = st.sw[i]; }
  const int nH = st.nH, nS = st.nS;
  const uint32_t mmask = (1u << lnm) - 1u;
  for (int i = threadIdx.x; i < items; i += blockDim.x) {
    const int j = i >> lnm;
    const uint32_t m = (uint32_t)i & mmask;
    const uint64_t* pj = pw + j * NW;
    int hidx = 0;
    if (!PLAIN) {
#pragma unroll
      for (int t = 0; t < kMaxSlices; ++t)
        if (t < nS) hidx += (int)bit_of_prefix(pj, sq[t]) * sw[t];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < nH) hidx += (int)((m >> hm[t]) & 1u) * hw[t];
    }
    uint32_t abase = m, cbase = m;
#pragma unroll
    for (int t = 0; t < NK; ++t) abase = ((abase >> kpos[t]) << (kpos[t] + 1)) | (abase & ((1u << kpos[t]) - 1u));
#pragma unroll
    for (int t = 0; t < NN; ++t) cbase = ((cbase >> npos[t]) << (npos[t] + 1)) | (cbase & ((1u << npos[t]) - 1u));
    const float2* Aj = bufA + (size_t)j * buf_elems;
    const float2* Gj = G + 16 * slot[j] + hidx;
    float2 a[nk], gv[nn][nk];
#pragma unroll
    for (int k = 0; k < nk; ++k) a[k] = Aj[abase + koff[k]];
#pragma unroll
    for (int n = 0; n < nn; ++n)
#pragma unroll
      for (int k = 0; k < nk; ++k) gv[n][k] = PLAIN ? Gj[n * nk + k] : Gj[nB[n] + kB[k]];
    float2* Cj = Cb + (int64_t)j * c_stride + cbase;
#pragma unroll
    for (int n = 0; n < nn; ++n) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int k = 0; k < nk; ++k) acc = cfma(a[k], gv[n][k], acc);
      Cj[noff[n]] = acc;
    }
  }
}

__device__ inline uint32_t init_offset(const InitArgs& in, uint32_t m, const uint64_t* pw) {
  for (int i = 0; i < in.nsl; ++i) {
    const int p = in.pos[i];
    const uint32_t lo = m & ((1u << p) - 1u);
    m = ((m >> p) << (p + 1)) | (bit_of_prefix(pw, in.q[i]) << p) | lo;
  }
  return m;
}

// gate entries staged per chunk of steps: [chunk steps][trajectory slots][16] float2
constexpr int kVmGateEntries = 512;
constexpr int kVmMaxJobs = 64;        // jobs per workgroup (one wavefront assigns the trajectory slots)

__global__ void __launch_bounds__(256) part_vm_kernel(const AbsorbStep* __restrict__ steps, int n_steps,
                                                      int buf_elems, int J, GateCtx g, int64_t n_jobs,
                                                      const int32_t* __restrict__ job_traj, int32_t traj_base,
                                                      const uint64_t* __restrict__ job_prefix, int NW,
                                                      InitArgs init, float2* __restrict__ out, int out_rank,
                                                      int direct) {
  // J jobs per workgroup run the same step list in lockstep: each step's
  // descriptor is decoded once for all of them and the threads take
  // (job, kept index) work items.  Consecutive jobs of one trajectory (the
  // elements of a batch are grouped by trajectory) share one slot of gate
  // entries, so a step stages 16 entries per distinct trajectory, not per job.
  extern __shared__ float2 lds[];
  __shared__ int slot[kVmMaxJobs], slot_traj[kVmMaxJobs], n_slots_s;
  float2* bufA = lds;                                   // [J][buf_elems]
  float2* bufC = lds + (size_t)J * buf_elems;           // [J][buf_elems]
  float2* Gm = lds + 2 * (size_t)J * buf_elems;         // [chunk][slots][16] gates of a chunk of steps
  int4* stab = reinterpret_cast<int4*>(Gm + kVmGateEntries);   // [n_steps] gate | conj << 31, gperm
  uint64_t* pw = reinterpret_cast<uint64_t*>(stab + n_steps);  // [J][NW] prefixes
  const int tid = threadIdx.x, nt = blockDim.x;
  // the step list's gate indices, once per workgroup (visible after the first barrier)
  for (int s = tid; s < n_steps; s += nt)
    stab[s] = make_int4(steps[s].gate | (steps[s].conj ? (int)0x80000000 : 0), (int)steps[s].gperm[0],
                        (int)steps[s].gperm[1], 0);
  const int64_t n_groups = (n_jobs + J - 1) / J;
  for (int64_t grp = blockIdx.x; grp < n_groups; grp += gridDim.x) {
    const int64_t job0 = grp * J;
    const int nj = (int)(n_jobs - job0 < J ? n_jobs - job0 : J);
    for (int i = tid; i < nj * NW; i += nt) pw[i] = job_prefix ? job_prefix[job0 * NW + i] : 0ull;
    if (tid < 64) {   // wavefront 0: a slot per run of equal trajectories
      const bool live = tid < nj;
      const int tj = live ? (job_traj ? job_traj[job0 + tid] : traj_base + (int)(job0 + tid)) : -1;
      const int tprev = __shfl_up(tj, 1);
      const bool start = live && (tid == 0 || tprev != tj);
      const uint64_t starts = __ballot(start);
      const int sl = __popcll(starts & ((2ull << tid) - 1ull)) - 1;
      if (live) slot[tid] = sl;
      if (start) slot_traj[sl] = tj;
      if (tid == 0) n_slots_s = __popcll(starts);
    }
    __syncthreads();
    const int n_slots = n_slots_s;
    const int per_step = 16 * n_slots;
    const int chunk = kVmGateEntries / per_step > 1 ? kVmGateEntries / per_step : 1;
    // gates of the steps [c0, c1) in LDS, every (step, slot, entry) of the chunk
    // spread over all threads, two loads per thread in flight together
    // (unconditional, from a clamped valid entry), the bra conjugation applied at
    // the store
    auto stage = [&](int c0, int c1) {
      const int E = (c1 - c0) * per_step;
      for (int e0 = 0; e0 < E; e0 += 2 * nt) {
        float2 v[2];
        int dst[2];
        bool neg[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int e = e0 + u * nt + tid;
          dst[u] = e < E ? e : -1;
          const int ec = e < E ? e : E - 1;
          const int q = ec >> 4, gi = ec & 15;
          const int si = q / n_slots, sl = q - si * n_slots;
          const int4 sd = stab[c0 + si];
          const uint32_t perm = (uint32_t)(gi < 8 ? sd.y : sd.z);
          const uint32_t src = (perm >> (4 * (gi & 7))) & 15u;
          neg[u] = sd.x < 0;
          v[u] = g.merged[((int64_t)slot_traj[sl] * g.G + (sd.x & 0x7fffffff)) * 16 + src];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
          if (dst[u] >= 0) Gm[dst[u]] = neg[u] ? make_float2(v[u].x, -v[u].y) : v[u];
      }
    };
    if (init.Vprev) {
      // nt / J threads per job: one parent index per thread, and every entry's
      // load issued before the first store (at most 8 per thread: J 2^r0 <= 2048)
      const uint32_t n0 = 1u << init.r0;
      const int tpj = nt / J, j = tid / tpj, jl = tid - j * tpj;
      if (j < nj) {
        const float2* src = init.Vprev + (int64_t)init.parent[job0 + j] * init.stride;
        const uint64_t* pj = pw + j * NW;
        float2* dst = bufA + (size_t)j * buf_elems;
        float2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const uint32_t m = (uint32_t)(jl + u * tpj);
          if (m < n0) v[u] = src[init_offset(init, m, pj)];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const uint32_t m = (uint32_t)(jl + u * tpj);
          if (m < n0) dst[m] = v[u];
        }
        for (uint32_t m = (uint32_t)(jl + 8 * tpj); m < n0; m += tpj) dst[m] = src[init_offset(init, m, pj)];
      }
    } else {
      for (int j = tid; j < nj; j += nt) bufA[(size_t)j * buf_elems] = make_float2(1.f, 0.f);
    }
    int cs = 0;
    if (n_steps > 0) stage(0, n_steps < chunk ? n_steps : chunk);
    for (int s = 0; s < n_steps; ++s) {
      const AbsorbStep& st = steps[s];
      if (s == cs + chunk) {
        cs = s;
        __syncthreads();   // every thread is done with the previous chunk's gates
        stage(cs, n_steps - cs < chunk ? n_steps : cs + chunk);
      }
      const float2* G = Gm + (size_t)(s - cs) * per_step;
      __syncthreads();     // gates visible; previous step's C complete
      const int lnm = st.rC - st.nN;
      if (direct && s == n_steps - 1) {
        // the last step writes the output in HBM (its rank exceeds the LDS buffers)
        float2* Co = out + job0 * ((int64_t)1 << out_rank);
        const int64_t cst = (int64_t)1 << out_rank;
        switch (st.nK * 8 + st.nN) {
#define VM_OUT(K, N)                                                                       \
          case K * 8 + N:                                                                  \
            if (st.nH == 0 && st.nS == 0)                                                  \
              vm_step<K, N, true>(st, nj, lnm, buf_elems, bufA, Co, cst, G, slot, pw, NW); \
            else                                                                           \
              vm_step<K, N, false>(st, nj, lnm, buf_elems, bufA, Co, cst, G, slot, pw, NW); \
            break;
          VM_OUT(0, 1) VM_OUT(0, 2) VM_OUT(0, 3) VM_OUT(0, 4) VM_OUT(1, 2) VM_OUT(1, 3)
#undef VM_OUT
          default: break;   // not reached: the host sets direct for these leg counts only
        }
        continue;
      }
      switch (st.nK * 8 + st.nN) {    // uniform: every thread takes the same case
#define VM_CASE(K, N)                                                                     \
        case K * 8 + N:                                                                   \
          if (st.nH == 0 && st.nS == 0)                                                   \
            vm_step<K, N, true>(st, nj, lnm, buf_elems, bufA, bufC, buf_elems, G, slot, pw, NW);  \
          else                                                                            \
            vm_step<K, N, false>(st, nj, lnm, buf_elems, bufA, bufC, buf_elems, G, slot, pw, NW); \
          break;
        VM_CASE(0, 0) VM_CASE(0, 1) VM_CASE(0, 2) VM_CASE(0, 3) VM_CASE(0, 4)
        VM_CASE(1, 0) VM_CASE(1, 1) VM_CASE(1, 2) VM_CASE(1, 3)
        VM_CASE(2, 0) VM_CASE(2, 1) VM_CASE(2, 2)
        VM_CASE(3, 0) VM_CASE(3, 1)
        VM_CASE(4, 0)
#undef VM_CASE
        default: {   // not reached: a gate tensor has at most four legs, and the cases above take
                     // every step with nK + nN <= 4 (the gate is staged in B's order for these only
                     // when the step has hyper or sliced legs)
          const int items = nj << lnm;
          for (int i = tid; i < items; i += nt) {
            const int j = i >> lnm;
            const uint32_t m = (uint32_t)i & ((1u << lnm) - 1u);
            absorb_one(st, slice_base(st, pw + j * NW), m, bufA + (size_t)j * buf_elems,
                       bufC + (size_t)j * buf_elems, G + 16 * slot[j]);
          }
        }
      }
      float2* t = bufA; bufA = bufC; bufC = t;
    }
    __syncthreads();
    const int64_t n_out = (int64_t)1 << out_rank;
    if (!direct || n_steps == 0)
      for (int64_t i = tid; i < (int64_t)nj * n_out; i += nt) {
        const int64_t j = i >> out_rank, k = i & (n_out - 1);
        out[(job0 + j) * n_out + k] = bufA[j * buf_elems + k];
      }
    __syncthreads();   // LDS is reused by the next group of this workgroup
  }
}

// --------------------------------------------------------------- HBM sweep step
constexpr uint32_t kAbsorbPerBlock = 2048;

template <int NK>
__global__ void absorb_global_kernel(const AbsorbStep* __restrict__ st_dev, GateCtx g, int64_t n_jobs,
                                     int64_t blocks_per_job, const int32_t* __restrict__ job_traj,
                                     int32_t traj_base, const uint64_t* __restrict__ job_prefix, int NW,
                                     const float2* A, float2* C) {   // A == C allowed for in-place steps
  __shared__ float2 Gm[16];
  __shared__ uint64_t pw[16];
  const AbsorbStep& st = *st_dev;
  for (int64_t bid = blockIdx.x; bid < n_jobs * blocks_per_job; bid += gridDim.x) {
  const int64_t job = bid / blocks_per_job;
  const int64_t chunk = bid % blocks_per_job;
  const int traj = job_traj ? job_traj[job] : traj_base + (int)job;
  if (threadIdx.x < NW) pw[threadIdx.x] = job_prefix ? job_prefix[job * NW + threadIdx.x] : 0ull;
  if (threadIdx.x < 16) Gm[threadIdx.x] = gate_entry(g, st.gate, traj, st.conj, threadIdx.x);
  __syncthreads();
  const int sb = slice_base(st, pw);
  const uint32_t nm = 1u << (st.rC - st.nN);
  const float2* Aj = A + (job << st.rA);
  float2* Cj = C + (job << st.rC);
  // each block covers kAbsorbPerBlock kept indices (the gate load is amortised);
  // a thread takes 4 of them at a time, blockDim.x apart (coalesced per u)
  const uint32_t m0 = (uint32_t)(chunk * kAbsorbPerBlock);
  if (NK > 4) {
    for (uint32_t i = threadIdx.x; i < kAbsorbPerBlock; i += blockDim.x) {
      const uint32_t m = m0 + i;
      if (m >= nm) break;
      absorb_one(st, sb, m, Aj, Cj, Gm);
    }
  } else {
    for (uint32_t i0 = 0; i0 < kAbsorbPerBlock; i0 += 4 * blockDim.x) {
      uint32_t m[4];
      int nu = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        m[u] = m0 + i0 + threadIdx.x + u * blockDim.x;
        nu += m[u] < nm && i0 + threadIdx.x + u * blockDim.x < kAbsorbPerBlock;
      }
      if (nu == 0) break;
      absorb_multi<NK, 4>(st, sb, m, nu, Aj, Cj, Gm);
    }
  }
  __syncthreads();   // Gm and pw are rewritten for the next block of this workgroup
  }
}

// A fused run of in-place steps: one workgroup per (job, tile); the tile is the
// 2^np entries whose non-P bits equal the tile index; every step of the run is
// applied to the tile in LDS before it is written back.
struct FusedArgs {
  const FusedStep* fs; int n_fs;
  int r, np;
  int P[kFuseMax];
  int64_t tiles_per_job;
  const float2* Ucl; int n_cl;    // gate-cluster matrices [job][n_cl][256], or null
};


// Gate-cluster matrices, one workgroup per (job, cluster): the members' merged
// gate matrices of the job's trajectory are staged in LDS and multiplied up.
__global__ void __launch_bounds__(256) cluster_build_kernel(const ClusterDesc* __restrict__ cl, int n_cl,
                                                           const FusedStep* __restrict__ fused, GateCtx g,
                                                           int64_t n_jobs, const int32_t* __restrict__ job_traj,
                                                           int32_t traj_base, float2* __restrict__ Ucl) {
  __shared__ float2 Gm[16 * kGateChunk];
  __shared__ float2 Ua[256], Ub[256];
  for (int64_t bid = blockIdx.x; bid < n_jobs * n_cl; bid += gridDim.x) {
    const int64_t job = bid / n_cl;
    const int c = (int)(bid % n_cl);
    const int traj = job_traj ? job_traj[job] : traj_base + (int)job;
    const ClusterDesc& cd = cl[c];
    const FusedStep* fs = fused + cd.first;
    for (int i = threadIdx.x; i < 16 * cd.len; i += blockDim.x)
      Gm[i] = gate_entry(g, fs[i / 16].gate, traj, fs[i / 16].conj, i % 16);
    __syncthreads();
    const float2* U = build_cluster(fs, cd.len, Gm, Ua, Ub);
    Ucl[bid * 256 + threadIdx.x] = U[threadIdx.x];
    __syncthreads();   // Gm, Ua, Ub are reused by the next (job, cluster) of this workgroup
  }
}

template <bool CLUSTERS>
__global__ void __launch_bounds__(256) fused_inplace_kernel(FusedArgs f, GateCtx g, int64_t n_jobs,
                                                           const int32_t* __restrict__ job_traj, int32_t traj_base,
                                                           const uint64_t* __restrict__ job_prefix, int NW,
                                                           float2* A) {
  extern __shared__ float2 tile[];
  float2* Gm = tile + ((int64_t)1 << f.np);
  __shared__ uint64_t pw[16];
  // each workgroup takes a contiguous range of (job, tile) pairs, so that
  // consecutive tiles of one job reuse the staged gate matrices
  const int64_t total = n_jobs * f.tiles_per_job;
  const int64_t per = (total + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per, b1 = b0 + per < total ? b0 + per : total;
  int last_traj = -1;
  for (int64_t bid = b0; bid < b1; ++bid) {
    const int64_t job = bid / f.tiles_per_job;
    const uint32_t t = (uint32_t)(bid % f.tiles_per_job);
    const int traj = job_traj ? job_traj[job] : traj_base + (int)job;
    if ((int)threadIdx.x < NW) pw[threadIdx.x] = job_prefix ? job_prefix[job * NW + threadIdx.x] : 0ull;
    const bool ready = traj == last_traj && f.n_fs <= kGateChunk;
    window_tile_pass<CLUSTERS>(f.fs, f.n_fs, f.P, f.np, f.r, t, A + (job << f.r), g, traj, pw, tile, Gm,
                               CLUSTERS ? f.Ucl + job * (int64_t)f.n_cl * 256 : nullptr, ready);   // ends with a barrier
    last_traj = traj;
  }
}

__global__ void init_gather_kernel(InitArgs init, int64_t n_jobs, const uint64_t* __restrict__ job_prefix, int NW,
                                   float2* __restrict__ out) {
  const int64_t per = (int64_t)1 << init.r0;
  for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < per * n_jobs; id += (int64_t)gridDim.x * blockDim.x) {
    const int64_t job = id / per;
    const uint32_t m = (uint32_t)(id % per);
    const uint64_t* pw = job_prefix + job * NW;
    out[id] = init.Vprev[(int64_t)init.parent[job] * init.stride + init_offset(init, m, pw)];
  }
}

__global__ void fill_one_kernel(float2* buf, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    buf[i] = make_float2(1.f, 0.f);
}

// ------------------------------------------------------------------------ join
__device__ inline int64_t tab(const int64_t* base, int64_t lo_off, int64_t hi_off, int lo_bits, uint32_t g) {
  return base[lo_off + (g & ((1u << lo_bits) - 1u))] + base[hi_off + (g >> lo_bits)];
}

__global__ void join_kernel(JoinArgs a) {
  const int64_t rows = (int64_t)1 << a.xb_bits;
  const int64_t nx = (int64_t)1 << a.xT_bits;
  const int64_t total = a.n_elems * rows * nx;
  for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < total; id += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t x = (uint32_t)(id % nx);
    const uint32_t row = (uint32_t)((id / nx) % rows);
    const int64_t e = id / (nx * rows);
    const int lo_x = a.xT_bits < 12 ? a.xT_bits : 12;
    const int lo_b = a.xb_bits < 12 ? a.xb_bits : 12;
    const int lo_k = a.lk_bits < 12 ? a.lk_bits : 12;
    const float2* V = a.V + e * a.v_stride;
    const int32_t ti = a.elem_traj[e] - a.traj_base;
    const float2* T = a.T + (int64_t)(a.tslot ? a.tslot[ti] : ti) * a.t_stride;
    const int64_t vr = tab(a.tab, a.jd.vr_lo, a.jd.vr_hi, lo_b, row);
    const int64_t tx = tab(a.tab, a.jd.tx_lo, a.jd.tx_hi, lo_x, x);
    const int nk = 1 << a.lk_bits;
    const int64_t oidx = tab(a.tab, a.jd.ox_lo, a.jd.ox_hi, lo_x, x) + tab(a.tab, a.jd.ob_lo, a.jd.ob_hi, lo_b, row);
    const int64_t nout = (int64_t)1 << a.b;
    if (a.doubled) {
      float acc = 0.f;
      for (int k2 = 0; k2 < nk; ++k2) {
        const float2 v2 = V[vr + tab(a.tab, a.jd.vc_lo, a.jd.vc_hi, lo_k, k2)];
        const int64_t tb = tab(a.tab, a.jd.tb_lo, a.jd.tb_hi, lo_k, k2);
        float2 y = make_float2(0.f, 0.f);
        for (int k = 0; k < nk; ++k) {
          const float2 v = V[vr + tab(a.tab, a.jd.vc_lo, a.jd.vc_hi, lo_k, k)];
          y = cfma(v, T[tx + tab(a.tab, a.jd.tk_lo, a.jd.tk_hi, lo_k, k) + tb], y);
        }
        acc += y.x * v2.x + y.y * v2.y;   // Re(y * conj(v2))
      }
      a.pop[e * nout + oidx] = acc;
    } else {
      float2 y = make_float2(0.f, 0.f);
      for (int k = 0; k < nk; ++k) {
        const float2 v = V[vr + tab(a.tab, a.jd.vc_lo, a.jd.vc_hi, lo_k, k)];
        y = cfma(v, T[tx + tab(a.tab, a.jd.tk_lo, a.jd.tk_hi, lo_k, k)], y);
      }
      if (a.amp) a.amp[e * nout + oidx] = y;
      if (a.pop) a.pop[e * nout + oidx] = y.x * y.x + y.y * y.y;
    }
  }
}

// Last-batch join when every element has at most four rows (2^xb <= 4) and its
// trajectory few elements: amp[e][o(x, r)] = sum_k V[e][r][k] T[t][x][k] with T
// read in the right part's own layout through the plan's tables, so T crosses
// HBM once per element and needs no canonical copy (an HBM-bound GEMV: 1 flop
// per byte of T).  A workgroup takes 256 consecutive x of one element; the
// element's V rows and the k offsets of T are staged in LDS.
template <int ROWS>
__global__ void __launch_bounds__(256) ketjoin_gemv_kernel(JoinArgs a) {
  __shared__ float2 Vs[ROWS][64];
  __shared__ int64_t tk[64];
  const int nk = 1 << a.lk_bits;
  const int64_t tiles = (int64_t)1 << (a.xT_bits - 8);
  const int lo_x = a.xT_bits < 12 ? a.xT_bits : 12;
  const int lo_b = a.xb_bits < 12 ? a.xb_bits : 12;
  const int lo_k = a.lk_bits < 12 ? a.lk_bits : 12;
  const int tid = threadIdx.x;
  if (tid < nk) tk[tid] = tab(a.tab, a.jd.tk_lo, a.jd.tk_hi, lo_k, (uint32_t)tid);
  const int64_t nout = (int64_t)1 << a.b;
  for (int64_t bid = blockIdx.x; bid < a.n_elems * tiles; bid += gridDim.x) {
    const int64_t e = bid >> (a.xT_bits - 8);
    const uint32_t x = (uint32_t)(((bid & (tiles - 1)) << 8) + tid);
    __syncthreads();                       // the previous element's Vs is no longer read
    if (tid < ROWS * nk) {
      const int r = tid / nk, k = tid % nk;
      Vs[r][k] = a.V[e * a.v_stride + tab(a.tab, a.jd.vr_lo, a.jd.vr_hi, lo_b, (uint32_t)r) +
                     tab(a.tab, a.jd.vc_lo, a.jd.vc_hi, lo_k, (uint32_t)k)];
    }
    __syncthreads();
    const int32_t ti = a.elem_traj[e] - a.traj_base;
    const float2* T = a.T + (int64_t)(a.tslot ? a.tslot[ti] : ti) * a.t_stride +
                      tab(a.tab, a.jd.tx_lo, a.jd.tx_hi, lo_x, x);
    float2 acc[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) acc[r] = make_float2(0.f, 0.f);
#pragma unroll 8
    for (int k = 0; k < nk; ++k) {
      const float2 t = T[tk[k]];
#pragma unroll
      for (int r = 0; r < ROWS; ++r) acc[r] = cfma(Vs[r][k], t, acc[r]);
    }
    const int64_t ox = tab(a.tab, a.jd.ox_lo, a.jd.ox_hi, lo_x, x);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      const int64_t o = e * nout + ox + tab(a.tab, a.jd.ob_lo, a.jd.ob_hi, lo_b, (uint32_t)r);
      if (a.amp) a.amp[o] = acc[r];
      if (a.pop) a.pop[o] = acc[r].x * acc[r].x + acc[r].y * acc[r].y;
    }
  }
}

// The same GEMV over tiles of 4096 values of x (GemvTiling): thread t reads the
// 16 values i = t + 256 j of the tile (i's bits are the tile bits in order of
// their T offsets, so a wavefront's reads are contiguous runs), accumulates all
// k in registers, and the populations pass through LDS to be written in order
// of their output offsets.
// k is taken in chunks of kGemvKChunk (the chunk's V rows and T offsets staged in
// LDS), so that crossings of up to 12 wires (a sliced last batch keeps many) fit.
constexpr int kGemvKChunk = 512;

template <int ROWS>
__global__ void __launch_bounds__(256) ketjoin_gemv_tiled_kernel(JoinArgs a, GemvTiling g) {
  __shared__ float2 Vs[ROWS][kGemvKChunk];
  __shared__ int64_t tk[kGemvKChunk];
  __shared__ float outs[ROWS][4096];
  const int nk = 1 << a.lk_bits;
  const int lo_b = a.xb_bits < 12 ? a.xb_bits : 12;
  const int lo_k = a.lk_bits < 12 ? a.lk_bits : 12;
  const int tid = threadIdx.x;
  int64_t t_lo = 0, or_lo = 0, w_lo = 0;
  int l_lo = 0;
#pragma unroll
  for (int s = 0; s < 8; ++s)
    if ((tid >> s) & 1) {
      t_lo += g.t_off[s];
      or_lo += g.o_read[s];
      l_lo += 1 << g.w_of[s];
      w_lo += g.o_off[s];
    }
  const int64_t nout = (int64_t)1 << a.b;
  const int64_t tiles = (int64_t)1 << g.n_hi;
  int64_t obr[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) obr[r] = tab(a.tab, a.jd.ob_lo, a.jd.ob_hi, lo_b, (uint32_t)r);
  for (int64_t bid = blockIdx.x; bid < a.n_elems * tiles; bid += gridDim.x) {
    const int64_t e = bid >> g.n_hi;
    const int64_t tile = bid & (tiles - 1);
    int64_t tbase = 0, obase = 0;
    for (int h = 0; h < g.n_hi; ++h)
      if ((tile >> h) & 1) { tbase += g.t_hi[h]; obase += g.o_hi[h]; }
    const int32_t ti = a.elem_traj[e] - a.traj_base;
    const float2* T = a.T + (int64_t)(a.tslot ? a.tslot[ti] : ti) * a.t_stride + tbase + t_lo;
    float2 acc[16][ROWS];
#pragma unroll
    for (int j = 0; j < 16; ++j)
#pragma unroll
      for (int r = 0; r < ROWS; ++r) acc[j][r] = make_float2(0.f, 0.f);
    for (int k0 = 0; k0 < nk; k0 += kGemvKChunk) {
      const int kn = nk - k0 < kGemvKChunk ? nk - k0 : kGemvKChunk;
      __syncthreads();                     // Vs, tk and outs of the previous chunk or tile are no longer read
      for (int i = tid; i < ROWS * kn; i += 256) {
        const int r = i / kn, k = i % kn;
        Vs[r][k] = a.V[e * a.v_stride + tab(a.tab, a.jd.vr_lo, a.jd.vr_hi, lo_b, (uint32_t)r) +
                       tab(a.tab, a.jd.vc_lo, a.jd.vc_hi, lo_k, (uint32_t)(k0 + k))];
      }
      for (int k = tid; k < kn; k += 256) tk[k] = tab(a.tab, a.jd.tk_lo, a.jd.tk_hi, lo_k, (uint32_t)(k0 + k));
      __syncthreads();
      for (int k = 0; k < kn; ++k) {
        const float2* Tk = T + tk[k];
        float2 v[ROWS];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) v[r] = Vs[r][k];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          int64_t hj = 0;
#pragma unroll
          for (int s = 0; s < 4; ++s)
            if ((j >> s) & 1) hj += g.t_off[8 + s];
          const float2 t = Tk[hj];
#pragma unroll
          for (int r = 0; r < ROWS; ++r) acc[j][r] = cfma(v[r], t, acc[j][r]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      int li = l_lo;
      int64_t orj = or_lo;
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if ((j >> s) & 1) { li += 1 << g.w_of[8 + s]; orj += g.o_read[8 + s]; }
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        outs[r][li] = acc[j][r].x * acc[j][r].x + acc[j][r].y * acc[j][r].y;
        if (a.amp) a.amp[e * nout + obase + orj + obr[r]] = acc[j][r];
      }
    }
    __syncthreads();
    if (a.pop) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        int64_t oj = w_lo;
#pragma unroll
        for (int s = 0; s < 4; ++s)
          if ((j >> s) & 1) oj += g.o_off[8 + s];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) a.pop[e * nout + obase + oj + obr[r]] = outs[r][tid + 256 * j];
      }
    }
  }
}

// GEMV join with the six lowest-offset bits of T on the lanes (GemvLanes): a
// wavefront reads 64 neighbouring entries of T per k value off the lanes, each
// lane accumulates its own k values, and the k lane bits are summed by a fixed
// butterfly of shuffles.  A workgroup stages one element's V rows and the k
// offsets off the lanes in LDS; its wavefronts take values of the x bits off the
// lanes in turn.
template <int ROWS>
__global__ void __launch_bounds__(256) ketjoin_gemv_lanes_kernel(JoinArgs a, GemvLanes g, int64_t wg_per_elem) {
  extern __shared__ float2 lds_gl[];
  const int nk = 1 << a.lk_bits, nkh = 1 << g.n_hk;
  float2* Vs = lds_gl;                                              // [ROWS][nk]
  int64_t* khoff = reinterpret_cast<int64_t*>(Vs + ROWS * nk);      // [nkh] T offset of the k bits off the lanes
  int* khval = reinterpret_cast<int*>(khoff + nkh);                 // [nkh] their k value
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lo_b = a.xb_bits < 12 ? a.xb_bits : 12, lo_k = a.lk_bits < 12 ? a.lk_bits : 12;
  int64_t ltoff = 0, looff = 0;
  int lkv = 0, kred = 0;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    if ((lane >> i) & 1) { ltoff += g.lane_toff[i]; looff += g.lane_ooff[i]; lkv |= g.lane_kbit[i]; }
    if (g.lane_is_k[i]) kred |= 1 << i;
  }
  const bool writer = (lane & kred) == 0;
  for (int i = tid; i < nkh; i += 256) {
    int64_t o = 0;
    int v = 0;
    for (int h = 0; h < g.n_hk; ++h)
      if ((i >> h) & 1) { o += g.hk_toff[h]; v |= g.hk_kbit[h]; }
    khoff[i] = o;
    khval[i] = v;
  }
  const int64_t nxb = (int64_t)1 << g.n_hx;
  const int64_t nout = (int64_t)1 << a.b;
  int64_t obr[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) obr[r] = tab(a.tab, a.jd.ob_lo, a.jd.ob_hi, lo_b, (uint32_t)r);
  for (int64_t bid = blockIdx.x; bid < a.n_elems * wg_per_elem; bid += gridDim.x) {
    const int64_t e = bid / wg_per_elem, gi = bid % wg_per_elem;
    __syncthreads();                       // the previous element's V rows are no longer read
    for (int i = tid; i < ROWS * nk; i += 256) {
      const int r = i / nk, k = i % nk;
      Vs[i] = a.V[e * a.v_stride + tab(a.tab, a.jd.vr_lo, a.jd.vr_hi, lo_b, (uint32_t)r) +
                  tab(a.tab, a.jd.vc_lo, a.jd.vc_hi, lo_k, (uint32_t)k)];
    }
    __syncthreads();
    const int32_t ti = a.elem_traj[e] - a.traj_base;
    const float2* T = a.T + (int64_t)(a.tslot ? a.tslot[ti] : ti) * a.t_stride + ltoff;
    for (int64_t xb = gi * 4 + wave; xb < nxb; xb += wg_per_elem * 4) {
      int64_t xto = 0, xoo = 0;
      for (int h = 0; h < g.n_hx; ++h)
        if ((xb >> h) & 1) { xto += g.hx_toff[h]; xoo += g.hx_ooff[h]; }
      float2 acc[ROWS];
#pragma unroll
      for (int r = 0; r < ROWS; ++r) acc[r] = make_float2(0.f, 0.f);
#pragma unroll 8
      for (int kh = 0; kh < nkh; ++kh) {
        const float2 t = T[xto + khoff[kh]];
        const int kv = lkv | khval[kh];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) acc[r] = cfma(Vs[r * nk + kv], t, acc[r]);
      }
#pragma unroll
      for (int i = 0; i < 6; ++i)
        if ((kred >> i) & 1)
#pragma unroll
          for (int r = 0; r < ROWS; ++r) {
            acc[r].x += __shfl_xor(acc[r].x, 1 << i);
            acc[r].y += __shfl_xor(acc[r].y, 1 << i);
          }
      if (writer)
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
          const int64_t o = e * nout + looff + xoo + obr[r];
          if (a.amp) a.amp[o] = acc[r];
          if (a.pop) a.pop[o] = acc[r].x * acc[r].x + acc[r].y * acc[r].y;
        }
    }
  }
}

// Gather the per-trajectory part T into the canonical layout used by the MFMA
// join: Tc[x][k][k'] with k' fastest (K = 2^lk_bits), via the plan's tables.
__global__ void permute_T_kernel(const float2* __restrict__ T, int64_t t_stride, int64_t n_traj,
                                 const int64_t* __restrict__ tables, Plan::JoinDev jd, int xT_bits, int lk_bits,
                                 int lb_bits, float2* __restrict__ Tc) {
  const int64_t per = (int64_t)1 << (xT_bits + lk_bits + lb_bits);
  for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < per * n_traj; id += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = id / per, r = id % per;
    const uint32_t kb = (uint32_t)(r & ((1u << lb_bits) - 1u));
    const uint32_t k = (uint32_t)((r >> lb_bits) & ((1u << lk_bits) - 1u));
    const uint32_t x = (uint32_t)(r >> (lb_bits + lk_bits));
    const int lo_x = xT_bits < 12 ? xT_bits : 12, lo_k = lk_bits < 12 ? lk_bits : 12;
    const int lo_b = lb_bits < 12 ? lb_bits : 12;
    const int64_t off = tab(tables, jd.tx_lo, jd.tx_hi, lo_x, x) + tab(tables, jd.tk_lo, jd.tk_hi, lo_k, k) +
                        tab(tables, jd.tb_lo, jd.tb_hi, lo_b, kb);
    Tc[id] = T[t * t_stride + off];
  }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// MFMA join of the last (ket-only) batch: amp[e][o(x, xb)] = sum_k V[e][xb][k] Tc[t][x][k]
// and pi = |amp|^2.  Rows (element, xb) of one trajectory are the M dimension, x
// the N dimension (tiles of 16), k the reduction (K = 2^crossing).
template <int K>
__global__ void __launch_bounds__(256) ketjoin_mfma_kernel(QformArgs a) {
  constexpr int ROWS = 64;
  constexpr int KS = K / 4;
  __shared__ float Tr[K][17], Ti[K][17];
  __shared__ float2 Vs[ROWS][K + 1];
  uint32_t bx, by, bz;
  {
    const uint32_t nbx = gridDim.x, nby = gridDim.y, total = nbx * nby * gridDim.z;
    const uint32_t phys = blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z);
    const uint32_t xcd = phys % 8u, slot = phys / 8u, q = total / 8u, r = total % 8u;
    const uint32_t logical = xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
    bx = logical % nbx;
    by = (logical / nbx) % nby;
    bz = logical / (nbx * nby);
  }
  const int t = a.traj0 + (int)by;
  const int64_t e_begin = a.first[t] > a.e_lo ? a.first[t] : a.e_lo;
  const int64_t e_end = a.first[t + 1] < a.e_hi ? a.first[t + 1] : a.e_hi;
  const int xb_bits = a.xb_bits;
  const int64_t rows_t = (e_end - e_begin) << xb_bits;
  const int64_t row0 = (int64_t)bx * ROWS;
  if (row0 >= rows_t) return;
  const int nx = 1 << a.xT_bits;
  const int ntile = (nx + 15) / 16;
  const int t_per = (ntile + gridDim.z - 1) / gridDim.z;
  const int tile_begin = (int)bz * t_per;
  const int tile_end = tile_begin + t_per < ntile ? tile_begin + t_per : ntile;
  if (tile_begin >= tile_end) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lo_b = xb_bits < 12 ? xb_bits : 12, lo_k = a.lk_bits < 12 ? a.lk_bits : 12;
  const int lo_x = a.xT_bits < 12 ? a.xT_bits : 12;
  for (int i = tid; i < ROWS * K; i += 256) {
    const int rr = i / K, k = i % K;
    const int64_t row = row0 + rr;
    float2 v = make_float2(0.f, 0.f);
    if (row < rows_t) {
      const int64_t e = e_begin + (row >> xb_bits);
      const uint32_t xb = (uint32_t)(row & ((1 << xb_bits) - 1));
      v = a.V[(e - a.v_base) * a.v_stride + tab(a.tab, a.jd.vr_lo, a.jd.vr_hi, lo_b, xb) +
              tab(a.tab, a.jd.vc_lo, a.jd.vc_hi, lo_k, (uint32_t)k)];
    }
    Vs[rr][k] = v;
  }
  __syncthreads();
  float ar[KS], ai[KS];
  const int arow = wave * 16 + (lane & 15);
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const float2 v = Vs[arow][4 * s + (lane >> 4)];
    ar[s] = v.x;
    ai[s] = v.y;
  }
  const int32_t ts = a.tslot ? a.tslot[t - a.traj_base] : t - a.traj_base;
  const float2* Tt = a.Tc + (int64_t)ts * ((int64_t)nx * K);
  const int nout = 1 << a.b;
  for (int tl = tile_begin; tl < tile_end; ++tl) {
    const int x0 = tl * 16;
    for (int i = tid; i < 16 * K; i += 256) {       // Tc[x0 + xi][k] -> Tr[k][xi]
      const int xi = i / K, k = i % K;
      const float2 v = x0 + xi < nx ? Tt[(int64_t)(x0 + xi) * K + k] : make_float2(0.f, 0.f);
      Tr[k][xi] = v.x;
      Ti[k][xi] = v.y;
    }
    __syncthreads();
    floatx4 yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const float br = Tr[4 * s + (lane >> 4)][lane & 15], bim = Ti[4 * s + (lane >> 4)][lane & 15];
      yr = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[s], br, yr, 0, 0, 0);
      yr = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[s], bim, yr, 0, 0, 0);
      yi = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[s], bim, yi, 0, 0, 0);
      yi = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[s], br, yi, 0, 0, 0);
    }
    const int x = x0 + (lane & 15);
    if (x < nx) {
      const int64_t ox = tab(a.tab, a.jd.ox_lo, a.jd.ox_hi, lo_x, (uint32_t)x);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + wave * 16 + 4 * (lane >> 4) + i;
        if (row < rows_t) {
          const int64_t e = e_begin + (row >> xb_bits);
          const uint32_t xb = (uint32_t)(row & ((1 << xb_bits) - 1));
          const int64_t o = (e - a.v_base) * nout + ox + tab(a.tab, a.jd.ob_lo, a.jd.ob_hi, lo_b, xb);
          if (a.pop) a.pop[o] = yr[i] * yr[i] + yi[i] * yi[i];
          if (a.amp) a.amp[o] = make_float2(yr[i], yi[i]);
        }
      }
    }
    __syncthreads();
  }
}

// MFMA join of the doubled network (Sec. II-B marginals) as one real GEMM.  For
// an element row v (K = 2^lk_bits complex entries) and T = Tc[x] (K x K,
// rows k, columns k'), the population pi = Re sum_{a,b} v_a T_ab conj(v_b) is
// a real bilinear form in the products v_a conj(v_b).  Folding each unordered
// pair {a, b} (Re(v_a conj v_b) is symmetric, Im antisymmetric) leaves exactly
// K^2 terms, one per slot f = a K + b:
//   a == b:  M_f = |v_a|^2,              Theta_f = Re T_aa
//   a <  b:  M_f = Re(v_a conj v_b),     Theta_f = Re T_ab + Re T_ba
//   a >  b:  M_f = Im(v_b conj v_a),     Theta_f = Im T_ab - Im T_ba
// and pi = sum_f M_f(v) Theta_f(T) exactly (T need not be Hermitian).  The
// populations of a tile of rows and a tile of x values are the real product
// M Theta with inner dimension K^2: 2 K^2 flops per row and x, against 8 K^2
// for the complex product followed by the second contraction.
//
// theta_T_kernel: one workgroup per (trajectory, x) gathers T[x] into LDS through
// the plan's tables and writes Theta[traj][x][f] (f contiguous).
//
// With split != 0 the kernel writes Theta as two 16-bit planes, hi = h(theta) and
// lo = h(theta - hi), hi at Th and the lo plane n_traj 2^xT K^2 elements later:
// split 1: bf16; split 2: fp16 of theta 2^s with s chosen per (trajectory, x) so
// that max |theta| 2^s lies in [1/2, 1) (s stored as int32 after the lo plane).
template <typename H>
__device__ inline void put_split(H* hi, H* lo, int f, float v) {
  const H h = (H)v;
  hi[f] = h;
  lo[f] = (H)(v - (float)h);
}

template <int K>
__global__ void __launch_bounds__(256) theta_T_kernel(const float2* __restrict__ T, int64_t t_stride, int64_t n_traj,
                                                       const int64_t* __restrict__ tables, Plan::JoinDev jd,
                                                       int xT_bits, float* __restrict__ Th, int split) {
  constexpr int KK = K * K, PERT = KK / 256;
  constexpr int LK = K == 16 ? 4 : 5;
  static_assert(KK % 256 == 0, "K = 16 or 32");
  __shared__ float2 Ts[K][K + 1];
  __shared__ float red[4];
  const int tid = threadIdx.x;
  const int lo_x = xT_bits < 12 ? xT_bits : 12;
  int64_t koff[PERT];
#pragma unroll
  for (int i = 0; i < PERT; ++i) {
    const int idx = tid + 256 * i;
    koff[i] = tab(tables, jd.tk_lo, jd.tk_hi, LK, (uint32_t)(idx / K)) +
              tab(tables, jd.tb_lo, jd.tb_hi, LK, (uint32_t)(idx % K));
  }
  const int64_t nx = (int64_t)1 << xT_bits;
  for (int64_t g = blockIdx.x; g < n_traj * nx; g += gridDim.x) {
    const int64_t t = g >> xT_bits;
    const uint32_t x = (uint32_t)(g & (nx - 1));
    const float2* Tx = T + t * t_stride + tab(tables, jd.tx_lo, jd.tx_hi, lo_x, x);
#pragma unroll
    for (int i = 0; i < PERT; ++i) {
      const int idx = tid + 256 * i;
      Ts[idx / K][idx % K] = Tx[koff[i]];
    }
    __syncthreads();
    float th[PERT];
    float mx = 0.f;
#pragma unroll
    for (int i = 0; i < PERT; ++i) {
      const int f = tid + 256 * i;
      const int a = f / K, b = f % K;
      if (a == b) th[i] = Ts[a][a].x;
      else if (a < b) th[i] = Ts[a][b].x + Ts[b][a].x;
      else th[i] = Ts[a][b].y - Ts[b][a].y;
      mx = fmaxf(mx, fabsf(th[i]));
    }
    if (split == 0) {
      float* out = Th + g * KK;
#pragma unroll
      for (int i = 0; i < PERT; ++i) out[tid + 256 * i] = th[i];
    } else if (split == 1) {
      __bf16* hi = reinterpret_cast<__bf16*>(Th) + g * KK;
      __bf16* lo = reinterpret_cast<__bf16*>(Th) + (n_traj * nx + g) * KK;
#pragma unroll
      for (int i = 0; i < PERT; ++i) put_split(hi, lo, tid + 256 * i, th[i]);
    } else {
#pragma unroll
      for (int d = 32; d > 0; d >>= 1) mx = fmaxf(mx, __shfl_xor(mx, d));
      if ((tid & 63) == 0) red[tid >> 6] = mx;
      __syncthreads();
      mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
      int ex = 0;
      if (mx > 0.f) frexpf(mx, &ex);
      _Float16* hi = reinterpret_cast<_Float16*>(Th) + g * KK;
      _Float16* lo = reinterpret_cast<_Float16*>(Th) + (n_traj * nx + g) * KK;
#pragma unroll
      for (int i = 0; i < PERT; ++i) put_split(hi, lo, tid + 256 * i, ldexpf(th[i], -ex));
      if (tid == 0) reinterpret_cast<int32_t*>(reinterpret_cast<_Float16*>(Th) + 2 * n_traj * nx * KK)[g] = -ex;
    }
    __syncthreads();
  }
}

// One workgroup = 4 wavefronts = 64 rows of one trajectory (16 per wave) x a tile
// of XT = 16 NC values of x.  The inner dimension runs in chunks of 32 slots:
// Theta[x][chunk] is staged in LDS in MFMA fragment order (double-buffered, the
// next chunk in flight during the MFMAs), and each lane builds its A operand
// M_f(row) on the fly from the row's V entries (for K = 32 the chunk fixes a and
// the lane's b runs over 8 values it keeps in registers).  Output: v_mfma
// accumulators hold pi[row][x] directly.
template <int K, int NC>
__global__ void __launch_bounds__(256) qform_mfma_kernel(QformArgs a) {
  constexpr int ROWS = 64, KK = K * K, KC = 32, NS = KC / 4, XT = 16 * NC, NCH = KK / KC, KB = K / 4;
  constexpr int F4C = KC * XT / 4;              // float4 of Theta per chunk
  constexpr int PL = (F4C + 255) / 256;          // float4 per thread per chunk
  static_assert(PL <= 4, "four float4 per thread at most");
  __shared__ float Thl[2][KC * XT];
  __shared__ float2 Vs[ROWS][K + 1];
  // Workgroups go round-robin to the 8 XCDs in linear launch order; renumber them
  // so that consecutive logical tiles (the x tiles, then the row tiles of one
  // trajectory, which share its Theta and V) run on the same XCD and share its L2.
  uint32_t bx, by, bz;
  {
    const uint32_t nbx = gridDim.x, nby = gridDim.y, nbz = gridDim.z, total = nbx * nby * nbz;
    const uint32_t phys = blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z);
    const uint32_t xcd = phys % 8u, slot = phys / 8u, q = total / 8u, r = total % 8u;
    const uint32_t logical = xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
    bz = logical % nbz;
    bx = (logical / nbz) % nbx;
    by = logical / (nbz * nbx);
  }
  const int t = a.traj0 + (int)by;                    // trajectory of this tile
  const int64_t e_begin = a.first[t] > a.e_lo ? a.first[t] : a.e_lo;
  const int64_t e_end = a.first[t + 1] < a.e_hi ? a.first[t + 1] : a.e_hi;
  const int xb_bits = a.xb_bits;
  const int64_t rows_t = (e_end - e_begin) << xb_bits;
  const int64_t row0 = (int64_t)bx * ROWS;
  if (row0 >= rows_t) return;
  const int nx = 1 << a.xT_bits;
  const int x0 = (int)bz * XT;
  if (x0 >= nx) return;
  const int xv = nx - x0 < XT ? nx - x0 : XT;         // valid x of this tile
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lo_b = xb_bits < 12 ? xb_bits : 12, lo_k = a.lk_bits < 12 ? a.lk_bits : 12;
  // stage the 64 rows of V (zero beyond the trajectory's rows)
  for (int i = tid; i < ROWS * K; i += 256) {
    const int rr = i / K, k = i % K;
    const int64_t row = row0 + rr;
    float2 v = make_float2(0.f, 0.f);
    if (row < rows_t) {
      const int64_t e = e_begin + (row >> xb_bits);
      const uint32_t xb = (uint32_t)(row & ((1 << xb_bits) - 1));
      v = a.V[(e - a.v_base) * a.v_stride + tab(a.tab, a.jd.vr_lo, a.jd.vr_hi, lo_b, xb) +
              tab(a.tab, a.jd.vc_lo, a.jd.vc_hi, lo_k, (uint32_t)k)];
    }
    Vs[rr][k] = v;
  }
  // Theta chunk loader: float4 number idx holds slots 4s..4s+3 of the chunk at
  // x = x0 + idx % XT (s = idx / XT); in LDS slot 4s + q of x = x0 + 16c + j sits
  // at ((s * 64 + 16 q + j) * NC + c), the B operand of lane 16 q + j at k-step s.
  const int32_t ts = a.tslot ? a.tslot[t - a.traj_base] : t - a.traj_base;
  const float* Tt = a.Th + ((int64_t)ts * nx + x0) * KK;
  int xlq[PL], sq[PL];
  bool hq[PL], vq[PL];
#pragma unroll
  for (int i = 0; i < PL; ++i) {
    const int idx = tid + 256 * i;
    hq[i] = idx < F4C;
    xlq[i] = idx % XT;
    sq[i] = (idx / XT) % NS;
    vq[i] = hq[i] && xlq[i] < xv;
  }
  auto ld = [&](int ch, int xl, int s, bool ok) -> float4 {
    return ok ? *reinterpret_cast<const float4*>(Tt + (int64_t)xl * KK + ch * KC + 4 * s)
              : make_float4(0.f, 0.f, 0.f, 0.f);
  };
  auto st = [&](float* d, int xl, int s, float4 v) {
    float* p = d + (s * 64 + (xl & 15)) * NC + (xl >> 4);
    p[0] = v.x; p[16 * NC] = v.y; p[32 * NC] = v.z; p[48 * NC] = v.w;
  };
  float4 rq[PL];
#pragma unroll
  for (int i = 0; i < PL; ++i) rq[i] = ld(0, xlq[i], sq[i], vq[i]);
#pragma unroll
  for (int i = 0; i < PL; ++i)
    if (hq[i]) st(Thl[0], xlq[i], sq[i], rq[i]);
  __syncthreads();
  // per lane: row rl, slot offset q; vb[i] = v[rl][4 i + q]
  const int rl = wave * 16 + (lane & 15), q = lane >> 4;
  float2 vb[KB];
#pragma unroll
  for (int i = 0; i < KB; ++i) vb[i] = Vs[rl][4 * i + q];
  const int nout = 1 << a.b;
  int64_t obase[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = row0 + wave * 16 + 4 * q + i;
    obase[i] = -1;
    if (row < rows_t) {
      const int64_t e = e_begin + (row >> xb_bits);
      const uint32_t xb = (uint32_t)(row & ((1 << xb_bits) - 1));
      obase[i] = (e - a.v_base) * nout + tab(a.tab, a.jd.ob_lo, a.jd.ob_hi, lo_b, xb);
    }
  }
  floatx4 acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int ch = 0; ch < NCH; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < NCH;
    const int cn = more ? ch + 1 : ch;            // the last chunk reloads itself (not stored)
#pragma unroll
    for (int i = 0; i < PL; ++i) rq[i] = ld(cn, xlq[i], sq[i], vq[i]);
    __builtin_amdgcn_sched_barrier(0);          // keep the loads ahead of the MFMAs
    const float* B = Thl[buf];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int kstep = ch * NS + s;
      const int av = (4 * kstep) / K;               // the slot's a: uniform
      const int ib = s % KB;                         // kstep % KB: static
      const int b = 4 * ib + q;
      const float2 va = Vs[rl][av];
      const float2 w = vb[ib];
      const float R = va.x * w.x + va.y * w.y;       // Re(v_a conj v_b)
      const float I = w.y * va.x - w.x * va.y;       // Im(v_b conj v_a)
      const float m = av <= b ? R : I;
      if constexpr (NC == 8) {
        const float4 bq = *reinterpret_cast<const float4*>(B + (s * 64 + lane) * 8);
        const float4 bp = *reinterpret_cast<const float4*>(B + (s * 64 + lane) * 8 + 4);
        acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, bq.x, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, bq.y, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, bq.z, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, bq.w, acc[3], 0, 0, 0);
        acc[4] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, bp.x, acc[4], 0, 0, 0);
        acc[5] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, bp.y, acc[5], 0, 0, 0);
        acc[6] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, bp.z, acc[6], 0, 0, 0);
        acc[7] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, bp.w, acc[7], 0, 0, 0);
      } else if constexpr (NC == 4) {
        const float4 bq = *reinterpret_cast<const float4*>(B + (s * 64 + lane) * 4);
        acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, bq.x, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, bq.y, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, bq.z, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, bq.w, acc[3], 0, 0, 0);
      } else if constexpr (NC == 2) {
        const float2 bq = *reinterpret_cast<const float2*>(B + (s * 64 + lane) * 2);
        acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, bq.x, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, bq.y, acc[1], 0, 0, 0);
      } else {
        acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, B[s * 64 + lane], acc[0], 0, 0, 0);
      }
    }
    if (more) {
#pragma unroll
      for (int i = 0; i < PL; ++i)
        if (hq[i]) st(Thl[buf ^ 1], xlq[i], sq[i], rq[i]);
    }
    __syncthreads();
  }
  // acc[c][i] = pi[row wave*16 + 4 q + i][x0 + 16 c + lane % 16]
  const int lo_x = a.xT_bits < 12 ? a.xT_bits : 12;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int xl = 16 * c + (lane & 15);
    if (xl < xv) {
      const int64_t ox = tab(a.tab, a.jd.ox_lo, a.jd.ox_hi, lo_x, (uint32_t)(x0 + xl));
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (obase[i] >= 0) a.pop[obase[i] + ox] = acc[c][i];
    }
  }
}

// Split-precision slot GEMM: M and Theta as hi + lo 16-bit values (hi = h(x),
// lo = h(x - hi)), three products hi*hi + hi*lo + lo*hi per tile on
// v_mfma_f32_16x16x32_bf16 / _f16, FP32 accumulation.  One MFMA k-step covers 32
// slots: lane 16 q + j takes slots 8q..8q+7 of the step, for row j (A) or for
// x = 16c + j (B).  Theta planes are staged in LDS two k-steps at a time
// (double-buffered).  fp16 (F16): each row's M is scaled by 2^e_r with max |v|^2
// 2^e_r in [1/2, 1) (|M_f| <= max |v|^2), Theta by its stored 2^e_x, and the FP32
// result is multiplied by 2^-(e_r + e_x) (exact).
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
template <bool F16> struct Split16;
template <> struct Split16<false> {
  typedef __bf16 E; typedef bf16x8 V;
  static __device__ floatx4 mfma(V x, V y, floatx4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0); }
};
template <> struct Split16<true> {
  typedef _Float16 E; typedef f16x8 V;
  static __device__ floatx4 mfma(V x, V y, floatx4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c, 0, 0, 0); }
};

template <int K, int NC, bool F16>
__global__ void __launch_bounds__(256) qform_split_kernel(QformArgs a) {
  typedef typename Split16<F16>::E E;
  typedef typename Split16<F16>::V bf16x8;
  // NC = 8: one A operand (built and split per lane) feeds 24 MFMAs; the Theta
  // chunk is then one k-step (LDS stays under 64 KB)
  constexpr int ROWS = 64, KK = K * K, XT = 16 * NC, NST = KK / 32, KS = NC >= 8 ? 1 : 2, NCH = NST / KS;
  constexpr int U16 = KS * 2 * XT * 4;            // 16-byte units of Theta per chunk
  static_assert(NCH >= 1 && NST % KS == 0, "chunking");
  __shared__ bf16x8 Tb[2][KS][2][NC][64];          // [buf][k-step][plane][c][lane]
  __shared__ float2 Vs[ROWS][K + 1];
  uint32_t bx, by, bz;
  {
    const uint32_t nbx = gridDim.x, nby = gridDim.y, nbz = gridDim.z, total = nbx * nby * nbz;
    const uint32_t phys = blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z);
    const uint32_t xcd = phys % 8u, slot = phys / 8u, q = total / 8u, r = total % 8u;
    const uint32_t logical = xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
    bz = logical % nbz;
    bx = (logical / nbz) % nbx;
    by = logical / (nbz * nbx);
  }
  const int t = a.traj0 + (int)by;
  const int64_t e_begin = a.first[t] > a.e_lo ? a.first[t] : a.e_lo;
  const int64_t e_end = a.first[t + 1] < a.e_hi ? a.first[t + 1] : a.e_hi;
  const int xb_bits = a.xb_bits;
  const int64_t rows_t = (e_end - e_begin) << xb_bits;
  const int64_t row0 = (int64_t)bx * ROWS;
  if (row0 >= rows_t) return;
  const int nx = 1 << a.xT_bits;
  const int x0 = (int)bz * XT;
  if (x0 >= nx) return;
  const int xv = nx - x0 < XT ? nx - x0 : XT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lo_b = xb_bits < 12 ? xb_bits : 12, lo_k = a.lk_bits < 12 ? a.lk_bits : 12;
  for (int i = tid; i < ROWS * K; i += 256) {
    const int rr = i / K, k = i % K;
    const int64_t row = row0 + rr;
    float2 v = make_float2(0.f, 0.f);
    if (row < rows_t) {
      const int64_t e = e_begin + (row >> xb_bits);
      const uint32_t xb = (uint32_t)(row & ((1 << xb_bits) - 1));
      v = a.V[(e - a.v_base) * a.v_stride + tab(a.tab, a.jd.vr_lo, a.jd.vr_hi, lo_b, xb) +
              tab(a.tab, a.jd.vc_lo, a.jd.vc_hi, lo_k, (uint32_t)k)];
    }
    Vs[rr][k] = v;
  }
  // Theta planes: hi at a.Th (bf16), lo n_all = (#slots of the launch's trajectories) later
  const int32_t ts = a.tslot ? a.tslot[t - a.traj_base] : t - a.traj_base;
  const E* Hp = reinterpret_cast<const E*>(a.Th) + ((int64_t)ts * nx + x0) * KK;
  const int64_t plane = a.th_plane;                   // elements between the hi and lo planes
  // chunk loader: 16-byte unit u = (plane, k-step, x, q) with q fastest; every lane
  // loads (rows past the tile's x read row x0, in bounds) and masks when storing
  auto ld = [&](int ch, int u) -> bf16x8 {
    const int q = u & 3, xl = (u >> 2) % XT, ks = (u / (4 * XT)) % KS, pl = u / (4 * XT * KS);
    const int xr = xl < xv ? xl : 0;
    return *reinterpret_cast<const bf16x8*>(Hp + pl * plane + (int64_t)xr * KK + (ch * KS + ks) * 32 + 8 * q);
  };
  auto st = [&](int buf, int u, bf16x8 v) {
    const int q = u & 3, xl = (u >> 2) % XT, ks = (u / (4 * XT)) % KS, pl = u / (4 * XT * KS);
    if (xl >= xv) v = bf16x8{};
    Tb[buf][ks][pl][xl >> 4][16 * q + (xl & 15)] = v;
  };
  constexpr int PU = (U16 + 255) / 256;
  static_assert(PU <= 4, "four units per thread at most");
  bf16x8 r[4];
#pragma unroll
  for (int i = 0; i < PU; ++i) {
    const int u = tid + 256 * i;
    r[i] = ld(0, u < U16 ? u : U16 - 1);
  }
#pragma unroll
  for (int i = 0; i < PU; ++i)
    if (tid + 256 * i < U16) st(0, tid + 256 * i, r[i]);
  __syncthreads();
  // lane: row rl, slot group q (slots 8q..8q+7 of each k-step)
  const int rl = wave * 16 + (lane & 15), q = lane >> 4;
  constexpr int BQ = K == 32 ? 1 : 2;                // K = 16: a k-step spans two values of a
  float2 vb[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) vb[i] = Vs[rl][(8 * (q % (4 / BQ)) + i) & (K - 1)];
  // fp16: row scale 2^er from max |v|^2 over the row (lanes 16 q + j, q = 0..3, share row j)
  int er = 0;
  float rsc = 1.f;
  if constexpr (F16) {
    float mr = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) mr = fmaxf(mr, vb[i].x * vb[i].x + vb[i].y * vb[i].y);
    if (K == 32) {                                    // K = 16: 8 (q % 2) + i covers the row already
      mr = fmaxf(mr, __shfl_xor(mr, 16));
      mr = fmaxf(mr, __shfl_xor(mr, 32));
    } else {
      mr = fmaxf(mr, __shfl_xor(mr, 16));
    }
    int ex = 0;
    if (mr > 0.f) frexpf(mr, &ex);
    er = -ex;
    rsc = ldexpf(1.f, er);
  }
  const int nout = 1 << a.b;
  int64_t obase[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = row0 + wave * 16 + 4 * q + i;
    obase[i] = -1;
    if (row < rows_t) {
      const int64_t e = e_begin + (row >> xb_bits);
      const uint32_t xb = (uint32_t)(row & ((1 << xb_bits) - 1));
      obase[i] = (e - a.v_base) * nout + tab(a.tab, a.jd.ob_lo, a.jd.ob_hi, lo_b, xb);
    }
  }
  floatx4 acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int ch = 0; ch < NCH; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < NCH;
    const int cn = more ? ch + 1 : ch;
#pragma unroll
    for (int i = 0; i < PU; ++i) {
      const int u = tid + 256 * i;
      r[i] = ld(cn, u < U16 ? u : U16 - 1);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int kstep = ch * KS + ks;
      // slot f = 32 kstep + 8 q + i = a K + b
      const int av = (32 * kstep + 8 * q) / K;
      const int b0 = (32 * kstep + 8 * q) % K;
      const float2 va = Vs[rl][av];
      bf16x8 ah, al;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const float2 w = vb[i];
        const float R = va.x * w.x + va.y * w.y;       // Re(v_a conj v_b)
        const float I = w.y * va.x - w.x * va.y;       // Im(v_b conj v_a)
        const float m = (av <= b0 + i ? R : I) * rsc;
        const E h = (E)m;
        ah[i] = h;
        al[i] = (E)(m - (float)h);
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const bf16x8 bh = Tb[buf][ks][0][c][lane], bl = Tb[buf][ks][1][c][lane];
        acc[c] = Split16<F16>::mfma(ah, bh, acc[c]);
        acc[c] = Split16<F16>::mfma(ah, bl, acc[c]);
        acc[c] = Split16<F16>::mfma(al, bh, acc[c]);
      }
    }
    if (more) {
#pragma unroll
      for (int i = 0; i < PU; ++i)
        if (tid + 256 * i < U16) st(buf ^ 1, tid + 256 * i, r[i]);
    }
    __syncthreads();
  }
  const int lo_x = a.xT_bits < 12 ? a.xT_bits : 12;
  // fp16: the output rows' scales (row 4 q + i of the wave is held by lane 4 q + i)
  int eo[4] = {0, 0, 0, 0};
  if constexpr (F16) {
#pragma unroll
    for (int i = 0; i < 4; ++i) eo[i] = __shfl(er, 4 * q + i);
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int xl = 16 * c + (lane & 15);
    if (xl < xv) {
      const int64_t ox = tab(a.tab, a.jd.ox_lo, a.jd.ox_hi, lo_x, (uint32_t)(x0 + xl));
      int exs = 0;
      if constexpr (F16) exs = a.th_scale[(int64_t)ts * nx + x0 + xl];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (obase[i] >= 0) a.pop[obase[i] + ox] = F16 ? ldexpf(acc[c][i], -(eo[i] + exs)) : acc[c][i];
    }
  }
}

__global__ void row_totals_kernel(const float* pop, int64_t n_elems, int b, double* totals) {
  __shared__ double red[256];
  const int64_t n = (int64_t)1 << b;
  for (int64_t e = blockIdx.x; e < n_elems; e += gridDim.x) {
  // thread t sums the float4 groups t, t + 256, ... (coalesced) into four FP64
  // accumulators (independent add chains), combined in a fixed order, then a fixed
  // tree: deterministic
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if ((n & 3) == 0 && (reinterpret_cast<uintptr_t>(pop) & 15) == 0) {   // 16-byte aligned rows
    const float4* p4 = reinterpret_cast<const float4*>(pop + e * n);
    for (int64_t i = threadIdx.x; i < (n >> 2); i += blockDim.x) {
      const float4 v = p4[i];
      s0 += (double)v.x; s1 += (double)v.y; s2 += (double)v.z; s3 += (double)v.w;
    }
  } else {
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s0 += (double)pop[e * n + i];
  }
  const double s = (s0 + s1) + (s2 + s3);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) totals[e] = red[0];
  __syncthreads();
  }
}

// --------------------------------------------------------------------- sampling
// Sampling and non-degenerate batching run one wavefront per element, with no
// workgroup-wide scans: lane L owns the contiguous chunk [L per, (L+1) per) of
// the 2^b values.
//
// The CDF (Sec. II-B inverse-CDF draw) in FP64: a lane sums its chunk in index
// order (s_L), a fixed shuffle tree gives the exclusive prefix exc_L of the
// chunk sums, and C(x) = exc_L + (sum of the chunk's values up to x, in index
// order).  cend_L = exc_L + s_L is C at the chunk's end, computed by the same
// operations, so the lane found by a search over cend always contains the
// first x with C(x) > target.  Z = C(2^b - 1).
__device__ inline void chunk_of(int n, int lane, int& c0, int& c1) {
  const int per = n >= 64 ? n >> 6 : 1;
  c0 = lane * per;
  c1 = c0 + per < n ? c0 + per : n;
  if (c0 > n) c0 = n;
}

// One element sampled by the whole wavefront (hist: [2^b] shot counts per x,
// used for child counts; cend, exc: [64] per-lane chunk ends and starts).
__device__ void sample_element_wave(const SampleArgs& a, int64_t e, int* hist, double* cend, double* exc) {
  const int n = 1 << a.b;
  const int lane = threadIdx.x;
  const int nl = n < 64 ? n : 64;         // lanes with a non-empty chunk
  int c0, c1;
  chunk_of(n, lane, c0, c1);
  {
    const float* pi = a.pop + e * (int64_t)n;
    const int off = a.elem_shot_off[e];
    const int cnt = a.elem_shot_cnt[e];
    const bool want_hist = a.child_cnt && cnt > 1;
    if (want_hist)
      for (int x = c0; x < c1; ++x) hist[x] = 0;
    double s = 0.0;
    int lp = -1;
    if (((c1 - c0) & 3) == 0) {
      for (int x = c0; x < c1; x += 4) {
        const float4 v = *reinterpret_cast<const float4*>(pi + x);
        s += (double)v.x; s += (double)v.y; s += (double)v.z; s += (double)v.w;
        if (v.x > 0.f) lp = x;
        if (v.y > 0.f) lp = x + 1;
        if (v.z > 0.f) lp = x + 2;
        if (v.w > 0.f) lp = x + 3;
      }
    } else {
      for (int x = c0; x < c1; ++x) {
        const float v = pi[x];
        s += (double)v;
        if (v > 0.f) lp = x;
      }
    }
    double incl = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const double t = __shfl_up(incl, d);
      if (lane >= d) incl += t;
    }
    double ex = __shfl_up(incl, 1);
    if (lane == 0) ex = 0.0;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      const int o = __shfl_xor(lp, d);
      lp = o > lp ? o : lp;
    }
    const int last_pos = lp;                   // largest x with pi(x) > 0, or -1
    exc[lane] = ex;
    cend[lane] = ex + s;
    __syncthreads();
    const double Z = cend[nl - 1];
    if (lane == 0) {
      a.elem_total[e] = Z;
      // Z == 0: the trajectory's inserted operators annihilated the state (weight 0,
      // all-zero shots); only a non-finite or negative total is an error
      if (!(Z >= 0.0) || !isfinite(Z)) atomicExch(a.bad_flag, 1);
    }
    const int traj = a.elem_traj[e];
    const int64_t tbase = a.traj_shot_base[traj];
    for (int i = lane; i < cnt; i += 64) {
      const int row = a.shot_ids[off + i];
      const uint32_t t = (uint32_t)(row - tbase);
      const double u = philox_uniform(a.seed, a.tag, (uint32_t)traj, (uint32_t)a.j, t, 0u);
      const double target = u * Z;
      int lo = 0, hi = nl;                      // first lane with cend > target
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cend[mid] > target) hi = mid; else lo = mid + 1;
      }
      int x = last_pos;
      if (lo < nl) {
        int b0, b1;
        chunk_of(n, lo, b0, b1);
        const double el = exc[lo];
        double sx = 0.0;
        for (int k = b0; k < b1; ++k) {
          sx += (double)pi[k];
          if (el + sx > target) { x = k; break; }
        }
      }
      if (x < 0) x = 0;
      a.shot_x[row] = x;
      if (a.p_cond) a.p_cond[row] = Z > 0.0 ? (double)pi[x] / Z : 0.0;
      if (a.shots) {   // write the batch bits at qubits [start, start + b)
        uint64_t* w = a.shots + (int64_t)row * a.NW;
        const int q0 = a.start;
        const int wi = q0 >> 6, sh = q0 & 63;
        w[wi] |= (uint64_t)x << sh;
        if (sh + a.b > 64) w[wi + 1] |= (uint64_t)x >> (64 - sh);
      }
      if (want_hist) atomicAdd(&hist[x], 1);
    }
    if (a.child_cnt) {
      int c = cnt > 0 ? 1 : 0;
      if (want_hist) {
        __syncthreads();
        c = 0;
        for (int x = c0; x < c1; ++x) c += hist[x] > 0;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d);
      }
      if (lane == 0) a.child_cnt[e] = c;
    }
    __syncthreads();   // LDS is reused by the next element
  }
}

__global__ void __launch_bounds__(64) sample_kernel(SampleArgs a) {
  extern __shared__ int hist[];
  __shared__ double cend[64], exc[64];
  for (int64_t e = blockIdx.x; e < a.n_elems; e += gridDim.x) sample_element_wave(a, e, hist, cend, exc);
}

// Elements with few shots and b <= 5, one lane per element (64 elements per
// wavefront): a lane recomputes, in registers, exactly the FP64 operations of
// sample_element_wave for 2^B <= 32 values (one value per chunk: the same
// Hillis-Steele partial sums in the same order, the same chunk ends, the same
// binary search), so both give the same draws bit for bit; elements with more
// than kLaneShots shots are taken by the whole wavefront afterwards.  This
// turns a chain of dependent loads per element into one per 64 elements.
constexpr int kLaneShots = 16;

template <int B>
__global__ void __launch_bounds__(64) sample_lanes_kernel(SampleArgs a) {
  extern __shared__ int hist[];
  __shared__ double cend_s[64], exc_s[64];
  constexpr int n = 1 << B;
  const int lane = threadIdx.x;
  for (int64_t base = (int64_t)blockIdx.x * 64; base < a.n_elems; base += (int64_t)gridDim.x * 64) {
    const int64_t e = base + lane;
    const bool mine = e < a.n_elems;
    const int cnt = mine ? a.elem_shot_cnt[e] : 0;
    const bool small = mine && cnt <= kLaneShots;
    if (small) {
      const float* pi = a.pop + e * (int64_t)n;
      float p[n];
      if (n >= 4 && (reinterpret_cast<uintptr_t>(a.pop) & 15) == 0) {
#pragma unroll
        for (int k = 0; k < n / 4; ++k) {
          const float4 v = reinterpret_cast<const float4*>(pi)[k];
          p[4 * k] = v.x; p[4 * k + 1] = v.y; p[4 * k + 2] = v.z; p[4 * k + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int k = 0; k < n; ++k) p[k] = pi[k];
      }
      double sv[n], incl[n], cend[n];
      int last_pos = -1;
#pragma unroll
      for (int L = 0; L < n; ++L) {
        sv[L] = 0.0 + (double)p[L];
        incl[L] = sv[L];
        if (p[L] > 0.f) last_pos = L;
      }
#pragma unroll
      for (int d = 1; d < n; d <<= 1)
#pragma unroll
        for (int L = n - 1; L >= d; --L) incl[L] = incl[L] + incl[L - d];
      cend[0] = 0.0 + sv[0];
#pragma unroll
      for (int L = 1; L < n; ++L) cend[L] = incl[L - 1] + sv[L];
      const double Z = cend[n - 1];
      a.elem_total[e] = Z;
      if (!(Z >= 0.0) || !isfinite(Z)) atomicExch(a.bad_flag, 1);
      uint32_t seen = 0u;
      if (cnt > 0) {
        const int traj = a.elem_traj[e];
        const int64_t tbase = a.traj_shot_base[traj];
        const int off = a.elem_shot_off[e];
        for (int i = 0; i < cnt; ++i) {
          const int row = a.shot_ids[off + i];
          const uint32_t t = (uint32_t)(row - tbase);
          const double u = philox_uniform(a.seed, a.tag, (uint32_t)traj, (uint32_t)a.j, t, 0u);
          const double target = u * Z;
          int lo = 0, hi = n;
#pragma unroll
          for (int it = 0; it <= B; ++it) {
            if (lo < hi) {
              const int mid = (lo + hi) >> 1;
              double cm = cend[0];
#pragma unroll
              for (int L = 1; L < n; ++L) cm = mid == L ? cend[L] : cm;
              if (cm > target) hi = mid; else lo = mid + 1;
            }
          }
          int x = lo < n ? lo : last_pos;
          if (x < 0) x = 0;
          a.shot_x[row] = x;
          if (a.p_cond) {
            float px = p[0];
#pragma unroll
            for (int L = 1; L < n; ++L) px = x == L ? p[L] : px;
            a.p_cond[row] = Z > 0.0 ? (double)px / Z : 0.0;
          }
          if (a.shots) {
            uint64_t* w = a.shots + (int64_t)row * a.NW;
            const int wi = a.start >> 6, sh = a.start & 63;
            w[wi] |= (uint64_t)x << sh;
            if (sh + B > 64) w[wi + 1] |= (uint64_t)x >> (64 - sh);
          }
          seen |= 1u << x;
        }
      }
      if (a.child_cnt) a.child_cnt[e] = __popc(seen);
    }
    // elements with more shots: the whole wavefront, one element at a time
    uint64_t big = __ballot(mine && !small);
    while (big) {
      const int l = __ffsll((unsigned long long)big) - 1;
      big &= big - 1;
      sample_element_wave(a, base + l, hist, cend_s, exc_s);
    }
  }
}

// The children of one element, by the whole wavefront (ism: 3 * 2^b ints).
__device__ void children_element_wave(const ChildArgs& a, int64_t e, int* ism) {
  const int n = 1 << a.b;
  int* hist = ism;          // counts per x
  int* start = ism + n;     // exclusive scan of counts (then the scatter cursor)
  int* rank = ism + 2 * n;  // exclusive scan of (count > 0)
  const int lane = threadIdx.x;
  int c0, c1;
  chunk_of(n, lane, c0, c1);
  {
    const int off = a.elem_shot_off[e], cnt = a.elem_shot_cnt[e];
    if (cnt <= 0) return;                 // uniform over the wavefront
    const int traj = a.elem_traj[e];
    const int64_t cbase = a.child_off[e];
    const uint64_t* pp = a.elem_prefix + e * a.NW;
    const int wi = a.start >> 6, sh = a.start & 63;
    if (cnt == 1) {                       // one shot: one child
      if (lane == 0) {
        const int row = a.shot_ids[off];
        const int x = a.shot_x[row];
        a.out_traj[cbase] = traj;
        a.out_parent[cbase] = (int32_t)e;
        a.out_shot_off[cbase] = off;
        a.out_shot_cnt[cbase] = 1;
        uint64_t* op = a.out_prefix + cbase * a.NW;
        for (int w = 0; w < a.NW; ++w) op[w] = pp[w];
        op[wi] |= (uint64_t)x << sh;
        if (sh + a.b > 64) op[wi + 1] |= (uint64_t)x >> (64 - sh);
        a.out_shot_ids[off] = row;
      }
      return;
    }
    for (int x = c0; x < c1; ++x) hist[x] = 0;
    __syncthreads();
    for (int i = lane; i < cnt; i += 64) atomicAdd(&hist[a.shot_x[a.shot_ids[off + i]]], 1);
    __syncthreads();
    // exclusive scans of hist and of (hist > 0) over the lanes' chunks
    int ls = 0, lr = 0;
    for (int x = c0; x < c1; ++x) { ls += hist[x]; lr += hist[x] > 0; }
    int is = ls, ir = lr;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int ts = __shfl_up(is, d), tr = __shfl_up(ir, d);
      if (lane >= d) { is += ts; ir += tr; }
    }
    int sacc = is - ls, racc = ir - lr;
    for (int x = c0; x < c1; ++x) {
      const int h = hist[x];
      start[x] = sacc; rank[x] = racc;
      if (h > 0) {
        const int64_t c = cbase + racc;
        a.out_traj[c] = traj;
        a.out_parent[c] = (int32_t)e;
        a.out_shot_off[c] = off + sacc;
        a.out_shot_cnt[c] = h;
        uint64_t* op = a.out_prefix + c * a.NW;
        for (int w = 0; w < a.NW; ++w) op[w] = pp[w];
        op[wi] |= (uint64_t)x << sh;
        if (sh + a.b > 64) op[wi + 1] |= (uint64_t)x >> (64 - sh);
      }
      sacc += h; racc += h > 0;
    }
    __syncthreads();
    // scatter shot ids into the children's ranges (order within a child is free)
    for (int i = lane; i < cnt; i += 64) {
      const int row = a.shot_ids[off + i];
      const int x = a.shot_x[row];
      const int pos = atomicAdd(&start[x], 1);
      a.out_shot_ids[off + pos] = row;
    }
    __syncthreads();   // LDS is reused by the next element
  }
}

__global__ void __launch_bounds__(64) children_kernel(ChildArgs a) {
  extern __shared__ int ism[];
  for (int64_t e = blockIdx.x; e < a.n_elems; e += gridDim.x) children_element_wave(a, e, ism);
}

// Elements with at most kLaneChildShots shots and b <= 5, one lane per element:
// the same children as children_element_wave (ascending x, each child's shots
// contiguous from off + the number of the element's shots with smaller x), with
// the shots of a child in their order within the element.
constexpr int kLaneChildShots = 4;

__global__ void __launch_bounds__(64) children_lanes_kernel(ChildArgs a) {
  extern __shared__ int ism[];
  const int lane = threadIdx.x;
  constexpr int T = kLaneChildShots;
  for (int64_t base = (int64_t)blockIdx.x * 64; base < a.n_elems; base += (int64_t)gridDim.x * 64) {
    const int64_t e = base + lane;
    const bool mine = e < a.n_elems;
    const int cnt = mine ? a.elem_shot_cnt[e] : 0;
    if (mine && cnt > 0 && cnt <= T) {
      const int off = a.elem_shot_off[e];
      const int traj = a.elem_traj[e];
      const int64_t cbase = a.child_off[e];
      const uint64_t* pp = a.elem_prefix + e * a.NW;
      const int wi = a.start >> 6, sh = a.start & 63;
      int r[T], x[T];
      uint32_t mask = 0u;
#pragma unroll
      for (int i = 0; i < T; ++i) {
        r[i] = 0; x[i] = 0;
        if (i < cnt) {
          r[i] = a.shot_ids[off + i];
          x[i] = a.shot_x[r[i]];
          mask |= 1u << x[i];
        }
      }
#pragma unroll
      for (int i = 0; i < T; ++i) {
        if (i >= cnt) break;
        int less = 0, before = 0, same = 0;
#pragma unroll
        for (int k = 0; k < T; ++k) {
          if (k < cnt) {
            less += x[k] < x[i];
            same += x[k] == x[i];
            if (k < i) before += x[k] == x[i];
          }
        }
        a.out_shot_ids[off + less + before] = r[i];
        if (before == 0) {               // first shot of its child
          const int64_t c = cbase + __popc(mask & ((1u << x[i]) - 1u));
          a.out_traj[c] = traj;
          a.out_parent[c] = (int32_t)e;
          a.out_shot_off[c] = off + less;
          a.out_shot_cnt[c] = same;
          uint64_t* op = a.out_prefix + c * a.NW;
          for (int w = 0; w < a.NW; ++w) op[w] = pp[w];
          op[wi] |= (uint64_t)x[i] << sh;
          if (sh + a.b > 64) op[wi + 1] |= (uint64_t)x[i] >> (64 - sh);
        }
      }
    }
    uint64_t big = __ballot(mine && cnt > T);
    while (big) {
      const int l = __ffsll((unsigned long long)big) - 1;
      big &= big - 1;
      children_element_wave(a, base + l, ism);
    }
  }
}

// ------------------------------------------- non-proportional NBS (Sec. III-B)
__global__ void np_init_kernel(int64_t E, int64_t t0, int32_t* elem_traj, uint64_t* elem_prefix, int NW) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
    elem_traj[e] = (int32_t)(t0 + e);
    for (int w = 0; w < NW; ++w) elem_prefix[e * NW + w] = 0ull;
  }
}

__global__ void np_direct_rows_kernel(int64_t n_elems, int draws, const int32_t* elem_traj,
                                      const uint64_t* elem_prefix, int NW, uint64_t* bits, int32_t* row_traj) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n_elems * draws;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = r / draws;
    for (int w = 0; w < NW; ++w) bits[r * NW + w] = elem_prefix[e * NW + w];
    if (row_traj) row_traj[r] = elem_traj[e];
  }
}

__global__ void np_direct_prefix_p_kernel(int64_t n_elems, int draws, const int32_t* elem_traj,
                                          const double* elem_total, const double* traj_norm, double* p_prefix) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n_elems * draws;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = r / draws;
    const double Z = elem_total[e];
    p_prefix[r] = Z > 0.0 ? (traj_norm ? Z / traj_norm[elem_traj[e]] : 1.0) : 0.0;
  }
}

__global__ void np_rows_kernel(int64_t n_elems, int draws, const int32_t* elem_traj, int32_t* off, int32_t* cnt,
                               int32_t* ids, int64_t* traj_base) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_elems;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r0 = e * draws;
    off[e] = (int32_t)r0;
    cnt[e] = draws;
    for (int d = 0; d < draws; ++d) ids[r0 + d] = (int32_t)(r0 + d);
    if (e == 0 || elem_traj[e] != elem_traj[e - 1]) traj_base[elem_traj[e]] = r0;
  }
}

// Thread t of a tile owns the values [t per, (t + 1) per) of the tile; the
// threshold decision is the same expression in both kernels.
__device__ inline bool exh_pass(float v, double Z, double thr) { return Z > 0.0 && (double)v / Z > thr; }

__global__ void __launch_bounds__(256) exh_count_kernel(ExhArgs a) {
  __shared__ int red[256];
  const int64_t X = (int64_t)1 << a.b;
  const int tileX = X < kExhTile ? (int)X : kExhTile;
  const int per = tileX >= 256 ? tileX >> 8 : 1;
  const int64_t n_units = a.n_elems << a.tile_bits;
  for (int64_t u = blockIdx.x; u < n_units; u += gridDim.x) {
    const int64_t e = u >> a.tile_bits;
    const int64_t x0 = (u & (((int64_t)1 << a.tile_bits) - 1)) * tileX;
    const double Z = a.elem_total[e];
    const float* pi = a.pop + e * X + x0;
    int c = 0;
    for (int i = 0; i < per; ++i) {   // x = 256 i + t: coalesced
      const int x = 256 * i + (int)threadIdx.x;
      if (x < tileX) c += exh_pass(pi[x], Z, a.threshold);
    }
    red[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.tile_cnt[u] = red[0];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) exh_write_kernel(ExhArgs a) {
  // Rows of a tile in x order: round i covers x = 256 i + t; within a round the
  // four wavefronts hold consecutive x ranges, and a lane's place among them is
  // the popcount of the passing lanes below it (ballot).  Consecutive lanes write
  // consecutive rows.
  __shared__ int wcnt[kExhTile / 256][4];
  const int64_t X = (int64_t)1 << a.b;
  const int tileX = X < kExhTile ? (int)X : kExhTile;
  const int per = tileX >= 256 ? tileX >> 8 : 1;
  const int64_t n_units = a.n_elems << a.tile_bits;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int wi = a.start >> 6, sh = a.start & 63;
  for (int64_t u = blockIdx.x; u < n_units; u += gridDim.x) {
    const int64_t e = u >> a.tile_bits;
    const int64_t x0 = (u & (((int64_t)1 << a.tile_bits) - 1)) * tileX;
    const double Z = a.elem_total[e];
    const float* pi = a.pop + e * X + x0;
    __syncthreads();   // wcnt of the previous unit is no longer read
    for (int i = 0; i < per; ++i) {
      const int x = 256 * i + tid;
      const bool pass = x < tileX && exh_pass(pi[x], Z, a.threshold);
      const uint64_t m = __ballot(pass);
      if (lane == 0) wcnt[i][wv] = __popcll(m);
    }
    __syncthreads();
    const int traj = a.elem_traj[e];
    const uint64_t* pp = a.elem_prefix + e * a.NW;
    const double pref = a.traj_norm ? Z / a.traj_norm[traj] : 1.0;
    int64_t row = a.row_base + a.tile_off[u];
    for (int i = 0; i < per; ++i) {
      const int x = 256 * i + tid;
      const float v = x < tileX ? pi[x] : 0.f;
      const bool pass = x < tileX && exh_pass(v, Z, a.threshold);
      const uint64_t m = __ballot(pass);
      int before = 0;
      for (int w = 0; w < wv; ++w) before += wcnt[i][w];
      if (pass) {
        const int64_t r = row + before + __popcll(m & below);
        if (r < a.capacity) {
          const uint64_t xv = (uint64_t)(x0 + x);
          uint64_t* w = a.bits + r * a.NW;
          for (int k = 0; k < a.NW; ++k) w[k] = pp[k];
          w[wi] |= xv << sh;
          if (sh + a.b > 64) w[wi + 1] |= xv >> (64 - sh);
          if (a.row_traj) a.row_traj[r] = traj;
          if (a.p_cond) a.p_cond[r] = (double)v / Z;
          if (a.p_prefix) a.p_prefix[r] = pref;
        }
      }
      row += wcnt[i][0] + wcnt[i][1] + wcnt[i][2] + wcnt[i][3];
    }
  }
}

// ---------------------------------------------------------------------- scans
constexpr int kScanBlock = 1024;

__global__ void scan_block_sums(const int32_t* in, int64_t n, int32_t* sums) {
  __shared__ int32_t red[256];
  const int64_t base = blockIdx.x * (int64_t)kScanBlock;
  int32_t s = 0;
  for (int i = threadIdx.x; i < kScanBlock; i += 256)
    if (base + i < n) s += in[base + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

// Exclusive scan of the block sums in place, one workgroup: thread t takes a
// contiguous run of the sums, the run totals are scanned in LDS (integers, so
// the result does not depend on the order of the additions).
__global__ void __launch_bounds__(1024) scan_sums_block(int32_t* sums, int64_t nb, int32_t* total) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (nb + 1023) / 1024;
  const int64_t lo = t * per < nb ? t * per : nb, hi = lo + per < nb ? lo + per : nb;
  int32_t own = 0;
  for (int64_t i = lo; i < hi; ++i) own += sums[i];
  part[t] = own;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int32_t v = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t acc = part[t] - own;
  for (int64_t i = lo; i < hi; ++i) { const int32_t v = sums[i]; sums[i] = acc; acc += v; }
  if (t == 1023) *total = part[1023];
}

__global__ void scan_apply(const int32_t* in, int64_t n, const int32_t* sums, int32_t* out) {
  __shared__ int32_t vals[kScanBlock];
  __shared__ int32_t part[256];
  const int64_t base = blockIdx.x * (int64_t)kScanBlock;
  for (int i = threadIdx.x; i < kScanBlock; i += 256) vals[i] = base + i < n ? in[base + i] : 0;
  __syncthreads();
  const int per = kScanBlock / 256;
  const int lo = threadIdx.x * per;
  int32_t s = 0;
  for (int i = 0; i < per; ++i) s += vals[lo + i];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t acc = sums[blockIdx.x];
    for (int t = 0; t < 256; ++t) { int32_t v = part[t]; part[t] = acc; acc += v; }
  }
  __syncthreads();
  int32_t acc = part[threadIdx.x];
  for (int i = 0; i < per; ++i) {
    int32_t v = vals[lo + i];
    if (base + lo + i < n) out[base + lo + i] = acc;
    acc += v;
  }
}

// -------------------------------------------------------------------- weights
__global__ void weights_kernel(WeightArgs a) {
  __shared__ double red[1024];
  double s = 0.0;
  // fixed assignment of trajectories to threads and a fixed tree: deterministic
  for (int64_t i = threadIdx.x; i < a.E; i += blockDim.x) {
    double m = a.mult ? (double)a.mult[i] : 1.0;
    s += m * a.norms[i];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double tot = red[0];
  for (int64_t i = threadIdx.x; i < a.E; i += blockDim.x) {
    double m = a.mult ? (double)a.mult[i] : 1.0;
    if (a.weights) a.weights[i] = m * a.norms[i] / tot;
    if (a.norm_out) a.norm_out[i] = a.norms[i];
  }
}

__global__ void init_traj_kernel(int64_t E, const int64_t* m, const int64_t* base, int32_t* elem_traj,
                                 uint64_t* elem_prefix, int NW, int32_t* shot_off, int32_t* shot_cnt) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= E) return;
  elem_traj[i] = (int32_t)i;
  for (int w = 0; w < NW; ++w) elem_prefix[i * NW + w] = 0ull;
  shot_off[i] = (int32_t)base[i];
  shot_cnt[i] = (int32_t)m[i];
}

__global__ void init_shots_kernel(int64_t M, int64_t E, const int64_t* base, int32_t* shot_ids,
                                  int32_t* shot_traj, uint64_t* shots, int NW) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= M) return;
  shot_ids[g] = (int32_t)g;
  for (int w = 0; w < NW; ++w) shots[g * NW + w] = 0ull;
  if (shot_traj) {
    // trajectory owning row g: last i with base[i] <= g (base non-decreasing)
    int64_t lo = 0, hi = E - 1;
    while (lo < hi) {
      int64_t mid = (lo + hi + 1) >> 1;
      if (base[mid] <= g) lo = mid; else hi = mid - 1;
    }
    // the last such i is the one that owns rows (earlier ones with equal base have no shots)
    shot_traj[g] = (int32_t)lo;
  }
}

__global__ void traj_first_kernel(const int32_t* elem_traj, int64_t U, int64_t E, int32_t* first) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e > U) return;
  int lo_t = (e == 0) ? 0 : elem_traj[e - 1] + 1;
  int hi_t = (e == U) ? (int)E : elem_traj[e];
  for (int t = lo_t; t <= hi_t; ++t) first[t] = (int32_t)e;
}

}  // namespace

// ---------------------------------------------------------------------- launchers
hipError_t launch_init_gather(const InitArgs& init, int64_t n_jobs, const uint64_t* job_prefix, int NW,
                              float2* out, hipStream_t stream) {
  const int64_t total = n_jobs << init.r0;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(init_gather_kernel, dim3(grid_blocks((total + 255) / 256)), dim3(256), 0, stream, init, n_jobs,
                     job_prefix, NW, out);
  return hipGetLastError();
}

hipError_t launch_part_vm(const AbsorbStep* d_steps, int n_steps, int peak, GateCtx g, int64_t n_jobs,
                          const int32_t* job_traj, int32_t traj_base, const uint64_t* job_prefix, int NW,
                          const InitArgs& init, float2* out, int out_rank, int direct, hipStream_t stream) {
  if (n_jobs <= 0) return hipSuccess;
  const int buf = 1 << (peak > 0 ? peak : 0);
  // small tensors: up to 64 jobs share a 256-thread workgroup (2048 entries of
  // tensors in the A and C buffers; peak is the largest rank held in LDS: with
  // direct, the last step's larger output goes to HBM); one job per workgroup at
  // 2^11 entries
  const int J = buf >= 2048 ? 1 : (2048 / buf > kVmMaxJobs ? kVmMaxJobs : 2048 / buf);
  const int threads = J > 1 ? 256 : (buf / 2 < 64 ? 64 : (buf / 2 > 256 ? 256 : buf / 2));
  // jobs' tensors one entry apart beyond their size: the same index of
  // neighbouring jobs falls in different LDS banks
  const int stride = J > 1 ? buf + 1 : buf;
  const size_t shmem = (size_t)(2 * J * stride + kVmGateEntries) * sizeof(float2) + (size_t)n_steps * sizeof(int4) +
                       (size_t)J * NW * sizeof(uint64_t);
  hipLaunchKernelGGL(part_vm_kernel, dim3(grid_blocks((n_jobs + J - 1) / J)), dim3(threads), shmem, stream,
                     d_steps, n_steps, stride, J, g, n_jobs, job_traj, traj_base, job_prefix, NW, init, out, out_rank,
                     direct);
  return hipGetLastError();
}

hipError_t launch_upv_merge(GateCtx g, int64_t E, float2* merged, hipStream_t stream) {
  const int64_t n = E * g.G;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(upv_merge_kernel, dim3(grid_blocks((n + 127) / 128)), dim3(128), 0, stream, g, E, merged);
  return hipGetLastError();
}

hipError_t launch_absorb_global(const AbsorbStep& st, const AbsorbStep* d_st, GateCtx g, int64_t n_jobs,
                                const int32_t* job_traj, int32_t traj_base, const uint64_t* job_prefix,
                                int NW, const float2* A, float2* C, hipStream_t stream) {
  if (n_jobs <= 0) return hipSuccess;
  const int64_t nm = (int64_t)1 << (st.rC - st.nN);
  const int threads = 256;
  const int64_t bpj = (nm + kAbsorbPerBlock - 1) / kAbsorbPerBlock;
  const dim3 grid(grid_blocks(bpj * n_jobs));
  if (st.nK <= 1)
    hipLaunchKernelGGL(absorb_global_kernel<2>, grid, dim3(threads), 0, stream, d_st, g, n_jobs, bpj, job_traj,
                       traj_base, job_prefix, NW, A, C);
  else if (st.nK == 2)
    hipLaunchKernelGGL(absorb_global_kernel<4>, grid, dim3(threads), 0, stream, d_st, g, n_jobs, bpj, job_traj,
                       traj_base, job_prefix, NW, A, C);
  else
    hipLaunchKernelGGL(absorb_global_kernel<16>, grid, dim3(threads), 0, stream, d_st, g, n_jobs, bpj, job_traj,
                       traj_base, job_prefix, NW, A, C);
  return hipGetLastError();
}

hipError_t launch_fused(const Segment& seg, const FusedStep* d_fs, GateCtx g, int64_t n_jobs, const int32_t* job_traj,
                        int32_t traj_base, const uint64_t* job_prefix, int NW, float2* A, hipStream_t stream,
                        const float2* Ucl, int n_cl) {
  if (n_jobs <= 0) return hipSuccess;
  FusedArgs f{};
  f.Ucl = seg.np >= 10 ? Ucl : nullptr;
  f.n_cl = n_cl;
  f.fs = d_fs + seg.fused_off;
  f.n_fs = seg.count;
  f.r = seg.r;
  f.np = seg.np;
  for (int i = 0; i < kFuseMax; ++i) f.P[i] = seg.P[i];
  f.tiles_per_job = (int64_t)1 << (seg.r - seg.np);
  const size_t shmem = (((size_t)1 << seg.np) + 16 * kGateChunk) * sizeof(float2);
  // a few workgroups per CU, each walking a contiguous range of tiles
  const int64_t total = f.tiles_per_job * n_jobs;
  const dim3 grid((unsigned)std::min<int64_t>(total, 8192));
  if (f.Ucl)
    hipLaunchKernelGGL(fused_inplace_kernel<true>, grid, dim3(256), shmem, stream, f, g, n_jobs, job_traj, traj_base,
                       job_prefix, NW, A);
  else
    hipLaunchKernelGGL(fused_inplace_kernel<false>, grid, dim3(256), shmem, stream, f, g, n_jobs, job_traj, traj_base,
                       job_prefix, NW, A);
  return hipGetLastError();
}

hipError_t launch_cluster_build(const ClusterDesc* d_cl, int n_cl, const FusedStep* d_fused, GateCtx g, int64_t n_jobs,
                                const int32_t* job_traj, int32_t traj_base, float2* Ucl, hipStream_t stream) {
  if (n_jobs <= 0 || n_cl <= 0) return hipSuccess;
  hipLaunchKernelGGL(cluster_build_kernel, dim3(grid_blocks(n_jobs * n_cl)), dim3(256), 0, stream, d_cl, n_cl, d_fused,
                     g, n_jobs, job_traj, traj_base, Ucl);
  return hipGetLastError();
}

hipError_t launch_fill_one(float2* buf, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_one_kernel, dim3(grid_blocks((n + 255) / 256)), dim3(256), 0, stream, buf, n);
  return hipGetLastError();
}

hipError_t launch_join(const JoinArgs& a, hipStream_t stream) {
  const int64_t total = a.n_elems * ((int64_t)1 << (a.xb_bits + a.xT_bits));
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(join_kernel, dim3(grid_blocks((total + 255) / 256)), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_ketjoin_gemv(const JoinArgs& a, hipStream_t stream) {
  if (a.n_elems <= 0) return hipSuccess;
  if (!ketjoin_gemv_supported(a.xb_bits, a.lk_bits, a.xT_bits) || a.doubled) return hipErrorInvalidValue;
  const dim3 grid(grid_blocks(a.n_elems << (a.xT_bits - 8)));
  switch (a.xb_bits) {
    case 0: hipLaunchKernelGGL(ketjoin_gemv_kernel<1>, grid, dim3(256), 0, stream, a); break;
    case 1: hipLaunchKernelGGL(ketjoin_gemv_kernel<2>, grid, dim3(256), 0, stream, a); break;
    default: hipLaunchKernelGGL(ketjoin_gemv_kernel<4>, grid, dim3(256), 0, stream, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_ketjoin_gemv_tiled(const JoinArgs& a, const GemvTiling& g, hipStream_t stream) {
  if (a.n_elems <= 0) return hipSuccess;
  if (a.doubled || a.xb_bits > 1 || a.lk_bits > 12 || a.xT_bits < 12 || g.n_hi != a.xT_bits - 12 || g.n_hi > 32)
    return hipErrorInvalidValue;
  const dim3 grid(grid_blocks(a.n_elems << g.n_hi));
  if (a.xb_bits == 0) hipLaunchKernelGGL(ketjoin_gemv_tiled_kernel<1>, grid, dim3(256), 0, stream, a, g);
  else hipLaunchKernelGGL(ketjoin_gemv_tiled_kernel<2>, grid, dim3(256), 0, stream, a, g);
  return hipGetLastError();
}

hipError_t launch_ketjoin_gemv_lanes(const JoinArgs& a, const GemvLanes& g, hipStream_t stream) {
  if (a.n_elems <= 0) return hipSuccess;
  if (a.doubled || a.xb_bits > 1 || a.lk_bits > 12 || g.n_hk > 10 || g.n_hx > 32) return hipErrorInvalidValue;
  const int rows = 1 << a.xb_bits, nk = 1 << a.lk_bits, nkh = 1 << g.n_hk;
  const size_t shmem = (size_t)rows * nk * sizeof(float2) + (size_t)nkh * (sizeof(int64_t) + sizeof(int));
  const int64_t nxb = (int64_t)1 << g.n_hx;
  // about 32 values of the off-lane x bits per wavefront, at most 2^20 workgroups
  int64_t wpe = (nxb + 127) / 128;
  if (wpe < 1) wpe = 1;
  while (wpe > 1 && a.n_elems * wpe > ((int64_t)1 << 20)) wpe = (wpe + 1) / 2;
  const dim3 grid(grid_blocks(a.n_elems * wpe));
  if (rows == 1) hipLaunchKernelGGL(ketjoin_gemv_lanes_kernel<1>, grid, dim3(256), shmem, stream, a, g, wpe);
  else hipLaunchKernelGGL(ketjoin_gemv_lanes_kernel<2>, grid, dim3(256), shmem, stream, a, g, wpe);
  return hipGetLastError();
}

hipError_t launch_permute_T(const float2* T, int64_t t_stride, int64_t n_traj, const int64_t* tab,
                            const Plan::JoinDev& jd, int xT_bits, int lk_bits, int lb_bits, float2* Tc,
                            hipStream_t stream) {
  const int64_t total = n_traj << (xT_bits + lk_bits + lb_bits);
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(permute_T_kernel, dim3(grid_blocks((total + 255) / 256)), dim3(256), 0, stream, T, t_stride,
                     n_traj, tab, jd, xT_bits, lk_bits, lb_bits, Tc);
  return hipGetLastError();
}

bool qform_supported(int lk_bits) { return lk_bits == 4 || lk_bits == 5; }
bool qform_split_supported(int lk_bits) { return lk_bits == 4 || lk_bits == 5; }

hipError_t launch_qform_split(const QformArgs& a, int n_traj, int max_rows, bool f16, hipStream_t stream) {
  if (n_traj <= 0 || max_rows <= 0) return hipSuccess;
  const int tiles = (max_rows + 63) / 64;
  const int nx = 1 << a.xT_bits;
  const int nc = nx >= 128 ? 8 : (nx >= 64 ? 4 : (nx >= 32 ? 2 : 1));
  const int xtiles = (nx + 16 * nc - 1) / (16 * nc);
  dim3 grid((unsigned)tiles, (unsigned)n_traj, (unsigned)xtiles);
#define PTSBE_QSPLIT(KV, NCV)                                                                         \
  do {                                                                                                \
    if (f16) hipLaunchKernelGGL((qform_split_kernel<KV, NCV, true>), grid, dim3(256), 0, stream, a);  \
    else hipLaunchKernelGGL((qform_split_kernel<KV, NCV, false>), grid, dim3(256), 0, stream, a);     \
  } while (0)
  if (a.lk_bits == 4) {
    if (nc == 8) PTSBE_QSPLIT(16, 8); else if (nc == 4) PTSBE_QSPLIT(16, 4);
    else if (nc == 2) PTSBE_QSPLIT(16, 2); else PTSBE_QSPLIT(16, 1);
  } else if (a.lk_bits == 5) {
    if (nc == 8) PTSBE_QSPLIT(32, 8); else if (nc == 4) PTSBE_QSPLIT(32, 4);
    else if (nc == 2) PTSBE_QSPLIT(32, 2); else PTSBE_QSPLIT(32, 1);
  } else {
    return hipErrorInvalidValue;
  }
#undef PTSBE_QSPLIT
  return hipGetLastError();
}
bool ketjoin_supported(int lk_bits) { return lk_bits >= 2 && lk_bits <= 6; }

size_t qform_theta_bytes(int xT_bits, int lk_bits) {
  return ((size_t)4 << (xT_bits + 2 * lk_bits)) + ((size_t)4 << xT_bits);   // + fp16 split scales
}

hipError_t launch_theta_T(const float2* T, int64_t t_stride, int64_t n_traj, const int64_t* tab,
                          const Plan::JoinDev& jd, int xT_bits, int lk_bits, float* Th, int split,
                          hipStream_t stream) {
  if (n_traj <= 0) return hipSuccess;
  if (!qform_supported(lk_bits)) return hipErrorInvalidValue;
  const dim3 grid(grid_blocks(n_traj << xT_bits));
  if (lk_bits == 4)
    hipLaunchKernelGGL(theta_T_kernel<16>, grid, dim3(256), 0, stream, T, t_stride, n_traj, tab, jd, xT_bits, Th,
                       split);
  else
    hipLaunchKernelGGL(theta_T_kernel<32>, grid, dim3(256), 0, stream, T, t_stride, n_traj, tab, jd, xT_bits, Th,
                       split);
  return hipGetLastError();
}

hipError_t launch_qform(const QformArgs& a, int n_traj, int max_rows, hipStream_t stream) {
  if (n_traj <= 0 || max_rows <= 0) return hipSuccess;
  const int tiles = (max_rows + 63) / 64;
  const int nx = 1 << a.xT_bits;
  const int nc = nx >= 128 ? 8 : (nx >= 64 ? 4 : (nx >= 32 ? 2 : 1));
  const int xtiles = (nx + 16 * nc - 1) / (16 * nc);
  dim3 grid((unsigned)tiles, (unsigned)n_traj, (unsigned)xtiles);
#define PTSBE_QFORM(KV, NCV) hipLaunchKernelGGL((qform_mfma_kernel<KV, NCV>), grid, dim3(256), 0, stream, a)
  if (a.lk_bits == 4) {
    if (nc == 8) PTSBE_QFORM(16, 8); else if (nc == 4) PTSBE_QFORM(16, 4); else if (nc == 2) PTSBE_QFORM(16, 2);
    else PTSBE_QFORM(16, 1);
  } else if (a.lk_bits == 5) {
    if (nc == 8) PTSBE_QFORM(32, 8); else if (nc == 4) PTSBE_QFORM(32, 4); else if (nc == 2) PTSBE_QFORM(32, 2);
    else PTSBE_QFORM(32, 1);
  } else {
    return hipErrorInvalidValue;
  }
#undef PTSBE_QFORM
  return hipGetLastError();
}

hipError_t launch_ketjoin(const QformArgs& a, int n_traj, int max_rows, hipStream_t stream) {
  if (n_traj <= 0 || max_rows <= 0) return hipSuccess;
  const int tiles = (max_rows + 63) / 64;
  const int ntile = ((1 << a.xT_bits) + 15) / 16;
  int64_t wg = (int64_t)tiles * n_traj;
  int zs = 1;
  while (zs < ntile && wg * zs < 4096) zs *= 2;
  dim3 grid((unsigned)tiles, (unsigned)n_traj, (unsigned)zs);
  switch (a.lk_bits) {
    case 2: hipLaunchKernelGGL(ketjoin_mfma_kernel<4>, grid, dim3(256), 0, stream, a); break;
    case 3: hipLaunchKernelGGL(ketjoin_mfma_kernel<8>, grid, dim3(256), 0, stream, a); break;
    case 4: hipLaunchKernelGGL(ketjoin_mfma_kernel<16>, grid, dim3(256), 0, stream, a); break;
    case 5: hipLaunchKernelGGL(ketjoin_mfma_kernel<32>, grid, dim3(256), 0, stream, a); break;
    case 6: hipLaunchKernelGGL(ketjoin_mfma_kernel<64>, grid, dim3(256), 0, stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_row_totals(const float* pop, int64_t n_elems, int b, double* totals, hipStream_t stream) {
  if (n_elems <= 0) return hipSuccess;
  hipLaunchKernelGGL(row_totals_kernel, dim3(grid_blocks(n_elems)), dim3(256), 0, stream, pop, n_elems, b, totals);
  return hipGetLastError();
}

__global__ void prefix_or_kernel(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst, int64_t n, int NW,
                                 int wi, uint64_t bits) {
  for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < n * NW; id += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t v = src ? src[id] : 0ull;
    dst[id] = (int)(id % NW) == wi ? (v | bits) : v;
  }
}

__global__ void amp_accumulate_kernel(float2* __restrict__ acc, const float2* __restrict__ amp, int64_t n) {
  for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < n; id += (int64_t)gridDim.x * blockDim.x) {
    const float2 a = acc[id], b = amp[id];
    acc[id] = make_float2(a.x + b.x, a.y + b.y);
  }
}

__global__ void amp_population_kernel(const float2* __restrict__ acc, float* __restrict__ pop, int64_t n) {
  for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < n; id += (int64_t)gridDim.x * blockDim.x) {
    const float2 a = acc[id];
    pop[id] = a.x * a.x + a.y * a.y;
  }
}

hipError_t launch_prefix_or(const uint64_t* src, uint64_t* dst, int64_t n, int NW, int wi, uint64_t bits,
                            hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(prefix_or_kernel, dim3(grid_blocks((n * NW + 255) / 256)), dim3(256), 0, stream, src, dst, n,
                     NW, wi, bits);
  return hipGetLastError();
}

hipError_t launch_amp_accumulate(float2* acc, const float2* amp, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(amp_accumulate_kernel, dim3(grid_blocks((n + 255) / 256)), dim3(256), 0, stream, acc, amp, n);
  return hipGetLastError();
}

hipError_t launch_amp_population(const float2* acc, float* pop, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(amp_population_kernel, dim3(grid_blocks((n + 255) / 256)), dim3(256), 0, stream, acc, pop, n);
  return hipGetLastError();
}

hipError_t launch_sample(const SampleArgs& a, hipStream_t stream) {
  if (a.n_elems <= 0) return hipSuccess;
  const int n = 1 << a.b;
  const size_t shmem = (size_t)n * sizeof(int);
  if (a.lane_path && a.b <= 5) {
    const unsigned grid = grid_blocks((a.n_elems + 63) / 64);
    switch (a.b) {
      case 0: hipLaunchKernelGGL(sample_lanes_kernel<0>, dim3(grid), dim3(64), shmem, stream, a); break;
      case 1: hipLaunchKernelGGL(sample_lanes_kernel<1>, dim3(grid), dim3(64), shmem, stream, a); break;
      case 2: hipLaunchKernelGGL(sample_lanes_kernel<2>, dim3(grid), dim3(64), shmem, stream, a); break;
      case 3: hipLaunchKernelGGL(sample_lanes_kernel<3>, dim3(grid), dim3(64), shmem, stream, a); break;
      case 4: hipLaunchKernelGGL(sample_lanes_kernel<4>, dim3(grid), dim3(64), shmem, stream, a); break;
      default: hipLaunchKernelGGL(sample_lanes_kernel<5>, dim3(grid), dim3(64), shmem, stream, a); break;
    }
    return hipGetLastError();
  }
  hipLaunchKernelGGL(sample_kernel, dim3(grid_blocks(a.n_elems)), dim3(64), shmem, stream, a);
  return hipGetLastError();
}

hipError_t launch_children(const ChildArgs& a, hipStream_t stream) {
  if (a.n_elems <= 0) return hipSuccess;
  const int n = 1 << a.b;
  const size_t shmem = (size_t)3 * n * sizeof(int);
  if (a.lane_path && a.b <= 5)
    hipLaunchKernelGGL(children_lanes_kernel, dim3(grid_blocks((a.n_elems + 63) / 64)), dim3(64), shmem, stream, a);
  else
    hipLaunchKernelGGL(children_kernel, dim3(grid_blocks(a.n_elems)), dim3(64), shmem, stream, a);
  return hipGetLastError();
}

hipError_t launch_np_init(int64_t E, int64_t t0, int32_t* elem_traj, uint64_t* elem_prefix, int NW,
                          hipStream_t stream) {
  if (E <= 0) return hipSuccess;
  hipLaunchKernelGGL(np_init_kernel, dim3(grid_blocks((E + 255) / 256)), dim3(256), 0, stream, E, t0, elem_traj,
                     elem_prefix, NW);
  return hipGetLastError();
}

hipError_t launch_np_direct_rows(int64_t n_elems, int draws, const int32_t* elem_traj, const uint64_t* elem_prefix,
                                 int NW, uint64_t* bits, int32_t* row_traj, hipStream_t stream) {
  if (n_elems <= 0) return hipSuccess;
  hipLaunchKernelGGL(np_direct_rows_kernel, dim3(grid_blocks((n_elems * draws + 255) / 256)), dim3(256), 0, stream,
                     n_elems, draws, elem_traj, elem_prefix, NW, bits, row_traj);
  return hipGetLastError();
}

hipError_t launch_np_direct_prefix_p(int64_t n_elems, int draws, const int32_t* elem_traj, const double* elem_total,
                                     const double* traj_norm, double* p_prefix, hipStream_t stream) {
  if (n_elems <= 0 || !p_prefix) return hipSuccess;
  hipLaunchKernelGGL(np_direct_prefix_p_kernel, dim3(grid_blocks((n_elems * draws + 255) / 256)), dim3(256), 0,
                     stream, n_elems, draws, elem_traj, elem_total, traj_norm, p_prefix);
  return hipGetLastError();
}

hipError_t launch_np_rows(int64_t n_elems, int draws, const int32_t* elem_traj, int32_t* shot_off,
                          int32_t* shot_cnt, int32_t* shot_ids, int64_t* traj_base, hipStream_t stream) {
  if (n_elems <= 0) return hipSuccess;
  if (draws < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(np_rows_kernel, dim3(grid_blocks((n_elems + 255) / 256)), dim3(256), 0, stream, n_elems, draws,
                     elem_traj, shot_off, shot_cnt, shot_ids, traj_base);
  return hipGetLastError();
}

hipError_t launch_exh_count(const ExhArgs& a, hipStream_t stream) {
  if (a.n_elems <= 0) return hipSuccess;
  if (a.b < 0 || a.b > kMaxBatch || a.tile_bits != (a.b > 12 ? a.b - 12 : 0)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(exh_count_kernel, dim3(grid_blocks(a.n_elems << a.tile_bits)), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_exh_write(const ExhArgs& a, hipStream_t stream) {
  if (a.n_elems <= 0) return hipSuccess;
  if (a.b < 0 || a.b > kMaxBatch || a.tile_bits != (a.b > 12 ? a.b - 12 : 0) || !a.bits) return hipErrorInvalidValue;
  hipLaunchKernelGGL(exh_write_kernel, dim3(grid_blocks(a.n_elems << a.tile_bits)), dim3(256), 0, stream, a);
  return hipGetLastError();
}

size_t scan_scratch_bytes(int64_t n) {
  return (size_t)((n + kScanBlock - 1) / kScanBlock + 1) * sizeof(int32_t);
}

hipError_t launch_scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* d_total, int32_t* d_scratch,
                           hipStream_t stream) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (n <= 0) {
    hipLaunchKernelGGL(scan_sums_block, dim3(1), dim3(1024), 0, stream, d_scratch, (int64_t)0, d_total);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(scan_block_sums, dim3((unsigned)nb), dim3(256), 0, stream, in, n, d_scratch);
  hipLaunchKernelGGL(scan_sums_block, dim3(1), dim3(1024), 0, stream, d_scratch, nb, d_total);
  hipLaunchKernelGGL(scan_apply, dim3((unsigned)nb), dim3(256), 0, stream, in, n, d_scratch, out);
  return hipGetLastError();
}

hipError_t launch_weights(const WeightArgs& a, hipStream_t stream) {
  hipLaunchKernelGGL(weights_kernel, dim3(1), dim3(1024), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_init_elements(int64_t E, const int64_t* shots_per_traj, int32_t* elem_traj, uint64_t* elem_prefix,
                                int NW, int32_t* shot_off, int32_t* shot_cnt, int64_t* traj_shot_base,
                                int32_t* shot_ids, int32_t* shot_traj, uint64_t* shots, int64_t M,
                                hipStream_t stream) {
  if (E > 0)
    hipLaunchKernelGGL(init_traj_kernel, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, stream, E,
                       shots_per_traj, traj_shot_base, elem_traj, elem_prefix, NW, shot_off, shot_cnt);
  if (M > 0)
    hipLaunchKernelGGL(init_shots_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, stream, M, E,
                       traj_shot_base, shot_ids, shot_traj, shots, NW);
  return hipGetLastError();
}

hipError_t launch_init_shots(int64_t M, int64_t E, const int64_t* traj_shot_base, int32_t* shot_ids,
                             int32_t* shot_traj, uint64_t* shots, int NW, hipStream_t stream) {
  if (M > 0)
    hipLaunchKernelGGL(init_shots_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, stream, M, E,
                       traj_shot_base, shot_ids, shot_traj, shots, NW);
  return hipGetLastError();
}

hipError_t launch_traj_ranges(const int32_t* elem_traj, int64_t n_elems, int64_t E, int32_t* traj_first,
                              hipStream_t stream) {
  hipLaunchKernelGGL(traj_first_kernel, dim3((unsigned)((n_elems + 1 + 255) / 256)), dim3(256), 0, stream,
                     elem_traj, n_elems, E, traj_first);
  return hipGetLastError();
}

}  // namespace ptsbe
