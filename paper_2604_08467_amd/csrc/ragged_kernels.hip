// Kernels of ragged sets: the statevector method for many circuits at once.
// Every kernel is persistent (a fixed grid that walks its task list with a
// grid-stride loop) and reads data-dependent counts from device memory, so a
// wave's whole launch sequence needs no host round trip and can be captured as
// one graph.  Tasks of a level are independent; the kernel boundary between
// levels is the dependency barrier.  Per element, the circuit-specific data
// (qubit count, batch layout, gate windows, shot rows) comes from its piece.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.h"
#include "internal.h"
#include "philox.h"
#include "sv_tile.h"

namespace ptsbe {
namespace {

__device__ inline double norm2(float2 v) { return (double)v.x * v.x + (double)v.y * v.y; }

__device__ inline int find_le(const int64_t* starts, int n, int64_t v) {   // largest i < n with starts[i] <= v
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (starts[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Sum over y in [y0, y0 + ys) of |P[(y << (start + b)) + (x << start) + s]|^2
// for every x < 2^b (FP64); out(x, value) receives the sums.  Wide batches give
// each thread the values x = tid + 256 i; narrow ones share a value between
// 256 / 2^b threads, combined in a fixed order.  Uniform over the workgroup.
template <typename Out>
__device__ inline void marg_sum(const float2* P, int start, int b, uint64_t s, int64_t y0, int64_t ys,
                                double* red, Out out) {
  const int tid = threadIdx.x;
  const int X = 1 << b, sb = start + b;
  if (X >= kRgThreads) {
    const int nx = X / kRgThreads;
    double acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0;
    for (int64_t y = y0; y < y0 + ys; ++y) {
      const float2* row = P + (y << sb) + s;
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (i < nx) acc[i] += norm2(row[(int64_t)(tid + kRgThreads * i) << start]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (i < nx) out(tid + kRgThreads * i, acc[i]);
  } else {
    const int R = kRgThreads >> b;
    const int x = tid & (X - 1), r = tid >> b;
    double acc = 0.0;
    for (int64_t y = y0 + r; y < y0 + ys; y += R) acc += norm2(P[(y << sb) + ((int64_t)x << start) + s]);
    red[tid] = acc;
    __syncthreads();
    if (tid < X) {
      double t = 0.0;
      for (int k = 0; k < R; ++k) t += red[k * X + tid];
      out(tid, t);
    }
    __syncthreads();
  }
}

__global__ void rg_start_kernel(RgWave w) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (w.done) {
    for (int i = 0; i < w.n_jobs; ++i) w.done[i] = 0ull;
    w.done[w.n_jobs] = (uint64_t)wall_clock64();
  }
  *w.bad_flag = 0;
}

// |0...0> states, UPV-merged gates of every piece, shot rows and first-batch elements.
__global__ void __launch_bounds__(kRgThreads) rg_prepare_kernel(RgWave w) {
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int p = 0; p < w.n_pieces; ++p) {
    const RgPiece& pc = w.pieces[p];
    const int64_t sz = (int64_t)pc.nj << pc.n, mask = ((int64_t)1 << pc.n) - 1;
    for (int64_t i = gid; i < sz; i += stride) pc.psi[i] = make_float2((i & mask) == 0 ? 1.f : 0.f, 0.f);
    float2* merged = const_cast<float2*>(pc.g.merged);
    for (int64_t id = gid; id < (int64_t)pc.nj * pc.g.G; id += stride) {
      float2 m[16];
      merge_gate(pc.g, (int)(id % pc.g.G), (int)(id / pc.g.G), m);
      for (int i = 0; i < 16; ++i) merged[id * 16 + i] = m[i];
    }
  }
  for (int64_t r = gid; r < w.R; r += stride) {
    w.ids[0][r] = (int32_t)r;
    const int wt = find_le(w.traj_row0, w.T, r);
    const RgPiece& pc = w.pieces[w.traj_piece[wt]];
    pc.shots[r - pc.row0 + pc.job_row0] = 0ull;
  }
  for (int64_t t = gid; t < w.T; t += stride) {
    w.el_wt[0][t] = (int32_t)t;
    w.el_prefix[0][t] = 0ull;
    w.el_off[0][t] = (int32_t)w.traj_row0[t];
    w.el_cnt[0][t] = (int32_t)(w.traj_row0[t + 1] - w.traj_row0[t]);
  }
  if (gid == 0) {
    w.counts[0] = w.T;
    for (int j = 1; j <= kRgMaxBatches; ++j) w.counts[j] = 0;
  }
}

// Window level `level`: every 2^np tile of every trajectory of every piece that
// has that many windows; tiles of heavier circuits come first in the queue.
__global__ void __launch_bounds__(kRgThreads) rg_window_kernel(RgWave w, RgLevel lv, int level) {
  extern __shared__ float2 lds[];
  float2* tile = lds;
  float2* Gm = lds + (1 << kFuseMax);   // staged gates: generic chunks, or one 16-entry slot per op
  __shared__ uint64_t pw[1];
  if (threadIdx.x == 0) pw[0] = 0ull;
  // contiguous task ranges per workgroup: consecutive tiles of one trajectory
  // reuse the staged gate matrices
  const int64_t per = (lv.tasks + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per, b1 = b0 + per < lv.tasks ? b0 + per : lv.tasks;
  const RgPiece* last_pc = nullptr;
  int64_t last_traj = -1;
  for (int64_t task = b0; task < b1; ++task) {
    const int e = find_le(lv.start, lv.n, task);
    const RgPiece& pc = w.pieces[lv.piece[e]];
    const RgWindow& wd = pc.win[level];
    const int tb = pc.n - wd.np;
    const int64_t local = task - lv.start[e];
    const int64_t traj = local >> tb;
    const uint32_t t = (uint32_t)(local & (((int64_t)1 << tb) - 1));
    const bool same = &pc == last_pc && traj == last_traj;
    if (pc.swin) {
      // compact plain ops (scalar-cache reads), gates staged once per trajectory
      const SvWin& sw = pc.swin[level];
      const SvOp* ops = pc.sops + sw.op_off;
      if (!same) {
        __syncthreads();   // nobody reads the previous trajectory's gates any more
        for (int i = threadIdx.x; i < 16 * sw.n_ops; i += kRgThreads) {
          const SvOp& op = ops[i >> 4];
          const int el = i & 15, d2 = op.kind == kSvOpGate1 ? 4 : 16;
          Gm[i] = el < d2 ? pc.g.merged[(traj * pc.g.G + op.gate) * 16 + op.idx[el]] : make_float2(0.f, 0.f);
        }
        __syncthreads();
      }
      float2* A = pc.psi + (traj << pc.n) + deposit_other(t, sw.other);
      if (sw.np == 12) plain_tile_pass<12>(ops, sw.n_ops, sw.P, A, A, tile, Gm);
      else if (sw.np == 11) plain_tile_pass<11>(ops, sw.n_ops, sw.P, A, A, tile, Gm);
      else plain_tile_pass<10>(ops, sw.n_ops, sw.P, A, A, tile, Gm);
    } else {
      const bool ready = same && wd.n_fs <= kGateChunk && last_pc && !last_pc->swin;
      window_tile_pass(pc.fused + wd.fused_off, wd.n_fs, wd.P, wd.np, pc.n, t, pc.psi + (traj << pc.n), pc.g,
                       (int)traj, pw, tile, Gm, nullptr, ready);
    }
    last_pc = &pc;
    last_traj = traj;
  }
}

// First batch: partial sums over slices of the later qubits, per trajectory.
__global__ void __launch_bounds__(kRgThreads) rg_marg0_kernel(RgWave w, int64_t tasks) {
  __shared__ double red[kRgThreads];
  for (int64_t task = blockIdx.x; task < tasks; task += gridDim.x) {
    const int p = find_le(w.m0_start, w.n_pieces, task);
    const RgPiece& pc = w.pieces[p];
    const int ls = pc.log_split0;
    const int64_t local = task - w.m0_start[p];
    const int64_t traj = local >> ls, sl = local & (((int64_t)1 << ls) - 1);
    const int b = pc.b[0];
    const int64_t ys = (int64_t)1 << (pc.n - b - ls);
    double* out = w.part + ((pc.part_off + (traj << ls) + sl) << w.xbits);
    marg_sum(pc.psi + (traj << pc.n), 0, b, 0ull, sl * ys, ys, red, [&](int x, double v) { out[x] = v; });
  }
}

__global__ void rg_reduce0_kernel(RgWave w) {
  const int64_t X = (int64_t)1 << w.xbits;
  for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < (int64_t)w.T * X;
       id += (int64_t)gridDim.x * blockDim.x) {
    const int64_t wt = id >> w.xbits, x = id & (X - 1);
    const RgPiece& pc = w.pieces[w.traj_piece[wt]];
    if (x >= ((int64_t)1 << pc.b[0])) continue;
    const int ls = pc.log_split0;
    const int64_t traj = wt - pc.traj_off;
    double t = 0.0;
    for (int64_t sl = 0; sl < ((int64_t)1 << ls); ++sl) t += w.part[((pc.part_off + (traj << ls) + sl) << w.xbits) + x];
    w.pop[id] = (float)t;
  }
}

// Batch j >= 1: the marginal of every element from its trajectory's state.
__global__ void __launch_bounds__(kRgThreads) rg_marg_kernel(RgWave w, int j, int cur) {
  __shared__ double red[kRgThreads];
  const int64_t U = w.counts[j];
  for (int64_t e = blockIdx.x; e < U; e += gridDim.x) {
    const int wt = w.el_wt[cur][e];
    const RgPiece& pc = w.pieces[w.traj_piece[wt]];
    const int start = pc.start[j], b = pc.b[j];
    const uint64_t s = w.el_prefix[cur][e] & ((1ull << start) - 1ull);
    const int64_t ys = (int64_t)1 << (pc.n - start - b);
    float* out = w.pop + (e << w.xbits);
    marg_sum(pc.psi + ((int64_t)(wt - pc.traj_off) << pc.n), start, b, s, 0, ys, red,
             [&](int x, double v) { out[x] = (float)v; });
  }
}

__device__ void block_scan_f64_rg(double* c, int n, double* part) {
  const int T = kRgThreads;
  const int per = (n + T - 1) / T;
  const int lo = threadIdx.x * per;
  const int hi = lo + per < n ? lo + per : n;
  double s = 0.0;
  for (int i = lo; i < hi; ++i) { s += c[i]; c[i] = s; }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {
    const double v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0.0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  const double add = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0.0;
  for (int i = lo; i < hi; ++i) c[i] += add;
  __syncthreads();
}

// FP64 cumulative sums and inverse-CDF draws of every element of batch j, as in
// the single-circuit sampler (same Philox counters: job trajectory, batch, shot
// index within the trajectory).
__global__ void __launch_bounds__(kRgThreads) rg_sample_kernel(RgWave w, int j, int cur) {
  extern __shared__ double sm[];
  const int Xmax = 1 << w.xbits;
  double* C = sm;
  double* part = sm + Xmax;
  int* hist = reinterpret_cast<int*>(part + kRgThreads);
  __shared__ int last_pos, nchild;
  const int64_t U = w.counts[j];
  for (int64_t e = blockIdx.x; e < U; e += gridDim.x) {
    const int wt = w.el_wt[cur][e];
    const RgPiece& pc = w.pieces[w.traj_piece[wt]];
    const int b = pc.b[j], start = pc.start[j];
    const int n = 1 << b;
    const float* pi = w.pop + (e << w.xbits);
    for (int i = threadIdx.x; i < n; i += kRgThreads) {
      C[i] = (double)pi[i];
      hist[i] = 0;
    }
    if (threadIdx.x == 0) { last_pos = -1; nchild = 0; }
    __syncthreads();
    {
      int lp = -1;
      for (int i = threadIdx.x; i < n; i += kRgThreads)
        if (C[i] > 0.0) lp = i;
      atomicMax(&last_pos, lp);
    }
    __syncthreads();
    block_scan_f64_rg(C, n, part);
    const double Z = C[n - 1];
    const int traj = pc.t0 + (wt - pc.traj_off);
    if (threadIdx.x == 0) {
      if (!(Z >= 0.0) || !isfinite(Z)) atomicExch(w.bad_flag, 1);   // Z == 0: weight-0 trajectory
      if (j == 0) pc.norms[traj] = Z;
    }
    const int off = w.el_off[cur][e], cnt = w.el_cnt[cur][e];
    const int64_t tbase = w.traj_row0[wt];
    for (int i = threadIdx.x; i < cnt; i += kRgThreads) {
      const int row = w.ids[cur][off + i];
      const uint32_t t = (uint32_t)(row - tbase);
      const double u = philox_uniform(pc.seed, 2u, (uint32_t)traj, (uint32_t)j, t, 0u);
      const double target = u * Z;
      int lo = 0, hi = n;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (C[mid] > target) hi = mid; else lo = mid + 1;
      }
      int x = lo < n ? lo : last_pos;
      if (x < 0) x = 0;
      w.shot_x[row] = x;
      pc.shots[row - pc.row0 + pc.job_row0] |= (uint64_t)x << start;
      atomicAdd(&hist[x], 1);
    }
    __syncthreads();
    int c = 0;
    for (int i = threadIdx.x; i < n; i += kRgThreads) c += hist[i] > 0;
    atomicAdd(&nchild, c);
    __syncthreads();
    if (threadIdx.x == 0) {
      w.child_cnt[e] = (j + 1 < pc.f) ? nchild : 0;
      if (j == pc.f - 1 && w.done) atomicMax((unsigned long long*)&w.done[pc.job], (unsigned long long)wall_clock64());
    }
    __syncthreads();
  }
}

// exclusive scan of child counts of batch j: per 1024-block sums, one block scans
// the sums (total -> counts[j + 1]), then every block scans its entries
constexpr int kRgScan = 1024;

__global__ void rg_scan_sums_kernel(RgWave w, int j) {
  __shared__ int red[kRgThreads];
  const int64_t n = w.counts[j];
  const int64_t b0 = (int64_t)blockIdx.x * kRgScan;
  if (b0 >= n) return;
  int s = 0;
  for (int64_t i = b0 + threadIdx.x; i < b0 + kRgScan && i < n; i += kRgThreads) s += w.child_cnt[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = kRgThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) w.scan_sums[blockIdx.x] = red[0];
}

__global__ void rg_scan_top_kernel(RgWave w, int j) {
  __shared__ int part[kRgThreads];
  const int64_t n = w.counts[j];
  const int nb = (int)((n + kRgScan - 1) / kRgScan);
  const int per = (nb + kRgThreads - 1) / kRgThreads;
  const int lo = threadIdx.x * per, hi = lo + per < nb ? lo + per : nb;
  int s = 0;
  for (int i = lo; i < hi; ++i) s += w.scan_sums[i];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int t = 0; t < kRgThreads; ++t) { const int v = part[t]; part[t] = acc; acc += v; }
    w.counts[j + 1] = acc;
  }
  __syncthreads();
  int acc = part[threadIdx.x];
  for (int i = lo; i < hi; ++i) { const int v = w.scan_sums[i]; w.scan_sums[i] = acc; acc += v; }
}

__global__ void rg_scan_apply_kernel(RgWave w, int j) {
  __shared__ int part[kRgThreads];
  const int64_t n = w.counts[j];
  const int64_t b0 = (int64_t)blockIdx.x * kRgScan;
  if (b0 >= n) return;
  constexpr int per = kRgScan / kRgThreads;
  const int64_t lo = b0 + threadIdx.x * per;
  int v[per];
  int s = 0;
  for (int i = 0; i < per; ++i) {
    v[i] = (lo + i < n) ? w.child_cnt[lo + i] : 0;
    s += v[i];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = w.scan_sums[blockIdx.x];
    for (int t = 0; t < kRgThreads; ++t) { const int x = part[t]; part[t] = acc; acc += x; }
  }
  __syncthreads();
  int acc = part[threadIdx.x];
  for (int i = 0; i < per; ++i) {
    if (lo + i < n) w.child_off[lo + i] = acc;
    acc += v[i];
  }
}

// Next batch's elements: the distinct (prefix, x) of each element's shots, in x order.
__global__ void __launch_bounds__(kRgThreads) rg_children_kernel(RgWave w, int j, int cur) {
  extern __shared__ int ism[];
  const int Xmax = 1 << w.xbits;
  int* hist = ism;
  int* startx = ism + Xmax;
  int* rank = ism + 2 * Xmax;
  __shared__ int part_s[kRgThreads];
  __shared__ int part_r[kRgThreads];
  const int nxt = cur ^ 1;
  const int64_t U = w.counts[j];
  for (int64_t e = blockIdx.x; e < U; e += gridDim.x) {
    const int wt = w.el_wt[cur][e];
    const RgPiece& pc = w.pieces[w.traj_piece[wt]];
    if (j + 1 >= pc.f) continue;                       // the circuit's last batch: no children
    const int b = pc.b[j], start = pc.start[j];
    const int n = 1 << b;
    for (int i = threadIdx.x; i < n; i += kRgThreads) hist[i] = 0;
    __syncthreads();
    const int off = w.el_off[cur][e], cnt = w.el_cnt[cur][e];
    for (int i = threadIdx.x; i < cnt; i += kRgThreads) atomicAdd(&hist[w.shot_x[w.ids[cur][off + i]]], 1);
    __syncthreads();
    const int per = (n + kRgThreads - 1) / kRgThreads;
    const int lo = threadIdx.x * per, hi = lo + per < n ? lo + per : n;
    int s = 0, r = 0;
    for (int i = lo; i < hi; ++i) { s += hist[i]; r += hist[i] > 0; }
    part_s[threadIdx.x] = s;
    part_r[threadIdx.x] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
      int as = 0, ar = 0;
      for (int t = 0; t < kRgThreads; ++t) {
        const int ts = part_s[t], tr = part_r[t];
        part_s[t] = as; part_r[t] = ar;
        as += ts; ar += tr;
      }
    }
    __syncthreads();
    s = part_s[threadIdx.x];
    r = part_r[threadIdx.x];
    for (int i = lo; i < hi; ++i) {
      startx[i] = s; rank[i] = r;
      s += hist[i]; r += hist[i] > 0;
    }
    __syncthreads();
    const int64_t cbase = w.child_off[e];
    const uint64_t pp = w.el_prefix[cur][e];
    for (int x = threadIdx.x; x < n; x += kRgThreads) {
      if (hist[x] == 0) continue;
      const int64_t c = cbase + rank[x];
      w.el_wt[nxt][c] = wt;
      w.el_prefix[nxt][c] = pp | ((uint64_t)x << start);
      w.el_off[nxt][c] = off + startx[x];
      w.el_cnt[nxt][c] = hist[x];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += kRgThreads) {
      const int row = w.ids[cur][off + i];
      const int x = w.shot_x[row];
      const int pos = atomicAdd(&startx[x], 1);
      w.ids[nxt][off + pos] = row;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_rg_start(const RgWave& w, hipStream_t s) {
  hipLaunchKernelGGL(rg_start_kernel, dim3(1), dim3(64), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_rg_prepare(const RgWave& w, int grid, hipStream_t s) {
  hipLaunchKernelGGL(rg_prepare_kernel, dim3((unsigned)grid), dim3(kRgThreads), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_rg_window(const RgWave& w, const RgLevel& lv, int level, int n_cu, hipStream_t s) {
  if (lv.tasks <= 0) return hipSuccess;
  const size_t shmem = (((size_t)1 << kFuseMax) + 16 * (size_t)std::max(kGateChunk, (int)lv.max_ops)) * sizeof(float2);
  // a persistent grid is only as large as what fits on the chip at once
  int per_cu = 0;
  hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, rg_window_kernel, kRgThreads, shmem);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(rg_window_kernel, dim3((unsigned)(n_cu * std::max(per_cu, 1))), dim3(kRgThreads), shmem, s, w,
                     lv, level);
  return hipGetLastError();
}

hipError_t launch_rg_marginal0(const RgWave& w, int64_t tasks, int grid, hipStream_t s) {
  if (tasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(rg_marg0_kernel, dim3((unsigned)grid), dim3(kRgThreads), 0, s, w, tasks);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(rg_reduce0_kernel, dim3((unsigned)grid), dim3(kRgThreads), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_rg_marginal(const RgWave& w, int j, int cur, int grid, hipStream_t s) {
  hipLaunchKernelGGL(rg_marg_kernel, dim3((unsigned)grid), dim3(kRgThreads), 0, s, w, j, cur);
  return hipGetLastError();
}

hipError_t launch_rg_sample(const RgWave& w, int j, int cur, int grid, hipStream_t s) {
  const size_t X = (size_t)1 << w.xbits;
  const size_t shmem = X * 8 + kRgThreads * 8 + X * 4;
  hipLaunchKernelGGL(rg_sample_kernel, dim3((unsigned)grid), dim3(kRgThreads), shmem, s, w, j, cur);
  return hipGetLastError();
}

hipError_t launch_rg_scan(const RgWave& w, int j, hipStream_t s) {
  const unsigned nb = (unsigned)std::max<int64_t>(1, (w.cap + kRgScan - 1) / kRgScan);
  hipLaunchKernelGGL(rg_scan_sums_kernel, dim3(nb), dim3(kRgThreads), 0, s, w, j);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(rg_scan_top_kernel, dim3(1), dim3(kRgThreads), 0, s, w, j);
  err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(rg_scan_apply_kernel, dim3(nb), dim3(kRgThreads), 0, s, w, j);
  return hipGetLastError();
}

hipError_t launch_rg_children(const RgWave& w, int j, int cur, int grid, hipStream_t s) {
  const size_t shmem = ((size_t)3 << w.xbits) * 4;
  hipLaunchKernelGGL(rg_children_kernel, dim3((unsigned)grid), dim3(kRgThreads), shmem, s, w, j, cur);
  return hipGetLastError();
}

}  // namespace ptsbe
