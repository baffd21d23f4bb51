// Statevector method of the unified path.  The ket network of every trajectory
// is contracted in circuit order into its full statevector: one gate schedule
// (LDS windows of at most 12 qubits) shared by all trajectories, each applying
// its own UPV-merged gates (Sec. III-A).  The marginal of batch j for an element
// (trajectory, prefix) is then a partial sum of |psi|^2 over the later qubits
// (Sec. II-B), and the proportional sampling loop (Sec. III-B) runs unchanged on
// those marginals: FP64 prefix sums, inverse-CDF draws, prefix deduplication.
// Trajectories are processed in chunks whose states fit the workspace; shot rows,
// Philox counters and weights use global trajectory ids, so results do not
// depend on the chunking.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

namespace ptsbe {

namespace {

constexpr int64_t kSvElemCap = 16384;     // elements per marginal launch (contract_batch)

// Slices of the later-qubit range per element: enough (element, slice) tasks to
// fill the chip.  The partial-sum rows n_elems << ls are < kSplitRows whenever
// ls > 0 (ls grows only while n_elems << (ls - 1) < kSplitRows / 2).
constexpr int64_t kSplitRows = 4096;
int pick_log_split(int64_t n_elems, int ybits) {
  int ls = 0;
  while (ls < ybits && (n_elems << ls) < kSplitRows / 2) ++ls;
  return ls;
}

int max_batch_bits(const Plan& p) {
  int b = 1;
  for (int x : p.batch_sizes) b = std::max(b, x);
  return b;
}

// per-element device bytes of the sampling loop (marginal, sampling, children)
size_t sv_elem_bytes(const Plan& p) {
  const size_t X = (size_t)1 << max_batch_bits(p);
  return X * 12 + 2 * (4 + 4 + 4 + 8 * (size_t)p.NW) + 4 + 4 + 4 + 8 + 16;
}

size_t sv_global_bytes(const Plan& p, int64_t E, int64_t M) {
  size_t b = 0;
  auto add = [&](size_t x) { b += (x + 255) & ~(size_t)255; };
  add((size_t)std::max<int64_t>(M, 1) * 4 * 3);   // shot ids (x2), shot x
  add((size_t)E * 8 * 2);                          // shot base, norms
  add(64);
  add((size_t)E * p.G * 16 * sizeof(float2));      // merged gates
  add(((size_t)kSplitRows << max_batch_bits(p)) * 8);   // split partial sums of the first batch
  return b + (1 << 20);
}

}  // namespace

// Device bytes of one trajectory's state and its gate-cluster matrices.
static size_t sv_traj_bytes(const Plan& p) { return ((size_t)8 << p.n) + p.sv_cl[2].size() * 256 * sizeof(float2) + 512; }

ptsbe_status_t collect_window_events(Plan& p) {
  for (auto& e : p.win_evs) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e.first, e.second));
    p.win_ms += ms;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  p.win_evs.clear();
  return PTSBE_OK;
}

ptsbe_status_t sv_evolve(Plan& p, const GateCtx& g, int64_t t0, int64_t nj, float2* psi, float2* Ucl,
                         hipStream_t s) {
  HIP_TRY(launch_state_init(psi, nj, p.n, s));
  const int n_cl = Ucl ? (int)p.sv_cl[2].size() : 0;
  if (n_cl > 0) HIP_TRY(launch_cluster_build(p.d_sv_cl[2], n_cl, p.d_fused, g, nj, nullptr, (int32_t)t0, Ucl, s));
  const bool compact = p.sv_wins[2].size() == p.sv_segs.size() && p.d_sv_ops[2];
  for (size_t k = 0; k < p.sv_segs.size(); ++k) {
    const Segment& sg = p.sv_segs[k];
    if (compact && sv_window_lds_bytes(p.sv_wins[2][k]) != 0 && sv_window_lds_bytes(p.sv_wins[2][k]) <= 64 * 1024) {
      std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
      if (p.profile) {
        HIP_TRY(hipEventCreate(&ev.first));
        HIP_TRY(hipEventCreate(&ev.second));
        HIP_TRY(hipEventRecord(ev.first, s));
      }
      HIP_TRY(launch_sv_window(p.sv_wins[2][k], p.d_sv_ops[2], g.merged, p.G, Ucl, n_cl, nj, (int32_t)t0, psi, p.n,
                               p.precision, s));
      if (p.profile) {
        HIP_TRY(hipEventRecord(ev.second, s));
        p.win_evs.push_back(ev);
        ++p.win_launches;
        p.win_bytes += (double)nj * 16.0 * std::ldexp(1.0, p.n);   // every state read and written once
      }
      continue;
    }
    // windows of fewer than 10 qubits (small circuits) take the generic fused pass
    HIP_TRY(launch_fused(sg, p.d_fused, g, nj, nullptr, (int32_t)t0, nullptr, p.NW, psi, s, n_cl > 0 ? Ucl : nullptr,
                         n_cl));
  }
  return PTSBE_OK;
}

// Gate-cluster matrices of nj trajectories (null when the windows have none).
static float2* take_clusters(const Plan& p, Arena& ar, int64_t nj) {
  const size_t n_cl = p.sv_cl[2].size();
  return n_cl ? (float2*)ar.take((size_t)nj * n_cl * 256 * sizeof(float2)) : nullptr;
}

size_t sv_sample_workspace(const Plan& p, int64_t E, int64_t M) {
  const size_t state = sv_traj_bytes(p);
  const int64_t avg_m = E > 0 ? (M + E - 1) / E : 0;
  const size_t per_traj = state + (size_t)(avg_m + 1) * sv_elem_bytes(p);
  const int64_t k = std::max<int64_t>(1, std::min<int64_t>(E, (int64_t)(((size_t)16 << 30) / per_traj)));
  return sv_global_bytes(p, E, M) + (size_t)k * per_traj + ((size_t)4 << 20);
}

size_t sv_contract_workspace(const Plan& p, int j, int64_t E, int64_t n_elems) {
  const size_t X = (size_t)1 << p.batches[j].size;
  const int64_t ec = std::min<int64_t>(std::max<int64_t>(n_elems, 1), kSvElemCap);
  const size_t state = sv_traj_bytes(p);
  const int64_t k = std::max<int64_t>(1, std::min<int64_t>(E, (int64_t)(((size_t)16 << 30) / state)));
  return (size_t)E * p.G * 16 * sizeof(float2) + (size_t)(E + 1) * 4 + (size_t)std::max<int64_t>(ec, kSplitRows) * X * 8 +
         (size_t)k * state + ((size_t)4 << 20);
}

ptsbe_status_t sv_sample_shots(Plan& p, const uint8_t* d_kraus, int64_t E, const int64_t* d_mult,
                               const int64_t* d_m, uint64_t seed, uint64_t* d_shots, int32_t* d_shot_traj,
                               double* d_w, double* d_norm, int64_t* stats, void* d_workspace,
                               size_t workspace_bytes, hipStream_t s) {
  std::vector<int64_t> m((size_t)E), base((size_t)E + 1);
  HIP_TRY(hipMemcpyAsync(m.data(), d_m, (size_t)E * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int64_t M = 0;
  for (int64_t i = 0; i < E; ++i) {
    if (m[i] < 0) return fail(PTSBE_ERR_INVALID_ARG, "negative shot count");
    base[i] = M;
    M += m[i];
  }
  base[E] = M;
  if (M >= ((int64_t)1 << 31)) return fail(PTSBE_ERR_UNSUPPORTED, "more than 2^31 shots");
  Arena ar;
  ar.base = (char*)d_workspace;
  ar.cap = workspace_bytes;
  const int64_t M1 = std::max<int64_t>(M, 1);
  int32_t* ids[2];
  for (int k = 0; k < 2; ++k) ids[k] = (int32_t*)ar.take((size_t)M1 * 4);
  int32_t* shot_x = (int32_t*)ar.take((size_t)M1 * 4);
  int64_t* d_base = (int64_t*)ar.take((size_t)E * 8);
  double* norms = (double*)ar.take((size_t)E * 8);
  int32_t* counters = (int32_t*)ar.take(64);
  float2* merged = (float2*)ar.take((size_t)E * p.G * 16 * sizeof(float2));
  const int bmax = max_batch_bits(p);
  const int64_t Xmax = (int64_t)1 << bmax;
  if (!ids[0] || !ids[1] || !shot_x || !d_base || !norms || !counters || !merged)
    return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for the shot arrays and merged gates");
  // chunks of trajectories: at most NJ states and CE elements (elements of a
  // batch never outnumber max(trajectories, shots) of the chunk)
  const size_t state = (size_t)8 << p.n, tb = sv_traj_bytes(p);
  const size_t per_elem = sv_elem_bytes(p);
  const size_t fixed = (size_t)kSplitRows * Xmax * 8 + ((size_t)1 << 20);   // first-batch split sums + alignment
  const size_t avail = ar.left() > fixed ? ar.left() - fixed : 0;
  int64_t max_m = 0;
  for (int64_t t = 0; t < E; ++t) max_m = std::max(max_m, m[t]);
  int64_t CE = std::min<int64_t>(std::max<int64_t>(E, M), (int64_t)(avail / 2 / per_elem));
  CE = std::max<int64_t>(CE, max_m + 1);
  const size_t elem_bytes = (size_t)CE * per_elem + scan_scratch_bytes(CE);
  if (elem_bytes + tb > avail) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for one trajectory's state");
  const int64_t NJ = std::min<int64_t>({(int64_t)((avail - elem_bytes) / tb), 65535, CE});
  std::vector<int64_t> cuts = {0};
  {
    int64_t nj = 0, mc = 0;
    for (int64_t t = 0; t < E; ++t) {
      if (nj + 1 > NJ || mc + m[t] > CE) {
        cuts.push_back(t);
        nj = 0;
        mc = 0;
      }
      ++nj;
      mc += m[t];
    }
    cuts.push_back(E);
  }
  const int64_t cap = CE;
  struct Elems { int32_t* traj; uint64_t* prefix; int32_t* off; int32_t* cnt; } el[2];
  for (int k = 0; k < 2; ++k) {
    el[k].traj = (int32_t*)ar.take((size_t)cap * 4);
    el[k].prefix = (uint64_t*)ar.take((size_t)cap * 8 * p.NW);
    el[k].off = (int32_t*)ar.take((size_t)cap * 4);
    el[k].cnt = (int32_t*)ar.take((size_t)cap * 4);
  }
  int32_t* child_cnt = (int32_t*)ar.take((size_t)cap * 4);
  int32_t* child_off = (int32_t*)ar.take((size_t)cap * 4);
  double* totals = (double*)ar.take((size_t)cap * 8);
  int32_t* scan_scratch = (int32_t*)ar.take(scan_scratch_bytes(cap));
  int32_t* parents = (int32_t*)ar.take((size_t)cap * 4);
  float* pop = (float*)ar.take((size_t)cap * Xmax * 4);
  const int64_t part_rows = std::max<int64_t>(cap, kSplitRows);
  double* part = (double*)ar.take((size_t)part_rows * Xmax * 8);
  bool ok = child_cnt && child_off && totals && scan_scratch && parents && pop && part;
  for (int k = 0; k < 2; ++k) ok = ok && el[k].traj && el[k].prefix && el[k].off && el[k].cnt;
  if (!ok) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for the element arrays");
  const size_t mark = ar.used;
  HIP_TRY(hipMemcpyAsync(d_base, base.data(), (size_t)E * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(counters, 0, 64, s));
  // shot rows: ids = identity, shots zeroed, row -> trajectory (no elements are made here)
  HIP_TRY(launch_init_shots(M, E, d_base, ids[0], d_shot_traj, d_shots, p.NW, s));
  // error injection: UPV merge of every trajectory's operators into its gates
  GateCtx g{};
  g.gates = p.d_gates;
  g.gate_site_list = p.d_gate_site_list;
  g.site_ops = p.d_site_ops;
  g.kraus = d_kraus;
  g.S = p.S;
  g.max_kraus = p.max_kraus;
  g.G = p.G;
  HIP_TRY(launch_upv_merge(g, E, merged, s));
  g.merged = merged;
  const int f = (int)p.batches.size();
  if (stats)
    for (int j = 0; j < f; ++j) stats[j] = 0;
  for (size_t c = 0; c + 1 < cuts.size(); ++c) {
    const int64_t t0 = cuts[c], t1 = cuts[c + 1], nj = t1 - t0;
    ar.used = mark;
    float2* psi = (float2*)ar.take((size_t)nj * state);
    float2* Ucl = take_clusters(p, ar, nj);
    if (!psi || (!Ucl && !p.sv_cl[2].empty()))
      return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for the chunk's states");
    HIP_TRY(launch_init_traj_range(t0, nj, d_m, d_base, el[0].traj, el[0].prefix, p.NW, el[0].off, el[0].cnt, s));
    ptsbe_status_t st = sv_evolve(p, g, t0, nj, psi, Ucl, s);
    if (st != PTSBE_OK) return st;
    int cur = 0;
    int64_t U = nj;
    for (int j = 0; j < f && U > 0; ++j) {
      const BatchPlan& bp = p.batches[j];
      if (stats) stats[j] += U;
      SvMargArgs ma{};
      ma.psi = psi; ma.n = p.n; ma.start = bp.start; ma.b = bp.size; ma.NW = p.NW;
      ma.n_elems = U; ma.elem_traj = el[cur].traj; ma.traj_base = (int32_t)t0; ma.elem_prefix = el[cur].prefix;
      ma.log_split = pick_log_split(U, p.n - bp.start - bp.size);
      ma.part = part; ma.part_rows = part_rows; ma.pop = pop;
      HIP_TRY(launch_sv_marginal(ma, s));
      SampleArgs sa{};
      sa.pop = pop; sa.b = bp.size; sa.start = bp.start; sa.NW = p.NW;
      sa.n_elems = U; sa.elem_traj = el[cur].traj;
      sa.elem_shot_off = el[cur].off; sa.elem_shot_cnt = el[cur].cnt;
      sa.shot_ids = ids[cur]; sa.traj_shot_base = d_base;
      sa.seed = seed; sa.j = j;
      sa.shots = d_shots; sa.shot_x = shot_x;
      sa.elem_total = totals;
      sa.child_cnt = (j + 1 < f) ? child_cnt : nullptr;
      sa.bad_flag = counters + 1;
      HIP_TRY(launch_sample(sa, s));
      if (j == 0)   // first-batch elements are the chunk's trajectories: totals = squared norms
        HIP_TRY(hipMemcpyAsync(norms + t0, totals, (size_t)nj * 8, hipMemcpyDeviceToDevice, s));
      if (j + 1 < f) {
        HIP_TRY(launch_scan_i32(child_cnt, child_off, U, counters, scan_scratch, s));
        int32_t nU = 0;
        HIP_TRY(hipMemcpyAsync(&nU, counters, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        ChildArgs ca{};
        ca.n_elems = U; ca.b = bp.size; ca.start = bp.start; ca.NW = p.NW;
        ca.elem_traj = el[cur].traj; ca.elem_prefix = el[cur].prefix;
        ca.elem_shot_off = el[cur].off; ca.elem_shot_cnt = el[cur].cnt;
        ca.shot_ids = ids[cur]; ca.shot_x = shot_x; ca.child_off = child_off;
        ca.out_traj = el[1 - cur].traj; ca.out_prefix = el[1 - cur].prefix;
        ca.out_shot_off = el[1 - cur].off; ca.out_shot_cnt = el[1 - cur].cnt; ca.out_shot_ids = ids[1 - cur];
        ca.out_parent = parents;   // not needed by this method (no left tensors to resume from)
        HIP_TRY(launch_children(ca, s));
        cur = 1 - cur;
        U = nU;
      }
    }
  }
  if (d_w || d_norm) {
    WeightArgs wa{norms, d_mult, E, d_w, d_norm};
    HIP_TRY(launch_weights(wa, s));
  }
  int32_t bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, counters + 1, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (p.profile) {
    const ptsbe_status_t st = collect_window_events(p);
    if (st != PTSBE_OK) return st;
  }
  if (bad) return fail(PTSBE_ERR_NUMERIC, "an element had a non-finite marginal total");
  return PTSBE_OK;
}

ptsbe_status_t sv_contract_batch(Plan& p, int j, const uint8_t* d_kraus, int64_t E, const int32_t* d_elem_traj,
                                 const uint64_t* d_elem_prefix, int64_t n_elems, int32_t out_kind, void* d_out,
                                 double* d_elem_total, void* d_workspace, size_t workspace_bytes, hipStream_t s) {
  const BatchPlan& bp = p.batches[j];
  if (out_kind == PTSBE_OUT_AMPLITUDE && bp.start + bp.size != p.n)
    return fail(PTSBE_ERR_INVALID_ARG, "amplitudes exist only for the last batch");
  Arena ar;
  ar.base = (char*)d_workspace;
  ar.cap = workspace_bytes;
  float2* merged = (float2*)ar.take((size_t)E * p.G * 16 * sizeof(float2));
  int32_t* d_first = (int32_t*)ar.take((size_t)(E + 1) * 4);
  const int64_t X = (int64_t)1 << bp.size;
  const int64_t ec = std::min<int64_t>(n_elems, kSvElemCap);
  const int64_t part_rows = std::max<int64_t>(ec, kSplitRows);
  double* part = (double*)ar.take((size_t)part_rows * X * 8);
  if (!merged || !d_first || !part) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small (merged gates, ranges)");
  GateCtx g{};
  g.gates = p.d_gates;
  g.gate_site_list = p.d_gate_site_list;
  g.site_ops = p.d_site_ops;
  g.kraus = d_kraus;
  g.S = p.S;
  g.max_kraus = p.max_kraus;
  g.G = p.G;
  HIP_TRY(launch_upv_merge(g, E, merged, s));
  g.merged = merged;
  HIP_TRY(launch_traj_ranges(d_elem_traj, n_elems, E, d_first, s));
  std::vector<int32_t> first((size_t)E + 1);
  HIP_TRY(hipMemcpyAsync(first.data(), d_first, (size_t)(E + 1) * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const size_t state = (size_t)8 << p.n;
  const int64_t nj_cap = std::min<int64_t>((int64_t)(ar.left() / sv_traj_bytes(p)), 65535);
  if (nj_cap < 1) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for one trajectory's state");
  float2* psi = (float2*)ar.take((size_t)nj_cap * state);
  float2* Ucl = take_clusters(p, ar, nj_cap);
  if (!psi || (!Ucl && !p.sv_cl[2].empty()))
    return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for one trajectory's state");
  int64_t t0 = 0;
  while (t0 < E) {
    while (t0 < E && first[t0 + 1] == first[t0]) ++t0;   // skip trajectories without elements
    if (t0 >= E) break;
    const int64_t t1 = std::min<int64_t>(E, t0 + nj_cap);
    const int64_t e0 = first[t0], e1 = first[t1];
    ptsbe_status_t st = sv_evolve(p, g, t0, t1 - t0, psi, Ucl, s);
    if (st != PTSBE_OK) return st;
    for (int64_t a0 = e0; a0 < e1; a0 += kSvElemCap) {
      const int64_t ne = std::min<int64_t>(kSvElemCap, e1 - a0);
      SvMargArgs ma{};
      ma.psi = psi; ma.n = p.n; ma.start = bp.start; ma.b = bp.size; ma.NW = p.NW;
      ma.n_elems = ne; ma.elem_traj = d_elem_traj + a0; ma.traj_base = (int32_t)t0;
      ma.elem_prefix = d_elem_prefix + a0 * p.NW;
      if (out_kind == PTSBE_OUT_AMPLITUDE) {
        HIP_TRY(launch_sv_amplitudes(ma, (float2*)d_out + a0 * X, s));
      } else {
        ma.log_split = pick_log_split(ne, p.n - bp.start - bp.size);
        ma.part = part;
        ma.part_rows = part_rows;
        ma.pop = (float*)d_out + a0 * X;
        HIP_TRY(launch_sv_marginal(ma, s));
        if (d_elem_total) HIP_TRY(launch_row_totals(ma.pop, ne, bp.size, d_elem_total + a0, s));
      }
    }
    t0 = t1;
  }
  HIP_TRY(hipStreamSynchronize(s));
  return p.profile ? collect_window_events(p) : PTSBE_OK;
}


// ------------------------------------------------ non-proportional NBS (Sec. III-B)
// The statevector form of the non-proportional mode: the same draws, element
// order, Philox counters and final-batch rows as the network method, with every
// marginal taken from the trajectory's state.  Trajectories run in chunks whose
// states fit the workspace; a trajectory's elements stay in its chunk, so draw
// rows (and their counters) are chunk-local and results do not depend on chunking.
namespace {
struct SvNpLayout {
  float2* merged; double* norms; int64_t* base; int32_t* counters; double* part;
  int32_t* traj[2]; uint64_t* prefix[2]; int32_t* off[2]; int32_t* cnt[2]; int32_t* ids[2];
  int32_t *shot_x, *child_cnt, *child_off, *parents, *scan_scratch, *tile_cnt, *tile_off, *exh_scan, *exh_total;
  double* totals; float* pop;
};

bool take_sv_np(const Plan& p, int64_t E, int64_t cap, int32_t R, Arena& ar, SvNpLayout& L) {
  const size_t Xmax = (size_t)1 << max_batch_bits(p);
  const size_t rows = (size_t)cap * (size_t)R;
  bool ok = true;
  auto take = [&](size_t bytes) {   // every array is taken, so a probe arena measures the whole layout
    void* q = ar.take(bytes);
    ok = ok && q != nullptr;
    return q;
  };
  L.merged = (float2*)take((size_t)E * p.G * 16 * sizeof(float2));
  L.norms = (double*)take((size_t)E * 8);
  L.base = (int64_t*)take((size_t)E * 8);
  L.counters = (int32_t*)take(64);
  L.part = (double*)take((size_t)std::max<int64_t>(cap, kSplitRows) * Xmax * 8);
  for (int k = 0; k < 2; ++k) {
    L.traj[k] = (int32_t*)take((size_t)cap * 4);
    L.prefix[k] = (uint64_t*)take((size_t)cap * 8 * p.NW);
    L.off[k] = (int32_t*)take((size_t)cap * 4);
    L.cnt[k] = (int32_t*)take((size_t)cap * 4);
    L.ids[k] = (int32_t*)take(rows * 4);
  }
  L.shot_x = (int32_t*)take(rows * 4);
  L.child_cnt = (int32_t*)take((size_t)cap * 4);
  L.child_off = (int32_t*)take((size_t)cap * 4);
  L.parents = (int32_t*)take((size_t)cap * 4);
  L.scan_scratch = (int32_t*)take(scan_scratch_bytes(cap));
  L.tile_cnt = (int32_t*)take((size_t)cap * 4);
  L.tile_off = (int32_t*)take((size_t)cap * 4);
  L.exh_scan = (int32_t*)take(scan_scratch_bytes(cap));
  L.exh_total = (int32_t*)take(64);
  L.totals = (double*)take((size_t)cap * 8);
  L.pop = (float*)take((size_t)cap * Xmax * 4);
  return ok;
}
}  // namespace

size_t sv_np_workspace(const Plan& p, int64_t E, int64_t cap, int32_t rows_per_elem) {
  Arena probe;                       // an arena without memory measures the layout
  probe.base = nullptr;
  probe.cap = ~(size_t)0 >> 1;
  SvNpLayout L;
  take_sv_np(p, E, cap, rows_per_elem, probe, L);
  const size_t state = sv_traj_bytes(p);
  const int64_t k = std::max<int64_t>(1, std::min<int64_t>(E, (int64_t)(((size_t)16 << 30) / state)));
  return probe.used + (size_t)k * state + ((size_t)4 << 20);
}

ptsbe_status_t sv_sample_nonproportional(Plan& p, const uint8_t* d_kraus, int64_t E, const int64_t* d_mult,
                                         int32_t draws, int32_t final_draws, int64_t cap, uint64_t seed,
                                         double threshold, uint64_t* d_bits, int32_t* d_row_traj, double* d_p_cond,
                                         double* d_p_prefix, int64_t capacity, int64_t* n_rows_out, double* d_w,
                                         double* d_norm, int64_t* stats, void* d_workspace, size_t workspace_bytes,
                                         hipStream_t s) {
  const int32_t R = std::max(draws, final_draws);
  Arena ar;
  ar.base = (char*)d_workspace;
  ar.cap = workspace_bytes;
  SvNpLayout L;
  if (!take_sv_np(p, E, cap, R, ar, L))
    return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for the element arrays");
  const size_t state = sv_traj_bytes(p);
  const int64_t NJ = std::min<int64_t>({(int64_t)(ar.left() / (state + 256)), 65535, E});
  if (NJ < 1) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for one trajectory's state");
  const int64_t part_rows = std::max<int64_t>(cap, kSplitRows);
  HIP_TRY(hipMemsetAsync(L.counters, 0, 64, s));
  GateCtx g{};
  g.gates = p.d_gates;
  g.gate_site_list = p.d_gate_site_list;
  g.site_ops = p.d_site_ops;
  g.kraus = d_kraus;
  g.S = p.S;
  g.max_kraus = p.max_kraus;
  g.G = p.G;
  HIP_TRY(launch_upv_merge(g, E, L.merged, s));
  g.merged = L.merged;
  const int f = (int)p.batches.size();
  if (stats)
    for (int j = 0; j < f; ++j) stats[j] = 0;
  int64_t rows = 0;             // rows found so far
  bool room = true;             // direct mode: every chunk so far fitted the capacity
  const size_t mark = ar.used;
  for (int64_t t0 = 0; t0 < E; t0 += NJ) {
    const int64_t nj = std::min<int64_t>(NJ, E - t0);
    ar.used = mark;
    float2* psi = (float2*)ar.take((size_t)nj * state);
    float2* Ucl = take_clusters(p, ar, nj);
    if (!psi || (!Ucl && !p.sv_cl[2].empty()))
      return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for the chunk's states");
    HIP_TRY(launch_np_init(nj, t0, L.traj[0], L.prefix[0], p.NW, s));
    ptsbe_status_t st = sv_evolve(p, g, t0, nj, psi, Ucl, s);
    if (st != PTSBE_OK) return st;
    int cur = 0;
    int64_t U = nj;
    for (int j = 0; j < f; ++j) {
      const BatchPlan& bp = p.batches[j];
      const bool last = j + 1 == f;
      if (stats) stats[j] += U;
      SvMargArgs ma{};
      ma.psi = psi; ma.n = p.n; ma.start = bp.start; ma.b = bp.size; ma.NW = p.NW;
      ma.n_elems = U; ma.elem_traj = L.traj[cur]; ma.traj_base = (int32_t)t0; ma.elem_prefix = L.prefix[cur];
      ma.log_split = pick_log_split(U, p.n - bp.start - bp.size);
      ma.part = L.part; ma.part_rows = part_rows; ma.pop = L.pop;
      HIP_TRY(launch_sv_marginal(ma, s));
      if (last && final_draws == 0) {   // exhaustive final batch
        HIP_TRY(launch_row_totals(L.pop, U, bp.size, L.totals, s));
        if (j == 0) HIP_TRY(hipMemcpyAsync(L.norms + t0, L.totals, (size_t)nj * 8, hipMemcpyDeviceToDevice, s));
        // element ranges whose rows stay below 2^31 (the row scan is int32)
        const int64_t X = (int64_t)1 << bp.size;
        const int64_t sub = std::max<int64_t>(1, (((int64_t)1 << 31) - 1) / X);
        for (int64_t a0 = 0; a0 < U; a0 += sub) {
          const int64_t ne = std::min<int64_t>(sub, U - a0);
          ExhArgs a{};
          a.pop = L.pop + a0 * X; a.b = bp.size; a.start = bp.start; a.NW = p.NW;
          a.n_elems = ne; a.elem_traj = L.traj[cur] + a0; a.elem_prefix = L.prefix[cur] + a0 * p.NW;
          a.elem_total = L.totals + a0; a.traj_norm = f > 1 ? L.norms : nullptr;
          a.threshold = threshold;
          a.tile_cnt = L.tile_cnt; a.tile_off = L.tile_off; a.tile_bits = 0;   // b <= 12: one tile per element
          a.row_base = rows; a.capacity = capacity;
          a.bits = d_bits; a.row_traj = d_row_traj; a.p_cond = d_p_cond; a.p_prefix = d_p_prefix;
          HIP_TRY(launch_exh_count(a, s));
          HIP_TRY(launch_scan_i32(L.tile_cnt, L.tile_off, ne, L.exh_total, L.exh_scan, s));
          int32_t found = 0;
          HIP_TRY(hipMemcpyAsync(&found, L.exh_total, 4, hipMemcpyDeviceToHost, s));
          HIP_TRY(hipStreamSynchronize(s));
          if (found > 0 && rows < capacity) HIP_TRY(launch_exh_write(a, s));
          rows += found;
        }
        break;
      }
      const int32_t Rj = last ? final_draws : draws;
      HIP_TRY(launch_np_rows(U, Rj, L.traj[cur], L.off[cur], L.cnt[cur], L.ids[cur], L.base, s));
      const bool write = last && room && rows + U * Rj <= capacity;
      if (last && !write) room = false;
      if (write)
        HIP_TRY(launch_np_direct_rows(U, Rj, L.traj[cur], L.prefix[cur], p.NW, d_bits + rows * p.NW,
                                      d_row_traj ? d_row_traj + rows : nullptr, s));
      SampleArgs sa{};
      sa.pop = L.pop; sa.b = bp.size; sa.start = bp.start; sa.NW = p.NW;
      sa.n_elems = U; sa.elem_traj = L.traj[cur];
      sa.elem_shot_off = L.off[cur]; sa.elem_shot_cnt = L.cnt[cur];
      sa.shot_ids = L.ids[cur]; sa.traj_shot_base = L.base;
      sa.seed = seed; sa.j = j; sa.tag = 3u;
      sa.shots = write ? d_bits + rows * p.NW : nullptr;
      sa.p_cond = write && d_p_cond ? d_p_cond + rows : nullptr;
      sa.shot_x = L.shot_x;
      sa.elem_total = L.totals;
      sa.child_cnt = last ? nullptr : L.child_cnt;
      sa.bad_flag = L.counters + 1;
      HIP_TRY(launch_sample(sa, s));
      if (j == 0) HIP_TRY(hipMemcpyAsync(L.norms + t0, L.totals, (size_t)nj * 8, hipMemcpyDeviceToDevice, s));
      if (last) {
        if (write)
          HIP_TRY(launch_np_direct_prefix_p(U, Rj, L.traj[cur], L.totals, f > 1 ? L.norms : nullptr,
                                            d_p_prefix ? d_p_prefix + rows : nullptr, s));
        rows += U * Rj;
        break;
      }
      HIP_TRY(launch_scan_i32(L.child_cnt, L.child_off, U, L.counters, L.scan_scratch, s));
      int32_t nU = 0;
      HIP_TRY(hipMemcpyAsync(&nU, L.counters, 4, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (nU > cap)
        return fail(PTSBE_ERR_OUT_OF_MEMORY, "batch " + std::to_string(j + 1) + " has more elements than max_elems");
      ChildArgs ca{};
      ca.n_elems = U; ca.b = bp.size; ca.start = bp.start; ca.NW = p.NW;
      ca.elem_traj = L.traj[cur]; ca.elem_prefix = L.prefix[cur];
      ca.elem_shot_off = L.off[cur]; ca.elem_shot_cnt = L.cnt[cur];
      ca.shot_ids = L.ids[cur]; ca.shot_x = L.shot_x; ca.child_off = L.child_off;
      ca.out_traj = L.traj[1 - cur]; ca.out_prefix = L.prefix[1 - cur];
      ca.out_shot_off = L.off[1 - cur]; ca.out_shot_cnt = L.cnt[1 - cur]; ca.out_shot_ids = L.ids[1 - cur];
      ca.out_parent = L.parents;   // not needed by this method (no left tensors to resume from)
      HIP_TRY(launch_children(ca, s));
      cur = 1 - cur;
      U = nU;
    }
  }
  if (d_w || d_norm) {
    WeightArgs wa{L.norms, d_mult, E, d_w, d_norm};
    HIP_TRY(launch_weights(wa, s));
  }
  int32_t bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, L.counters + 1, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (p.profile) {
    const ptsbe_status_t st = collect_window_events(p);
    if (st != PTSBE_OK) return st;
  }
  *n_rows_out = rows;
  if (bad) return fail(PTSBE_ERR_NUMERIC, "an element had a non-finite marginal total");
  if (rows > capacity)
    return fail(PTSBE_ERR_OUT_OF_MEMORY, std::to_string(rows) + " rows found, capacity " + std::to_string(capacity));
  return PTSBE_OK;
}

}  // namespace ptsbe
