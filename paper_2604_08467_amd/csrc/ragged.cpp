// Ragged sets: the trajectories of several statevector-method plans (different
// circuits, qubit counts and batch layouts) sampled in shared launches.  The
// host cuts the jobs' trajectories into waves that fit the workspace, writes
// each wave's tables (pieces, trajectory -> piece, shot-row bases, window-level
// task queues), and issues one fixed launch sequence per wave; with
// PTSBE_RAGGED_GRAPH the sequence is captured once as a hipGraph and replayed.
// The autotuner times the gate-window pass of each plan for three tile sizes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"

using ptsbe::Arena;
using ptsbe::fail;
using ptsbe::Plan;

struct ptsbe_ragged_s {
  int device = 0;
  int n_cu = 256;
  double khz = 0.0;
  std::unordered_map<const Plan*, int> choice;   // window size index per plan
  std::vector<hipGraphExec_t> execs;
  std::vector<int64_t> key;
  int last_waves = 0, last_replayed = 0;
  int64_t last_launches = 0;
  void drop_graphs() {
    for (auto e : execs) (void)hipGraphExecDestroy(e);
    execs.clear();
    key.clear();
  }
};

namespace {

using ptsbe::RgLevel;
using ptsbe::RgPiece;
using ptsbe::RgWave;

int plan_xbits(const Plan& p) {
  int b = 1;
  for (int x : p.batch_sizes) b = std::max(b, x);
  return b;
}

ptsbe_status_t check_jobs(const ptsbe_ragged_s& set, const ptsbe_ragged_job_t* jobs, int32_t n_jobs) {
  if (!jobs || n_jobs < 1) return fail(PTSBE_ERR_INVALID_ARG, "no jobs");
  for (int c = 0; c < n_jobs; ++c) {
    const Plan* p = reinterpret_cast<const Plan*>(jobs[c].plan);
    const std::string id = "job " + std::to_string(c) + ": ";
    if (!p) return fail(PTSBE_ERR_INVALID_ARG, id + "null plan");
    if (p->method != PTSBE_METHOD_STATEVECTOR) return fail(PTSBE_ERR_UNSUPPORTED, id + "ragged sets take statevector-method plans");
    if (p->device != set.device) return fail(PTSBE_ERR_INVALID_ARG, id + "plan is on another device");
    if (p->batch_sizes.size() > (size_t)ptsbe::kRgMaxBatches) return fail(PTSBE_ERR_UNSUPPORTED, id + "too many batches");
    if (jobs[c].E < 1) return fail(PTSBE_ERR_INVALID_ARG, id + "E < 1");
    if (jobs[c].E >= ((int64_t)1 << 31)) return fail(PTSBE_ERR_UNSUPPORTED, id + "E >= 2^31");
    if (!jobs[c].d_kraus_idx || !jobs[c].shots_per_traj || !jobs[c].d_shots)
      return fail(PTSBE_ERR_INVALID_ARG, id + "null pointer");
    for (int64_t i = 0; i < jobs[c].E; ++i)
      if (jobs[c].shots_per_traj[i] < 0) return fail(PTSBE_ERR_INVALID_ARG, id + "negative shot count");
  }
  return PTSBE_OK;
}

int window_choice(const ptsbe_ragged_s& set, const Plan* p) {
  auto it = set.choice.find(p);
  return it == set.choice.end() ? 2 : it->second;
}

// one job's trajectories [t0, t0 + nj) in a wave
struct PieceSpec { int job; int64_t t0, nj; };

struct WavePlan {
  std::vector<PieceSpec> pieces;
  int64_t T = 0, R = 0;
};

// per-trajectory bytes of a wave (state, merged gates, first-batch partial sums,
// elements at every level, shot rows)
size_t traj_bytes(const Plan& p, int xbits, int64_t m) {
  const size_t X = (size_t)1 << xbits;
  const size_t elem = X * 4 + 2 * (4 + 8 + 4 + 4) + 4 + 4 + 4;
  return ((size_t)8 << p.n) + (size_t)p.G * 128 + 16 * X * 8 + (size_t)(m + 1) * elem + (size_t)m * 12 + 16 + 512;
}

size_t wave_fixed_bytes() { return (size_t)64 << 10; }

}  // namespace

extern "C" {

ptsbe_status_t ptsbe_ragged_create(int32_t device, ptsbe_ragged_t* out) {
  if (!out) return fail(PTSBE_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  auto* s = new ptsbe_ragged_s();
  s->device = device;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&s->n_cu, hipDeviceAttributeMultiprocessorCount, device);
  int khz = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device);
  if (e != hipSuccess) {
    delete s;
    return fail(PTSBE_ERR_DEVICE, std::string("HIP: ") + hipGetErrorString(e));
  }
  s->khz = khz;
  *out = s;
  return PTSBE_OK;
}

void ptsbe_ragged_destroy(ptsbe_ragged_t set) {
  if (!set) return;
  set->drop_graphs();
  delete set;
}

ptsbe_status_t ptsbe_ragged_info(ptsbe_ragged_t set, ptsbe_ragged_info_t* out) {
  if (!set || !out) return fail(PTSBE_ERR_INVALID_ARG, "null argument");
  out->n_waves = set->last_waves;
  out->graphs_replayed = set->last_replayed;
  out->launches = set->last_launches;
  out->wall_clock_khz = set->khz;
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_ragged_workspace_size(ptsbe_ragged_t set, const ptsbe_ragged_job_t* jobs, int32_t n_jobs,
                                           size_t* bytes) {
  if (!set || !bytes) return fail(PTSBE_ERR_INVALID_ARG, "null argument");
  ptsbe_status_t st = check_jobs(*set, jobs, n_jobs);
  if (st != PTSBE_OK) return st;
  int xbits = 1;
  size_t persistent = 0, biggest = 0, total = 0;
  for (int c = 0; c < n_jobs; ++c) xbits = std::max(xbits, plan_xbits(*reinterpret_cast<const Plan*>(jobs[c].plan)));
  for (int c = 0; c < n_jobs; ++c) {
    const Plan& p = *reinterpret_cast<const Plan*>(jobs[c].plan);
    persistent += (size_t)jobs[c].E * 8 + 256;
    for (int64_t i = 0; i < jobs[c].E; ++i) {
      const size_t b = traj_bytes(p, xbits, jobs[c].shots_per_traj[i]);
      biggest = std::max(biggest, b);
      total += b;
    }
  }
  // everything in one wave if it is under 32 GB, else waves of 32 GB
  const size_t wave = std::max(biggest, std::min(total, (size_t)32 << 30));
  *bytes = persistent + wave + (size_t)n_jobs * 4096 + ((size_t)64 << 20);
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_ragged_autotune(ptsbe_ragged_t set, const ptsbe_ragged_job_t* jobs, int32_t n_jobs,
                                     int32_t* best_window, float* ms_per_traj, void* d_workspace,
                                     size_t workspace_bytes, void* stream) {
  if (!set) return fail(PTSBE_ERR_INVALID_ARG, "null set");
  ptsbe_status_t st = check_jobs(*set, jobs, n_jobs);
  if (st != PTSBE_OK) return st;
  HIP_TRY(hipSetDevice(set->device));
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t ev[4];
  for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  std::unordered_map<const Plan*, std::array<float, 3>> seen;
  for (int c = 0; c < n_jobs; ++c) {
    Plan& p = *reinterpret_cast<Plan*>(jobs[c].plan);
    std::array<float, 3> ms{};
    auto it = seen.find(&p);
    if (it != seen.end()) {
      ms = it->second;
    } else {
      const int64_t nt = std::min<int64_t>(jobs[c].E, 2);
      Arena ar;
      ar.base = (char*)d_workspace;
      ar.cap = workspace_bytes;
      float2* merged = (float2*)ar.take((size_t)nt * p.G * 128);
      float2* psi = (float2*)ar.take((size_t)nt * ((size_t)8 << p.n));
      if (!merged || !psi) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for the autotuner");
      ptsbe::GateCtx g{};
      g.gates = p.d_gates;
      g.gate_site_list = p.d_gate_site_list;
      g.site_ops = p.d_site_ops;
      g.kraus = jobs[c].d_kraus_idx;
      g.S = p.S;
      g.max_kraus = p.max_kraus;
      g.G = p.G;
      HIP_TRY(ptsbe::launch_upv_merge(g, nt, merged, s));
      g.merged = merged;
      for (int w = 0; w < 3; ++w) {
        for (int rep = 0; rep < 2; ++rep) {   // the first pass warms up
          HIP_TRY(hipEventRecord(ev[0], s));
          HIP_TRY(ptsbe::launch_state_init(psi, nt, p.n, s));
          // the pass the set runs: compact plain ops for 10..12-qubit windows, else the generic one
          const bool compact = p.d_sv_ops_plain[w] && p.sv_wins_plain[w].size() == p.sv_win[w].size();
          for (size_t k = 0; k < p.sv_win[w].size(); ++k) {
            if (compact && p.sv_wins_plain[w][k].np >= 10 && p.sv_wins_plain[w][k].n_ops <= 224)
              HIP_TRY(ptsbe::launch_sv_window(p.sv_wins_plain[w][k], p.d_sv_ops_plain[w], merged, p.G, nullptr, 0,
                                              nt, 0, psi, p.n, PTSBE_C64, s));
            else
              HIP_TRY(ptsbe::launch_fused(p.sv_win[w][k], p.d_fused, g, nt, nullptr, 0, nullptr, p.NW, psi, s));
          }
          HIP_TRY(hipEventRecord(ev[1], s));
        }
        HIP_TRY(hipEventSynchronize(ev[1]));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, ev[0], ev[1]));
        ms[w] = t / (float)nt;
      }
      seen[&p] = ms;
    }
    const int best = (int)(std::min_element(ms.begin(), ms.end()) - ms.begin());
    set->choice[&p] = best;
    if (best_window) best_window[c] = ptsbe::kSvWindowMin + best;
    if (ms_per_traj)
      for (int w = 0; w < 3; ++w) ms_per_traj[3 * c + w] = ms[w];
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  set->drop_graphs();   // window choices are baked into captured graphs
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_ragged_sample_shots(ptsbe_ragged_t set, const ptsbe_ragged_job_t* jobs, int32_t n_jobs,
                                         int32_t flags, uint64_t* d_done_ticks, void* d_workspace,
                                         size_t workspace_bytes, void* stream) {
  if (!set) return fail(PTSBE_ERR_INVALID_ARG, "null set");
  ptsbe_status_t st = check_jobs(*set, jobs, n_jobs);
  if (st != PTSBE_OK) return st;
  if (!d_workspace) return fail(PTSBE_ERR_INVALID_ARG, "null workspace");
  const bool use_graph = (flags & PTSBE_RAGGED_GRAPH) != 0;
  if (use_graph && stream == nullptr) return fail(PTSBE_ERR_INVALID_ARG, "graph capture needs a non-null stream");
  HIP_TRY(hipSetDevice(set->device));
  hipStream_t s = (hipStream_t)stream;
  int xbits = 1;
  for (int c = 0; c < n_jobs; ++c) xbits = std::max(xbits, plan_xbits(*reinterpret_cast<const Plan*>(jobs[c].plan)));
  // shot layout of every job
  std::vector<std::vector<int64_t>> base(n_jobs);
  for (int c = 0; c < n_jobs; ++c) {
    base[c].resize((size_t)jobs[c].E + 1);
    int64_t M = 0;
    for (int64_t i = 0; i < jobs[c].E; ++i) {
      base[c][i] = M;
      M += jobs[c].shots_per_traj[i];
    }
    base[c][jobs[c].E] = M;
  }
  Arena ar;
  ar.base = (char*)d_workspace;
  ar.cap = workspace_bytes;
  std::vector<double*> norms(n_jobs);
  for (int c = 0; c < n_jobs; ++c) {
    norms[c] = (double*)ar.take((size_t)jobs[c].E * 8);
    if (!norms[c]) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for the trajectory norms");
  }
  int32_t* bad_flag = (int32_t*)ar.take(256);
  if (!bad_flag) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small");
  // waves: jobs lightest first (per-trajectory cost 2^n x windows), trajectories in
  // order, so that light circuits complete in the first waves; inside a wave the
  // heaviest pieces come first in the task queues (no long task at the tail)
  std::vector<int> order(n_jobs);
  std::iota(order.begin(), order.end(), 0);
  auto cost = [&](int c) {
    const Plan& p = *reinterpret_cast<const Plan*>(jobs[c].plan);
    return (double)((int64_t)1 << p.n) * (double)p.sv_win[window_choice(*set, &p)].size();
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) < cost(b); });
  // tables take at most this much; the rest is the wave arena
  int64_t total_T = 0;
  for (int c = 0; c < n_jobs; ++c) total_T += jobs[c].E;
  const size_t table_bytes = std::max<size_t>((size_t)16 << 20, (size_t)total_T * 32 + (size_t)n_jobs * (16 << 10));
  char* tables = (char*)ar.take(table_bytes);
  const size_t arena_bytes = ar.left();
  if (!tables || arena_bytes < ((size_t)1 << 20)) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for the wave tables");
  char* arena = (char*)ar.take(arena_bytes - 4096);
  const size_t budget = arena_bytes - 4096 - wave_fixed_bytes();
  std::vector<WavePlan> waves;
  {
    WavePlan cur;
    size_t used = 0;
    for (int c : order) {
      const Plan& p = *reinterpret_cast<const Plan*>(jobs[c].plan);
      for (int64_t i = 0; i < jobs[c].E; ++i) {
        const size_t b = traj_bytes(p, xbits, jobs[c].shots_per_traj[i]);
        if (b > budget) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for one trajectory of job " + std::to_string(c));
        if (used + b > budget && cur.T > 0) {
          waves.push_back(cur);
          cur = WavePlan();
          used = 0;
        }
        if (cur.pieces.empty() || cur.pieces.back().job != c) cur.pieces.push_back({c, i, 0});
        cur.pieces.back().nj++;
        cur.T++;
        cur.R += jobs[c].shots_per_traj[i];
        used += b;
      }
    }
    if (cur.T > 0) waves.push_back(cur);
    for (auto& wv : waves) std::reverse(wv.pieces.begin(), wv.pieces.end());
  }
  // tables and launch descriptors of every wave
  struct WaveLaunch {
    RgWave w;
    std::vector<RgLevel> levels;
    int64_t m0_tasks = 0;
    int maxf = 0;
  };
  std::vector<WaveLaunch> wl(waves.size());
  Arena tb;
  tb.base = tables;
  tb.cap = table_bytes;
  std::vector<int64_t> key = {n_jobs, flags, (int64_t)(intptr_t)d_workspace, (int64_t)workspace_bytes,
                              (int64_t)(intptr_t)d_done_ticks};
  for (int c = 0; c < n_jobs; ++c) {
    const ptsbe_ragged_job_t& jb = jobs[c];
    for (int64_t v : {(int64_t)(intptr_t)jb.plan, (int64_t)(intptr_t)jb.d_kraus_idx, jb.E,
                      (int64_t)(intptr_t)jb.d_mult, (int64_t)jb.seed, (int64_t)(intptr_t)jb.d_shots,
                      (int64_t)window_choice(*set, reinterpret_cast<const Plan*>(jb.plan))})
      key.push_back(v);
    key.insert(key.end(), base[c].begin(), base[c].end());
  }
  for (size_t wi = 0; wi < waves.size(); ++wi) {
    const WavePlan& wp = waves[wi];
    WaveLaunch& L = wl[wi];
    RgWave& w = L.w;
    std::memset(&w, 0, sizeof(w));
    const int P = (int)wp.pieces.size();
    // first-batch slices: a fixed 16 per trajectory (fewer if the state is
    // smaller), so that the FP64 sums do not depend on how jobs fall into waves
    const int ls_target = 4;
    std::vector<RgPiece> pcs(P);
    std::vector<int32_t> traj_piece((size_t)wp.T);
    std::vector<int64_t> traj_row0((size_t)wp.T + 1), m0_start((size_t)P + 1);
    Arena wa;
    wa.base = arena;
    wa.cap = arena_bytes - 4096;
    int64_t toff = 0, row = 0, part_rows = 0, mt = 0;
    const int64_t cap = wp.T + wp.R;
    for (int k = 0; k < P; ++k) {
      const PieceSpec& ps = wp.pieces[k];
      const ptsbe_ragged_job_t& jb = jobs[ps.job];
      Plan& p = *reinterpret_cast<Plan*>(jb.plan);
      const int wc = window_choice(*set, &p);
      RgPiece& pc = pcs[k];
      std::memset(&pc, 0, sizeof(pc));
      pc.g.gates = p.d_gates;
      pc.g.gate_site_list = p.d_gate_site_list;
      pc.g.site_ops = p.d_site_ops;
      pc.g.kraus = jb.d_kraus_idx + ps.t0 * p.S;
      pc.g.S = p.S;
      pc.g.max_kraus = p.max_kraus;
      pc.g.G = p.G;
      pc.g.merged = (const float2*)wa.take((size_t)ps.nj * p.G * 128);
      pc.psi = (float2*)wa.take((size_t)ps.nj * ((size_t)8 << p.n));
      pc.win = p.d_rg_win[wc];
      pc.fused = p.d_fused;
      // compact plain ops when every window of the set has them and a 10..12-qubit tile
      bool compact = p.d_sv_wins_plain[wc] && p.sv_wins_plain[wc].size() == p.sv_win[wc].size();
      for (const auto& wd : p.sv_wins_plain[wc]) compact = compact && wd.np >= 10 && wd.n_ops <= 224;
      pc.swin = compact ? p.d_sv_wins_plain[wc] : nullptr;
      pc.sops = compact ? p.d_sv_ops_plain[wc] : nullptr;
      pc.shots = jb.d_shots;
      pc.norms = norms[ps.job];
      pc.row0 = row;
      pc.job_row0 = base[ps.job][ps.t0];
      pc.seed = jb.seed;
      pc.job = ps.job;
      pc.n = p.n;
      pc.f = (int)p.batch_sizes.size();
      pc.n_win = (int)p.sv_win[wc].size();
      pc.t0 = (int32_t)ps.t0;
      pc.nj = (int32_t)ps.nj;
      pc.traj_off = (int32_t)toff;
      pc.log_split0 = std::min(ls_target, p.n - p.batch_sizes[0]);
      pc.part_off = part_rows;
      for (int j = 0; j < pc.f; ++j) {
        pc.start[j] = p.batches[j].start;
        pc.b[j] = p.batches[j].size;
      }
      if (!pc.g.merged || !pc.psi) return fail(PTSBE_ERR_OUT_OF_MEMORY, "wave arena too small (states)");
      for (int64_t i = 0; i < ps.nj; ++i) {
        traj_piece[(size_t)(toff + i)] = k;
        traj_row0[(size_t)(toff + i)] = row;
        row += jb.shots_per_traj[ps.t0 + i];
      }
      m0_start[k] = mt;
      mt += ps.nj << pc.log_split0;
      part_rows += ps.nj << pc.log_split0;
      toff += ps.nj;
      L.maxf = std::max(L.maxf, pc.f);
    }
    traj_row0[(size_t)wp.T] = row;
    m0_start[P] = mt;
    L.m0_tasks = mt;
    const size_t X = (size_t)1 << xbits;
    w.part = (double*)wa.take((size_t)part_rows * X * 8);
    w.pop = (float*)wa.take((size_t)cap * X * 4);
    bool ok = w.part && w.pop;
    for (int k = 0; k < 2; ++k) {
      w.el_wt[k] = (int32_t*)wa.take((size_t)cap * 4);
      w.el_prefix[k] = (uint64_t*)wa.take((size_t)cap * 8);
      w.el_off[k] = (int32_t*)wa.take((size_t)cap * 4);
      w.el_cnt[k] = (int32_t*)wa.take((size_t)cap * 4);
      w.ids[k] = (int32_t*)wa.take((size_t)std::max<int64_t>(wp.R, 1) * 4);
      ok = ok && w.el_wt[k] && w.el_prefix[k] && w.el_off[k] && w.el_cnt[k] && w.ids[k];
    }
    w.shot_x = (int32_t*)wa.take((size_t)std::max<int64_t>(wp.R, 1) * 4);
    w.child_cnt = (int32_t*)wa.take((size_t)cap * 4);
    w.child_off = (int32_t*)wa.take((size_t)cap * 4);
    w.scan_sums = (int32_t*)wa.take((size_t)((cap + 1023) / 1024 + 1) * 4);
    w.counts = (int32_t*)wa.take((size_t)(ptsbe::kRgMaxBatches + 1) * 4);
    ok = ok && w.shot_x && w.child_cnt && w.child_off && w.scan_sums && w.counts;
    if (!ok) return fail(PTSBE_ERR_OUT_OF_MEMORY, "wave arena too small (elements)");
    // tables
    auto put = [&](const void* src, size_t bytes) -> void* {
      void* d = tb.take(std::max<size_t>(bytes, 8));
      if (d && bytes) {
        if (hipMemcpy(d, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
      }
      return d;
    };
    w.pieces = (const RgPiece*)put(pcs.data(), pcs.size() * sizeof(RgPiece));
    w.traj_piece = (const int32_t*)put(traj_piece.data(), traj_piece.size() * 4);
    w.traj_row0 = (const int64_t*)put(traj_row0.data(), traj_row0.size() * 8);
    w.m0_start = (const int64_t*)put(m0_start.data(), m0_start.size() * 8);
    if (!w.pieces || !w.traj_piece || !w.traj_row0 || !w.m0_start)
      return fail(PTSBE_ERR_OUT_OF_MEMORY, "wave tables do not fit");
    w.n_pieces = P;
    w.T = (int32_t)wp.T;
    w.R = wp.R;
    w.xbits = xbits;
    w.cap = cap;
    w.done = d_done_ticks;
    w.bad_flag = bad_flag;
    w.n_jobs = n_jobs;
    // window levels: pieces in wave order (heaviest job first)
    int maxW = 0;
    for (auto& pc : pcs) maxW = std::max(maxW, pc.n_win);
    for (int l = 0; l < maxW; ++l) {
      std::vector<int32_t> lp;
      std::vector<int64_t> ls;
      int64_t tasks = 0;
      int32_t max_ops = 0;
      for (int k = 0; k < P; ++k) {
        if (pcs[k].n_win <= l) continue;
        const Plan& p = *reinterpret_cast<const Plan*>(jobs[pcs[k].job].plan);
        const int np = p.sv_win[window_choice(*set, &p)][l].np;
        if (pcs[k].swin) max_ops = std::max(max_ops, p.sv_wins_plain[window_choice(*set, &p)][l].n_ops);
        lp.push_back(k);
        ls.push_back(tasks);
        tasks += (int64_t)pcs[k].nj << (pcs[k].n - np);
      }
      RgLevel lv{};
      lv.piece = (const int32_t*)put(lp.data(), lp.size() * 4);
      lv.start = (const int64_t*)put(ls.data(), ls.size() * 8);
      if (!lv.piece || !lv.start) return fail(PTSBE_ERR_OUT_OF_MEMORY, "wave tables do not fit");
      lv.n = (int32_t)lp.size();
      lv.tasks = tasks;
      lv.max_ops = max_ops;
      L.levels.push_back(lv);
    }
  }
  // launch (or replay) every wave
  const bool replay = use_graph && set->key == key && set->execs.size() == waves.size();
  if (use_graph && !replay) set->drop_graphs();
  int64_t launches = 0;
  const int g_mem = set->n_cu * 8, g_samp = set->n_cu * 2;
  for (size_t wi = 0; wi < waves.size(); ++wi) {
    const WaveLaunch& L = wl[wi];
    if (replay) {
      HIP_TRY(hipGraphLaunch(set->execs[wi], s));
      continue;
    }
    if (use_graph) HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int64_t n0 = launches;
    if (wi == 0) { HIP_TRY(ptsbe::launch_rg_start(L.w, s)); ++launches; }
    HIP_TRY(ptsbe::launch_rg_prepare(L.w, g_mem, s));
    ++launches;
    for (size_t l = 0; l < L.levels.size(); ++l) {
      HIP_TRY(ptsbe::launch_rg_window(L.w, L.levels[l], (int)l, set->n_cu, s));
      ++launches;
    }
    HIP_TRY(ptsbe::launch_rg_marginal0(L.w, L.m0_tasks, g_mem, s));
    launches += 2;
    int cur = 0;
    for (int j = 0; j < L.maxf; ++j) {
      if (j > 0) { HIP_TRY(ptsbe::launch_rg_marginal(L.w, j, cur, g_mem, s)); ++launches; }
      HIP_TRY(ptsbe::launch_rg_sample(L.w, j, cur, g_samp, s));
      ++launches;
      if (j + 1 < L.maxf) {
        HIP_TRY(ptsbe::launch_rg_scan(L.w, j, s));
        HIP_TRY(ptsbe::launch_rg_children(L.w, j, cur, g_samp, s));
        launches += 4;
        cur ^= 1;
      }
    }
    (void)n0;
    if (use_graph) {
      hipGraph_t graph;
      HIP_TRY(hipStreamEndCapture(s, &graph));
      hipGraphExec_t exec;
      hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return fail(PTSBE_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
      set->execs.push_back(exec);
      HIP_TRY(hipGraphLaunch(exec, s));
    }
  }
  if (use_graph && !replay) set->key = key;
  // self-normalised weights per job
  for (int c = 0; c < n_jobs; ++c) {
    if (!jobs[c].d_traj_weight && !jobs[c].d_traj_norm) continue;
    ptsbe::WeightArgs wa{norms[c], jobs[c].d_mult, jobs[c].E, jobs[c].d_traj_weight, jobs[c].d_traj_norm};
    HIP_TRY(ptsbe::launch_weights(wa, s));
  }
  int32_t bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, bad_flag, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  set->last_waves = (int)waves.size();
  set->last_replayed = replay ? (int)waves.size() : 0;
  set->last_launches = replay ? 0 : launches;
  if (bad) return fail(PTSBE_ERR_NUMERIC, "an element had a non-finite marginal total");
  return PTSBE_OK;
}

}  // extern "C"
