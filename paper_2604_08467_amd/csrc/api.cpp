// C ABI of the PTSBE library: argument checking, the plan (host constants and
// the unified path of every batch), host-side pre-trajectory sampling, and the
// executor that drives the HIP kernels of one batch and of the whole
// non-degenerate batched sampling loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "philox.h"

using ptsbe::Plan;

namespace {
using ptsbe::fail;

using cd = std::complex<double>;

// Matrix of `op` (acting on `sq`, first listed qubit = high bit) in the space of
// the gate qubits `gq`; identity on gate qubits the operator does not touch.
void embed_op(const cd* op, const std::vector<int>& sq, const std::vector<int>& gq, cd* out) {
  const int nG = (int)gq.size(), nS = (int)sq.size();
  const int D = 1 << nG, d = 1 << nS;
  std::vector<int> spos(nS);
  for (int i = 0; i < nS; ++i)
    for (int k = 0; k < nG; ++k)
      if (gq[k] == sq[i]) spos[i] = k;
  for (int gx = 0; gx < D; ++gx)
    for (int gy = 0; gy < D; ++gy) {
      bool same = true;
      for (int k = 0; k < nG; ++k) {
        bool in_s = false;
        for (int i = 0; i < nS; ++i) in_s |= spos[i] == k;
        if (in_s) continue;
        if (((gx >> (nG - 1 - k)) & 1) != ((gy >> (nG - 1 - k)) & 1)) same = false;
      }
      if (!same) { out[gx * D + gy] = 0.0; continue; }
      int sx = 0, sy = 0;
      for (int i = 0; i < nS; ++i) {
        sx |= ((gx >> (nG - 1 - spos[i])) & 1) << (nS - 1 - i);
        sy |= ((gy >> (nG - 1 - spos[i])) & 1) << (nS - 1 - i);
      }
      out[gx * D + gy] = op[sx * d + sy];
    }
}

void matmul(const cd* a, const cd* b, cd* c, int d) {
  for (int r = 0; r < d; ++r)
    for (int cc = 0; cc < d; ++cc) {
      cd acc = 0.0;
      for (int x = 0; x < d; ++x) acc += a[r * d + x] * b[x * d + cc];
      c[r * d + cc] = acc;
    }
}

using ptsbe::Arena;

}  // namespace

namespace ptsbe {
thread_local std::string g_last_error;
ptsbe_status_t fail(ptsbe_status_t s, const std::string& msg) {
  g_last_error = msg;
  return s;
}
}  // namespace ptsbe

namespace {

ptsbe::GateCtx gate_ctx(const Plan& p, const uint8_t* kraus, const float2* merged) {
  ptsbe::GateCtx g;
  g.gates = p.d_gates;
  g.gate_site_list = p.d_gate_site_list;
  g.site_ops = p.d_site_ops;
  g.kraus = kraus;
  g.S = p.S;
  g.max_kraus = p.max_kraus;
  g.merged = merged;
  g.G = p.G;
  return g;
}

size_t merged_bytes(const Plan& p, int64_t E) { return (size_t)E * p.G * 16 * sizeof(float2); }

bool part_uses_vm(const ptsbe::PartPlan& pp) { return pp.peak <= ptsbe::kVmMaxRank; }

size_t part_scratch_per_job(const ptsbe::PartPlan& pp) {
  if (pp.steps.empty() || part_uses_vm(pp)) return 0;
  return 2 * ((size_t)8 << pp.peak);
}

// Workspace of one trajectory at batch bp: its right tensor, the join's layout of
// it (the larger of the folded blocks and the canonical copy) and sweep scratch.
size_t join_traj_bytes(const ptsbe::BatchPlan& bp) {
  const int lkb = (int)bp.lk.size();
  size_t layout = (size_t)8 << bp.right.labels.size();
  if (bp.doubled && ptsbe::qform_supported(lkb))
    layout = std::max(layout, ptsbe::qform_theta_bytes((int)bp.xT.size(), lkb));
  return ((size_t)8 << bp.right.labels.size()) + layout + part_scratch_per_job(bp.right);
}

// One LDS sweep launch (part_vm_kernel) over the first n_steps steps of a part;
// under profiling, HIP events on the launch stream and the steps' algorithmic
// flops (8 per complex multiply-add: 8 2^(rC + nK) per step and job).
ptsbe_status_t timed_part_vm(Plan& p, const ptsbe::PartPlan& pp, const ptsbe::AbsorbStep* d_steps, int n_steps,
                             int peak, const ptsbe::GateCtx& g, int64_t n_jobs, const int32_t* job_traj,
                             int32_t traj_base, const uint64_t* job_prefix, const ptsbe::InitArgs& init, float2* out,
                             int out_rank, hipStream_t s) {
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  if (p.profile) {
    HIP_TRY(hipEventCreate(&ev.first));
    HIP_TRY(hipEventCreate(&ev.second));
    HIP_TRY(hipEventRecord(ev.first, s));
  }
  // a last step that raises the rank past every other tensor of the sweep (the
  // per-element parts of small batches end so) writes its output straight to HBM,
  // so that the LDS buffers, and with them the jobs per workgroup, are sized for
  // the ranks before it
  int lds_peak = 0, direct = 0;
  for (int i = 0; i < n_steps; ++i) {
    const ptsbe::AbsorbStep& st = pp.steps[(size_t)i];
    lds_peak = std::max(lds_peak, st.rA);
    if (i + 1 < n_steps) lds_peak = std::max(lds_peak, st.rC);
  }
  if (n_steps > 0) {
    const ptsbe::AbsorbStep& last = pp.steps[(size_t)n_steps - 1];
    if (last.rC > lds_peak && last.rC == out_rank && last.nK <= 1 && last.nN > last.nK && last.nK + last.nN <= 4)
      direct = 1;
  }
  HIP_TRY(ptsbe::launch_part_vm(d_steps, n_steps, direct ? lds_peak : peak, g, n_jobs, job_traj, traj_base, job_prefix,
                                p.NW, init, out, out_rank, direct, s));
  if (p.profile) {
    HIP_TRY(hipEventRecord(ev.second, s));
    p.vm_evs.push_back(ev);
    ++p.vm_launches;
    double f = 0.0;
    for (int i = 0; i < n_steps; ++i) f += 8.0 * std::ldexp(1.0, pp.steps[(size_t)i].rC + pp.steps[(size_t)i].nK);
    p.vm_flops += f * (double)n_jobs;
  }
  return PTSBE_OK;
}

// Subtree reuse in a per-trajectory part (Sec. VI: cached intermediates between
// error sets): jobs whose error sets agree on every noise site absorbed so far share
// the running tensor, and a job gets its own copy only at the launch where a site it
// disagrees on is absorbed.  Jobs are the distinct error patterns of the part (one
// representative trajectory each); at each launch boundary the jobs are grouped by
// their Kraus choices on the sites absorbed up to there, each group running once on
// its first job's gates (identical for every member on those sites, so results are
// bit-identical to running every job alone).
struct PartTrie {
  const uint8_t* h_kraus = nullptr;                 // host [E][S]
  int64_t S = 0;
  const std::vector<int32_t>* reps = nullptr;       // absolute trajectory of each job
  std::vector<std::vector<int32_t>>* keep = nullptr;   // host sources of async uploads
};

// Jobs of the level that ends after step `end` (exclusive): the first job of every
// group of equal Kraus choices on the sites absorbed so far, ascending; pos[r] =
// index of job r's group in that list.  Incremental: `done` marks the sites
// already absorbed (steps before `from`), and the groups refine the previous
// level's (prev_pos, empty at the first level) by the choices on the new sites.
void trie_level(const Plan& p, const ptsbe::PartPlan& pp, const PartTrie& t, int from, int end,
                std::vector<char>& done, const std::vector<int32_t>& prev_pos, std::vector<int32_t>& first,
                std::vector<int32_t>& pos) {
  std::vector<int32_t> sites;
  for (int i = from; i < end; ++i) {
    const int gate = pp.steps[(size_t)i].gate;
    if (gate < 0 || gate >= p.n_user_gates) continue;
    for (int st : p.gate_sites[(size_t)gate])
      if (!done[(size_t)st]) {
        done[(size_t)st] = 1;
        sites.push_back(st);
      }
  }
  const std::vector<int32_t>& reps = *t.reps;
  first.clear();
  pos.assign(reps.size(), 0);
  if (sites.empty() && !prev_pos.empty()) {      // no new site: the previous groups
    std::vector<int32_t> seen_first;
    for (size_t r = 0; r < reps.size(); ++r) {
      const int32_t gi = prev_pos[r];
      if ((size_t)gi >= seen_first.size()) seen_first.resize((size_t)gi + 1, -1);
      if (seen_first[(size_t)gi] < 0) {
        seen_first[(size_t)gi] = (int32_t)first.size();
        first.push_back((int32_t)r);
      }
      pos[r] = seen_first[(size_t)gi];
    }
    return;
  }
  std::unordered_map<std::string, int32_t> seen;
  std::string key(4 + sites.size(), '\0');
  for (size_t r = 0; r < reps.size(); ++r) {
    const int32_t gi = prev_pos.empty() ? 0 : prev_pos[r];
    std::memcpy(&key[0], &gi, 4);
    const uint8_t* kr = t.h_kraus + (int64_t)reps[r] * t.S;
    for (size_t i = 0; i < sites.size(); ++i) key[4 + i] = (char)kr[sites[i]];
    auto it = seen.emplace(key, (int32_t)first.size());
    if (it.second) first.push_back((int32_t)r);
    pos[r] = it.first->second;
  }
}

// Run one part (left or right) for n_jobs jobs; the result (rank = labels.size())
// goes to out[job][2^rank].  With `trie` (per-trajectory parts; n_jobs ==
// trie->reps->size(), job_traj the representatives on the device) launches run once
// per group of jobs that agree on the sites absorbed so far.
ptsbe_status_t run_part(Plan& p, const ptsbe::PartPlan& pp, const ptsbe::AbsorbStep* d_steps,
                        const ptsbe::GateCtx& g, int64_t n_jobs, const int32_t* job_traj, int32_t traj_base,
                        const uint64_t* job_prefix, const ptsbe::InitArgs& init, float2* out, Arena& ar,
                        hipStream_t s, const PartTrie* trie = nullptr) {
  if (n_jobs <= 0) return PTSBE_OK;
  const int out_rank = (int)pp.labels.size();
  if (pp.steps.empty()) {
    if (init.Vprev) HIP_TRY(ptsbe::launch_init_gather(init, n_jobs, job_prefix, p.NW, out, s));
    else HIP_TRY(ptsbe::launch_fill_one(out, n_jobs, s));
    return PTSBE_OK;
  }
  if (part_uses_vm(pp))
    return timed_part_vm(p, pp, d_steps, (int)pp.steps.size(), pp.peak, g, n_jobs, job_traj, traj_base, job_prefix,
                         init, out, out_rank, s);
  const size_t mark = ar.used;
  float2* b0 = (float2*)ar.take((size_t)n_jobs * ((size_t)8 << pp.peak));
  float2* b1 = (float2*)ar.take((size_t)n_jobs * ((size_t)8 << pp.peak));
  if (!b0 || !b1) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for a sweep");
  // subtree reuse: the current level's jobs (first job of each group), their
  // trajectories on the device, and each job's group
  int64_t cur_n = n_jobs;
  const int32_t* cur_traj = job_traj;
  std::vector<int32_t> lv_first, lv_pos;
  auto upload = [&](std::vector<int32_t>&& v, int32_t** d) -> ptsbe_status_t {
    *d = (int32_t*)ar.take(std::max<size_t>(v.size(), 1) * 4);
    if (!*d) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small (subtree reuse tables)");
    trie->keep->push_back(std::move(v));
    HIP_TRY(hipMemcpyAsync(*d, trie->keep->back().data(), trie->keep->back().size() * 4, hipMemcpyHostToDevice, s));
    return PTSBE_OK;
  };
  // the jobs of the level ending after step `end`; returns the device gather index
  // from the previous level (null when the job set does not grow)
  std::vector<char> lv_done(trie ? p.site_gate.size() : 0, 0);
  int lv_end = 0;
  auto enter_level = [&](int end, int32_t** d_gather) -> ptsbe_status_t {
    *d_gather = nullptr;
    if (!trie) return PTSBE_OK;
    std::vector<int32_t> first, pos;
    trie_level(p, pp, *trie, lv_end, end, lv_done, lv_pos, first, pos);
    lv_end = end;
    if ((int64_t)first.size() == cur_n && !lv_first.empty()) {
      lv_pos = std::move(pos);      // the same partition (group order may differ: keep the list)
      return PTSBE_OK;
    }
    std::vector<int32_t> gidx(first.size()), trajs(first.size());
    for (size_t k = 0; k < first.size(); ++k) {
      gidx[k] = lv_first.empty() ? 0 : lv_pos[(size_t)first[k]];
      trajs[k] = (*trie->reps)[(size_t)first[k]];
    }
    int32_t* dt = nullptr;
    ptsbe_status_t st = upload(std::move(trajs), &dt);
    if (st != PTSBE_OK) return st;
    if (!lv_first.empty()) {
      st = upload(std::move(gidx), d_gather);
      if (st != PTSBE_OK) return st;
    }
    cur_n = (int64_t)first.size();
    cur_traj = dt;
    lv_first = std::move(first);
    lv_pos = std::move(pos);
    return PTSBE_OK;
  };
  // the leading segments whose tensors all fit 2^kVmMaxRank entries run as one
  // LDS sweep (one launch) instead of one launch per step
  const size_t nseg = pp.segs.size();
  size_t s0 = 0;
  int h = 0, hpeak = 0;
  while (s0 + 1 < nseg) {
    const ptsbe::Segment& sg = pp.segs[s0];
    int pk = hpeak;
    for (int i = sg.first; i < sg.first + sg.count; ++i)
      pk = std::max(pk, std::max(pp.steps[(size_t)i].rA, pp.steps[(size_t)i].rC));
    if (pk > ptsbe::kVmMaxRank) break;
    hpeak = pk;
    h = sg.first + sg.count;
    ++s0;
  }
  if (h < 2) s0 = 0;
  // the last rank-changing step writes the output; in-place runs after it work on
  // the output directly (no final copy; with subtree reuse the job set may still
  // grow, so the output is written by a final copy)
  size_t last_nf = nseg;
  for (size_t si = s0; si < nseg; ++si)
    if (!pp.segs[si].fused) last_nf = si;
  if (trie) last_nf = nseg + 1;
  float2* A = last_nf == nseg ? out : b0;
  int32_t* d_gather = nullptr;
  {
    const ptsbe_status_t st = enter_level(h >= 2 ? h : 0, &d_gather);
    if (st != PTSBE_OK) return st;
  }
  if (h >= 2) {
    const ptsbe_status_t st = timed_part_vm(p, pp, d_steps, h, hpeak, g, cur_n, cur_traj, traj_base, job_prefix,
                                            init, A, pp.steps[(size_t)h - 1].rC, s);
    if (st != PTSBE_OK) return st;
  } else {
    if (init.Vprev) HIP_TRY(ptsbe::launch_init_gather(init, cur_n, job_prefix, p.NW, A, s));
    else HIP_TRY(ptsbe::launch_fill_one(A, cur_n, s));   // rank-0 start: the scalar 1 per job
  }
  int cur_rank = h >= 2 ? pp.steps[(size_t)h - 1].rC : (init.Vprev ? init.r0 : 0);
  for (size_t si = s0; si < nseg; ++si) {
    const ptsbe::Segment& sg = pp.segs[si];
    if (trie) {
      // the jobs of this launch: groups that agree on every site absorbed by its end
      const ptsbe_status_t st = enter_level(sg.first + sg.count, &d_gather);
      if (st != PTSBE_OK) return st;
      if (d_gather) {
        float2* D = A == b0 ? b1 : b0;
        HIP_TRY(ptsbe::launch_gather_rows(A, d_gather, D, cur_n, cur_rank, s));
        A = D;
      }
    }
    if (sg.fused) {   // a run of in-place steps, one tile pass, in place
      HIP_TRY(ptsbe::launch_fused(sg, p.d_fused, g, cur_n, cur_traj, traj_base, job_prefix, p.NW, A, s));
      if (p.profile) p.fused_bytes += (double)cur_n * 16.0 * std::ldexp(1.0, sg.r);
      continue;
    }
    const size_t i = (size_t)sg.first;
    float2* C = (si == last_nf) ? out : (A == b0 ? b1 : b0);
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (p.profile >= 2) {
      HIP_TRY(hipEventCreate(&ev.first));
      HIP_TRY(hipEventCreate(&ev.second));
      HIP_TRY(hipEventRecord(ev.first, s));
    }
    HIP_TRY(ptsbe::launch_absorb_global(pp.steps[i], d_steps + i, g, cur_n, cur_traj, traj_base, job_prefix,
                                        p.NW, A, C, s));
    if (p.profile >= 2) {
      HIP_TRY(hipEventRecord(ev.second, s));
      p.sweep_evs.push_back(ev);
      ++p.sweep_launches;
    }
    A = C;
    cur_rank = pp.steps[i].rC;
    if (p.profile) p.sweep_bytes += (double)cur_n * 8.0 *
                                    (std::ldexp(1.0, pp.steps[i].rA) + std::ldexp(1.0, pp.steps[i].rC));
  }
  if (cur_n != n_jobs) return fail(PTSBE_ERR_DEVICE, "subtree reuse: the last level does not hold every job");
  if (A != out) HIP_TRY(ptsbe::launch_copy(A, out, n_jobs << out_rank, s));
  ar.used = mark;
  return PTSBE_OK;
}

struct BatchIO {
  // elements of this batch (device)
  const int32_t* elem_traj = nullptr;
  const uint64_t* elem_prefix = nullptr;
  int64_t U = 0;
  // contraction output mode: external full-size output, or per-chunk sampling
  float* pop_out = nullptr;     // [U][2^b] (contract_batch)
  float2* amp_out = nullptr;    // [U][2^b] (contract_batch, last batch)
  double* totals = nullptr;     // [U] FP64 sums (may be null for contract_batch)
  bool sample = false;
  ptsbe::SampleArgs sa{};       // template: per-element arrays at offset 0
  // prefix-tree reuse: left tensors of all elements kept for the next batch
  float2* V_out = nullptr;      // [U][2^rank] persistent left tensors of this batch, or null
  bool resume = false;          // start each element from its parent's left tensor
  const float2* V_prev = nullptr;
  int64_t V_prev_stride = 1;
  const int32_t* parent = nullptr;
  // host copy of the trajectories' Kraus indices [E][S]: trajectories that agree
  // on the sites of a batch's per-trajectory part share its tensor (null: no sharing)
  const uint8_t* h_kraus = nullptr;
  // exhaustive final-batch sampling: rows appended per element chunk (null: off)
  struct Exhaustive {
    ptsbe::ExhArgs tmpl{};      // threshold, traj_norm, outputs, capacity
    int64_t rows = 0;           // rows found so far (host)
  }* exh = nullptr;
};

// The noise sites whose Kraus choices enter the per-trajectory part of a batch.
std::vector<int32_t> right_sites(const Plan& p, const ptsbe::BatchPlan& bp) {
  std::vector<char> on((size_t)p.site_gate.size(), 0);
  for (const ptsbe::AbsorbStep& st : bp.right.steps)
    if (st.gate >= 0 && st.gate < p.n_user_gates)
      for (int s : p.gate_sites[(size_t)st.gate]) on[(size_t)s] = 1;
  std::vector<int32_t> out;
  for (size_t s = 0; s < on.size(); ++s)
    if (on[s]) out.push_back((int32_t)s);
  return out;
}

struct EventPair { hipEvent_t a, b; };

// Exhaustive final-batch sampling of one element chunk (Sec. III-B): FP64 totals,
// rows per (element, tile), their scan, and the ordered row writes.  The row
// count is read back so that the next chunk's rows follow these.
ptsbe_status_t exhaustive_chunk(const ptsbe::BatchPlan& bp, BatchIO& io, const float* pop, int64_t a0, int64_t ne,
                                int tile_bits, Arena& ar, hipStream_t s) {
  const size_t mark = ar.used;
  const int64_t n_units = ne << tile_bits;
  double* tot = (double*)ar.take((size_t)ne * 8);
  int32_t* cnt = (int32_t*)ar.take((size_t)n_units * 4);
  int32_t* off = (int32_t*)ar.take((size_t)n_units * 4);
  int32_t* scratch = (int32_t*)ar.take(ptsbe::scan_scratch_bytes(n_units));
  int32_t* total = (int32_t*)ar.take(64);
  if (!tot || !cnt || !off || !scratch || !total)
    return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small (exhaustive rows)");
  HIP_TRY(ptsbe::launch_row_totals(pop, ne, bp.size, tot, s));
  ptsbe::ExhArgs a = io.exh->tmpl;
  if (a.totals_out) HIP_TRY(hipMemcpyAsync(a.totals_out + a0, tot, (size_t)ne * 8, hipMemcpyDeviceToDevice, s));
  a.pop = pop; a.b = bp.size; a.start = bp.start;
  a.n_elems = ne;
  a.elem_traj = io.elem_traj + a0;
  a.elem_prefix = io.elem_prefix + a0 * a.NW;
  a.elem_total = tot;
  a.tile_cnt = cnt; a.tile_off = off; a.tile_bits = tile_bits;
  a.row_base = io.exh->rows;
  HIP_TRY(ptsbe::launch_exh_count(a, s));
  HIP_TRY(ptsbe::launch_scan_i32(cnt, off, n_units, total, scratch, s));
  int32_t found = 0;
  HIP_TRY(hipMemcpyAsync(&found, total, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (found > 0 && a.row_base < a.capacity) HIP_TRY(ptsbe::launch_exh_write(a, s));
  io.exh->rows += found;
  ar.used = mark;
  return PTSBE_OK;
}

// Bytes of the join's layout of one per-trajectory tensor: Theta (the doubled
// join's folded slot coefficients) or the canonical copy of the MFMA ket join.
size_t join_layout_bytes(const ptsbe::BatchPlan& bp) {
  const int lkb = (int)bp.lk.size();
  if (bp.doubled && ptsbe::qform_supported(lkb)) return ptsbe::qform_theta_bytes((int)bp.xT.size(), lkb);
  if (!bp.doubled && ptsbe::ketjoin_supported(lkb)) return (size_t)8 << bp.right.labels.size();
  return 0;
}

// Trajectories and elements per chunk of one batch when `avail` workspace bytes are
// left: half for the per-trajectory tensors (with their join layout and sweep
// scratch), half for the per-element tensors and populations.
struct ChunkCaps { int64_t t_cap = 0, e_cap = 0; };
ChunkCaps chunk_caps(const ptsbe::BatchPlan& bp, const ptsbe::PartPlan& left, int64_t E, bool own_V,
                     bool chunk_pop, bool exh, size_t avail, int NW = 0) {
  // NW > 0: sliced last batch (per job: prefix words with the slice bits; per
  // element: the amplitude sum and one slice's amplitudes)
  const size_t per_traj = ((size_t)8 << bp.right.labels.size()) + join_layout_bytes(bp) +
                          part_scratch_per_job(bp.right) + (size_t)NW * 8;
  const int exh_tile_bits = bp.size > 12 ? bp.size - 12 : 0;
  const size_t per_elem = (own_V ? ((size_t)8 << left.labels.size()) : 0) + part_scratch_per_job(left) +
                          (chunk_pop ? ((size_t)4 << bp.size) : 0) + (exh ? 16 + ((size_t)12 << exh_tile_bits) : 0) +
                          (NW > 0 ? ((size_t)16 << bp.size) + (size_t)NW * 8 : 0);
  ChunkCaps c;
  c.t_cap = (int64_t)std::min<size_t>((size_t)E, (avail / 2) / per_traj);
  c.e_cap = (int64_t)((avail / 2) / per_elem);
  c.e_cap = std::min<int64_t>(c.e_cap, 1 << 22);
  if (exh) c.e_cap = std::min<int64_t>(c.e_cap, std::max<int64_t>(1, (((int64_t)1 << 31) - 1) >> bp.size));
  c.t_cap = std::min<int64_t>(c.t_cap, 65535);   // one grid dimension of the MFMA join
  return c;
}

// Last batch with sliced crossing wires (slice_bits = s > 0): for each chunk of
// trajectories and each chunk of their elements, both parts are contracted once
// per slice value (the value's bits OR'ed into the jobs' prefix words at bits
// n..n+s-1, which the sliced legs read) and the join's amplitudes are summed over
// the 2^s values: the contraction over the sliced wires split into its terms.
// Populations (and the sampling, exhaustive and total outputs) are formed from
// the sums.  The per-trajectory part is recomputed per element chunk.
ptsbe_status_t run_batch_sliced(Plan& p, int j, const uint8_t* d_kraus, const float2* merged, int64_t E,
                                BatchIO& io, Arena& ar, hipStream_t s) {
  const ptsbe::BatchPlan& bp = p.batches[j];
  const ptsbe::GateCtx g = gate_ctx(p, d_kraus, merged);
  // the sliced batch is the last one: no later batch resumes from its left
  // tensors, so io.V_out (which would differ per slice) is not written
  const size_t mark0 = ar.used;
  int32_t* d_first = (int32_t*)ar.take((size_t)(E + 1) * 4);
  if (!d_first) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small (trajectory ranges)");
  HIP_TRY(ptsbe::launch_traj_ranges(io.elem_traj, io.U, E, d_first, s));
  std::vector<int32_t> first((size_t)E + 1);
  HIP_TRY(hipMemcpyAsync(first.data(), d_first, (size_t)(E + 1) * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const ptsbe::PartPlan& left = io.resume ? bp.left_resume : bp.left;
  const int rT = (int)bp.right.labels.size(), rV = (int)left.labels.size();
  const Plan::JoinDev& jdv = io.resume ? p.join_dev_r[j] : p.join_dev[j];
  const int lkb = (int)bp.lk.size();
  const bool use_ket = ptsbe::ketjoin_supported(lkb);
  const size_t layout_bytes = join_layout_bytes(bp);
  const size_t nb = (size_t)1 << bp.size;
  const bool chunk_pop = io.sample || io.exh;
  const int exh_tile_bits = bp.size > 12 ? bp.size - 12 : 0;
  const ChunkCaps caps = chunk_caps(bp, left, E, true, chunk_pop, io.exh != nullptr, ar.left(), p.NW);
  if (caps.t_cap < 1 || caps.e_cap < 1)
    return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for one trajectory of batch " + std::to_string(j));
  const ptsbe::AbsorbStep* d_left = p.d_steps + p.part_step_off[3 * j + (io.resume ? 2 : 0)];
  const ptsbe::AbsorbStep* d_right = p.d_steps + p.part_step_off[3 * j + 1];
  ptsbe::GemvTiling gtile{};
  const bool gemv_tiled = bp.xb.size() <= 1 && ptsbe::make_gemv_tiling(bp, gtile);
  ptsbe::GemvLanes glanes{};
  const bool gemv_lanes = ptsbe::make_gemv_lanes(bp, glanes);
  const int wi = p.n >> 6, sh = p.n & 63;
  const int64_t n_slices = (int64_t)1 << bp.slice_bits;
  for (int64_t t0 = 0; t0 < E; t0 += caps.t_cap) {
    const int64_t t1 = std::min<int64_t>(E, t0 + caps.t_cap), n_rt = t1 - t0;
    const int64_t e0 = first[t0], e1 = first[t1];
    if (e1 <= e0) continue;
    const bool gemv = ptsbe::ketjoin_gemv_supported((int)bp.xb.size(), lkb, (int)bp.xT.size()) &&
                      (lkb <= 6 || gemv_tiled || gemv_lanes) && e1 - e0 <= 2 * (t1 - t0);
    for (int64_t a0 = e0; a0 < e1; a0 += caps.e_cap) {
      const int64_t a1 = std::min<int64_t>(e1, a0 + caps.e_cap), ne = a1 - a0;
      const size_t mark = ar.used;
      float2* T = (float2*)ar.take((size_t)n_rt * ((size_t)8 << rT));
      float2* Tc = (!gemv && use_ket) ? (float2*)ar.take((size_t)n_rt * layout_bytes) : nullptr;
      uint64_t* rpre = (uint64_t*)ar.take((size_t)n_rt * p.NW * 8);
      float2* V = (float2*)ar.take((size_t)ne * ((size_t)8 << rV));
      uint64_t* epre = (uint64_t*)ar.take((size_t)ne * p.NW * 8);
      float2* acc = (float2*)ar.take((size_t)ne * nb * 8);
      float2* amp = (float2*)ar.take((size_t)ne * nb * 8);
      float* pop = chunk_pop ? (float*)ar.take((size_t)ne * nb * 4) : nullptr;
      if (!T || (!gemv && use_ket && !Tc) || !rpre || !V || !epre || !acc || !amp || (chunk_pop && !pop))
        return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small (sliced batch)");
      HIP_TRY(hipMemsetAsync(acc, 0, (size_t)ne * nb * 8, s));
      ptsbe::InitArgs init;
      if (io.resume) {
        init.Vprev = io.V_prev;
        init.stride = io.V_prev_stride;
        init.parent = io.parent + a0;
        init.r0 = bp.resume_rank0;
        init.nsl = (int)bp.resume_slice_pos.size();
        for (int i = 0; i < init.nsl; ++i) { init.pos[i] = bp.resume_slice_pos[i]; init.q[i] = bp.resume_slice_q[i]; }
      }
      int64_t tA = t0, tB = t1 - 1;
      while (tA + 1 < t1 && first[tA + 1] <= a0) ++tA;
      while (tB > tA && first[tB] >= a1) --tB;
      int64_t max_rows = 0;
      for (int64_t t = tA; t <= tB; ++t) {
        const int64_t lo = std::max<int64_t>(first[t], a0), hi = std::min<int64_t>(first[t + 1], a1);
        max_rows = std::max<int64_t>(max_rows, (hi - lo) << bp.xb.size());
      }
      for (int64_t sv = 0; sv < n_slices; ++sv) {
        const uint64_t bits = (uint64_t)sv << sh;
        HIP_TRY(ptsbe::launch_prefix_or(nullptr, rpre, n_rt, p.NW, wi, bits, s));
        ptsbe_status_t st = run_part(p, bp.right, d_right, g, n_rt, nullptr, (int32_t)t0, rpre, ptsbe::InitArgs(), T,
                                     ar, s);
        if (st != PTSBE_OK) return st;
        if (Tc)
          HIP_TRY(ptsbe::launch_permute_T(T, (int64_t)1 << rT, n_rt, p.d_tables, p.join_dev[j], (int)bp.xT.size(),
                                          lkb, 0, Tc, s));
        HIP_TRY(ptsbe::launch_prefix_or(io.elem_prefix + a0 * p.NW, epre, ne, p.NW, wi, bits, s));
        st = run_part(p, left, d_left, g, ne, io.elem_traj + a0, 0, epre, init, V, ar, s);
        if (st != PTSBE_OK) return st;
        ptsbe::JoinArgs ja{};
        ja.V = V; ja.v_stride = (int64_t)1 << rV;
        ja.T = T; ja.t_stride = (int64_t)1 << rT;
        ja.elem_traj = io.elem_traj + a0; ja.traj_base = (int32_t)t0; ja.tslot = nullptr;
        ja.n_elems = ne;
        ja.xb_bits = (int)bp.xb.size(); ja.lk_bits = lkb; ja.xT_bits = (int)bp.xT.size();
        ja.tab = p.d_tables; ja.jd = jdv;
        ja.b = bp.size; ja.doubled = 0;
        ja.pop = nullptr;
        ja.amp = amp;
        if (gemv) {
          if (gemv_lanes) HIP_TRY(ptsbe::launch_ketjoin_gemv_lanes(ja, glanes, s));
          else if (gemv_tiled) HIP_TRY(ptsbe::launch_ketjoin_gemv_tiled(ja, gtile, s));
          else HIP_TRY(ptsbe::launch_ketjoin_gemv(ja, s));
        } else if (use_ket) {
          ptsbe::QformArgs qa{};
          qa.V = V; qa.v_stride = (int64_t)1 << rV; qa.v_base = a0;
          qa.Tc = Tc; qa.Th = nullptr; qa.traj_base = (int32_t)t0; qa.tslot = nullptr;
          qa.traj0 = (int32_t)tA;
          qa.first = d_first; qa.e_lo = a0; qa.e_hi = a1;
          qa.xb_bits = (int)bp.xb.size(); qa.lk_bits = lkb; qa.xT_bits = (int)bp.xT.size();
          qa.b = bp.size; qa.tab = p.d_tables; qa.jd = jdv;
          qa.pop = nullptr;
          qa.amp = amp;
          HIP_TRY(ptsbe::launch_ketjoin(qa, (int)(tB - tA + 1), (int)max_rows, s));
        } else {
          HIP_TRY(ptsbe::launch_join(ja, s));
        }
        HIP_TRY(ptsbe::launch_amp_accumulate(acc, amp, (int64_t)ne * (int64_t)nb, s));
      }
      float* pop_dst = chunk_pop ? pop : (io.pop_out ? io.pop_out + a0 * (int64_t)nb : nullptr);
      if (pop_dst) HIP_TRY(ptsbe::launch_amp_population(acc, pop_dst, (int64_t)ne * (int64_t)nb, s));
      if (io.amp_out)
        HIP_TRY(hipMemcpyAsync(io.amp_out + a0 * (int64_t)nb, acc, (size_t)ne * nb * 8, hipMemcpyDeviceToDevice, s));
      if (io.sample) {
        ptsbe::SampleArgs sa = io.sa;
        sa.pop = pop;
        sa.n_elems = ne;
        sa.elem_traj = io.elem_traj + a0;
        sa.elem_shot_off = io.sa.elem_shot_off + a0;
        sa.elem_shot_cnt = io.sa.elem_shot_cnt + a0;
        sa.elem_total = io.sa.elem_total + a0;
        sa.child_cnt = io.sa.child_cnt ? io.sa.child_cnt + a0 : nullptr;
        HIP_TRY(ptsbe::launch_sample(sa, s));
      } else if (io.exh) {
        ptsbe_status_t st = exhaustive_chunk(bp, io, pop, a0, ne, exh_tile_bits, ar, s);
        if (st != PTSBE_OK) return st;
      } else if (io.totals && pop_dst) {
        HIP_TRY(ptsbe::launch_row_totals(pop_dst, ne, bp.size, io.totals + a0, s));
      }
      ar.used = mark;
    }
  }
  ar.used = mark0;
  return PTSBE_OK;
}

ptsbe_status_t run_batch(Plan& p, int j, const uint8_t* d_kraus, const float2* merged, int64_t E, BatchIO& io,
                         Arena& ar, hipStream_t s, std::vector<EventPair>& evs) {
  const ptsbe::BatchPlan& bp = p.batches[j];
  if (io.U <= 0) return PTSBE_OK;
  if (bp.slice_bits > 0) return run_batch_sliced(p, j, d_kraus, merged, E, io, ar, s);
  const ptsbe::GateCtx g = gate_ctx(p, d_kraus, merged);
  const size_t mark0 = ar.used;
  // element ranges per trajectory
  int32_t* d_first = (int32_t*)ar.take((size_t)(E + 1) * 4);
  if (!d_first) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small (trajectory ranges)");
  HIP_TRY(ptsbe::launch_traj_ranges(io.elem_traj, io.U, E, d_first, s));
  std::vector<int32_t> first((size_t)E + 1);
  HIP_TRY(hipMemcpyAsync(first.data(), d_first, (size_t)(E + 1) * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const ptsbe::PartPlan& left = io.resume ? bp.left_resume : bp.left;
  const int rT = (int)bp.right.labels.size(), rV = (int)left.labels.size();
  const Plan::JoinDev& jdv = io.resume ? p.join_dev_r[j] : p.join_dev[j];
  const int lkb = (int)bp.lk.size();
  const bool use_qform = bp.doubled && ptsbe::qform_supported(lkb);
  const bool use_ket = !bp.doubled && ptsbe::ketjoin_supported(lkb);
  const bool use_mfma = use_qform || use_ket;
  const bool use_split = use_qform && p.precision != PTSBE_C64 && ptsbe::qform_split_supported(lkb);
  const int split_kind = !use_split ? 0 : (p.precision == PTSBE_SPLIT_F16 ? 2 : 1);
  const bool use_fold = use_qform;               // Theta layout (FP32, or bf16 hi + lo planes)
  const size_t layout_bytes = join_layout_bytes(bp);
  const size_t nb = (size_t)1 << bp.size;
  const bool chunk_pop = io.sample || io.exh;     // populations live per element chunk
  const int exh_tile_bits = bp.size > 12 ? bp.size - 12 : 0;
  const ChunkCaps caps = chunk_caps(bp, left, E, !io.V_out, chunk_pop, io.exh != nullptr, ar.left());
  if (caps.t_cap < 1 || caps.e_cap < 1)
    return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for one trajectory of batch " + std::to_string(j));
  const int64_t t_cap = caps.t_cap, e_cap = caps.e_cap;
  const ptsbe::AbsorbStep* d_left = p.d_steps + p.part_step_off[3 * j + (io.resume ? 2 : 0)];
  const ptsbe::AbsorbStep* d_right = p.d_steps + p.part_step_off[3 * j + 1];
  const std::vector<int32_t> rsites = io.h_kraus ? right_sites(p, bp) : std::vector<int32_t>();
  ptsbe::GemvTiling gtile{};
  const bool gemv_tiled = !bp.doubled && bp.xb.size() <= 1 && ptsbe::make_gemv_tiling(bp, gtile);
  ptsbe::GemvLanes glanes{};
  const bool gemv_lanes = !bp.doubled && ptsbe::make_gemv_lanes(bp, glanes);
  const int64_t S = (int64_t)p.site_gate.size();
  std::vector<std::vector<int32_t>> keep;         // host sources of async uploads
  struct SyncOnExit {                             // on every return (errors included), the
    hipStream_t s;                                // uploads from `keep` finish before it is freed
    const std::vector<std::vector<int32_t>>& k;
    ~SyncOnExit() {
      if (!k.empty()) (void)hipStreamSynchronize(s);
    }
  } sync_on_exit{s, keep};
  std::vector<int32_t> trie_reps;                 // representatives of the chunk's right jobs (host)
  for (int64_t t0 = 0; t0 < E; t0 += t_cap) {
    const int64_t t1 = std::min<int64_t>(E, t0 + t_cap);
    const int64_t e0 = first[t0], e1 = first[t1];
    if (e1 <= e0) continue;                       // no elements for these trajectories
    const size_t mark = ar.used;
    // one per-trajectory tensor per distinct Kraus pattern on the part's sites
    int64_t n_rt = t1 - t0;
    const int32_t* d_rjob = nullptr;              // trajectory of each right job (null: t0 + job)
    const int32_t* d_slot = nullptr;              // right job of each trajectory (null: t - t0)
    if (io.h_kraus && n_rt > 1) {
      std::unordered_map<std::string, int32_t> seen;
      std::vector<int32_t> reps, slot((size_t)n_rt);
      std::string key(rsites.size(), '\0');
      for (int64_t t = t0; t < t1; ++t) {
        const uint8_t* kr = io.h_kraus + t * S;
        for (size_t i = 0; i < rsites.size(); ++i) key[i] = (char)kr[rsites[i]];
        auto it = seen.emplace(key, (int32_t)reps.size());
        if (it.second) reps.push_back((int32_t)t);
        slot[(size_t)(t - t0)] = it.first->second;
      }
      if ((int64_t)reps.size() < n_rt) {
        n_rt = (int64_t)reps.size();
        int32_t* dr = (int32_t*)ar.take(reps.size() * 4);
        int32_t* ds = (int32_t*)ar.take(slot.size() * 4);
        if (!dr || !ds) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small (trajectory sharing)");
        keep.push_back(std::move(reps));
        HIP_TRY(hipMemcpyAsync(dr, keep.back().data(), keep.back().size() * 4, hipMemcpyHostToDevice, s));
        keep.push_back(std::move(slot));
        HIP_TRY(hipMemcpyAsync(ds, keep.back().data(), keep.back().size() * 4, hipMemcpyHostToDevice, s));
        d_rjob = dr;
        d_slot = ds;
      }
    }
    float2* T = (float2*)ar.take((size_t)n_rt * ((size_t)8 << rT));
    if (!T) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small (right part)");
    PartTrie trie;
    if (p.subtree_reuse && io.h_kraus && n_rt > 1 && !part_uses_vm(bp.right)) {
      trie.h_kraus = io.h_kraus;
      trie.S = S;
      trie.keep = &keep;
      trie_reps.clear();
      if (d_rjob) {
        trie_reps = keep[keep.size() - 2];                       // the representatives uploaded above
      } else {
        for (int64_t t = t0; t < t1; ++t) trie_reps.push_back((int32_t)t);
      }
      trie.reps = &trie_reps;
    }
    ptsbe_status_t st = run_part(p, bp.right, d_right, g, n_rt, d_rjob, (int32_t)t0, nullptr,
                                 ptsbe::InitArgs(), T, ar, s, trie.reps ? &trie : nullptr);
    if (st != PTSBE_OK) return st;
    // last batch with at most two elements per trajectory: a GEMV on T's own layout
    // (T read once per element) beats the canonical copy plus the MFMA join
    const bool gemv = !bp.doubled && ptsbe::ketjoin_gemv_supported((int)bp.xb.size(), lkb, (int)bp.xT.size()) &&
                      (lkb <= 6 || gemv_tiled || gemv_lanes) && e1 - e0 <= 2 * (t1 - t0);
    float2* Tc = nullptr;
    float* Th = nullptr;
    if (gemv) {
      // T is read in place
    } else if (use_fold) {   // Theta (folded bilinear-form coefficients) for the FP32 MFMA doubled join
      Th = (float*)ar.take((size_t)n_rt * layout_bytes);
      if (!Th) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small (join layout)");
      HIP_TRY(ptsbe::launch_theta_T(T, (int64_t)1 << rT, n_rt, p.d_tables, p.join_dev[j], (int)bp.xT.size(),
                                    lkb, Th, split_kind, s));
    } else if (use_mfma) {   // canonical [x][k][k'] (split doubled) or [x][k] (ket) layout
      Tc = (float2*)ar.take((size_t)n_rt * layout_bytes);
      if (!Tc) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small (join layout)");
      HIP_TRY(ptsbe::launch_permute_T(T, (int64_t)1 << rT, n_rt, p.d_tables, p.join_dev[j], (int)bp.xT.size(),
                                      lkb, bp.doubled ? lkb : 0, Tc, s));
    }
    for (int64_t a0 = e0; a0 < e1; a0 += e_cap) {
      const int64_t a1 = std::min<int64_t>(e1, a0 + e_cap), ne = a1 - a0;
      const size_t mark2 = ar.used;
      float2* V = io.V_out ? io.V_out + a0 * ((int64_t)1 << rV) : (float2*)ar.take((size_t)ne * ((size_t)8 << rV));
      float* pop = chunk_pop ? (float*)ar.take((size_t)ne * nb * 4) : nullptr;
      if (!V || (chunk_pop && !pop)) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small (elements)");
      ptsbe::InitArgs init;
      if (io.resume) {
        init.Vprev = io.V_prev;
        init.stride = io.V_prev_stride;
        init.parent = io.parent + a0;
        init.r0 = bp.resume_rank0;
        init.nsl = (int)bp.resume_slice_pos.size();
        for (int i = 0; i < init.nsl; ++i) { init.pos[i] = bp.resume_slice_pos[i]; init.q[i] = bp.resume_slice_q[i]; }
      }
      st = run_part(p, left, d_left, g, ne, io.elem_traj + a0, 0, io.elem_prefix + a0 * p.NW, init, V, ar, s);
      if (st != PTSBE_OK) return st;
      ptsbe::JoinArgs ja{};
      ja.V = V; ja.v_stride = (int64_t)1 << rV;
      ja.T = T; ja.t_stride = (int64_t)1 << rT;
      ja.elem_traj = io.elem_traj + a0; ja.traj_base = (int32_t)t0; ja.tslot = d_slot;
      ja.n_elems = ne;
      ja.xb_bits = (int)bp.xb.size(); ja.lk_bits = (int)bp.lk.size(); ja.xT_bits = (int)bp.xT.size();
      ja.tab = p.d_tables; ja.jd = jdv;
      ja.b = bp.size; ja.doubled = bp.doubled ? 1 : 0;
      if (chunk_pop) {
        ja.pop = pop;
      } else {
        ja.pop = io.pop_out ? io.pop_out + a0 * (int64_t)nb : nullptr;
        ja.amp = io.amp_out ? io.amp_out + a0 * (int64_t)nb : nullptr;
      }
      EventPair ev{};
      const bool timed = p.profile && use_qform;   // the MFMA join is the measured kernel
      if (timed) {
        HIP_TRY(hipEventCreate(&ev.a));
        HIP_TRY(hipEventCreate(&ev.b));
        HIP_TRY(hipEventRecord(ev.a, s));
      }
      if (gemv) {
        if (gemv_lanes) HIP_TRY(ptsbe::launch_ketjoin_gemv_lanes(ja, glanes, s));
        else if (gemv_tiled) HIP_TRY(ptsbe::launch_ketjoin_gemv_tiled(ja, gtile, s));
        else HIP_TRY(ptsbe::launch_ketjoin_gemv(ja, s));
      } else if (use_mfma) {
        ptsbe::QformArgs qa{};
        qa.V = V; qa.v_stride = (int64_t)1 << rV; qa.v_base = a0;
        qa.Tc = Tc; qa.Th = Th; qa.traj_base = (int32_t)t0; qa.tslot = d_slot;
        qa.th_plane = n_rt * ((int64_t)1 << ((int)bp.xT.size() + 2 * lkb));
        qa.th_scale = Th ? reinterpret_cast<const int32_t*>(reinterpret_cast<const uint16_t*>(Th) + 2 * qa.th_plane)
                         : nullptr;
        int64_t tA = t0, tB = t1 - 1;
        while (tA + 1 < t1 && first[tA + 1] <= a0) ++tA;     // trajectory holding element a0
        while (tB > tA && first[tB] >= a1) --tB;             // trajectory holding element a1-1
        int64_t max_rows = 0;
        for (int64_t t = tA; t <= tB; ++t) {
          int64_t lo = std::max<int64_t>(first[t], a0), hi = std::min<int64_t>(first[t + 1], a1);
          max_rows = std::max<int64_t>(max_rows, (hi - lo) << bp.xb.size());
        }
        qa.traj0 = (int32_t)tA;
        qa.first = d_first; qa.e_lo = a0; qa.e_hi = a1;
        qa.xb_bits = (int)bp.xb.size(); qa.lk_bits = (int)bp.lk.size(); qa.xT_bits = (int)bp.xT.size();
        qa.b = bp.size; qa.tab = p.d_tables; qa.jd = jdv;
        qa.pop = ja.pop;
        qa.amp = ja.amp;
        if (use_qform) {
          if (!qa.pop) return fail(PTSBE_ERR_INVALID_ARG, "population output required");
          if (use_split)
            HIP_TRY(ptsbe::launch_qform_split(qa, (int)(tB - tA + 1), (int)max_rows, split_kind == 2, s));
          else
            HIP_TRY(ptsbe::launch_qform(qa, (int)(tB - tA + 1), (int)max_rows, s));
        } else {
          HIP_TRY(ptsbe::launch_ketjoin(qa, (int)(tB - tA + 1), (int)max_rows, s));
        }
      } else {
        HIP_TRY(ptsbe::launch_join(ja, s));
      }
      if (timed) {
        HIP_TRY(hipEventRecord(ev.b, s));
        evs.push_back(ev);
        p.join_launches++;
        p.join_flops += bp.join_flops_per_elem * (double)ne;
      }
      if (io.sample) {
        ptsbe::SampleArgs sa = io.sa;
        sa.pop = pop;
        sa.n_elems = ne;
        sa.elem_traj = io.elem_traj + a0;
        sa.elem_shot_off = io.sa.elem_shot_off + a0;
        sa.elem_shot_cnt = io.sa.elem_shot_cnt + a0;
        sa.elem_total = io.sa.elem_total + a0;
        sa.child_cnt = io.sa.child_cnt ? io.sa.child_cnt + a0 : nullptr;
        HIP_TRY(ptsbe::launch_sample(sa, s));
      } else if (io.exh) {
        st = exhaustive_chunk(bp, io, pop, a0, ne, exh_tile_bits, ar, s);
        if (st != PTSBE_OK) return st;
      } else if (io.totals && ja.pop) {
        HIP_TRY(ptsbe::launch_row_totals(ja.pop, ne, bp.size, io.totals + a0, s));
      }
      ar.used = mark2;
    }
    ar.used = mark;
  }
  ar.used = mark0;
  return PTSBE_OK;
}

ptsbe_status_t collect_events(Plan& p, std::vector<EventPair>& evs) {
  for (auto& e : evs) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e.a, e.b));
    p.join_ms += ms;
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  evs.clear();
  for (auto& e : p.sweep_evs) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e.first, e.second));
    p.sweep_ms += ms;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  p.sweep_evs.clear();
  for (auto& e : p.vm_evs) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e.first, e.second));
    p.vm_ms += ms;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  p.vm_evs.clear();
  return PTSBE_OK;
}

}  // namespace

extern "C" {

const char* ptsbe_last_error(void) { return ptsbe::g_last_error.c_str(); }

// Elements per trajectory and batch assumed by the automatic method choice.
constexpr double kAutoElems = 64.0;

ptsbe_status_t ptsbe_plan(const ptsbe_circuit_t* c, const ptsbe_plan_opts_t* o, ptsbe_plan_t* out) {
  if (!c || !o || !out) return fail(PTSBE_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (c->n_qubits < 1 || c->n_qubits > ptsbe::kMaxQubits) return fail(PTSBE_ERR_INVALID_ARG, "n_qubits out of range");
  if (c->n_gates < 0 || (c->n_gates > 0 && (!c->gate_arity || !c->gate_qubits || !c->gate_mats)))
    return fail(PTSBE_ERR_INVALID_ARG, "bad gate arrays");
  if (c->n_channels < 0 || c->n_sites < 0) return fail(PTSBE_ERR_INVALID_ARG, "bad channel/site counts");
  if (c->n_sites > 0 && (!c->site_gate || !c->site_qubits || !c->site_channel))
    return fail(PTSBE_ERR_INVALID_ARG, "bad site arrays");
  if (c->n_channels > 0 && (!c->ch_arity || !c->ch_nkraus || !c->ch_kraus))
    return fail(PTSBE_ERR_INVALID_ARG, "bad channel arrays");
  if (o->n_batches < 1 || !o->batch_sizes) return fail(PTSBE_ERR_INVALID_ARG, "no batches");
  if (o->precision != PTSBE_C64 && o->precision != PTSBE_SPLIT_BF16 && o->precision != PTSBE_SPLIT_F16)
    return fail(PTSBE_ERR_INVALID_ARG, "precision must be PTSBE_C64, PTSBE_SPLIT_BF16 or PTSBE_SPLIT_F16");
  auto p = new Plan();
  std::unique_ptr<Plan> guard(p);
  p->n = c->n_qubits;
  p->NW = (p->n + 63) / 64;
  p->precision = o->precision;
  p->device = o->device;
  p->hypersamples = std::max(1, o->hypersamples);
  p->path_seed = o->path_seed;
  int sum = 0;
  for (int j = 0; j < o->n_batches; ++j) {
    int b = o->batch_sizes[j];
    if (b < 1) return fail(PTSBE_ERR_INVALID_ARG, "batch size < 1");
    if (b > ptsbe::kMaxBatch) return fail(PTSBE_ERR_UNSUPPORTED, "batch size > 30");
    sum += b;
    p->batch_sizes.push_back(b);
  }
  if (sum != p->n) return fail(PTSBE_ERR_INVALID_ARG, "batch sizes must sum to n_qubits");
  // gates
  std::vector<bool> touched(p->n, false);
  size_t moff = 0;
  for (int g = 0; g < c->n_gates; ++g) {
    int ar = c->gate_arity[g];
    if (ar > 2) return fail(PTSBE_ERR_UNSUPPORTED, "gate arity > 2");
    if (ar < 1) return fail(PTSBE_ERR_INVALID_ARG, "gate arity < 1");
    std::array<int, 2> q = {c->gate_qubits[2 * g], ar == 2 ? c->gate_qubits[2 * g + 1] : -1};
    for (int a = 0; a < ar; ++a) {
      if (q[a] < 0 || q[a] >= p->n) return fail(PTSBE_ERR_INVALID_ARG, "gate qubit out of range");
      touched[q[a]] = true;
    }
    if (ar == 2 && q[0] == q[1]) return fail(PTSBE_ERR_INVALID_ARG, "two-qubit gate on one qubit");
    int d = 1 << ar;
    std::array<double, 32> m{};
    for (int i = 0; i < 2 * d * d; ++i) {
      m[i] = c->gate_mats[moff + i];
      if (!std::isfinite(m[i])) return fail(PTSBE_ERR_INVALID_ARG, "non-finite gate entry");
    }
    moff += 2 * d * d;
    p->arity.push_back(ar);
    p->qubits.push_back(q);
    p->mats.push_back(m);
  }
  p->n_user_gates = c->n_gates;
  // untouched qubits get an explicit identity so that every output leg is on a gate
  for (int q = 0; q < p->n; ++q)
    if (!touched[q]) {
      std::array<double, 32> m{};
      m[0] = 1.0; m[6] = 1.0;
      p->arity.push_back(1);
      p->qubits.push_back({q, -1});
      p->mats.push_back(m);
    }
  p->G = (int)p->arity.size();
  // channels
  size_t koff = 0, poff = 0;
  std::vector<char> ch_unitary;
  for (int ch = 0; ch < c->n_channels; ++ch) {
    int ar = c->ch_arity[ch], nk = c->ch_nkraus[ch];
    if (ar < 1 || ar > 2) return fail(PTSBE_ERR_UNSUPPORTED, "channel arity must be 1 or 2");
    if (nk < 1 || nk > 256) return fail(PTSBE_ERR_INVALID_ARG, "channel Kraus count out of range");
    int d = 1 << ar;
    std::vector<std::vector<cd>> K(nk, std::vector<cd>(d * d));
    for (int k = 0; k < nk; ++k)
      for (int i = 0; i < d * d; ++i) {
        const size_t o = koff + (size_t)k * 2 * d * d + 2 * (size_t)i;
        K[k][i] = cd(c->ch_kraus[o], c->ch_kraus[o + 1]);
        if (!std::isfinite(K[k][i].real()) || !std::isfinite(K[k][i].imag()))
          return fail(PTSBE_ERR_INVALID_ARG, "non-finite Kraus entry");
      }
    koff += (size_t)nk * 2 * d * d;
    // completeness: sum_k K^dag K = I
    for (int r = 0; r < d; ++r)
      for (int cc = 0; cc < d; ++cc) {
        cd acc = 0.0;
        for (int k = 0; k < nk; ++k)
          for (int x = 0; x < d; ++x) acc += std::conj(K[k][x * d + r]) * K[k][x * d + cc];
        if (std::abs(acc - (r == cc ? 1.0 : 0.0)) > 1e-10)
          return fail(PTSBE_ERR_INVALID_ARG, "channel " + std::to_string(ch) + " is not trace preserving");
      }
    std::vector<double> q(nk);
    double qs = 0;
    for (int k = 0; k < nk; ++k) {
      double given = c->ch_prob ? c->ch_prob[poff + k] : -1.0;
      if (given >= 0) {
        q[k] = given;
      } else {
        double tr = 0;
        for (int i = 0; i < d * d; ++i) tr += std::norm(K[k][i]);
        q[k] = tr / d;
      }
      qs += q[k];
    }
    poff += nk;
    if (std::abs(qs - 1.0) > 1e-10) return fail(PTSBE_ERR_INVALID_ARG, "Kraus probabilities do not sum to 1");
    std::vector<std::array<double, 32>> ops(nk);
    for (int k = 0; k < nk; ++k) {
      if (!(q[k] > 0)) {
        double nrm = 0;
        for (auto& v : K[k]) nrm += std::norm(v);
        if (nrm > 0) return fail(PTSBE_ERR_INVALID_ARG, "zero probability for a non-zero Kraus operator");
      }
      double sc = q[k] > 0 ? 1.0 / std::sqrt(q[k]) : 0.0;
      for (int i = 0; i < d * d; ++i) {
        ops[k][2 * i] = K[k][i].real() * sc;
        ops[k][2 * i + 1] = K[k][i].imag() * sc;
      }
    }
    // an inserted operator K / sqrt(q) that is unitary leaves the norm alone and
    // can be undone by its adjoint (the windowed adjoint pass and the light cone
    // use that)
    bool ch_unit = true;
    for (int k = 0; k < nk; ++k) {
      if (!(q[k] > 0)) continue;
      for (int r = 0; r < d; ++r)
        for (int cc = 0; cc < d; ++cc) {
          cd acc = 0;
          for (int x = 0; x < d; ++x)
            acc += std::conj(cd(ops[k][2 * (x * d + r)], ops[k][2 * (x * d + r) + 1])) *
                   cd(ops[k][2 * (x * d + cc)], ops[k][2 * (x * d + cc) + 1]);
          if (std::abs(acc - (r == cc ? 1.0 : 0.0)) > 1e-9) p->inserted_unitary = false;
          if (std::abs(acc - (r == cc ? 1.0 : 0.0)) > ptsbe::kUnitaryTol) ch_unit = false;
        }
    }
    ch_unitary.push_back(ch_unit ? 1 : 0);
    p->ch_ops.push_back(ops);
    p->ch_q.push_back(q);
    p->max_kraus = std::max(p->max_kraus, nk);
  }
  // sites
  p->gate_sites.assign(p->G, {});
  for (int s = 0; s < c->n_sites; ++s) {
    int g = c->site_gate[s], ch = c->site_channel[s];
    if (g < 0 || g >= c->n_gates) return fail(PTSBE_ERR_INVALID_ARG, "site gate out of range");
    if (ch < 0 || ch >= c->n_channels) return fail(PTSBE_ERR_INVALID_ARG, "site channel out of range");
    std::array<int, 2> sq = {c->site_qubits[2 * s], c->site_qubits[2 * s + 1]};
    int ar = c->ch_arity[ch];
    if ((ar == 1 && sq[1] != -1) || (ar == 2 && sq[1] < 0)) return fail(PTSBE_ERR_INVALID_ARG, "site qubits do not match channel arity");
    for (int a = 0; a < ar; ++a) {
      bool ok = false;
      for (int b = 0; b < p->arity[g]; ++b) ok |= p->qubits[g][b] == sq[a];
      if (!ok) return fail(PTSBE_ERR_INVALID_ARG, "site qubit is not a qubit of its gate");
    }
    if (ar == 2 && sq[0] == sq[1]) return fail(PTSBE_ERR_INVALID_ARG, "two-qubit site on one qubit");
    p->site_gate.push_back(g);
    p->site_channel.push_back(ch);
    p->site_qubits.push_back(sq);
    p->gate_sites[g].push_back(s);
  }
  p->S = c->n_sites;
  // light cone of doubled networks: which gates are unitary for every trajectory
  if (o->light_cone != 0 && o->light_cone != 1) return fail(PTSBE_ERR_INVALID_ARG, "light_cone must be 0 or 1");
  p->light_cone = o->light_cone == 1;
  if (o->subtree_reuse != 0 && o->subtree_reuse != 1)
    return fail(PTSBE_ERR_INVALID_ARG, "subtree_reuse must be 0 or 1");
  p->subtree_reuse = o->subtree_reuse == 1;
  if (o->sample_kernel != 0 && o->sample_kernel != 1)
    return fail(PTSBE_ERR_INVALID_ARG, "sample_kernel must be 0 or 1");
  p->sample_kernel = o->sample_kernel;
  if (o->max_part_rank != 0 && (o->max_part_rank < 4 || o->max_part_rank > 31))
    return fail(PTSBE_ERR_INVALID_ARG, "max_part_rank must be 0 or 4..31");
  p->max_part_rank = o->max_part_rank ? o->max_part_rank : 31;
  p->gate_unitary.assign((size_t)p->G, 1);
  for (int g = 0; g < p->G; ++g) {
    const int d = 1 << p->arity[(size_t)g];
    const auto& m = p->mats[(size_t)g];
    for (int r = 0; r < d; ++r)
      for (int cc = 0; cc < d; ++cc) {
        cd acc = 0;
        for (int x = 0; x < d; ++x)
          acc += std::conj(cd(m[2 * (x * d + r)], m[2 * (x * d + r) + 1])) * cd(m[2 * (x * d + cc)], m[2 * (x * d + cc) + 1]);
        if (std::abs(acc - (r == cc ? 1.0 : 0.0)) > ptsbe::kUnitaryTol) p->gate_unitary[(size_t)g] = 0;
      }
    for (int st : p->gate_sites[(size_t)g])
      if (!ch_unitary[(size_t)p->site_channel[(size_t)st]]) p->gate_unitary[(size_t)g] = 0;
  }
  // statevector schedule: every gate in circuit order, in place on qubit positions
  if (p->n <= ptsbe::kSvMaxQubits) {
    for (int g = 0; g < p->G; ++g) {
      ptsbe::AbsorbStep st{};
      st.gate = g;
      st.rA = st.rC = p->n;
      const int ar = p->arity[g];
      std::vector<std::pair<int, int>> ins, outs;   // (position, weight)
      for (int a = 0; a < ar; ++a) {
        const int q = p->qubits[g][a];
        outs.push_back({q, ar == 2 ? (a == 0 ? 8 : 4) : 2});
        ins.push_back({q, ar == 2 ? (a == 0 ? 2 : 1) : 1});
      }
      std::sort(ins.begin(), ins.end());
      std::sort(outs.begin(), outs.end());
      st.nK = st.nN = ar;
      for (int i = 0; i < ar; ++i) {
        st.kpos[i] = ins[i].first; st.kw[i] = ins[i].second;
        st.npos[i] = outs[i].first; st.nw[i] = outs[i].second;
      }
      for (int k = 0; k < (1 << st.nK); ++k) {
        st.koff[k] = 0; st.kB[k] = 0; st.noff[k] = 0; st.nB[k] = 0;
        for (int i = 0; i < st.nK; ++i)
          if ((k >> i) & 1) {
            st.koff[k] += 1u << st.kpos[i]; st.kB[k] += st.kw[i];
            st.noff[k] += 1u << st.npos[i]; st.nB[k] += st.nw[i];
          }
      }
      p->sv_steps.push_back(st);
    }
  }
  // contraction method and path
  if (o->method < PTSBE_METHOD_AUTO || o->method > PTSBE_METHOD_STATEVECTOR)
    return fail(PTSBE_ERR_INVALID_ARG, "unknown method");
  std::string err;
  bool sv_fits = p->n <= ptsbe::kSvMaxQubits;   // the statevector sampler takes batches of <= 12 qubits
  for (int b : p->batch_sizes) sv_fits = sv_fits && b <= 12;
  bool use_sv = o->method == PTSBE_METHOD_STATEVECTOR || (o->method == PTSBE_METHOD_AUTO && p->n <= 20 && sv_fits);
  if (!use_sv) {
    const bool net_ok = ptsbe::build_batch_plans(*p, err);
    if (!net_ok) {
      if (o->method == PTSBE_METHOD_NETWORK || !sv_fits) return fail(PTSBE_ERR_UNSUPPORTED, err);
      use_sv = true;
    } else if (o->method == PTSBE_METHOD_AUTO && sv_fits) {
      // both methods run: a cost per trajectory in HBM-byte equivalents.  The
      // network method pays its per-trajectory parts plus, per element, the left
      // part and the join, counted for kAutoElems elements per batch (the shot
      // count is not known here) at 25 flops per byte on MFMA joins and 0.5 on
      // the generic join (measured on the ragged mix: generic joins of crossing
      // 7..10 ran near 1 TFLOP/s); the statevector method pays its window passes
      // and marginal reads.
      double net = 0.0;
      for (const auto& bp : p->batches) {
        const int lkb = (int)bp.lk.size();
        const bool mfma = bp.doubled ? ptsbe::qform_supported(lkb) : ptsbe::ketjoin_supported(lkb);
        net += bp.right.bytes + kAutoElems * (bp.left.flops / 25.0 + bp.join_flops_per_elem / (mfma ? 25.0 : 0.5));
      }
      const double sv = (16.0 * ptsbe::count_sv_windows(*p, ptsbe::kFuseMax) + 8.0 * p->batch_sizes.size()) *
                        std::ldexp(1.0, p->n);
      use_sv = sv < net;
    }
  }
  if (use_sv) {
    if (p->n > ptsbe::kSvMaxQubits) return fail(PTSBE_ERR_UNSUPPORTED, "the statevector method needs n_qubits <= 30");
    for (int b : p->batch_sizes)
      if (b > 12) return fail(PTSBE_ERR_UNSUPPORTED, "the statevector method samples batches of at most 12 qubits");
    p->method = PTSBE_METHOD_STATEVECTOR;
    ptsbe::build_sv_batches(*p);
  }
  // device constants
  std::vector<ptsbe::DeviceGate> dg(p->G);
  std::vector<int32_t> site_list;
  std::vector<float2> site_ops((size_t)std::max(1, p->S) * p->max_kraus * 16, make_float2(0.f, 0.f));
  for (int g = 0; g < p->G; ++g) {
    const int ar = p->arity[g], d = 1 << ar;
    std::vector<int> gq = {p->qubits[g][0]};
    if (ar == 2) gq.push_back(p->qubits[g][1]);
    std::vector<cd> m(d * d), t(d * d), e(d * d);
    for (int i = 0; i < d * d; ++i) m[i] = cd(p->mats[g][2 * i], p->mats[g][2 * i + 1]);
    for (int i = 0; i < 16; ++i) dg[g].raw[i] = make_float2(0.f, 0.f);
    for (int i = 0; i < d * d; ++i) dg[g].raw[i] = make_float2((float)m[i].real(), (float)m[i].imag());
    dg[g].site_begin = (int)site_list.size();
    for (int s : p->gate_sites[g]) {
      site_list.push_back(s);
      const int ch = p->site_channel[s];
      const int car = c->ch_arity[ch];
      std::vector<int> sq = {p->site_qubits[s][0]};
      if (car == 2) sq.push_back(p->site_qubits[s][1]);
      const int dk = 1 << car;
      for (int k = 0; k < (int)p->ch_ops[ch].size(); ++k) {
        std::vector<cd> op(dk * dk);
        for (int i = 0; i < dk * dk; ++i) op[i] = cd(p->ch_ops[ch][k][2 * i], p->ch_ops[ch][k][2 * i + 1]);
        embed_op(op.data(), sq, gq, e.data());
        for (int i = 0; i < d * d; ++i)
          site_ops[((size_t)s * p->max_kraus + k) * 16 + i] = make_float2((float)e[i].real(), (float)e[i].imag());
        if (k == 0) {   // default branch: every site at Kraus index 0, later sites on the left
          matmul(e.data(), m.data(), t.data(), d);
          m = t;
        }
      }
    }
    dg[g].site_end = (int)site_list.size();
    dg[g].arity = ar;
    for (int i = 0; i < 16; ++i) dg[g].def[i] = make_float2(0.f, 0.f);
    for (int i = 0; i < d * d; ++i) dg[g].def[i] = make_float2((float)m[i].real(), (float)m[i].imag());
  }
  for (auto& bp : p->batches)
    for (ptsbe::PartPlan* pp : {&bp.left, &bp.right, &bp.left_resume})
      ptsbe::build_segments(pp->steps, pp->segs, p->fused);
  if (p->method == PTSBE_METHOD_STATEVECTOR) {
    ptsbe::build_sv_schedule(*p);
    ptsbe::build_sv_ops(*p);
  }
  std::vector<ptsbe::AbsorbStep> steps;
  std::vector<int64_t> tables;
  for (auto& bp : p->batches) {
    p->part_step_off.push_back((int64_t)steps.size());
    steps.insert(steps.end(), bp.left.steps.begin(), bp.left.steps.end());
    p->part_step_off.push_back((int64_t)steps.size());
    steps.insert(steps.end(), bp.right.steps.begin(), bp.right.steps.end());
    p->part_step_off.push_back((int64_t)steps.size());
    steps.insert(steps.end(), bp.left_resume.steps.begin(), bp.left_resume.steps.end());
    Plan::JoinDev jd{};
    auto put = [&](const ptsbe::SplitTable& t, int64_t& lo, int64_t& hi) {
      lo = (int64_t)tables.size();
      tables.insert(tables.end(), t.lo.begin(), t.lo.end());
      hi = (int64_t)tables.size();
      tables.insert(tables.end(), t.hi.begin(), t.hi.end());
    };
    put(bp.v_row, jd.vr_lo, jd.vr_hi);
    put(bp.v_col, jd.vc_lo, jd.vc_hi);
    put(bp.t_x, jd.tx_lo, jd.tx_hi);
    put(bp.t_k, jd.tk_lo, jd.tk_hi);
    put(bp.t_b, jd.tb_lo, jd.tb_hi);
    put(bp.o_x, jd.ox_lo, jd.ox_hi);
    put(bp.o_b, jd.ob_lo, jd.ob_hi);
    p->join_dev.push_back(jd);
    Plan::JoinDev jr = jd;   // the resumed left part may order its legs differently
    put(bp.v_row_r.lo.empty() ? bp.v_row : bp.v_row_r, jr.vr_lo, jr.vr_hi);
    put(bp.v_col_r.lo.empty() ? bp.v_col : bp.v_col_r, jr.vc_lo, jr.vc_hi);
    p->join_dev_r.push_back(jr);
  }
  if (steps.empty()) steps.push_back(ptsbe::AbsorbStep{});
  if (site_list.empty()) site_list.push_back(0);
  size_t bytes = dg.size() * sizeof(ptsbe::DeviceGate) + site_list.size() * 4 + site_ops.size() * sizeof(float2) +
                 steps.size() * sizeof(ptsbe::AbsorbStep) + tables.size() * 8 +
                 p->fused.size() * sizeof(ptsbe::FusedStep);
  p->device_bytes = (int64_t)bytes;
  if (o->device_budget_bytes && bytes > o->device_budget_bytes)
    return fail(PTSBE_ERR_OUT_OF_MEMORY, "plan constants exceed device_budget_bytes");
  if (p->device < 0) {   // host-only plan: path and pre-sampling only, no device constants
    *out = reinterpret_cast<ptsbe_plan_t>(guard.release());
    return PTSBE_OK;
  }
  HIP_TRY(hipSetDevice(p->device));
  HIP_TRY(hipMalloc(&p->d_gates, dg.size() * sizeof(ptsbe::DeviceGate)));
  HIP_TRY(hipMalloc(&p->d_gate_site_list, site_list.size() * 4));
  HIP_TRY(hipMalloc(&p->d_site_ops, site_ops.size() * sizeof(float2)));
  HIP_TRY(hipMalloc(&p->d_steps, steps.size() * sizeof(ptsbe::AbsorbStep)));
  HIP_TRY(hipMalloc(&p->d_tables, tables.size() * 8));
  if (!p->fused.empty()) {
    HIP_TRY(hipMalloc(&p->d_fused, p->fused.size() * sizeof(ptsbe::FusedStep)));
    HIP_TRY(hipMemcpy(p->d_fused, p->fused.data(), p->fused.size() * sizeof(ptsbe::FusedStep),
                      hipMemcpyHostToDevice));
  }
  if (p->method == PTSBE_METHOD_STATEVECTOR) {
    for (int i = 0; i < 3; ++i) {
      std::vector<ptsbe::RgWindow> w(p->sv_win[i].size());
      for (size_t k = 0; k < w.size(); ++k) {
        const ptsbe::Segment& sg = p->sv_win[i][k];
        w[k].np = sg.np;
        w[k].n_fs = sg.count;
        for (int q = 0; q < ptsbe::kFuseMax; ++q) w[k].P[q] = sg.P[q];
        w[k].fused_off = sg.fused_off;
      }
      HIP_TRY(hipMalloc(&p->d_rg_win[i], std::max<size_t>(1, w.size()) * sizeof(ptsbe::RgWindow)));
      HIP_TRY(hipMemcpy(p->d_rg_win[i], w.data(), w.size() * sizeof(ptsbe::RgWindow), hipMemcpyHostToDevice));
      if (!p->sv_ops_plain[i].empty()) {
        const auto& pw = p->sv_wins_plain[i];
        const auto& po = p->sv_ops_plain[i];
        HIP_TRY(hipMalloc(&p->d_sv_wins_plain[i], pw.size() * sizeof(ptsbe::SvWin)));
        HIP_TRY(hipMemcpy(p->d_sv_wins_plain[i], pw.data(), pw.size() * sizeof(ptsbe::SvWin), hipMemcpyHostToDevice));
        HIP_TRY(hipMalloc(&p->d_sv_ops_plain[i], po.size() * sizeof(ptsbe::SvOp)));
        HIP_TRY(hipMemcpy(p->d_sv_ops_plain[i], po.data(), po.size() * sizeof(ptsbe::SvOp), hipMemcpyHostToDevice));
      }
      const auto& so = p->sv_ops[i];
      if (!so.empty()) {
        HIP_TRY(hipMalloc(&p->d_sv_ops[i], so.size() * sizeof(ptsbe::SvOp)));
        HIP_TRY(hipMemcpy(p->d_sv_ops[i], so.data(), so.size() * sizeof(ptsbe::SvOp), hipMemcpyHostToDevice));
      }
      const auto& cl = p->sv_cl[i];
      HIP_TRY(hipMalloc(&p->d_sv_cl[i], std::max<size_t>(1, cl.size()) * sizeof(ptsbe::ClusterDesc)));
      if (!cl.empty())
        HIP_TRY(hipMemcpy(p->d_sv_cl[i], cl.data(), cl.size() * sizeof(ptsbe::ClusterDesc), hipMemcpyHostToDevice));
    }
  }
  if (!p->sv_steps.empty()) {
    HIP_TRY(hipMalloc(&p->d_sv_steps, p->sv_steps.size() * sizeof(ptsbe::AbsorbStep)));
    HIP_TRY(hipMemcpy(p->d_sv_steps, p->sv_steps.data(), p->sv_steps.size() * sizeof(ptsbe::AbsorbStep),
                      hipMemcpyHostToDevice));
  }
  HIP_TRY(hipMemcpy(p->d_gates, dg.data(), dg.size() * sizeof(ptsbe::DeviceGate), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->d_gate_site_list, site_list.data(), site_list.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->d_site_ops, site_ops.data(), site_ops.size() * sizeof(float2), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->d_steps, steps.data(), steps.size() * sizeof(ptsbe::AbsorbStep), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(p->d_tables, tables.data(), tables.size() * 8, hipMemcpyHostToDevice));
  *out = reinterpret_cast<ptsbe_plan_t>(guard.release());
  return PTSBE_OK;
}

void ptsbe_plan_destroy(ptsbe_plan_t plan) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return;
  for (auto& e : p->sweep_evs) {   // events of a profiled call that returned early
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto& e : p->vm_evs) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto& e : p->win_evs) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  if (p->d_gates) (void)hipFree(p->d_gates);
  if (p->d_gate_site_list) (void)hipFree(p->d_gate_site_list);
  if (p->d_site_ops) (void)hipFree(p->d_site_ops);
  if (p->d_steps) (void)hipFree(p->d_steps);
  if (p->d_tables) (void)hipFree(p->d_tables);
  if (p->d_sv_steps) (void)hipFree(p->d_sv_steps);
  if (p->d_fused) (void)hipFree(p->d_fused);
  for (auto* w : p->d_rg_win)
    if (w) (void)hipFree(w);
  for (auto* c : p->d_sv_cl)
    if (c) (void)hipFree(c);
  for (auto* o : p->d_sv_ops)
    if (o) (void)hipFree(o);
  for (auto* o : p->d_sv_ops_plain)
    if (o) (void)hipFree(o);
  for (auto* o : p->d_sv_wins_plain)
    if (o) (void)hipFree(o);
  delete p;
}

ptsbe_status_t ptsbe_plan_query(ptsbe_plan_t plan, ptsbe_plan_info_t* out) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p || !out) return fail(PTSBE_ERR_INVALID_ARG, "null argument");
  out->n_qubits = p->n;
  out->n_gates = p->G;
  out->n_sites = p->S;
  out->n_batches = (int32_t)p->batches.size();
  out->n_words = p->NW;
  out->max_kraus = p->max_kraus;
  out->plan_device_bytes = p->device_bytes;
  out->method = p->method;
  out->sv_windows = p->method == PTSBE_METHOD_STATEVECTOR ? (int32_t)p->sv_segs.size() : 0;
  for (int i = 0; i < 3; ++i)
    out->sv_windows_by_size[i] = p->method == PTSBE_METHOD_STATEVECTOR ? (int32_t)p->sv_win[i].size() : 0;
  out->sv_clusters = 0;
  out->sv_cluster_steps = 0;
  if (p->method == PTSBE_METHOD_STATEVECTOR)
    for (const auto& cd : p->sv_cl[2]) {
      ++out->sv_clusters;
      out->sv_cluster_steps += cd.len;
    }
  out->precision = p->precision;
  out->light_cone = p->light_cone ? 1 : 0;
  out->subtree_reuse = p->subtree_reuse ? 1 : 0;
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_plan_sv_schedule(ptsbe_plan_t plan, int32_t window_qubits, int32_t* gate_order,
                                      int32_t* window_first, int32_t* window_qubits_out, int32_t* n_windows_out) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(PTSBE_ERR_INVALID_ARG, "null plan");
  if (p->method != PTSBE_METHOD_STATEVECTOR) return fail(PTSBE_ERR_INVALID_ARG, "not a statevector-method plan");
  const int w = window_qubits - ptsbe::kSvWindowMin;
  if (w < 0 || w > 2) return fail(PTSBE_ERR_INVALID_ARG, "window_qubits must be 10, 11 or 12");
  const auto& segs = p->sv_win[w];
  int32_t pos = 0;
  for (size_t k = 0; k < segs.size(); ++k) {
    const ptsbe::Segment& sg = segs[k];
    if (window_first) window_first[k] = pos;
    for (int i = 0; i < sg.count; ++i, ++pos)
      if (gate_order) gate_order[pos] = p->fused[sg.fused_off + i].gate;
    if (window_qubits_out)
      for (int q = 0; q < ptsbe::kFuseMax; ++q) window_qubits_out[12 * k + q] = q < sg.np ? sg.P[q] : -1;
  }
  if (window_first) window_first[segs.size()] = pos;
  if (n_windows_out) *n_windows_out = (int32_t)segs.size();
  return PTSBE_OK;
}


ptsbe_status_t ptsbe_plan_right_sites(ptsbe_plan_t plan, int32_t j, int32_t* sites, int32_t* n_sites_out) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(PTSBE_ERR_INVALID_ARG, "null plan");
  if (p->method == PTSBE_METHOD_STATEVECTOR) return fail(PTSBE_ERR_INVALID_ARG, "statevector-method plan");
  if (j < 0 || j >= (int)p->batches.size()) return fail(PTSBE_ERR_INVALID_ARG, "batch index out of range");
  const std::vector<int32_t> v = right_sites(*p, p->batches[(size_t)j]);
  if (sites) std::copy(v.begin(), v.end(), sites);
  if (n_sites_out) *n_sites_out = (int32_t)v.size();
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_plan_join_tiling(ptsbe_plan_t plan, int32_t j, int64_t* t_read, int64_t* o_read,
                                      int32_t* w_of, int64_t* o_write, int64_t* t_hi, int64_t* o_hi,
                                      int32_t* n_hi, int64_t* x_t, int64_t* x_o, int32_t* n_x) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(PTSBE_ERR_INVALID_ARG, "null plan");
  if (p->method == PTSBE_METHOD_STATEVECTOR) return fail(PTSBE_ERR_INVALID_ARG, "statevector-method plan");
  if (j < 0 || j >= (int)p->batches.size()) return fail(PTSBE_ERR_INVALID_ARG, "batch index out of range");
  if (!t_read || !o_read || !w_of || !o_write || !t_hi || !o_hi || !n_hi || !x_t || !x_o || !n_x)
    return fail(PTSBE_ERR_INVALID_ARG, "null argument");
  const ptsbe::BatchPlan& bp = p->batches[(size_t)j];
  ptsbe::GemvTiling g{};
  if (bp.doubled || bp.xb.size() > 1 || !ptsbe::make_gemv_tiling(bp, g))
    return fail(PTSBE_ERR_UNSUPPORTED, "batch takes no GEMV tiling");
  for (int s = 0; s < 12; ++s) {
    t_read[s] = g.t_off[s];
    o_read[s] = g.o_read[s];
    w_of[s] = g.w_of[s];
    o_write[s] = g.o_off[s];
  }
  *n_hi = g.n_hi;
  for (int h = 0; h < g.n_hi; ++h) {
    t_hi[h] = g.t_hi[h];
    o_hi[h] = g.o_hi[h];
  }
  const int nx = (int)bp.xT.size();
  auto off = [](const ptsbe::SplitTable& t, int i) -> int64_t {
    return i < t.lo_bits ? t.lo[(size_t)1 << i] : t.hi[(size_t)1 << (i - t.lo_bits)];
  };
  for (int i = 0; i < nx; ++i) {
    x_t[i] = off(bp.t_x, i);
    x_o[i] = off(bp.o_x, i);
  }
  *n_x = nx;
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_plan_batch_info(ptsbe_plan_t plan, int32_t j, ptsbe_batch_info_t* out) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p || !out) return fail(PTSBE_ERR_INVALID_ARG, "null argument");
  if (j < 0 || j >= (int)p->batches.size()) return fail(PTSBE_ERR_INVALID_ARG, "batch index out of range");
  const auto& bp = p->batches[j];
  out->start = bp.start;
  out->size = bp.size;
  out->doubled = bp.doubled;
  out->n_left_steps = (int32_t)bp.left.steps.size();
  out->n_right_steps = (int32_t)bp.right.steps.size();
  out->n_resume_steps = j >= 1 ? (int32_t)bp.left_resume.steps.size() : 0;
  out->left_rank = (int32_t)bp.left.labels.size();
  out->right_rank = (int32_t)bp.right.labels.size();
  out->left_peak_rank = bp.left.peak;
  out->right_peak_rank = bp.right.peak;
  out->join_rows_log2 = (int32_t)bp.xb.size();
  out->crossing = (int32_t)bp.lk.size();
  out->flops_per_traj = bp.right.flops;
  out->flops_per_elem = bp.left.flops + bp.join_flops_per_elem;
  out->join_flops_per_elem = bp.join_flops_per_elem;
  out->bytes_per_traj = bp.right.bytes;
  out->n_right_launches = 0;
  out->n_right_fused_steps = 0;
  out->right_longest_run = 0;
  if (!part_uses_vm(bp.right))
    for (const ptsbe::Segment& sg : bp.right.segs) {
      ++out->n_right_launches;
      if (sg.fused) {
        out->n_right_fused_steps += sg.count;
        out->right_longest_run = std::max(out->right_longest_run, sg.count);
      }
    }
  out->kept_gates = bp.kept_gates;
  out->slice_bits = bp.slice_bits;
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_sample_trajectories(ptsbe_plan_t plan, uint64_t seed, int64_t n_unique, int64_t max_draws,
                                         uint8_t* kraus_idx, int64_t* mult, double* log_q, int64_t* n_unique_out,
                                         int64_t* n_draws_out) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(PTSBE_ERR_INVALID_ARG, "null plan");
  if (n_unique < 0 || max_draws < 0) return fail(PTSBE_ERR_INVALID_ARG, "negative count");
  if (n_unique > 0 && (!kraus_idx || !mult)) return fail(PTSBE_ERR_INVALID_ARG, "null output");
  const int S = p->S;
  std::vector<std::vector<double>> cum(S);
  for (int s = 0; s < S; ++s) {
    const auto& q = p->ch_q[p->site_channel[s]];
    double acc = 0;
    for (double v : q) { acc += v; cum[s].push_back(acc); }
  }
  // number of distinct error sets that can occur at all (capped): sampling stops
  // once every one of them has appeared
  double possible = 1.0;
  for (int s = 0; s < S; ++s) {
    int nz = 0;
    for (double v : p->ch_q[p->site_channel[s]]) nz += v > 0;
    possible *= nz;
    if (possible > 9e18) break;
  }
  const int64_t target = (int64_t)std::min<double>((double)n_unique, possible);
  std::unordered_map<std::string, int64_t> seen;
  std::string row(S, '\0');
  int64_t found = 0, d = 0;
  for (; d < max_draws && found < target; ++d) {
    for (int s = 0; s < S; ++s) {
      const double u = ptsbe::philox_uniform(seed, 1u, (uint32_t)d, (uint32_t)s, (uint32_t)(d >> 32), 0u);
      const auto& cs = cum[s];
      const auto& q = p->ch_q[p->site_channel[s]];
      int k = -1;
      for (size_t i = 0; i < cs.size(); ++i)
        if (cs[i] > u) { k = (int)i; break; }
      if (k < 0)
        for (int i = (int)q.size() - 1; i >= 0; --i)
          if (q[i] > 0) { k = i; break; }
      row[s] = (char)(uint8_t)k;
    }
    auto it = seen.find(row);
    if (it != seen.end()) {
      mult[it->second] += 1;
    } else {
      seen.emplace(row, found);
      std::memcpy(kraus_idx + found * S, row.data(), S);
      mult[found] = 1;
      if (log_q) {
        double lq = 0;
        for (int s = 0; s < S; ++s) lq += std::log(p->ch_q[p->site_channel[s]][(uint8_t)row[s]]);
        log_q[found] = lq;
      }
      ++found;
    }
  }
  if (n_unique_out) *n_unique_out = found;
  if (n_draws_out) *n_draws_out = d;
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_contract_workspace_size(ptsbe_plan_t plan, int32_t j, int64_t E, int64_t n_elems,
                                             size_t* bytes) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p || !bytes) return fail(PTSBE_ERR_INVALID_ARG, "null argument");
  if (j < 0 || j >= (int)p->batches.size()) return fail(PTSBE_ERR_INVALID_ARG, "batch index out of range");
  if (p->method == PTSBE_METHOD_STATEVECTOR) {
    *bytes = ptsbe::sv_contract_workspace(*p, j, E, n_elems);
    return PTSBE_OK;
  }
  const auto& bp = p->batches[j];
  // a sliced last batch also holds the jobs' prefix words with the slice bits and,
  // per element, the amplitude sum and one slice's amplitudes
  const size_t sl_traj = bp.slice_bits ? (size_t)p->NW * 8 : 0;
  const size_t sl_elem = bp.slice_bits ? ((size_t)16 << bp.size) + (size_t)p->NW * 8 : 0;
  const size_t per_traj = join_traj_bytes(bp) + sl_traj;
  const size_t per_elem = ((size_t)8 << bp.left.labels.size()) + part_scratch_per_job(bp.left) + sl_elem;
  size_t t = (size_t)std::min<int64_t>(E, 256), e = (size_t)std::min<int64_t>(n_elems, 65536);
  *bytes = merged_bytes(*p, E) + (size_t)(E + 1) * 4 +
           2 * (std::max<size_t>(t, 1) * per_traj + std::max<size_t>(e, 1) * per_elem) + (1 << 20);
  return PTSBE_OK;
}

namespace {
// Persistent arrays of ptsbe_sample_shots (network method), in the order they are
// taken from the workspace: element and shot arrays of two generations, the left
// tensors of every element (prefix-tree reuse), scan scratch, counters and the
// merged gates.
struct SampleLayout {
  struct Elems { int32_t* traj; uint64_t* prefix; int32_t* off; int32_t* cnt; int32_t* ids; int32_t* parent; } el[2];
  float2* Vbuf[2];
  int32_t *shot_x, *child_cnt, *child_off, *scan_scratch, *counters;
  double *totals, *norms;
  int64_t* base;
  float2* merged;
};

bool take_sample_layout(const Plan& p, int64_t E, int64_t M, Arena& ar, SampleLayout& L) {
  const int64_t cap = std::max<int64_t>(E, M);
  int rVmax = 0;
  for (auto& bp : p.batches) rVmax = std::max<int>(rVmax, (int)bp.left_resume.labels.size());
  for (int k = 0; k < 2; ++k) L.Vbuf[k] = (float2*)ar.take((size_t)cap * ((size_t)8 << rVmax));
  for (int k = 0; k < 2; ++k) {
    L.el[k].parent = (int32_t*)ar.take((size_t)cap * 4);
    L.el[k].traj = (int32_t*)ar.take((size_t)cap * 4);
    L.el[k].prefix = (uint64_t*)ar.take((size_t)cap * 8 * p.NW);
    L.el[k].off = (int32_t*)ar.take((size_t)cap * 4);
    L.el[k].cnt = (int32_t*)ar.take((size_t)cap * 4);
    L.el[k].ids = (int32_t*)ar.take((size_t)std::max<int64_t>(M, 1) * 4);
  }
  L.shot_x = (int32_t*)ar.take((size_t)std::max<int64_t>(M, 1) * 4);
  L.child_cnt = (int32_t*)ar.take((size_t)cap * 4);
  L.child_off = (int32_t*)ar.take((size_t)cap * 4);
  L.totals = (double*)ar.take((size_t)cap * 8);
  L.base = (int64_t*)ar.take((size_t)E * 8);
  L.norms = (double*)ar.take((size_t)E * 8);
  L.scan_scratch = (int32_t*)ar.take(ptsbe::scan_scratch_bytes(cap));
  L.counters = (int32_t*)ar.take(64);
  L.merged = (float2*)ar.take(merged_bytes(p, E));
  bool ok = L.shot_x && L.child_cnt && L.child_off && L.totals && L.base && L.norms && L.scan_scratch &&
            L.counters && L.merged;
  for (int k = 0; k < 2; ++k)
    ok = ok && L.el[k].traj && L.el[k].prefix && L.el[k].off && L.el[k].cnt && L.el[k].ids && L.el[k].parent &&
         L.Vbuf[k];
  return ok;
}
}  // namespace

namespace {
size_t sample_persistent_bytes(const Plan& p, int64_t E, int64_t M) {
  const int64_t cap = std::max<int64_t>(E, M);
  size_t b = 0;
  auto add = [&](size_t x) { b += (x + 255) & ~(size_t)255; };
  for (int k = 0; k < 2; ++k) {
    add((size_t)cap * 4);                 // elem traj
    add((size_t)cap * 8 * p.NW);          // elem prefix
    add((size_t)cap * 4);                 // shot off
    add((size_t)cap * 4);                 // shot cnt
    add((size_t)std::max<int64_t>(M, 1) * 4);  // shot ids
  }
  add((size_t)std::max<int64_t>(M, 1) * 4);    // shot x
  add((size_t)cap * 4);                   // child cnt
  add((size_t)cap * 4);                   // child off
  add((size_t)cap * 8);                   // totals
  add((size_t)E * 8);                     // traj shot base
  add((size_t)E * 8);                     // norms
  add(ptsbe::scan_scratch_bytes(cap));
  add(64);                                // counters
  add((size_t)E * p.G * 16 * 8);          // merged gates
  int rVmax = 0;
  for (auto& bp : p.batches) rVmax = std::max<int>(rVmax, (int)bp.left_resume.labels.size());
  for (int k = 0; k < 2; ++k) {
    add((size_t)cap * ((size_t)8 << rVmax));   // left tensors
    add((size_t)cap * 4);                      // parents
  }
  return b;
}
}  // namespace

ptsbe_status_t ptsbe_sample_workspace_size(ptsbe_plan_t plan, int64_t E, int64_t total_shots, size_t* bytes) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p || !bytes) return fail(PTSBE_ERR_INVALID_ARG, "null argument");
  if (p->method == PTSBE_METHOD_STATEVECTOR) {
    *bytes = ptsbe::sv_sample_workspace(*p, E, total_shots);
    return PTSBE_OK;
  }
  size_t chunk = 0;
  for (auto& bp : p->batches) {
    const size_t per_traj = join_traj_bytes(bp);
    const size_t per_elem = ((size_t)8 << bp.left.labels.size()) + part_scratch_per_job(bp.left) +
                            ((size_t)4 << bp.size);
    chunk = std::max(chunk, 2 * (std::min<size_t>(E, 256) * per_traj + 65536 * per_elem));
  }
  *bytes = sample_persistent_bytes(*p, E, total_shots) + (size_t)(E + 1) * 4 + chunk + (1 << 20);
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_plan_chunking(ptsbe_plan_t plan, int32_t call, int64_t E, int64_t count,
                                   size_t workspace_bytes, int64_t* traj_per_chunk) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p || !traj_per_chunk) return fail(PTSBE_ERR_INVALID_ARG, "null argument");
  if (p->method != PTSBE_METHOD_NETWORK) return fail(PTSBE_ERR_INVALID_ARG, "chunking applies to network-method plans");
  if (call != 0 && call != 1) return fail(PTSBE_ERR_INVALID_ARG, "call must be 0 (contract) or 1 (sample)");
  if (E < 1 || count < 0) return fail(PTSBE_ERR_INVALID_ARG, "bad counts");
  Arena probe;                       // an arena without memory measures the layout
  probe.base = nullptr;
  probe.cap = ~(size_t)0 >> 1;
  if (call == 1) {
    SampleLayout L;
    take_sample_layout(*p, E, count, probe, L);
  } else {
    probe.take(merged_bytes(*p, E));
  }
  probe.take((size_t)(E + 1) * 4);   // trajectory ranges, taken first by every batch
  const size_t off = (probe.used + 255) & ~(size_t)255;
  const size_t avail = off >= workspace_bytes ? 0 : workspace_bytes - off;
  for (size_t j = 0; j < p->batches.size(); ++j) {
    const auto& bp = p->batches[j];
    const bool resume = call == 1 && j >= 1;
    const ChunkCaps c = chunk_caps(bp, resume ? bp.left_resume : bp.left, E, call == 0, call == 1, false, avail);
    traj_per_chunk[j] = (c.t_cap < 1 || c.e_cap < 1) ? 0 : c.t_cap;
  }
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_contract_batch(ptsbe_plan_t plan, int32_t j, const uint8_t* d_kraus_idx, int64_t E,
                                    const int32_t* d_elem_traj, const uint64_t* d_elem_prefix, int64_t n_elems,
                                    int32_t out_kind, void* d_out, double* d_elem_total, void* d_workspace,
                                    size_t workspace_bytes, void* stream) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(PTSBE_ERR_INVALID_ARG, "null plan");
  if (p->device < 0) return fail(PTSBE_ERR_INVALID_ARG, "plan was built without a device");
  if (j < 0 || j >= (int)p->batches.size()) return fail(PTSBE_ERR_INVALID_ARG, "batch index out of range");
  if (E < 1 || n_elems < 0) return fail(PTSBE_ERR_INVALID_ARG, "bad counts");
  if (n_elems == 0) return PTSBE_OK;
  if (!d_kraus_idx || !d_elem_traj || !d_elem_prefix || !d_out || !d_workspace)
    return fail(PTSBE_ERR_INVALID_ARG, "null device pointer");
  if (out_kind == PTSBE_OUT_AMPLITUDE && p->batches[j].doubled)
    return fail(PTSBE_ERR_INVALID_ARG, "amplitudes exist only for the last batch");
  if (out_kind != PTSBE_OUT_AMPLITUDE && out_kind != PTSBE_OUT_POPULATION)
    return fail(PTSBE_ERR_INVALID_ARG, "bad out_kind");
  HIP_TRY(hipSetDevice(p->device));
  hipStream_t s = (hipStream_t)stream;
  {
    // per-trajectory buffers are indexed through elem_traj: it must be sorted and in range
    std::vector<int32_t> et((size_t)n_elems);
    HIP_TRY(hipMemcpyAsync(et.data(), d_elem_traj, (size_t)n_elems * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int64_t e = 0; e < n_elems; ++e)
      if (et[e] < 0 || et[e] >= E || (e > 0 && et[e] < et[e - 1]))
        return fail(PTSBE_ERR_INVALID_ARG, "d_elem_traj must be non-decreasing trajectory ids in [0, E)");
  }
  if (p->method == PTSBE_METHOD_STATEVECTOR)
    return ptsbe::sv_contract_batch(*p, j, d_kraus_idx, E, d_elem_traj, d_elem_prefix, n_elems, out_kind, d_out,
                                    d_elem_total, d_workspace, workspace_bytes, s);
  Arena ar;
  ar.base = (char*)d_workspace;
  ar.cap = workspace_bytes;
  std::vector<uint8_t> h_kraus((size_t)E * p->site_gate.size());
  if (!h_kraus.empty()) {
    HIP_TRY(hipMemcpyAsync(h_kraus.data(), d_kraus_idx, h_kraus.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  BatchIO io;
  io.h_kraus = h_kraus.empty() ? nullptr : h_kraus.data();
  io.elem_traj = d_elem_traj;
  io.elem_prefix = d_elem_prefix;
  io.U = n_elems;
  if (out_kind == PTSBE_OUT_AMPLITUDE) io.amp_out = (float2*)d_out;
  else io.pop_out = (float*)d_out;
  io.totals = out_kind == PTSBE_OUT_POPULATION ? d_elem_total : nullptr;
  std::vector<EventPair> evs;
  float2* merged = (float2*)ar.take(merged_bytes(*p, E));
  if (!merged) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for the merged gates");
  HIP_TRY(ptsbe::launch_upv_merge(gate_ctx(*p, d_kraus_idx, nullptr), E, merged, s));
  ptsbe_status_t st = run_batch(*p, j, d_kraus_idx, merged, E, io, ar, s, evs);
  if (st != PTSBE_OK) return st;
  if (p->profile) {
    HIP_TRY(hipStreamSynchronize(s));
    st = collect_events(*p, evs);
  }
  return st;
}

ptsbe_status_t ptsbe_sample_shots(ptsbe_plan_t plan, const uint8_t* d_kraus_idx, int64_t E, const int64_t* d_mult,
                                  const int64_t* d_shots_per_traj, int32_t mode, uint64_t seed, uint64_t* d_shots,
                                  int32_t* d_shot_traj, double* d_traj_weight, double* d_traj_norm,
                                  int64_t* stats_out, void* d_workspace, size_t workspace_bytes, void* stream) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(PTSBE_ERR_INVALID_ARG, "null plan");
  if (p->device < 0) return fail(PTSBE_ERR_INVALID_ARG, "plan was built without a device");
  if (mode != PTSBE_MODE_PROPORTIONAL) return fail(PTSBE_ERR_UNSUPPORTED, "only proportional mode is implemented");
  for (int b : p->batch_sizes)
    if (b > 12) return fail(PTSBE_ERR_UNSUPPORTED, "the sampler handles batches of at most 12 qubits");
  if (E < 1) return fail(PTSBE_ERR_INVALID_ARG, "E < 1");
  if (!d_kraus_idx || !d_shots_per_traj || !d_shots || !d_workspace)
    return fail(PTSBE_ERR_INVALID_ARG, "null device pointer");
  HIP_TRY(hipSetDevice(p->device));
  hipStream_t s = (hipStream_t)stream;
  if (p->method == PTSBE_METHOD_STATEVECTOR)
    return ptsbe::sv_sample_shots(*p, d_kraus_idx, E, d_mult, d_shots_per_traj, seed, d_shots, d_shot_traj,
                                  d_traj_weight, d_traj_norm, stats_out, d_workspace, workspace_bytes, s);
  // shot layout: trajectory i owns rows [base_i, base_i + m_i)
  std::vector<int64_t> m(E), base(E);
  HIP_TRY(hipMemcpyAsync(m.data(), d_shots_per_traj, (size_t)E * 8, hipMemcpyDeviceToHost, s));
  // host copy of the Kraus indices: trajectories that agree on the sites of a
  // batch's per-trajectory part share that part's tensor
  std::vector<uint8_t> h_kraus((size_t)E * p->site_gate.size());
  if (!h_kraus.empty())
    HIP_TRY(hipMemcpyAsync(h_kraus.data(), d_kraus_idx, h_kraus.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int64_t M = 0;
  for (int64_t i = 0; i < E; ++i) {
    if (m[i] < 0) return fail(PTSBE_ERR_INVALID_ARG, "negative shot count");
    base[i] = M;
    M += m[i];
  }
  if (M >= ((int64_t)1 << 31)) return fail(PTSBE_ERR_UNSUPPORTED, "more than 2^31 shots");
  Arena ar;
  ar.base = (char*)d_workspace;
  ar.cap = workspace_bytes;
  SampleLayout L;
  if (!take_sample_layout(*p, E, M, ar, L))
    return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for the shot and element arrays");
  auto& el = L.el;
  float2** Vbuf = L.Vbuf;
  int32_t *shot_x = L.shot_x, *child_cnt = L.child_cnt, *child_off = L.child_off;
  int32_t *scan_scratch = L.scan_scratch, *counters = L.counters;
  double *totals = L.totals, *norms = L.norms;
  int64_t* d_base = L.base;
  float2* merged = L.merged;
  HIP_TRY(hipMemcpyAsync(d_base, base.data(), (size_t)E * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(counters, 0, 64, s));
  HIP_TRY(ptsbe::launch_init_elements(E, d_shots_per_traj, el[0].traj, el[0].prefix, p->NW, el[0].off, el[0].cnt,
                                      d_base, el[0].ids, d_shot_traj, d_shots, M, s));
  // error injection: the UPV merge of every trajectory's operators into its gates
  HIP_TRY(ptsbe::launch_upv_merge(gate_ctx(*p, d_kraus_idx, nullptr), E, merged, s));
  int cur = 0;
  int64_t U = E;
  std::vector<EventPair> evs;
  const int f = (int)p->batches.size();
  for (int j = 0; j < f; ++j) {
    if (stats_out) stats_out[j] = U;
    const auto& bp = p->batches[j];
    BatchIO io;
    io.h_kraus = h_kraus.empty() ? nullptr : h_kraus.data();
    io.elem_traj = el[cur].traj;
    io.elem_prefix = el[cur].prefix;
    io.V_out = Vbuf[j & 1];
    if (j >= 1) {
      io.resume = true;
      io.V_prev = Vbuf[(j - 1) & 1];
      const auto& pv = p->batches[j - 1];
      io.V_prev_stride = (int64_t)1 << (j - 1 == 0 ? pv.left.labels.size() : pv.left_resume.labels.size());
      io.parent = el[cur].parent;
    }
    io.U = U;
    io.sample = true;
    ptsbe::SampleArgs& sa = io.sa;
    sa.b = bp.size; sa.start = bp.start; sa.NW = p->NW;
    sa.elem_shot_off = el[cur].off; sa.elem_shot_cnt = el[cur].cnt;
    sa.shot_ids = el[cur].ids;
    sa.traj_shot_base = d_base;
    sa.seed = seed; sa.j = j;
    sa.shots = d_shots; sa.shot_x = shot_x;
    sa.elem_total = totals;
    sa.child_cnt = (j + 1 < f) ? child_cnt : nullptr;
    sa.bad_flag = counters + 1;
    // few shots per element (later batches): one lane per element
    const int lane_path = p->sample_kernel == 0 && bp.size <= 5 && M <= 4 * U ? 1 : 0;
    sa.lane_path = lane_path;
    ptsbe_status_t st = run_batch(*p, j, d_kraus_idx, merged, E, io, ar, s, evs);
    if (st != PTSBE_OK) return st;
    if (j == 0) {
      // elements of batch 0 are the trajectories themselves: totals = squared norms
      HIP_TRY(hipMemcpyAsync(norms, totals, (size_t)E * 8, hipMemcpyDeviceToDevice, s));
      ptsbe::WeightArgs wa{norms, d_mult, E, d_traj_weight, d_traj_norm};
      if (d_traj_weight || d_traj_norm) HIP_TRY(ptsbe::launch_weights(wa, s));
    }
    if (j + 1 < f) {
      HIP_TRY(ptsbe::launch_scan_i32(child_cnt, child_off, U, counters, scan_scratch, s));
      int32_t nU = 0;
      HIP_TRY(hipMemcpyAsync(&nU, counters, 4, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      ptsbe::ChildArgs ca{};
      ca.n_elems = U; ca.b = bp.size; ca.start = bp.start; ca.NW = p->NW;
      ca.elem_traj = el[cur].traj; ca.elem_prefix = el[cur].prefix;
      ca.elem_shot_off = el[cur].off; ca.elem_shot_cnt = el[cur].cnt;
      ca.shot_ids = el[cur].ids; ca.shot_x = shot_x; ca.child_off = child_off;
      ca.out_traj = el[1 - cur].traj; ca.out_prefix = el[1 - cur].prefix;
      ca.out_shot_off = el[1 - cur].off; ca.out_shot_cnt = el[1 - cur].cnt; ca.out_shot_ids = el[1 - cur].ids;
      ca.out_parent = el[1 - cur].parent;
      ca.lane_path = lane_path;
      HIP_TRY(ptsbe::launch_children(ca, s));
      cur = 1 - cur;
      U = nU;
    }
  }
  int32_t bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, counters + 1, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (p->profile) {
    ptsbe_status_t st = collect_events(*p, evs);
    if (st != PTSBE_OK) return st;
  }
  if (bad) return fail(PTSBE_ERR_NUMERIC, "an element had a non-finite marginal total");
  return PTSBE_OK;
}

namespace {
// Persistent arrays of ptsbe_sample_nonproportional, in the order they are taken.
struct ExhLayout {
  int32_t* traj[2]; uint64_t* prefix[2]; int32_t* off[2]; int32_t* cnt[2]; int32_t* ids[2]; int32_t* parent[2];
  float2* V[2];
  int32_t *shot_x, *child_cnt, *child_off, *scan_scratch, *counters;
  double *totals, *norms;
  int64_t* base;
  float2* merged;
};

bool take_exh_layout(const Plan& p, int64_t E, int64_t cap, int32_t draws, Arena& ar, ExhLayout& L) {
  int rVmax = 0;
  for (auto& bp : p.batches) rVmax = std::max<int>(rVmax, (int)bp.left_resume.labels.size());
  const size_t rows = (size_t)cap * (size_t)draws;
  bool ok = true;
  auto take = [&](size_t bytes) {   // every array is taken, so a probe arena measures the whole layout
    void* q = ar.take(bytes);
    ok = ok && q != nullptr;
    return q;
  };
  for (int k = 0; k < 2; ++k) {
    L.traj[k] = (int32_t*)take((size_t)cap * 4);
    L.prefix[k] = (uint64_t*)take((size_t)cap * 8 * p.NW);
    L.off[k] = (int32_t*)take((size_t)cap * 4);
    L.cnt[k] = (int32_t*)take((size_t)cap * 4);
    L.ids[k] = (int32_t*)take(rows * 4);
    L.parent[k] = (int32_t*)take((size_t)cap * 4);
    L.V[k] = (float2*)take((size_t)cap * ((size_t)8 << rVmax));
  }
  L.shot_x = (int32_t*)take(rows * 4);
  L.child_cnt = (int32_t*)take((size_t)cap * 4);
  L.child_off = (int32_t*)take((size_t)cap * 4);
  L.scan_scratch = (int32_t*)take(ptsbe::scan_scratch_bytes(cap));
  L.counters = (int32_t*)take(64);
  L.totals = (double*)take((size_t)cap * 8);
  L.norms = (double*)take((size_t)E * 8);
  L.base = (int64_t*)take((size_t)E * 8);
  L.merged = (float2*)take(merged_bytes(p, E));
  return ok;
}
}  // namespace

ptsbe_status_t ptsbe_nonproportional_workspace_size(ptsbe_plan_t plan, int64_t E, int32_t draws, int32_t final_draws,
                                                    int64_t max_elems, size_t* bytes) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p || !bytes) return fail(PTSBE_ERR_INVALID_ARG, "null argument");
  if (E < 1 || draws < 1 || final_draws < 0) return fail(PTSBE_ERR_INVALID_ARG, "E < 1, draws < 1 or final_draws < 0");
  const int64_t cap = std::max<int64_t>(E, max_elems);
  if (p->method == PTSBE_METHOD_STATEVECTOR) {
    *bytes = ptsbe::sv_np_workspace(*p, E, cap, std::max(draws, final_draws));
    return PTSBE_OK;
  }
  Arena probe;                       // an arena without memory measures the layout
  probe.base = nullptr;
  probe.cap = ~(size_t)0 >> 1;
  ExhLayout L;
  take_exh_layout(*p, E, cap, std::max(draws, final_draws), probe, L);
  size_t chunk = 0;
  for (auto& bp : p->batches) {
    const size_t per_traj = join_traj_bytes(bp);
    const size_t tb = bp.size > 12 ? (size_t)1 << (bp.size - 12) : 1;
    const size_t per_elem = ((size_t)8 << bp.left.labels.size()) + part_scratch_per_job(bp.left) +
                            ((size_t)4 << bp.size) + 16 + 12 * tb;
    // trajectories and elements per chunk: up to 256 / 65536, within about 8 GiB each
    const size_t nt = std::max<size_t>(1, std::min<size_t>(std::min<size_t>(E, 256), ((size_t)8 << 30) / per_traj));
    const size_t ne = std::max<size_t>(1, std::min<size_t>(std::min<size_t>(cap, 65536), ((size_t)8 << 30) / per_elem));
    chunk = std::max(chunk, 2 * (nt * per_traj + ne * per_elem));
  }
  *bytes = probe.used + (size_t)(E + 1) * 4 + chunk + (1 << 20);
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_sample_nonproportional(ptsbe_plan_t plan, const uint8_t* d_kraus_idx, int64_t E,
                                            const int64_t* d_mult, int32_t draws, int32_t final_draws,
                                            int64_t max_elems, uint64_t seed, double threshold, uint64_t* d_bits,
                                            int32_t* d_row_traj, double* d_p_cond, double* d_p_prefix,
                                            int64_t capacity, int64_t* n_rows_out, double* d_traj_weight,
                                            double* d_traj_norm, int64_t* stats_out, void* d_workspace,
                                            size_t workspace_bytes, void* stream) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(PTSBE_ERR_INVALID_ARG, "null plan");
  if (p->device < 0) return fail(PTSBE_ERR_INVALID_ARG, "plan was built without a device");
  const int f = (int)p->batches.size();
  for (int j = 0; j + 1 < f; ++j)
    if (p->batches[j].size > 12) return fail(PTSBE_ERR_UNSUPPORTED, "non-final batches of at most 12 qubits");
  if (E < 1 || draws < 1 || final_draws < 0 || capacity < 0)
    return fail(PTSBE_ERR_INVALID_ARG, "E < 1, draws < 1, final_draws < 0 or capacity < 0");
  if (std::isnan(threshold)) return fail(PTSBE_ERR_INVALID_ARG, "threshold is NaN");
  if (final_draws > 0 && p->batches.back().size > 12)
    return fail(PTSBE_ERR_UNSUPPORTED, "direct final-batch sampling takes a last batch of at most 12 qubits");
  const int32_t rows_per_elem = std::max(draws, final_draws);
  if (!d_kraus_idx || !d_workspace || !n_rows_out || (capacity > 0 && !d_bits))
    return fail(PTSBE_ERR_INVALID_ARG, "null pointer");
  const int64_t cap = std::max<int64_t>(E, max_elems);
  if (cap * (int64_t)rows_per_elem >= ((int64_t)1 << 31))
    return fail(PTSBE_ERR_UNSUPPORTED, "max_elems * max(draws, final_draws) >= 2^31");
  *n_rows_out = 0;
  HIP_TRY(hipSetDevice(p->device));
  hipStream_t s = (hipStream_t)stream;
  if (p->method == PTSBE_METHOD_STATEVECTOR) {
    if (p->batches.back().size > 12)
      return fail(PTSBE_ERR_UNSUPPORTED, "the statevector method samples batches of at most 12 qubits");
    return ptsbe::sv_sample_nonproportional(*p, d_kraus_idx, E, d_mult, draws, final_draws, cap, seed, threshold,
                                            d_bits, d_row_traj, d_p_cond, d_p_prefix, capacity, n_rows_out,
                                            d_traj_weight, d_traj_norm, stats_out, d_workspace, workspace_bytes, s);
  }
  std::vector<uint8_t> h_kraus((size_t)E * p->site_gate.size());
  if (!h_kraus.empty()) {
    HIP_TRY(hipMemcpyAsync(h_kraus.data(), d_kraus_idx, h_kraus.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  Arena ar;
  ar.base = (char*)d_workspace;
  ar.cap = workspace_bytes;
  ExhLayout L;
  if (!take_exh_layout(*p, E, cap, rows_per_elem, ar, L))
    return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for the element arrays");
  HIP_TRY(hipMemsetAsync(L.counters, 0, 64, s));
  HIP_TRY(ptsbe::launch_np_init(E, 0, L.traj[0], L.prefix[0], p->NW, s));
  HIP_TRY(ptsbe::launch_upv_merge(gate_ctx(*p, d_kraus_idx, nullptr), E, L.merged, s));
  BatchIO::Exhaustive exh;
  exh.tmpl.NW = p->NW;
  exh.tmpl.traj_norm = f > 1 ? L.norms : nullptr;      // one batch: p(prefix) = 1
  exh.tmpl.threshold = threshold;
  exh.tmpl.capacity = capacity;
  exh.tmpl.bits = d_bits; exh.tmpl.row_traj = d_row_traj; exh.tmpl.p_cond = d_p_cond; exh.tmpl.p_prefix = d_p_prefix;
  exh.tmpl.totals_out = f > 1 ? nullptr : L.norms;    // one batch: its totals are the norms (copied in
                                                      // stream order before the weights read them)
  int cur = 0;
  int64_t U = E;
  std::vector<EventPair> evs;
  for (int j = 0; j < f; ++j) {
    if (stats_out) stats_out[j] = U;
    const auto& bp = p->batches[j];
    const bool last = j + 1 == f;
    BatchIO io;
    io.h_kraus = h_kraus.empty() ? nullptr : h_kraus.data();
    io.elem_traj = L.traj[cur];
    io.elem_prefix = L.prefix[cur];
    io.V_out = L.V[j & 1];
    if (j >= 1) {
      io.resume = true;
      io.V_prev = L.V[(j - 1) & 1];
      const auto& pv = p->batches[j - 1];
      io.V_prev_stride = (int64_t)1 << (j - 1 == 0 ? pv.left.labels.size() : pv.left_resume.labels.size());
      io.parent = L.parent[cur];
    }
    io.U = U;
    if (!last) {
      HIP_TRY(ptsbe::launch_np_rows(U, draws, L.traj[cur], L.off[cur], L.cnt[cur], L.ids[cur], L.base, s));
      io.sample = true;
      ptsbe::SampleArgs& sa = io.sa;
      sa.b = bp.size; sa.start = bp.start; sa.NW = p->NW;
      sa.elem_shot_off = L.off[cur]; sa.elem_shot_cnt = L.cnt[cur];
      sa.shot_ids = L.ids[cur];
      sa.traj_shot_base = L.base;
      sa.seed = seed; sa.j = j; sa.tag = 3u;
      sa.shots = nullptr; sa.shot_x = L.shot_x;
      sa.elem_total = L.totals;
      sa.child_cnt = L.child_cnt;
      sa.bad_flag = L.counters + 1;
    } else if (final_draws > 0) {   // direct sampling: final_draws rows per element
      const int64_t rows = U * (int64_t)final_draws;
      *n_rows_out = rows;
      if (rows > capacity)
        return fail(PTSBE_ERR_OUT_OF_MEMORY, std::to_string(rows) + " rows, capacity " + std::to_string(capacity));
      HIP_TRY(ptsbe::launch_np_rows(U, final_draws, L.traj[cur], L.off[cur], L.cnt[cur], L.ids[cur], L.base, s));
      HIP_TRY(ptsbe::launch_np_direct_rows(U, final_draws, L.traj[cur], L.prefix[cur], p->NW, d_bits, d_row_traj, s));
      io.sample = true;
      ptsbe::SampleArgs& sa = io.sa;
      sa.b = bp.size; sa.start = bp.start; sa.NW = p->NW;
      sa.elem_shot_off = L.off[cur]; sa.elem_shot_cnt = L.cnt[cur];
      sa.shot_ids = L.ids[cur];
      sa.traj_shot_base = L.base;
      sa.seed = seed; sa.j = j; sa.tag = 3u;
      sa.shots = d_bits; sa.shot_x = L.shot_x; sa.p_cond = d_p_cond;
      sa.elem_total = L.totals;
      sa.child_cnt = nullptr;
      sa.bad_flag = L.counters + 1;
    } else {
      io.exh = &exh;
    }
    ptsbe_status_t st = run_batch(*p, j, d_kraus_idx, L.merged, E, io, ar, s, evs);
    if (st != PTSBE_OK) return st;
    if (j == 0 && (!last || final_draws > 0))
      HIP_TRY(hipMemcpyAsync(L.norms, L.totals, (size_t)E * 8, hipMemcpyDeviceToDevice, s));
    if (last && final_draws > 0)
      HIP_TRY(ptsbe::launch_np_direct_prefix_p(U, final_draws, L.traj[cur], L.totals, f > 1 ? L.norms : nullptr,
                                               d_p_prefix, s));
    if (j == 0 && (d_traj_weight || d_traj_norm)) {
      ptsbe::WeightArgs wa{L.norms, d_mult, E, d_traj_weight, d_traj_norm};
      HIP_TRY(ptsbe::launch_weights(wa, s));
    }
    if (!last) {
      HIP_TRY(ptsbe::launch_scan_i32(L.child_cnt, L.child_off, U, L.counters, L.scan_scratch, s));
      int32_t nU = 0;
      HIP_TRY(hipMemcpyAsync(&nU, L.counters, 4, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (nU > cap) return fail(PTSBE_ERR_OUT_OF_MEMORY, "batch " + std::to_string(j + 1) + " has " +
                                                          std::to_string(nU) + " elements, more than max_elems");
      ptsbe::ChildArgs ca{};
      ca.n_elems = U; ca.b = bp.size; ca.start = bp.start; ca.NW = p->NW;
      ca.elem_traj = L.traj[cur]; ca.elem_prefix = L.prefix[cur];
      ca.elem_shot_off = L.off[cur]; ca.elem_shot_cnt = L.cnt[cur];
      ca.shot_ids = L.ids[cur]; ca.shot_x = L.shot_x; ca.child_off = L.child_off;
      ca.out_traj = L.traj[1 - cur]; ca.out_prefix = L.prefix[1 - cur];
      ca.out_shot_off = L.off[1 - cur]; ca.out_shot_cnt = L.cnt[1 - cur]; ca.out_shot_ids = L.ids[1 - cur];
      ca.out_parent = L.parent[1 - cur];
      HIP_TRY(ptsbe::launch_children(ca, s));
      cur = 1 - cur;
      U = nU;
    }
  }
  int32_t bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, L.counters + 1, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (p->profile) {
    ptsbe_status_t st = collect_events(*p, evs);
    if (st != PTSBE_OK) return st;
  }
  if (final_draws == 0) *n_rows_out = exh.rows;
  if (bad) return fail(PTSBE_ERR_NUMERIC, "an element had a non-finite marginal total");
  if (exh.rows > capacity)
    return fail(PTSBE_ERR_OUT_OF_MEMORY, std::to_string(exh.rows) + " rows found, capacity " + std::to_string(capacity));
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_profile_enable(ptsbe_plan_t plan, int32_t on) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(PTSBE_ERR_INVALID_ARG, "null plan");
  if (on < 0 || on > 2) return fail(PTSBE_ERR_INVALID_ARG, "profile level must be 0, 1 or 2");
  for (auto& e : p->sweep_evs) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  p->sweep_evs.clear();
  for (auto& e : p->win_evs) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  p->win_evs.clear();
  for (auto& e : p->vm_evs) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  p->vm_evs.clear();
  p->vm_ms = p->vm_flops = 0;
  p->vm_launches = 0;
  p->profile = on;
  p->join_ms = p->sweep_ms = p->join_flops = p->sweep_bytes = p->fused_bytes = 0;
  p->join_launches = p->sweep_launches = 0;
  p->win_ms = p->win_bytes = 0;
  p->win_launches = 0;
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_profile_read_windows(ptsbe_plan_t plan, double* ms, int64_t* launches, double* bytes) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(PTSBE_ERR_INVALID_ARG, "null plan");
  if (ms) *ms = p->win_ms;
  if (launches) *launches = p->win_launches;
  if (bytes) *bytes = p->win_bytes;
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_profile_read_sweeps(ptsbe_plan_t plan, double* step_ms, int64_t* step_launches,
                                         double* step_bytes, double* fused_bytes) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(PTSBE_ERR_INVALID_ARG, "null plan");
  if (step_ms) *step_ms = p->sweep_ms;
  if (step_launches) *step_launches = p->sweep_launches;
  if (step_bytes) *step_bytes = p->sweep_bytes;
  if (fused_bytes) *fused_bytes = p->fused_bytes;
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_profile_read_lds_sweeps(ptsbe_plan_t plan, double* ms, int64_t* launches, double* flops) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(PTSBE_ERR_INVALID_ARG, "null plan");
  if (ms) *ms = p->vm_ms;
  if (launches) *launches = p->vm_launches;
  if (flops) *flops = p->vm_flops;
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_profile_read(ptsbe_plan_t plan, double* join_ms, int64_t* join_launches, double* join_flops,
                                  double* sweep_ms, double* sweep_bytes) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(PTSBE_ERR_INVALID_ARG, "null plan");
  if (join_ms) *join_ms = p->join_ms;
  if (join_launches) *join_launches = p->join_launches;
  if (join_flops) *join_flops = p->join_flops;
  if (sweep_ms) *sweep_ms = p->sweep_ms;
  if (sweep_bytes) *sweep_bytes = p->sweep_bytes;
  return PTSBE_OK;
}

}  // extern "C"
