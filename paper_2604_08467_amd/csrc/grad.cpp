// Adjoint contraction: reverse-mode derivatives of trajectory-averaged
// quantities with respect to rotation angles and gate tensors (an addition to
// the paper's method, which reuses its unified gate schedule and UPV merge).
//
// The ket network of every trajectory is contracted in circuit order into its
// statevector through LDS gate windows of at most 11 qubits; the state after
// every window is kept as a checkpoint.  The backward pass starts from
// lambda = w O psi (O diagonal: ZZ terms or the caller's array) or from the
// caller's seed psi-bar = dL/d conj(psi), and walks the windows in reverse,
// propagating lambda_{k-1} = A_k^dag lambda_k and accumulating per gate
//   N_k = sum_i sum_rest lambda_{k-1} psi_{k-1}^dag,
// from which the derivative with respect to the bare gate U_k is
// d L / d conj(U_k) = U_k N_k, and for a rotation exp(-i theta P / 2)
// d L / d theta = Im <lambda_{k-1}|P|psi_{k-1}> summed over trajectories.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "internal.h"

using ptsbe::Arena;
using ptsbe::fail;
using ptsbe::Plan;

namespace {

constexpr int kAdjWindowQubits = 11;   // two (three when recomputing) 16 KB tiles per workgroup
constexpr int64_t kAdjChunkMax = 1024;

struct AdjSpec {
  int n_params = 0;
  std::vector<int32_t> gate_param, gate_axis;
  std::vector<int32_t> zq;
  std::vector<double> zc;
  const double* obs_diag = nullptr;
  bool has_obs = false;
};

ptsbe_status_t check_adj_spec(const Plan& p, const ptsbe_adjoint_spec_t* spec, AdjSpec& S) {
  if (!spec) return fail(PTSBE_ERR_INVALID_ARG, "null adjoint spec");
  if (p.n > ptsbe::kSvMaxQubits || p.sv_steps.empty())
    return fail(PTSBE_ERR_UNSUPPORTED, "differentiation needs n_qubits <= 30");
  if (spec->n_params < 0 || spec->n_terms < 0) return fail(PTSBE_ERR_INVALID_ARG, "negative counts");
  if (spec->n_params > 0 && (!spec->gate_param || !spec->gate_axis))
    return fail(PTSBE_ERR_INVALID_ARG, "null gate parameter arrays");
  if (spec->n_terms > 0 && (!spec->zz_qubits || !spec->zz_coef)) return fail(PTSBE_ERR_INVALID_ARG, "null terms");
  S.n_params = spec->n_params;
  S.gate_param.assign(p.G, -1);
  S.gate_axis.assign(p.G, 0);
  // gates after the caller's circuit are identities the plan added for untouched qubits
  if (spec->gate_param)
    for (int g = 0; g < p.n_user_gates; ++g) {
      const int prm = spec->gate_param[g];
      if (prm >= spec->n_params) return fail(PTSBE_ERR_INVALID_ARG, "parameter index out of range");
      if (prm < 0) continue;
      if (p.arity[g] != 1) return fail(PTSBE_ERR_UNSUPPORTED, "rotation gates must act on one qubit");
      const int ax = spec->gate_axis[g];
      if (ax < 0 || ax > 2) return fail(PTSBE_ERR_INVALID_ARG, "rotation axis must be 0, 1 or 2");
      S.gate_param[g] = prm;
      S.gate_axis[g] = ax;
    }
  for (int t = 0; t < spec->n_terms; ++t) {
    const int a = spec->zz_qubits[2 * t], b = spec->zz_qubits[2 * t + 1];
    if (a < 0 || a >= p.n || b < 0 || b >= p.n) return fail(PTSBE_ERR_INVALID_ARG, "observable qubit out of range");
    S.zq.push_back(a);
    S.zq.push_back(b);
    S.zc.push_back(spec->zz_coef[t]);
  }
  S.obs_diag = spec->d_obs_diag;
  S.has_obs = S.obs_diag != nullptr || spec->n_terms > 0;
  if (S.zq.empty()) {
    S.zq = {0, 0};
    S.zc = {0.0};
  }
  return PTSBE_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Largest number of ops per window whose LDS (tiles, staged gates, accumulators)
// fits 64 KB for the passes the call runs.
int adj_max_ops(const Plan& p, bool backward, bool recompute, bool want_adj) {
  const int np = std::min(kAdjWindowQubits, p.n);
  const size_t tiles = (size_t)(backward ? (recompute ? 3 : 2) : 1) << np;
  const size_t per_op = (size_t)(backward && recompute ? 2 : 1) * 16 * 8 + (backward ? 8 + (want_adj ? 256 : 0) : 0);
  const size_t fixed = tiles * 8 + (backward ? 2 * 4 * 33 * 8 : 0) + 64;
  return (int)std::min<size_t>(1024, (65536 - fixed) / per_op);
}

// Per-trajectory device bytes: the W + 1 window checkpoints and lambda (gradient),
// or two states (values only).
size_t adj_per_traj(const Plan& p, size_t n_windows, bool grad) {
  return (grad ? n_windows + 2 : 2) * ((size_t)8 << p.n);
}

size_t adj_fixed_bytes(const Plan& p, int64_t E, size_t n_ops, size_t width_total, size_t wg_width) {
  size_t b = 0;
  b += align256((size_t)E * p.G * 128) * 2;                  // merged gates and their adjoints
  b += align256(128) + align256((size_t)p.G * 4) * 3;        // (unused derivative slot), gate tables
  b += align256(n_ops * sizeof(ptsbe::AdjOp));
  b += align256(std::max<size_t>(n_ops, 1) * sizeof(ptsbe::AdjGroup));     // op groups (at most one per op)
  b += align256((size_t)E * 8);                              // per-trajectory values
  b += align256(64 * 4) + align256(64 * 8);                  // ZZ terms (at most 64 kept on device)
  b += align256(width_total * 8);                            // per-window totals
  b += align256((size_t)8 << p.n);                           // the observable's diagonal
  b += align256((size_t)std::min<int64_t>(E, kAdjChunkMax) * 64 * 8);   // partial values
  b += align256((size_t)8192 * wg_width * 8);                // per-workgroup sums of one window
  return b + ((size_t)1 << 20);
}

}  // namespace

extern "C" {

ptsbe_status_t ptsbe_adjoint_workspace_size(ptsbe_plan_t plan, const ptsbe_adjoint_spec_t* spec, int64_t E,
                                            size_t* bytes) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p || !bytes) return fail(PTSBE_ERR_INVALID_ARG, "null argument");
  AdjSpec S;
  ptsbe_status_t st = check_adj_spec(*p, spec, S);
  if (st != PTSBE_OK) return st;
  std::vector<ptsbe::AdjWin> wins;
  std::vector<ptsbe::AdjOp> ops;
  ptsbe::build_adj_windows(*p, kAdjWindowQubits, adj_max_ops(*p, true, !p->inserted_unitary, true), wins, ops);
  size_t max_ops = 0;
  for (const auto& w : wins) max_ops = std::max<size_t>(max_ops, (size_t)w.n_ops);
  *bytes = adj_fixed_bytes(*p, E, ops.size(), ops.size() * 33, max_ops * 33) +
           (size_t)std::min<int64_t>(E, 256) * adj_per_traj(*p, wins.size(), true);
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_contract_adjoint(ptsbe_plan_t plan, const ptsbe_adjoint_spec_t* spec,
                                      const uint8_t* d_kraus_idx, int64_t E, const double* d_weights,
                                      const double* d_theta, const void* d_psi_bar, double* d_traj_value,
                                      double* d_value, double* d_grad, double* d_gate_adj, void* d_workspace,
                                      size_t workspace_bytes, void* stream) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(PTSBE_ERR_INVALID_ARG, "null plan");
  if (p->device < 0) return fail(PTSBE_ERR_INVALID_ARG, "plan was built without a device");
  if (E < 1) return fail(PTSBE_ERR_INVALID_ARG, "E < 1");
  if (!d_kraus_idx || !d_weights || !d_workspace) return fail(PTSBE_ERR_INVALID_ARG, "null pointer");
  AdjSpec S;
  ptsbe_status_t st = check_adj_spec(*p, spec, S);
  if (st != PTSBE_OK) return st;
  if (S.n_params > 0 && !d_theta) return fail(PTSBE_ERR_INVALID_ARG, "null theta");
  if ((d_value || d_traj_value) && !S.has_obs)
    return fail(PTSBE_ERR_INVALID_ARG, "values need an observable (ZZ terms or a diagonal)");
  if ((d_grad != nullptr && S.n_params > 0 || d_gate_adj != nullptr) && !d_psi_bar && !S.has_obs)
    return fail(PTSBE_ERR_INVALID_ARG, "the backward pass needs an observable or a psi-bar seed");
  if ((int64_t)S.zc.size() > 64) return fail(PTSBE_ERR_UNSUPPORTED, "at most 64 ZZ terms");
  HIP_TRY(hipSetDevice(p->device));
  hipStream_t s = (hipStream_t)stream;
  const int n = p->n, G = p->G;
  // windows and their ops (host, once per call)
  const bool want_grad = d_grad != nullptr && S.n_params > 0;
  const bool want_adj = d_gate_adj != nullptr;
  const bool backward = want_grad || want_adj;
  const bool recompute = !p->inserted_unitary;
  std::vector<ptsbe::AdjWin> wins;
  std::vector<ptsbe::AdjOp> ops;
  ptsbe::build_adj_windows(*p, kAdjWindowQubits, adj_max_ops(*p, backward, recompute, want_adj), wins, ops);
  std::vector<ptsbe::AdjGroup> groups;
  ptsbe::build_adj_groups(wins, ops, groups);
  const int W = (int)wins.size();
  std::vector<int> width(W), tot_off(W + 1, 0);
  size_t max_width = 1;
  for (int w = 0; w < W; ++w) {
    const ptsbe::AdjWin& wd = wins[(size_t)w];
    for (int k = 0; k < wd.n_ops; ++k) {
      ptsbe::AdjOp& op = ops[(size_t)(wd.op_off + k)];
      op.axis = (int8_t)(want_grad && S.gate_param[(size_t)op.gate] >= 0 ? S.gate_axis[(size_t)op.gate] : -1);
      op.nslot = want_adj ? k : -1;
    }
    for (int gi = 0; gi < wd.n_groups; ++gi) {
      ptsbe::AdjGroup& gr = groups[(size_t)(wd.group_off + gi)];
      gr.rot_mask = 0;
      for (int j = 0; j < gr.n; ++j)
        if (ops[(size_t)(wd.op_off + gr.first + j)].axis >= 0) gr.rot_mask |= 1u << j;
    }
    width[(size_t)w] = wd.n_ops + (want_adj ? 32 * wd.n_ops : 0);
    tot_off[(size_t)w + 1] = tot_off[(size_t)w] + width[(size_t)w];
    max_width = std::max<size_t>(max_width, (size_t)width[(size_t)w]);
  }
  const int bmode = recompute ? 2 : 1;
  for (const auto& wd : wins) {
    const size_t lds = ptsbe::adj_window_lds_bytes(backward ? bmode : 0, wd.np, wd.n_ops, want_adj ? wd.n_ops : 0);
    if (lds > 64 * 1024) return fail(PTSBE_ERR_UNSUPPORTED, "an adjoint window holds too many gates for LDS");
  }
  // workspace
  Arena ar;
  ar.base = (char*)d_workspace;
  ar.cap = workspace_bytes;
  float2* merged = (float2*)ar.take((size_t)E * G * 128);
  float2* dagger = (float2*)ar.take((size_t)E * G * 128);
  float2* dslot = (float2*)ar.take(128);
  int32_t* d_gp = (int32_t*)ar.take((size_t)G * 4);
  int32_t* d_ga = (int32_t*)ar.take((size_t)G * 4);
  int32_t* d_gs = (int32_t*)ar.take((size_t)G * 4);
  ptsbe::AdjOp* d_ops = (ptsbe::AdjOp*)ar.take(std::max<size_t>(ops.size(), 1) * sizeof(ptsbe::AdjOp));
  ptsbe::AdjGroup* d_groups =
      (ptsbe::AdjGroup*)ar.take(std::max<size_t>(groups.size(), 1) * sizeof(ptsbe::AdjGroup));
  double* vals = (double*)ar.take((size_t)E * 8);
  int32_t* d_zq = (int32_t*)ar.take(64 * 4);
  double* d_zc = (double*)ar.take(64 * 8);
  double* d_tot = (double*)ar.take(std::max<size_t>((size_t)tot_off[(size_t)W], 1) * 8);
  double* d_diag = S.obs_diag ? nullptr : (double*)ar.take((size_t)8 << n);   // the ZZ terms' diagonal
  double* d_part = (double*)ar.take((size_t)std::min<int64_t>(E, kAdjChunkMax) * 64 * 8);
  if (!d_part || (!S.obs_diag && !d_diag)) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for the observable");
  double* d_wg = (double*)ar.take((size_t)8192 * max_width * 8);
  if (!d_wg) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for the merged gates and tables");
  std::vector<int32_t> gslot((size_t)G, -1);
  HIP_TRY(hipMemcpyAsync(d_gp, S.gate_param.data(), (size_t)G * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_ga, S.gate_axis.data(), (size_t)G * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_gs, gslot.data(), (size_t)G * 4, hipMemcpyHostToDevice, s));
  if (!ops.empty())
    HIP_TRY(hipMemcpyAsync(d_ops, ops.data(), ops.size() * sizeof(ptsbe::AdjOp), hipMemcpyHostToDevice, s));
  if (!groups.empty())
    HIP_TRY(hipMemcpyAsync(d_groups, groups.data(), groups.size() * sizeof(ptsbe::AdjGroup), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_zq, S.zq.data(), S.zq.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_zc, S.zc.data(), S.zc.size() * 8, hipMemcpyHostToDevice, s));
  std::vector<double> zeros((size_t)std::max(tot_off[(size_t)W], 1), 0.0);
  HIP_TRY(hipMemcpyAsync(d_tot, zeros.data(), zeros.size() * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));   // the host tables above are about to go out of scope
  // error injection + rotation angles: A = S U(theta) and A^dag of every (trajectory, gate)
  ptsbe::GateCtx g{};
  g.gates = p->d_gates;
  g.gate_site_list = p->d_gate_site_list;
  g.site_ops = p->d_site_ops;
  g.kraus = d_kraus_idx;
  g.S = p->S;
  g.max_kraus = p->max_kraus;
  g.G = G;
  ptsbe::GradGateArgs ga{g, E, d_gp, d_ga, d_gs, 0, d_theta, merged, dagger, dslot};
  HIP_TRY(ptsbe::launch_grad_gates(ga, s));
  if (!S.obs_diag) HIP_TRY(ptsbe::launch_adj_zz_diag(n, d_zq, d_zc, S.has_obs ? (int)S.zc.size() : 0, d_diag, s));
  const double* obs = S.obs_diag ? S.obs_diag : d_diag;
  // trajectory chunks
  const size_t per = adj_per_traj(*p, (size_t)W, backward);
  const size_t avail = ar.left() > ((size_t)1 << 20) ? ar.left() - ((size_t)1 << 20) : 0;
  const int64_t Ec = std::min<int64_t>({E, (int64_t)(avail / per), kAdjChunkMax});
  if (Ec < 1) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for one trajectory's checkpoints");
  const size_t SZ = (size_t)1 << n;
  for (int64_t t0 = 0; t0 < E; t0 += Ec) {
    const int64_t nj = std::min<int64_t>(Ec, E - t0);
    const size_t mark = ar.used;
    const int nbuf = backward ? W + 1 : 2;
    std::vector<float2*> ck((size_t)nbuf);
    for (auto& c : ck) c = (float2*)ar.take((size_t)nj * SZ * 8);
    float2* lam = backward ? (float2*)ar.take((size_t)nj * SZ * 8) : nullptr;
    if (!ck.back() || (backward && !lam)) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for the chunk");
    HIP_TRY(ptsbe::launch_state_init(ck[0], nj, n, s));
    // one window launch; under profiling, HIP events on the launch stream and the
    // algorithmic bytes (every state the mode streams, read or written once)
    auto timed_window = [&](int mode, const ptsbe::AdjArgs& a, const ptsbe::AdjOp* o, int grid,
                            double bytes_per_amp) -> hipError_t {
      std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
      if (p->profile) {
        hipError_t e = hipEventCreate(&ev.first);
        if (e == hipSuccess) e = hipEventCreate(&ev.second);
        if (e == hipSuccess) e = hipEventRecord(ev.first, s);
        if (e != hipSuccess) return e;
      }
      hipError_t e = ptsbe::launch_adj_window(mode, a, o, grid, s);
      if (e != hipSuccess || !p->profile) return e;
      e = hipEventRecord(ev.second, s);
      p->win_evs.push_back(ev);
      ++p->win_launches;
      p->win_bytes += (double)a.n_jobs * bytes_per_amp * std::ldexp(1.0, n);
      return e;
    };
    auto args_for = [&](const ptsbe::AdjWin& wd) {
      ptsbe::AdjArgs a{};
      a.n = n;
      a.np = wd.np;
      a.n_ops = wd.n_ops;
      a.G = G;
      uint32_t win = 0;
      for (int k = 0; k < 12; ++k) {
        a.P[k] = wd.P[k];
        if (k < wd.np) win |= 1u << wd.P[k];
      }
      a.other = (n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u)) & ~win;
      a.n_jobs = nj;
      a.traj_base = (int32_t)t0;
      a.A = merged;
      a.Ad = dagger;
      a.groups = d_groups + wd.group_off;
      a.n_groups = wd.n_groups;
      return a;
    };
    // forward: window w maps checkpoint w to checkpoint w + 1 (values only: two buffers)
    for (int w = 0; w < W; ++w) {
      const ptsbe::AdjWin& wd = wins[(size_t)w];
      ptsbe::AdjArgs a = args_for(wd);
      a.psi_in = ck[backward ? (size_t)w : (size_t)(w & 1)];
      a.psi_out = ck[backward ? (size_t)w + 1 : (size_t)((w + 1) & 1)];
      const size_t lds = ptsbe::adj_window_lds_bytes(0, wd.np, wd.n_ops, 0);
      const int grid = ptsbe::adj_window_grid(0, a, lds);
      if (grid < 1) return fail(PTSBE_ERR_DEVICE, "occupancy query failed");
      HIP_TRY(timed_window(0, a, d_ops + wd.op_off, grid, 16.0));
    }
    float2* final_state = ck[backward ? (size_t)W : (size_t)(W & 1)];
    ptsbe::AdjSeedArgs sd{};
    sd.psi = final_state;
    sd.lam = lam;
    sd.psi_bar = (const float2*)d_psi_bar;
    sd.obs_diag = obs;
    sd.part = d_part;
    sd.weights = d_weights;
    sd.values = S.has_obs ? vals : nullptr;
    sd.n = n;
    sd.traj_base = (int32_t)t0;
    HIP_TRY(ptsbe::launch_adj_seed(sd, nj, s));
    if (backward) {
      for (int w = W - 1; w >= 0; --w) {
        const ptsbe::AdjWin& wd = wins[(size_t)w];
        ptsbe::AdjArgs a = args_for(wd);
        a.psi_in = recompute ? ck[(size_t)w] : ck[(size_t)w + 1];
        a.lam = lam;
        a.n_nslots = want_adj ? wd.n_ops : 0;
        a.want_n = want_adj ? 1 : 0;
        a.wg_acc = d_wg;
        const size_t lds = ptsbe::adj_window_lds_bytes(bmode, wd.np, wd.n_ops, a.n_nslots);
        const int grid = std::min(8192, ptsbe::adj_window_grid(bmode, a, lds));
        if (grid < 1) return fail(PTSBE_ERR_DEVICE, "occupancy query failed");
        HIP_TRY(timed_window(bmode, a, d_ops + wd.op_off, grid, 24.0));
        HIP_TRY(ptsbe::launch_adj_reduce(d_wg, grid, width[(size_t)w], d_tot + tot_off[(size_t)w], s));
      }
    }
    ar.used = mark;
  }
  if (S.has_obs) {
    if (d_traj_value) HIP_TRY(hipMemcpyAsync(d_traj_value, vals, (size_t)E * 8, hipMemcpyDeviceToDevice, s));
    if (d_value) HIP_TRY(ptsbe::launch_value_sum(vals, d_weights, E, d_value, s));
  }
  if (backward) {
    // per-window totals -> angle derivatives and gate-tensor adjoints (host, FP64)
    std::vector<double> tot((size_t)std::max(tot_off[(size_t)W], 1));
    std::vector<double> theta((size_t)std::max(S.n_params, 1), 0.0);
    HIP_TRY(hipMemcpyAsync(tot.data(), d_tot, tot.size() * 8, hipMemcpyDeviceToHost, s));
    if (S.n_params > 0) HIP_TRY(hipMemcpyAsync(theta.data(), d_theta, (size_t)S.n_params * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<double> grad((size_t)std::max(S.n_params, 1), 0.0);
    std::vector<double> adj(want_adj ? (size_t)G * 32 : 0, 0.0);
    using cd = std::complex<double>;
    for (int w = 0; w < W; ++w) {
      const ptsbe::AdjWin& wd = wins[(size_t)w];
      const double* tw = tot.data() + tot_off[(size_t)w];
      for (int k = 0; k < wd.n_ops; ++k) {
        const ptsbe::AdjOp& op = ops[(size_t)(wd.op_off + k)];
        if (want_grad && op.axis >= 0) grad[(size_t)S.gate_param[(size_t)op.gate]] += tw[k];
        if (!want_adj) continue;
        // N in the gate's own layout, then M = U N with U the bare gate (theta substituted)
        const int d = op.kind == ptsbe::kSvOpGate1 ? 2 : 4;
        cd N[16], U[16];
        for (int i = 0; i < 16; ++i) N[i] = U[i] = 0;
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b) {
            const double* v = tw + wd.n_ops + 32 * k + 2 * (a * d + b);
            N[op.idx[a * d + b]] = cd(v[0], v[1]);
          }
        const int prm = S.gate_param[(size_t)op.gate];
        if (prm >= 0) {
          const double c = std::cos(0.5 * theta[(size_t)prm]), sn = std::sin(0.5 * theta[(size_t)prm]);
          const cd mi(0.0, -sn);    // U = c I - i s P
          const int ax = S.gate_axis[(size_t)op.gate];
          const cd P[3][4] = {{0, 1, 1, 0}, {0, cd(0, -1), cd(0, 1), 0}, {1, 0, 0, -1}};
          for (int i = 0; i < 4; ++i) U[i] = (i == 0 || i == 3 ? cd(c, 0) : cd(0, 0)) + mi * P[ax][i];
        } else {
          for (int i = 0; i < d * d; ++i)
            U[i] = cd(p->mats[(size_t)op.gate][2 * i], p->mats[(size_t)op.gate][2 * i + 1]);
        }
        for (int r = 0; r < d; ++r)
          for (int c2 = 0; c2 < d; ++c2) {
            cd m = 0;
            for (int x = 0; x < d; ++x) m += U[r * d + x] * N[x * d + c2];
            // torch's convention for a real loss: 2 dL / d conj(U)
            adj[(size_t)op.gate * 32 + 2 * (r * d + c2)] += 2.0 * m.real();
            adj[(size_t)op.gate * 32 + 2 * (r * d + c2) + 1] += 2.0 * m.imag();
          }
      }
    }
    if (want_grad) HIP_TRY(hipMemcpyAsync(d_grad, grad.data(), (size_t)S.n_params * 8, hipMemcpyHostToDevice, s));
    if (want_adj) HIP_TRY(hipMemcpyAsync(d_gate_adj, adj.data(), adj.size() * 8, hipMemcpyHostToDevice, s));
  } else if (d_grad && S.n_params > 0) {
    std::vector<double> z((size_t)S.n_params, 0.0);
    HIP_TRY(hipMemcpyAsync(d_grad, z.data(), z.size() * 8, hipMemcpyHostToDevice, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  return p->profile ? ptsbe::collect_window_events(*p) : PTSBE_OK;
}

// ZZ-observable form (value and angle gradient), on the adjoint contraction.
ptsbe_status_t ptsbe_expect_workspace_size(ptsbe_plan_t plan, const ptsbe_grad_spec_t* spec, int64_t E,
                                           size_t* bytes) {
  if (!spec) return fail(PTSBE_ERR_INVALID_ARG, "null gradient spec");
  if (spec->checkpoint_every < 1) return fail(PTSBE_ERR_INVALID_ARG, "checkpoint_every must be >= 1");
  ptsbe_adjoint_spec_t a{spec->n_params, spec->gate_param, spec->gate_axis, spec->n_terms, spec->zz_qubits,
                         spec->zz_coef, nullptr};
  return ptsbe_adjoint_workspace_size(plan, &a, E, bytes);
}

ptsbe_status_t ptsbe_expect_grad(ptsbe_plan_t plan, const ptsbe_grad_spec_t* spec, const uint8_t* d_kraus_idx,
                                 int64_t E, const double* d_weights, const double* d_theta, double* d_traj_value,
                                 double* d_value, double* d_grad, void* d_workspace, size_t workspace_bytes,
                                 void* stream) {
  if (!spec) return fail(PTSBE_ERR_INVALID_ARG, "null gradient spec");
  if (spec->checkpoint_every < 1) return fail(PTSBE_ERR_INVALID_ARG, "checkpoint_every must be >= 1");
  if (!d_value) return fail(PTSBE_ERR_INVALID_ARG, "null pointer");
  ptsbe_adjoint_spec_t a{spec->n_params, spec->gate_param, spec->gate_axis, spec->n_terms, spec->zz_qubits,
                         spec->zz_coef, nullptr};
  return ptsbe_contract_adjoint(plan, &a, d_kraus_idx, E, d_weights, d_theta, nullptr, d_traj_value, d_value, d_grad,
                                nullptr, d_workspace, workspace_bytes, stream);
}

}  // extern "C"
