// Adjoint contraction: value and gradient of a trajectory-averaged ZZ observable
// with respect to rotation angles (an addition to the paper's method, which
// reuses its unified network and UPV merge).  The ket network of each trajectory
// is contracted in circuit order into its statevector (forward), the states are
// checkpointed every C gates, and the backward pass walks the gates in reverse:
// recompute a segment's states from its checkpoint, reduce
// <lambda_k|(dA_k/dtheta) psi_{k-1}> for the rotation gates, and propagate
// lambda_{k-1} = A_k^dag lambda_k.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.h"

using ptsbe::Arena;
using ptsbe::fail;
using ptsbe::Plan;

namespace {

struct GradLayout {
  int G = 0, n_slots = 0, n_ck = 0, C = 1;
  std::vector<int32_t> gate_param, gate_axis, gate_slot, slot_param, zq;
  std::vector<double> zc;
};

ptsbe_status_t check_spec(const Plan& p, const ptsbe_grad_spec_t* spec, GradLayout& L) {
  if (!spec) return fail(PTSBE_ERR_INVALID_ARG, "null gradient spec");
  if (p.n > 30 || p.sv_steps.empty()) return fail(PTSBE_ERR_UNSUPPORTED, "differentiation needs n_qubits <= 30");
  if (spec->n_params < 0 || spec->n_terms < 0) return fail(PTSBE_ERR_INVALID_ARG, "negative counts");
  if (spec->checkpoint_every < 1) return fail(PTSBE_ERR_INVALID_ARG, "checkpoint_every must be >= 1");
  if (!spec->gate_param || !spec->gate_axis) return fail(PTSBE_ERR_INVALID_ARG, "null gate parameter arrays");
  if (spec->n_terms > 0 && (!spec->zz_qubits || !spec->zz_coef)) return fail(PTSBE_ERR_INVALID_ARG, "null terms");
  L.G = p.G;
  L.C = spec->checkpoint_every;
  L.gate_param.assign(p.G, -1);
  L.gate_axis.assign(p.G, 0);
  L.gate_slot.assign(p.G, -1);
  // gates after the caller's circuit are identities the plan added for untouched qubits
  for (int g = 0; g < p.n_user_gates; ++g) {
    const int prm = spec->gate_param[g];
    if (prm >= spec->n_params) return fail(PTSBE_ERR_INVALID_ARG, "parameter index out of range");
    if (prm >= 0) {
      if (p.arity[g] != 1) return fail(PTSBE_ERR_UNSUPPORTED, "rotation gates must act on one qubit");
      const int ax = spec->gate_axis[g];
      if (ax < 0 || ax > 2) return fail(PTSBE_ERR_INVALID_ARG, "rotation axis must be 0, 1 or 2");
      L.gate_param[g] = prm;
      L.gate_axis[g] = ax;
      L.gate_slot[g] = L.n_slots++;
      L.slot_param.push_back(prm);
    }
  }
  for (int t = 0; t < spec->n_terms; ++t) {
    const int a = spec->zz_qubits[2 * t], b = spec->zz_qubits[2 * t + 1];
    if (a < 0 || a >= p.n || b < 0 || b >= p.n) return fail(PTSBE_ERR_INVALID_ARG, "observable qubit out of range");
    L.zq.push_back(a);
    L.zq.push_back(b);
    L.zc.push_back(spec->zz_coef[t]);
  }
  if (L.slot_param.empty()) L.slot_param.push_back(-1);
  if (L.zq.empty()) { L.zq.push_back(0); L.zq.push_back(0); L.zc.push_back(0.0); }
  L.n_ck = (p.G + L.C - 1) / L.C;
  return PTSBE_OK;
}

size_t fixed_bytes(const Plan& p, const GradLayout& L, int64_t E) {
  size_t b = 0;
  auto add = [&](size_t x) { b += (x + 255) & ~(size_t)255; };
  add((size_t)E * p.G * 128);                    // merged
  add((size_t)E * p.G * 128);                    // dagger
  add((size_t)E * std::max(L.n_slots, 1) * 128); // dA
  add((size_t)E * std::max(L.n_slots, 1) * 8);   // partials
  add((size_t)E * 8);                            // per-trajectory values
  add((size_t)p.G * 4 * 3 + L.slot_param.size() * 4 + L.zq.size() * 4 + L.zc.size() * 8 + 4096);
  return b;
}

size_t per_traj_bytes(const Plan& p, const GradLayout& L) {
  return (size_t)(2 + L.n_ck + L.C) * ((size_t)8 << p.n);
}

}  // namespace

extern "C" {

ptsbe_status_t ptsbe_expect_workspace_size(ptsbe_plan_t plan, const ptsbe_grad_spec_t* spec, int64_t E,
                                           size_t* bytes) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p || !bytes) return fail(PTSBE_ERR_INVALID_ARG, "null argument");
  GradLayout L;
  ptsbe_status_t st = check_spec(*p, spec, L);
  if (st != PTSBE_OK) return st;
  *bytes = fixed_bytes(*p, L, E) + std::min<int64_t>(E, 64) * per_traj_bytes(*p, L) + (1 << 20);
  return PTSBE_OK;
}

ptsbe_status_t ptsbe_expect_grad(ptsbe_plan_t plan, const ptsbe_grad_spec_t* spec, const uint8_t* d_kraus_idx,
                                 int64_t E, const double* d_weights, const double* d_theta, double* d_traj_value,
                                 double* d_value, double* d_grad, void* d_workspace, size_t workspace_bytes,
                                 void* stream) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(PTSBE_ERR_INVALID_ARG, "null plan");
  if (p->device < 0) return fail(PTSBE_ERR_INVALID_ARG, "plan was built without a device");
  if (E < 1) return fail(PTSBE_ERR_INVALID_ARG, "E < 1");
  if (!d_kraus_idx || !d_weights || !d_value || !d_workspace) return fail(PTSBE_ERR_INVALID_ARG, "null pointer");
  GradLayout L;
  ptsbe_status_t st = check_spec(*p, spec, L);
  if (st != PTSBE_OK) return st;
  if (spec->n_params > 0 && !d_theta) return fail(PTSBE_ERR_INVALID_ARG, "null theta");
  HIP_TRY(hipSetDevice(p->device));
  hipStream_t s = (hipStream_t)stream;
  Arena ar;
  ar.base = (char*)d_workspace;
  ar.cap = workspace_bytes;
  const int n = p->n;
  const int ns = std::max(L.n_slots, 1);
  float2* merged = (float2*)ar.take((size_t)E * p->G * 128);
  float2* dagger = (float2*)ar.take((size_t)E * p->G * 128);
  float2* dmerged = (float2*)ar.take((size_t)E * ns * 128);
  double* partial = (double*)ar.take((size_t)E * ns * 8);
  double* vals = (double*)ar.take((size_t)E * 8);
  int32_t* d_gp = (int32_t*)ar.take((size_t)p->G * 4);
  int32_t* d_ga = (int32_t*)ar.take((size_t)p->G * 4);
  int32_t* d_gs = (int32_t*)ar.take((size_t)p->G * 4);
  int32_t* d_sp = (int32_t*)ar.take(L.slot_param.size() * 4);
  int32_t* d_zq = (int32_t*)ar.take(L.zq.size() * 4);
  double* d_zc = (double*)ar.take(L.zc.size() * 8);
  if (!d_zc) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for the gate tables");
  HIP_TRY(hipMemcpyAsync(d_gp, L.gate_param.data(), (size_t)p->G * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_ga, L.gate_axis.data(), (size_t)p->G * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_gs, L.gate_slot.data(), (size_t)p->G * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_sp, L.slot_param.data(), L.slot_param.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_zq, L.zq.data(), L.zq.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_zc, L.zc.data(), L.zc.size() * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));   // the host tables above are about to go out of scope
  // error injection + rotation angles: A, A^dag and dA/dtheta of every (trajectory, gate)
  ptsbe::GateCtx g{};
  g.gates = p->d_gates;
  g.gate_site_list = p->d_gate_site_list;
  g.site_ops = p->d_site_ops;
  g.kraus = d_kraus_idx;
  g.S = p->S;
  g.max_kraus = p->max_kraus;
  g.G = p->G;
  ptsbe::GradGateArgs ga{g, E, d_gp, d_ga, d_gs, L.n_slots, d_theta, merged, dagger, dmerged};
  HIP_TRY(ptsbe::launch_grad_gates(ga, s));
  ptsbe::GateCtx gf = g, gb = g;
  gf.merged = merged;
  gb.merged = dagger;
  const size_t per = per_traj_bytes(*p, L);
  const size_t avail = ar.left() > ((size_t)1 << 20) ? ar.left() - ((size_t)1 << 20) : 0;   // alignment slack
  const int64_t Ec = std::min<int64_t>(E, (int64_t)(avail / per));
  if (Ec < 1) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for one trajectory's states");
  const int64_t SZ = (int64_t)1 << n;
  const int G = p->G;
  for (int64_t t0 = 0; t0 < E; t0 += Ec) {
    const int64_t nj = std::min<int64_t>(Ec, E - t0);
    const size_t mark = ar.used;
    float2* psi = (float2*)ar.take((size_t)nj * SZ * 8);
    float2* lam = (float2*)ar.take((size_t)nj * SZ * 8);
    std::vector<float2*> ck(L.n_ck), seg(L.C + 1);
    for (auto& c : ck) c = (float2*)ar.take((size_t)nj * SZ * 8);
    for (int i = 1; i <= L.C; ++i) seg[i] = (float2*)ar.take((size_t)nj * SZ * 8);
    if (!seg[L.C] && L.C > 0) return fail(PTSBE_ERR_OUT_OF_MEMORY, "workspace too small for the checkpoints");
    // forward
    HIP_TRY(ptsbe::launch_state_init(psi, nj, n, s));
    for (int k = 0; k < G; ++k) {
      if (k % L.C == 0) HIP_TRY(ptsbe::launch_copy(psi, ck[k / L.C], nj * SZ, s));
      HIP_TRY(ptsbe::launch_absorb_global(p->sv_steps[k], p->d_sv_steps + k, gf, nj, nullptr, (int32_t)t0,
                                          nullptr, p->NW, psi, psi, s));
    }
    HIP_TRY(ptsbe::launch_observable(psi, lam, nj, n, d_zq, d_zc, (int)L.zc.size(), vals, t0, s));
    if (d_grad && L.n_slots > 0) {
      for (int c = L.n_ck - 1; c >= 0; --c) {
        const int k0 = c * L.C, k1 = std::min(G, k0 + L.C);
        seg[0] = ck[c];
        for (int k = k0; k < k1 - 1; ++k)
          HIP_TRY(ptsbe::launch_absorb_global(p->sv_steps[k], p->d_sv_steps + k, gf, nj, nullptr, (int32_t)t0,
                                              nullptr, p->NW, seg[k - k0], seg[k - k0 + 1], s));
        for (int k = k1 - 1; k >= k0; --k) {
          const int slot = L.gate_slot[k];
          if (slot >= 0)
            HIP_TRY(ptsbe::launch_grad_reduce(lam, seg[k - k0], nj, n, p->arity[k], p->qubits[k][0],
                                              p->arity[k] == 2 ? p->qubits[k][1] : 0, dmerged, L.n_slots, slot,
                                              d_weights, t0, partial, s));
          HIP_TRY(ptsbe::launch_absorb_global(p->sv_steps[k], p->d_sv_steps + k, gb, nj, nullptr, (int32_t)t0,
                                              nullptr, p->NW, lam, lam, s));
        }
      }
    }
    ar.used = mark;
  }
  if (d_traj_value) HIP_TRY(hipMemcpyAsync(d_traj_value, vals, (size_t)E * 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(ptsbe::launch_value_sum(vals, d_weights, E, d_value, s));
  if (d_grad && spec->n_params > 0) {
    if (L.n_slots > 0) {
      HIP_TRY(ptsbe::launch_grad_sum(partial, E, L.n_slots, d_sp, spec->n_params, d_grad, s));
    } else {
      HIP_TRY(hipMemsetAsync(d_grad, 0, (size_t)spec->n_params * 8, s));
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  return PTSBE_OK;
}

}  // extern "C"
