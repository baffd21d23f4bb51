// Host planner: one unified, error-independent contraction path per qubit batch.
//
// Unified path variations (Sec. III-A): every sampled noise operator is merged
// into the gate it follows, so every trajectory's network has the structure of
// the noiseless circuit and one path serves all error sets and all shots.  The
// path is found once per batch, on the host, outside the timed loop.
//
// Network of batch j (Sec. II-B; prefix s_<j projected):
//   * j < f-1: ket network x conjugate (bra) network; prefix outputs sliced to
//     the element's bits on both sides, batch outputs shared by ket and bra and
//     left open (diagonal), later outputs shared and summed (trace);
//   * j = f-1: ket network only, prefix outputs sliced, batch outputs open.
// The network is split into a per-element LEFT part (ket gates touching a
// prefix qubit; its bra copy is its complex conjugate and is never formed) and
// a per-trajectory RIGHT part (all other gates, ket and bra).  Each part is
// contracted as a sweep that absorbs one gate tensor at a time into a running
// tensor; the order is the cheapest of several structured sweeps and of
// `hypersamples` randomised greedy sweeps.  A final join contracts the two parts:
//   doubled: pi[xT, xb] = sum_{k,k'} V[xb, k] T[xT, k, k'] conj(V[xb, k'])
//   ket:     amp[xT, xb] = sum_k V[xb, k] T[xT, k]
// with k the wires crossing from the left to the right part.
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <random>
#include <set>

#include "internal.h"

namespace ptsbe {
namespace {

enum : int8_t { SL_NONE = 0, SL_ZERO = 1, SL_PREFIX = 2 };

struct NetTensor {
  int gate = 0, conj = 0, nlegs = 0, col = 0, time = 0;
  int label[4] = {-1, -1, -1, -1};
  int8_t slice[4] = {0, 0, 0, 0};
  int sq[4] = {0, 0, 0, 0};
  int weight[4] = {0, 0, 0, 0};
};

struct KetNet {
  std::vector<std::array<int, 2>> in_label, out_label;  // per gate, per qubit slot
  std::vector<int> final_label, last_gate;
  int n_labels = 0;
};

KetNet build_ket(const Plan& p) {
  KetNet k;
  k.in_label.assign(p.G, {-1, -1});
  k.out_label.assign(p.G, {-1, -1});
  std::vector<int> wire(p.n, -1);
  k.last_gate.assign(p.n, -1);
  int next = 0;
  for (int g = 0; g < p.G; ++g) {
    for (int a = 0; a < p.arity[g]; ++a) {
      int q = p.qubits[g][a];
      k.in_label[g][a] = wire[q];
      k.out_label[g][a] = next++;
      wire[q] = k.out_label[g][a];
      k.last_gate[q] = g;
    }
  }
  k.final_label = wire;
  k.n_labels = next;
  return k;
}

// Simulate absorbing `order` into a running tensor; keep_open labels survive.
bool simulate(const std::vector<const NetTensor*>& order, const std::set<int>& keep_open,
              const std::vector<int>& init, PartPlan& out, std::string& err) {
  std::map<int, int> cnt;
  for (const NetTensor* t : order)
    for (int i = 0; i < t->nlegs; ++i)
      if (t->label[i] >= 0) cnt[t->label[i]]++;
  std::vector<int> cur = init;
  out.peak = (int)init.size();
  out.steps.clear();
  out.flops = out.bytes = 0;
  for (const NetTensor* t : order) {
    AbsorbStep st{};
    st.gate = t->gate;
    st.conj = t->conj;
    st.rA = (int)cur.size();
    std::vector<std::pair<int, int>> K;   // (pos in A, weight)
    std::vector<std::pair<int, int>> H;   // (label, weight)
    std::vector<std::pair<int, int>> N;   // (label, weight)
    for (int i = 0; i < t->nlegs; ++i) {
      if (t->slice[i] == SL_ZERO) continue;
      if (t->slice[i] == SL_PREFIX) {
        if (st.nS >= kMaxSlices) { err = "too many sliced legs on one gate"; return false; }
        st.sq[st.nS] = t->sq[i];
        st.sw[st.nS] = t->weight[i];
        st.nS++;
        continue;
      }
      int L = t->label[i];
      cnt[L]--;
      auto it = std::find(cur.begin(), cur.end(), L);
      if (it != cur.end()) {
        int pos = (int)(it - cur.begin());
        if (cnt[L] == 0 && !keep_open.count(L)) K.push_back({pos, t->weight[i]});
        else H.push_back({L, t->weight[i]});
      } else {
        if (cnt[L] == 0 && !keep_open.count(L)) { err = "dangling label in network"; return false; }
        N.push_back({L, t->weight[i]});
      }
    }
    std::sort(K.begin(), K.end());
    std::vector<int> kept;
    {
      std::vector<char> drop(cur.size(), 0);
      for (auto& kk : K) drop[kk.first] = 1;
      for (size_t i = 0; i < cur.size(); ++i)
        if (!drop[i]) kept.push_back(cur[i]);
    }
    // C layout: new labels replace contracted ones in place (lowest first),
    // surplus contracted positions are dropped, surplus new labels go on top.
    std::vector<int> C = cur;
    size_t nrep = std::min(K.size(), N.size());
    for (size_t i = 0; i < nrep; ++i) C[K[i].first] = N[i].first;
    if (K.size() > N.size()) {
      std::vector<char> drop(C.size(), 0);
      for (size_t i = nrep; i < K.size(); ++i) drop[K[i].first] = 1;
      std::vector<int> c2;
      for (size_t i = 0; i < C.size(); ++i)
        if (!drop[i]) c2.push_back(C[i]);
      C.swap(c2);
    } else {
      for (size_t i = nrep; i < N.size(); ++i) C.push_back(N[i].first);
    }
    st.nK = (int)K.size();
    for (int i = 0; i < st.nK; ++i) { st.kpos[i] = K[i].first; st.kw[i] = K[i].second; }
    std::map<int, int> wN;
    for (auto& nn : N) wN[nn.first] = nn.second;
    std::vector<std::pair<int, int>> npos;
    for (size_t i = 0; i < C.size(); ++i)
      if (wN.count(C[i])) npos.push_back({(int)i, wN[C[i]]});
    std::sort(npos.begin(), npos.end());
    st.nN = (int)npos.size();
    for (int i = 0; i < st.nN; ++i) { st.npos[i] = npos[i].first; st.nw[i] = npos[i].second; }
    st.nH = (int)H.size();
    for (int i = 0; i < st.nH; ++i) {
      auto it = std::find(kept.begin(), kept.end(), H[i].first);
      st.hm[i] = (int)(it - kept.begin());
      st.hw[i] = H[i].second;
    }
    // sanity: C without the new positions equals kept
    {
      std::vector<int> chk;
      std::set<int> np;
      for (int i = 0; i < st.nN; ++i) np.insert(st.npos[i]);
      for (size_t i = 0; i < C.size(); ++i)
        if (!np.count((int)i)) chk.push_back(C[i]);
      if (chk != kept) { err = "internal layout error"; return false; }
    }
    st.rC = (int)C.size();
    if (st.rC > 31 || st.rA > 31) { err = "intermediate too large"; return false; }
    for (int k = 0; k < (1 << st.nK); ++k) {
      st.koff[k] = 0; st.kB[k] = 0;
      for (int i = 0; i < st.nK; ++i)
        if ((k >> i) & 1) { st.koff[k] += 1u << st.kpos[i]; st.kB[k] += st.kw[i]; }
    }
    for (int n = 0; n < (1 << st.nN); ++n) {
      st.noff[n] = 0; st.nB[n] = 0;
      for (int i = 0; i < st.nN; ++i)
        if ((n >> i) & 1) { st.noff[n] += 1u << st.npos[i]; st.nB[n] += st.nw[i]; }
    }
    st.gperm[0] = 0x76543210u; st.gperm[1] = 0xFEDCBA98u;
    if (st.nH == 0 && st.nS == 0) {
      const int nk = 1 << st.nK, nn = 1 << st.nN;
      for (int n = 0; n < nn; ++n)
        for (int k = 0; k < nk; ++k) {
          const int d = n * nk + k;
          const uint32_t src = (uint32_t)(st.nB[n] + st.kB[k]) & 15u;
          st.gperm[d >> 3] = (st.gperm[d >> 3] & ~(15u << (4 * (d & 7)))) | (src << (4 * (d & 7)));
        }
    }
    out.peak = std::max(out.peak, std::max(st.rA, st.rC));
    double m = std::ldexp(1.0, st.rC - st.nN);
    out.flops += 8.0 * m * std::ldexp(1.0, st.nN + st.nK);
    out.bytes += 8.0 * (std::ldexp(1.0, st.rA) + std::ldexp(1.0, st.rC));
    out.steps.push_back(st);
    cur = C;
  }
  for (int L : cur)
    if (!keep_open.count(L)) { err = "label left open"; return false; }
  out.labels = cur;
  out.cost = out.bytes + out.flops / 16.0;
  return true;
}

std::vector<const NetTensor*> sorted_order(const std::vector<NetTensor>& ts, int colsign, int timesign,
                                           bool time_major) {
  std::vector<const NetTensor*> o;
  for (auto& t : ts) o.push_back(&t);
  std::stable_sort(o.begin(), o.end(), [&](const NetTensor* a, const NetTensor* b) {
    if (time_major) {
      if (a->time != b->time) return timesign * a->time < timesign * b->time;
      if (a->col != b->col) return colsign * a->col < colsign * b->col;
      return a->conj < b->conj;
    }
    if (a->col != b->col) return colsign * a->col < colsign * b->col;
    if (a->time != b->time) return timesign * a->time < timesign * b->time;
    return a->conj < b->conj;
  });
  return o;
}

// Randomised greedy sweep: repeatedly absorb the tensor that gives the smallest
// running rank (ties: most contracted legs, then random).
std::vector<const NetTensor*> greedy_order(const std::vector<NetTensor>& ts, const std::set<int>& keep_open,
                                           const std::vector<int>& init, std::mt19937_64& rng) {
  std::map<int, int> cnt;
  for (auto& t : ts)
    for (int i = 0; i < t.nlegs; ++i)
      if (t.label[i] >= 0) cnt[t.label[i]]++;
  std::set<int> cur(init.begin(), init.end());
  std::vector<char> used(ts.size(), 0);
  std::vector<const NetTensor*> order;
  std::uniform_real_distribution<double> U(0.0, 1.0);
  for (size_t step = 0; step < ts.size(); ++step) {
    double best = 1e300;
    int bi = -1;
    for (size_t i = 0; i < ts.size(); ++i) {
      if (used[i]) continue;
      const NetTensor& t = ts[i];
      int delta = 0, kk = 0;
      bool touches = cur.empty();
      for (int l = 0; l < t.nlegs; ++l) {
        int L = t.label[l];
        if (L < 0) continue;
        if (cur.count(L)) {
          touches = true;
          if (cnt[L] == 1 && !keep_open.count(L)) { delta--; kk++; }
        } else {
          delta++;
        }
      }
      double score = (double)(cur.size() + delta) * 4.0 - kk + (touches ? 0.0 : 100.0) + U(rng) * 0.9;
      if (score < best) { best = score; bi = (int)i; }
    }
    used[bi] = 1;
    const NetTensor& t = ts[bi];
    order.push_back(&t);
    for (int l = 0; l < t.nlegs; ++l) {
      int L = t.label[l];
      if (L < 0) continue;
      cnt[L]--;
      if (cur.count(L)) {
        if (cnt[L] == 0 && !keep_open.count(L)) cur.erase(L);
      } else {
        cur.insert(L);
      }
    }
  }
  return order;
}

bool plan_part(const std::vector<NetTensor>& ts, const std::set<int>& keep_open, int hypersamples,
               uint64_t seed, PartPlan& best, std::string& err, const std::vector<int>& init = {}) {
  best = PartPlan();
  best.cost = 1e300;
  if (ts.empty()) {
    for (int L : init)
      if (!keep_open.count(L)) { err = "label left open"; return false; }
    best.cost = 0;
    best.order_name = "empty";
    best.labels = init;
    best.peak = (int)init.size();
    return true;
  }
  struct Cand { const char* name; int cs, tsg; bool tm; };
  const Cand cands[] = {{"col+time+", 1, 1, false}, {"col+time-", 1, -1, false},
                        {"col-time+", -1, 1, false}, {"col-time-", -1, -1, false},
                        {"time+", 1, 1, true},       {"time-", 1, -1, true}};
  bool any = false;
  std::string last_err;
  for (const Cand& c : cands) {
    PartPlan pp;
    std::string e;
    if (!simulate(sorted_order(ts, c.cs, c.tsg, c.tm), keep_open, init, pp, e)) { last_err = e; continue; }
    pp.order_name = c.name;
    if (pp.cost < best.cost) best = pp;
    any = true;
  }
  std::mt19937_64 rng(seed);
  for (int h = 0; h < hypersamples; ++h) {
    PartPlan pp;
    std::string e;
    if (!simulate(greedy_order(ts, keep_open, init, rng), keep_open, init, pp, e)) { last_err = e; continue; }
    pp.order_name = "greedy";
    if (pp.cost < best.cost) best = pp;
    any = true;
  }
  if (!any) { err = "no feasible sweep: " + last_err; return false; }
  return true;
}

SplitTable make_table(const std::vector<int>& group, const std::vector<int>& labels, int64_t unit = 1) {
  // offset of group index g = sum over set bits i of g of (unit << position of group[i])
  SplitTable t;
  t.bits = (int)group.size();
  t.lo_bits = std::min(t.bits, 12);
  std::vector<int64_t> w(group.size());
  for (size_t i = 0; i < group.size(); ++i) {
    auto it = std::find(labels.begin(), labels.end(), group[i]);
    w[i] = unit << (int)(it - labels.begin());
  }
  int hb = t.bits - t.lo_bits;
  t.lo.assign((size_t)1 << t.lo_bits, 0);
  t.hi.assign((size_t)1 << hb, 0);
  for (size_t g = 0; g < t.lo.size(); ++g)
    for (int i = 0; i < t.lo_bits; ++i)
      if ((g >> i) & 1) t.lo[g] += w[i];
  for (size_t g = 0; g < t.hi.size(); ++g)
    for (int i = 0; i < hb; ++i)
      if ((g >> i) & 1) t.hi[g] += w[t.lo_bits + i];
  return t;
}

SplitTable make_out_table(const std::vector<int>& group, const std::vector<int>& group_qubit, int start) {
  SplitTable t;
  t.bits = (int)group.size();
  t.lo_bits = std::min(t.bits, 12);
  int hb = t.bits - t.lo_bits;
  t.lo.assign((size_t)1 << t.lo_bits, 0);
  t.hi.assign((size_t)1 << hb, 0);
  for (size_t g = 0; g < t.lo.size(); ++g)
    for (int i = 0; i < t.lo_bits; ++i)
      if ((g >> i) & 1) t.lo[g] += (int64_t)1 << (group_qubit[i] - start);
  for (size_t g = 0; g < t.hi.size(); ++g)
    for (int i = 0; i < hb; ++i)
      if ((g >> i) & 1) t.hi[g] += (int64_t)1 << (group_qubit[t.lo_bits + i] - start);
  return t;
}

}  // namespace

// Gates of the doubled network for measured qubits [0, e) under the light cone
// (an extension of the unified path that Sec. VI names as open): in rho = U rho0
// U^dag traced over the later qubits, a unitary gate whose outputs reach no
// measured qubit and no kept non-unitary operator meets its own adjoint and
// cancels, U^dag U = I.  Walking back in time from the measured outputs, a gate is
// kept when it touches a live qubit or is not unitary for some trajectory (its
// sites may insert a non-unitary K / sqrt(q), whose K^dag K does not cancel); a
// kept gate makes all its qubits live.  The kept set depends on the channel
// types only, never on a trajectory's Kraus choices, so one path still serves
// every error set.
std::vector<char> light_cone_keep(const Plan& p, int e) {
  std::vector<char> keep((size_t)p.G, 0), live((size_t)p.n, 0);
  for (int q = 0; q < e; ++q) live[(size_t)q] = 1;
  for (int g = p.G - 1; g >= 0; --g) {
    bool k = !p.gate_unitary[(size_t)g];
    for (int a = 0; a < p.arity[(size_t)g]; ++a) k = k || live[(size_t)p.qubits[(size_t)g][(size_t)a]];
    if (!k) continue;
    keep[(size_t)g] = 1;
    for (int a = 0; a < p.arity[(size_t)g]; ++a) live[(size_t)p.qubits[(size_t)g][(size_t)a]] = 1;
  }
  return keep;
}

bool build_batch_plans(Plan& p, std::string& err) {
  const KetNet k = build_ket(p);
  const int NL = k.n_labels;
  int f = (int)p.batch_sizes.size();
  p.batches.clear();
  int start = 0;
  for (int j = 0; j < f; ++j) {
    BatchPlan bp;
    bp.start = start;
    bp.size = p.batch_sizes[j];
    bp.doubled = (j < f - 1);
    const int a = start, e = start + bp.size;
    auto cls = [&](int q) { return q < a ? 0 : (q < e ? 1 : 2); };  // prefix/batch/rest
    // gates of this batch's network; with the light cone, a qubit's output is the
    // last kept gate's (labels keep the full circuit's numbering), and a qubit
    // with no kept gate drops out (its |0><0| traces to 1)
    std::vector<char> keep = bp.doubled && p.light_cone ? light_cone_keep(p, e) : std::vector<char>((size_t)p.G, 1);
    std::vector<int> final_label((size_t)p.n, -1);
    for (int g = 0; g < p.G; ++g)
      if (keep[(size_t)g])
        for (int s = 0; s < p.arity[g]; ++s) final_label[(size_t)p.qubits[g][s]] = k.out_label[g][s];
    bp.kept_gates = (int)std::count(keep.begin(), keep.end(), (char)1);
    std::vector<int> final_of(NL, -1);  // label -> qubit whose final output it is
    for (int q = 0; q < p.n; ++q)
      if (final_label[(size_t)q] >= 0) final_of[final_label[(size_t)q]] = q;
    auto bra_label = [&](int L) {
      int q = final_of[L];
      if (q >= 0 && cls(q) != 0) return L;   // batch / rest outputs are shared
      return L + NL;
    };
    std::vector<NetTensor> left, right;
    for (int g = 0; g < p.G; ++g) {
      if (!keep[(size_t)g]) continue;
      bool is_left = false;
      for (int s = 0; s < p.arity[g]; ++s) is_left |= cls(p.qubits[g][s]) == 0;
      for (int side = 0; side < (bp.doubled ? 2 : 1); ++side) {
        if (is_left && side == 1) continue;  // bra of the left part = conj(V)
        NetTensor t;
        t.gate = g;
        t.conj = side;
        t.time = g;
        t.col = std::max(p.qubits[g][0], p.arity[g] == 2 ? p.qubits[g][1] : -1);
        int ar = p.arity[g];
        t.nlegs = 2 * ar;
        // legs: outputs then inputs, first listed qubit is the high index bit
        for (int s = 0; s < ar; ++s) {
          int wout = ar == 2 ? (s == 0 ? 8 : 4) : 2;
          int win = ar == 2 ? (s == 0 ? 2 : 1) : 1;
          int Lo = k.out_label[g][s], Li = k.in_label[g][s];
          // output leg
          int qo = final_of[Lo];
          if (qo >= 0 && cls(qo) == 0) {
            t.slice[s] = SL_PREFIX;
            t.sq[s] = qo;
            t.label[s] = -1;
          } else {
            t.label[s] = side ? bra_label(Lo) : Lo;
          }
          t.weight[s] = wout;
          // input leg
          if (Li < 0) {
            t.slice[ar + s] = SL_ZERO;
            t.label[ar + s] = -1;
          } else {
            t.label[ar + s] = side ? bra_label(Li) : Li;
          }
          t.weight[ar + s] = win;
        }
        (is_left ? left : right).push_back(t);
      }
    }
    // label groups
    std::set<int> left_labels, right_labels;
    for (auto& t : left)
      for (int i = 0; i < t.nlegs; ++i)
        if (t.label[i] >= 0) left_labels.insert(t.label[i]);
    for (auto& t : right)
      for (int i = 0; i < t.nlegs; ++i)
        if (t.label[i] >= 0) right_labels.insert(t.label[i]);
    std::vector<int> xb_q, xT_q;
    for (int q = a; q < e; ++q) {
      int L = final_label[(size_t)q];
      if (left_labels.count(L)) { bp.xb.push_back(L); xb_q.push_back(q); }
      else { bp.xT.push_back(L); xT_q.push_back(q); }
    }
    if (bp.doubled) {
      for (int q = e; q < p.n; ++q)
        if (final_label[(size_t)q] >= 0 && left_labels.count(final_label[(size_t)q])) {
          err = "unsupported network: a later qubit's output lies on a gate that touches the prefix";
          return false;
        }
    }
    for (int L : left_labels)
      if (L < NL && right_labels.count(L) && final_of[L] < 0) bp.lk.push_back(L);
    for (int L : bp.lk) bp.lb.push_back(L + NL);
    std::string e1;
    std::set<int> keep_right(bp.lk.begin(), bp.lk.end());
    keep_right.insert(bp.xT.begin(), bp.xT.end());
    if (bp.doubled) keep_right.insert(bp.lb.begin(), bp.lb.end());
    bool right_ok = plan_part(right, keep_right, p.hypersamples, p.path_seed * 1315423911ULL + 2 * j + 2, bp.right, e1);
    if (right_ok && !bp.doubled && bp.right.peak > p.max_part_rank) {
      right_ok = false;
      e1 = "per-trajectory tensor of rank " + std::to_string(bp.right.peak) + " above max_part_rank";
    }
    if (!right_ok && !bp.doubled) {
      // Slicing (last batch): fix the first s crossing wires (the earliest labels)
      // on both parts to each of their values in turn; sliced legs read prefix bit
      // n + i, which must lie in the last prefix word, past the qubits' bits.
      const std::vector<int> lk_all = bp.lk;
      for (int sb = 1; sb <= (int)lk_all.size() && !right_ok; ++sb) {
        if ((p.n >> 6) != ((p.n + sb - 1) >> 6) || p.n + sb > 64 * p.NW) break;
        std::map<int, int> sl_idx;
        for (int i = 0; i < sb; ++i) sl_idx[lk_all[(size_t)i]] = i;
        auto slice_legs = [&](std::vector<NetTensor>& ts) {
          for (auto& t : ts)
            for (int i = 0; i < t.nlegs; ++i) {
              auto it = t.label[i] >= 0 ? sl_idx.find(t.label[i]) : sl_idx.end();
              if (it == sl_idx.end()) continue;
              t.slice[i] = SL_PREFIX;
              t.sq[i] = p.n + it->second;
              t.label[i] = -1;
            }
        };
        std::vector<NetTensor> right_s = right;
        slice_legs(right_s);
        std::set<int> keep_s(lk_all.begin() + sb, lk_all.end());
        keep_s.insert(bp.xT.begin(), bp.xT.end());
        std::string e2;
        PartPlan rp;
        if (!plan_part(right_s, keep_s, p.hypersamples, p.path_seed * 1315423911ULL + 2 * j + 2, rp, e2)) continue;
        if (rp.peak > p.max_part_rank) continue;
        right_ok = true;
        bp.right = rp;
        right = right_s;
        slice_legs(left);
        bp.slice_bits = sb;
        bp.slice_labels.assign(lk_all.begin(), lk_all.begin() + sb);
        bp.lk.assign(lk_all.begin() + sb, lk_all.end());
      }
    }
    if (!right_ok) {
      err = "batch " + std::to_string(j) + " right part: " + e1;
      return false;
    }
    std::set<int> keep_left(bp.lk.begin(), bp.lk.end());
    keep_left.insert(bp.xb.begin(), bp.xb.end());
    if (!plan_part(left, keep_left, p.hypersamples, p.path_seed * 1315423911ULL + 2 * j + 1, bp.left, e1)) {
      err = "batch " + std::to_string(j) + " left part: " + e1;
      return false;
    }
    if ((int)bp.lk.size() > 12) {
      err = "batch " + std::to_string(j) + ": " + std::to_string(bp.lk.size()) +
            " wires cross between the prefix part and the rest (limit 12)";
      return false;
    }
    // Resume variant of the left part (used by the sampling loop): start from the
    // parent element's left tensor of batch j-1, whose open batch legs are now
    // prefix outputs and get sliced to the element's bits, and absorb only the
    // gates that touch the newly projected qubits.
    if (j >= 1) {
      const BatchPlan& pv = p.batches[j - 1];
      const std::vector<int>& plabels = (j - 1 == 0) ? pv.left.labels : pv.left_resume.labels;
      std::set<int> pgates(pv.left_gates.begin(), pv.left_gates.end());
      std::vector<int> init;
      std::vector<std::pair<int, int>> sl;   // (position in parent tensor, qubit)
      for (size_t i = 0; i < plabels.size(); ++i) {
        auto it = std::find(pv.xb.begin(), pv.xb.end(), plabels[i]);
        auto is = std::find(bp.slice_labels.begin(), bp.slice_labels.end(), plabels[i]);
        if (it != pv.xb.end()) sl.push_back({(int)i, pv.xb_qubits[it - pv.xb.begin()]});
        else if (is != bp.slice_labels.end()) sl.push_back({(int)i, p.n + (int)(is - bp.slice_labels.begin())});
        else init.push_back(plabels[i]);
      }
      std::vector<NetTensor> delta;
      for (auto& t : left)
        if (!pgates.count(t.gate)) delta.push_back(t);
      if (!plan_part(delta, keep_left, p.hypersamples, p.path_seed * 1315423911ULL + 2 * j + 7, bp.left_resume, e1,
                     init)) {
        err = "batch " + std::to_string(j) + " resumed left part: " + e1;
        return false;
      }
      bp.resume_rank0 = (int)init.size();
      bp.resume_parent_rank = (int)plabels.size();
      for (auto& x : sl) { bp.resume_slice_pos.push_back(x.first); bp.resume_slice_q.push_back(x.second); }
      if (bp.resume_slice_pos.size() > 8) {
        err = "batch " + std::to_string(j) + ": too many open batch legs on the prefix part";
        return false;
      }
      bp.v_row_r = make_table(bp.xb, bp.left_resume.labels);
      bp.v_col_r = make_table(bp.lk, bp.left_resume.labels);
    }
    for (auto& t : left) bp.left_gates.push_back(t.gate);
    bp.xb_qubits = xb_q;
    // join tables
    bp.v_row = make_table(bp.xb, bp.left.labels);
    bp.v_col = make_table(bp.lk, bp.left.labels);
    bp.t_x = make_table(bp.xT, bp.right.labels);
    bp.t_k = make_table(bp.lk, bp.right.labels);
    bp.t_b = make_table(bp.doubled ? bp.lb : std::vector<int>(), bp.right.labels);
    bp.o_x = make_out_table(bp.xT, xT_q, a);
    bp.o_b = make_out_table(bp.xb, xb_q, a);
    double rows = std::ldexp(1.0, (int)bp.xb.size() + bp.slice_bits);   // one join per slice
    double K = std::ldexp(1.0, (int)bp.lk.size());
    double X = std::ldexp(1.0, (int)bp.xT.size());
    if (bp.doubled && qform_supported((int)bp.lk.size())) {
      // MFMA join: the real bilinear form over K^2 folded slots, 2 flops per
      // slot, per row and x
      bp.join_flops_per_elem = rows * X * 2.0 * K * K;
    } else {
      bp.join_flops_per_elem = bp.doubled ? rows * X * (8.0 * K * K + 8.0 * K) : rows * X * 8.0 * K;
    }
    p.batches.push_back(bp);
    start = e;
  }
  return true;
}

}  // namespace ptsbe

namespace ptsbe {

// Group a step list into launches: maximal runs of in-place steps (rank and bit
// positions unchanged) whose positions fit in kFuseMax bits become one fused
// tile pass; every other step is launched alone.  P is padded with the lowest
// unused positions so that a tile covers contiguous memory where possible.
namespace {
// One in-place step re-expressed on the positions of a fused window P (sorted):
// window-local index bits for its legs, and the bits of hyper legs either inside
// the window (local) or outside it (taken from the tile's base offset).
FusedStep make_fused_step(const AbsorbStep& st, const std::vector<int>& Pv) {
  FusedStep fs{};
  auto in_P = [&](int pos) { return std::find(Pv.begin(), Pv.end(), pos) != Pv.end(); };
  fs.gate = st.gate; fs.conj = st.conj; fs.nK = st.nK; fs.nN = st.nN; fs.nH = st.nH; fs.nS = st.nS;
  auto loc = [&](int pos) { return (int)(std::find(Pv.begin(), Pv.end(), pos) - Pv.begin()); };
  for (int k = 0; k < st.nK; ++k) fs.kloc[k] = loc(st.kpos[k]);
  for (int k = 0; k < (1 << st.nK); ++k) {
    fs.koff[k] = 0;
    fs.kB[k] = st.kB[k];
    for (int b = 0; b < st.nK; ++b)
      if ((k >> b) & 1) fs.koff[k] += 1u << loc(st.kpos[b]);
  }
  for (int nn = 0; nn < (1 << st.nN); ++nn) {
    fs.noff[nn] = 0;
    fs.nB[nn] = st.nB[nn];
    for (int b = 0; b < st.nN; ++b)
      if ((nn >> b) & 1) fs.noff[nn] += 1u << loc(st.npos[b]);
  }
  // hyper legs: kept index bit hm -> tensor position (kept = all positions but kpos)
  for (int h = 0; h < st.nH; ++h) {
    int pos = -1, cnt = -1;
    for (int q = 0; q < st.rA; ++q) {
      bool is_k = false;
      for (int b = 0; b < st.nK; ++b) is_k |= st.kpos[b] == q;
      if (is_k) continue;
      if (++cnt == st.hm[h]) { pos = q; break; }
    }
    if (in_P(pos)) { fs.h_inP[h] = 1; fs.h_pos[h] = loc(pos); }
    else { fs.h_inP[h] = 0; fs.h_pos[h] = pos; }
    fs.hw[h] = st.hw[h];
  }
  for (int k = 0; k < st.nS; ++k) { fs.sq[k] = st.sq[k]; fs.sw[k] = st.sw[k]; }
  return fs;
}
}  // namespace

bool build_segments(const std::vector<AbsorbStep>& steps, std::vector<Segment>& segs,
                    std::vector<FusedStep>& fused) {
  segs.clear();
  auto in_place = [](const AbsorbStep& st) {
    if (st.rA != st.rC || st.nK != st.nN) return false;
    for (int i = 0; i < st.nK; ++i)
      if (st.kpos[i] != st.npos[i]) return false;
    return st.rA > kFuseMax;
  };
  size_t i = 0;
  while (i < steps.size()) {
    if (!in_place(steps[i])) {
      Segment sg;
      sg.first = (int)i;
      sg.count = 1;
      segs.push_back(sg);
      ++i;
      continue;
    }
    std::set<int> P;
    size_t j = i;
    const int r = steps[i].rA;
    while (j < steps.size() && in_place(steps[j]) && steps[j].rA == r) {
      std::set<int> P2 = P;
      for (int k = 0; k < steps[j].nK; ++k) P2.insert(steps[j].kpos[k]);
      if ((int)P2.size() > kFuseMax) break;
      P = P2;
      ++j;
    }
    if (j - i < 2) {
      Segment sg;
      sg.first = (int)i;
      sg.count = 1;
      segs.push_back(sg);
      ++i;
      continue;
    }
    for (int pos = 0; (int)P.size() < kFuseMax && pos < r; ++pos) P.insert(pos);
    Segment sg;
    sg.first = (int)i;
    sg.count = (int)(j - i);
    sg.fused = true;
    sg.r = r;
    sg.np = (int)P.size();
    std::vector<int> Pv(P.begin(), P.end());
    for (int k = 0; k < sg.np; ++k) sg.P[k] = Pv[k];
    sg.fused_off = (int64_t)fused.size();
    for (size_t s = i; s < j; ++s) fused.push_back(make_fused_step(steps[s], Pv));
    segs.push_back(sg);
    i = j;
  }
  return true;
}

void build_sv_batches(Plan& p) {
  p.batches.clear();
  int start = 0;
  const int f = (int)p.batch_sizes.size();
  for (int j = 0; j < f; ++j) {
    BatchPlan bp;
    bp.start = start;
    bp.size = p.batch_sizes[j];
    bp.doubled = j < f - 1;
    p.batches.push_back(bp);
    start += bp.size;
  }
}

namespace {
// Windows of at most `wmax` qubits (see build_sv_schedule); appends the fused
// steps to p.fused and returns the segments.
// A step the window pass applies in place as a plain 1- or 2-qubit gate.
bool plain_step(const AbsorbStep& st) {
  if (st.nH != 0 || st.nS != 0 || st.nK != st.nN || st.nK < 1 || st.nK > 2) return false;
  for (int k = 0; k < (1 << st.nK); ++k)
    if (st.noff[k] != st.koff[k]) return false;
  return true;
}

// Relative VALU cost of one step in the window pass (a dense two-qubit gate = 1);
// a 16 x 16 cluster on MFMA costs about 1.6 plus its build.
double step_cost(const Plan& p, const AbsorbStep& st) {
  bool mono = true;
  if (st.gate >= 0 && st.gate < (int)p.mats.size()) {
    const int d = 1 << p.arity[(size_t)st.gate];
    for (int r = 0; r < d; ++r) {
      int nz = 0;
      for (int c = 0; c < d; ++c) {
        const double re = p.mats[(size_t)st.gate][2 * (r * d + c)], im = p.mats[(size_t)st.gate][2 * (r * d + c) + 1];
        nz += (re != 0.0 || im != 0.0);
      }
      mono = mono && nz <= 1;
    }
  }
  if (mono) return 0.3;
  return st.nK == 1 ? 0.5 : 1.0;
}
constexpr double kClusterMinCost = 3.0;

// Regroup a window's steps (in a valid execution order) into clusters of steps on
// at most 4 qubits: a step joins the current group unless a step it must follow
// (one on a shared qubit) was left out, so the new order only moves steps past
// steps on disjoint qubits.  groups: (start, length) in the new order.
void cluster_order(const Plan& p, const std::vector<int>& steps, std::vector<int>& order,
                   std::vector<std::pair<int, int>>& groups) {
  std::vector<char> used(steps.size(), 0);
  order.clear();
  groups.clear();
  while (order.size() < steps.size()) {
    std::set<int> Q, blocked;
    const int start = (int)order.size();
    bool closed = false;
    for (size_t i = 0; i < steps.size(); ++i) {
      if (used[i]) continue;
      const AbsorbStep& st = p.sv_steps[(size_t)steps[i]];
      const bool first = (int)order.size() == start;   // the first unused step: nothing blocks it
      bool ok = !closed;
      std::set<int> Q2 = Q;
      for (int k = 0; k < st.nK; ++k) {
        ok = ok && !blocked.count(st.kpos[k]);
        Q2.insert(st.kpos[k]);
      }
      if (!first) ok = ok && plain_step(st) && Q2.size() <= 4;
      if (ok) {
        used[i] = 1;
        order.push_back(steps[i]);
        Q = Q2;
        if (first && !plain_step(st)) closed = true;   // a step the cluster pass cannot take stands alone
      } else {
        for (int k = 0; k < st.nK; ++k) blocked.insert(st.kpos[k]);
      }
    }
    groups.push_back({start, (int)order.size() - start});
  }
}

// One window of at most wmax qubits (qubits 0..3 always in it) from the steps
// `rest` still to apply, in order: a step joins if its qubits fit and no earlier
// step left out touches them (so it commutes with every step it overtakes).
// taken / left_out: the steps in order; Pv: the window's qubits, ascending.
void pack_window(const Plan& p, const std::vector<int>& rest, int wmax, std::vector<int>& taken,
                 std::vector<int>& left_out, std::vector<int>& Pv, size_t max_steps = (size_t)1 << 30) {
  const int n = p.n;
  const int cap = std::min(wmax, n);
  const int low = std::min(4, n);
  std::set<int> P, blocked;
  for (int q = 0; q < low; ++q) P.insert(q);
  taken.clear();
  left_out.clear();
  for (int g : rest) {
    const AbsorbStep& st = p.sv_steps[g];
    bool free = true;
    for (int k = 0; k < st.nK; ++k) free = free && !blocked.count(st.kpos[k]);
    std::set<int> P2 = P;
    for (int k = 0; k < st.nK; ++k) P2.insert(st.kpos[k]);
    if (free && (int)P2.size() <= cap && taken.size() < max_steps) {
      P = P2;
      taken.push_back(g);
    } else {
      for (int k = 0; k < st.nK; ++k) blocked.insert(st.kpos[k]);
      left_out.push_back(g);
    }
  }
  // pad the window with the lowest qubits not yet in it
  for (int q = 0; (int)P.size() < cap && q < n; ++q) P.insert(q);
  Pv.assign(P.begin(), P.end());
}

std::vector<Segment> sv_windows(Plan& p, int wmax, std::vector<AbsorbStep>* run, std::vector<ClusterDesc>& cls) {
  std::vector<Segment> segs;
  const int n = p.n;
  std::vector<int> rest(p.sv_steps.size());
  for (size_t i = 0; i < rest.size(); ++i) rest[i] = (int)i;
  int64_t first = 0;
  while (!rest.empty()) {
    std::vector<int> taken, left_out, Pv;
    pack_window(p, rest, wmax, taken, left_out, Pv);
    std::set<int> P(Pv.begin(), Pv.end());
    Segment sg;
    sg.first = (int)first;
    sg.count = (int)taken.size();
    sg.fused = true;
    sg.r = n;
    sg.np = (int)P.size();
    for (int k = 0; k < sg.np; ++k) sg.P[k] = Pv[k];
    sg.fused_off = (int64_t)p.fused.size();
    std::vector<int> order;
    std::vector<std::pair<int, int>> groups;
    cluster_order(p, taken, order, groups);
    for (int g : order) {
      if (run) run->push_back(p.sv_steps[g]);
      p.fused.push_back(make_fused_step(p.sv_steps[g], Pv));
    }
    // clusters worth the MFMA pass (windows of >= 10 positions: 4 wavefronts of
    // column tiles), split where the 32-step gate staging restarts
    if (sg.np >= 10)
      for (const auto& gr : groups) {
        int s0 = gr.first;
        const int end = gr.first + gr.second;
        while (s0 < end) {
          const int s1 = std::min(end, (s0 / kGateChunkHost + 1) * kGateChunkHost);
          double cost = 0.0;
          std::set<int> Q;
          for (int s = s0; s < s1; ++s) {
            const AbsorbStep& st = p.sv_steps[(size_t)order[(size_t)s]];
            cost += step_cost(p, st);
            for (int k = 0; k < st.nK; ++k) Q.insert(st.kpos[k]);
          }
          if (s1 - s0 >= 2 && cost >= kClusterMinCost) {
            FusedStep& f = p.fused[(size_t)sg.fused_off + (size_t)s0];
            f.cl_len = s1 - s0;
            f.cl_id = (int32_t)cls.size();
            std::vector<int> loc;
            for (int q : Q) loc.push_back((int)(std::find(Pv.begin(), Pv.end(), q) - Pv.begin()));
            for (int l = 0; (int)loc.size() < 4 && l < sg.np; ++l)      // pad with other tile positions
              if (std::find(loc.begin(), loc.end(), l) == loc.end()) loc.push_back(l);
            ClusterDesc cd{};
            cd.first = (int32_t)(sg.fused_off + s0);
            cd.len = s1 - s0;
            for (int i = 0; i < 4; ++i) cd.pos[i] = f.cl_pos[i] = loc[(size_t)i];
            cls.push_back(cd);
          }
          s0 = s1;
        }
      }
    first += (int64_t)taken.size();
    segs.push_back(sg);
    rest = left_out;
  }
  return segs;
}
}  // namespace

int count_sv_windows(const Plan& p, int wmax) {
  std::vector<int> rest(p.sv_steps.size());
  for (size_t i = 0; i < rest.size(); ++i) rest[i] = (int)i;
  int w = 0;
  while (!rest.empty()) {
    std::vector<int> taken, left_out, Pv;
    pack_window(p, rest, wmax, taken, left_out, Pv);
    rest = left_out;
    ++w;
  }
  return w;
}

void build_sv_schedule(Plan& p) {
  p.sv_run.clear();
  for (int i = 0; i < 3; ++i) {
    p.sv_cl[i].clear();
    p.sv_win[i] = sv_windows(p, kSvWindowMin + i, i == 2 ? &p.sv_run : nullptr, p.sv_cl[i]);
  }
  p.sv_segs = p.sv_win[2];
}

void build_adj_windows(const Plan& p, int wmax, int max_ops, std::vector<AdjWin>& wins, std::vector<AdjOp>& ops) {
  wins.clear();
  ops.clear();
  std::vector<int> rest(p.sv_steps.size());
  for (size_t i = 0; i < rest.size(); ++i) rest[i] = (int)i;
  while (!rest.empty()) {
    std::vector<int> taken, left_out, Pv;
    pack_window(p, rest, wmax, taken, left_out, Pv, (size_t)std::max(max_ops, 1));
    AdjWin w{};
    w.op_off = (int32_t)ops.size();
    w.n_ops = (int32_t)taken.size();
    w.np = (int32_t)Pv.size();
    for (int k = 0; k < w.np; ++k) w.P[k] = Pv[(size_t)k];
    auto loc = [&](int q) { return (int)(std::find(Pv.begin(), Pv.end(), q) - Pv.begin()); };
    for (int g : taken) {
      const AbsorbStep& st = p.sv_steps[(size_t)g];
      AdjOp op{};
      op.kind = (int8_t)(st.nK == 1 ? kSvOpGate1 : kSvOpGate2);
      op.p0 = (int8_t)loc(st.kpos[0]);
      op.p1 = (int8_t)(st.nK == 2 ? loc(st.kpos[1]) : 0);
      op.axis = -1;
      op.nslot = -1;
      op.slot = (int32_t)(ops.size() - (size_t)w.op_off);
      op.gate = st.gate;
      const int d = 1 << st.nK;
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) op.idx[a * d + b] = (int8_t)(st.nB[a] + st.kB[b]);
      ops.push_back(op);
    }
    wins.push_back(w);
    rest = left_out;
  }
}

void build_adj_groups(std::vector<AdjWin>& wins, std::vector<AdjOp>& ops, std::vector<AdjGroup>& groups) {
  groups.clear();
  std::vector<AdjOp> out;
  out.reserve(ops.size());
  for (AdjWin& w : wins) {
    std::vector<AdjOp> rest(ops.begin() + w.op_off, ops.begin() + w.op_off + w.n_ops);
    const int off = (int)out.size();
    w.group_off = (int32_t)groups.size();
    while (!rest.empty()) {
      std::vector<AdjOp> left;
      std::set<int> Q, blocked;
      AdjGroup g{};
      g.first = (int32_t)out.size() - off;
      int count = 0;
      for (AdjOp op : rest) {
        const bool two = op.kind == kSvOpGate2;
        std::set<int> Q2 = Q;
        Q2.insert(op.p0);
        if (two) Q2.insert(op.p1);
        const bool free = !blocked.count(op.p0) && (!two || !blocked.count(op.p1));
        if (free && Q2.size() <= 2 && count < kAdjGroupMax) {
          Q = Q2;
          op.slot = (int32_t)out.size() - off;
          out.push_back(op);
          ++count;
        } else {
          blocked.insert(op.p0);
          if (two) blocked.insert(op.p1);
          left.push_back(op);
        }
      }
      g.n = (int8_t)count;
      g.nq = (int8_t)Q.size();
      g.pa = (int8_t)*Q.begin();
      g.pb = (int8_t)*Q.rbegin();
      groups.push_back(g);
      rest = left;
    }
    w.op_off = off;
    w.n_groups = (int32_t)groups.size() - w.group_off;
  }
  ops = out;
}

void build_sv_ops(Plan& p) {
  const uint32_t all = p.n >= 32 ? 0xFFFFFFFFu : ((1u << p.n) - 1u);
  for (int i = 0; i < 3; ++i) {
    // plain form: every fused step of every window as its own op
    std::vector<SvWin>& pw = p.sv_wins_plain[i];
    std::vector<SvOp>& po = p.sv_ops_plain[i];
    pw.clear();
    po.clear();
    bool pok = true;
    for (const Segment& sg : p.sv_win[i]) {
      SvWin w{};
      w.op_off = (int32_t)po.size();
      w.np = sg.np;
      uint32_t win = 0;
      for (int k = 0; k < kFuseMax; ++k) {
        w.P[k] = sg.P[k];
        if (k < sg.np) win |= 1u << sg.P[k];
      }
      w.other = all & ~win;
      pok = pok && sg.P[0] == 0;
      for (int s = 0; s < sg.count && pok; ++s) {
        const FusedStep& f = p.fused[(size_t)(sg.fused_off + s)];
        const bool plain = f.nH == 0 && f.nS == 0 && f.nK == f.nN && f.nK >= 1 && f.nK <= 2 &&
                           f.noff[1] == f.koff[1] && (f.nK == 1 || (f.noff[2] == f.koff[2] && f.noff[3] == f.koff[3]));
        if (!plain) { pok = false; break; }
        SvOp op{};
        op.kind = f.nK == 1 ? kSvOpGate1 : kSvOpGate2;
        op.p0 = (int8_t)f.kloc[0];
        op.p1 = (int8_t)(f.nK == 2 ? f.kloc[1] : 0);
        op.conj = (int8_t)f.conj;
        op.gate = f.gate;
        op.slot = w.n_plain++;
        const int d = 1 << f.nK;
        for (int n = 0; n < d; ++n)
          for (int k = 0; k < d; ++k) op.idx[n * d + k] = (int8_t)(f.nB[n] + f.kB[k]);
        po.push_back(op);
      }
      if (!pok) break;
      w.n_ops = (int32_t)po.size() - w.op_off;
      pw.push_back(w);
    }
    if (!pok) {
      pw.clear();
      po.clear();
    }
    std::vector<SvWin>& wins = p.sv_wins[i];
    std::vector<SvOp>& ops = p.sv_ops[i];
    wins.clear();
    ops.clear();
    bool ok = true;
    for (const Segment& sg : p.sv_win[i]) {
      SvWin w{};
      w.op_off = (int32_t)ops.size();
      w.np = sg.np;
      uint32_t win = 0;
      for (int k = 0; k < kFuseMax; ++k) {
        w.P[k] = sg.P[k];
        if (k < sg.np) win |= 1u << sg.P[k];
      }
      w.other = all & ~win;
      ok = ok && sg.np >= 1 && sg.P[0] == 0;
      int cl_lo = -1, cl_hi = -1;
      for (int s = 0; s < sg.count && ok;) {
        const FusedStep& f = p.fused[(size_t)(sg.fused_off + s)];
        SvOp op{};
        if (f.cl_len > 0) {
          op.kind = kSvOpCluster;
          for (int k = 0; k < 4; ++k) op.cpos[k] = (int8_t)f.cl_pos[k];
          op.slot = f.cl_id;            // made window-relative below
          cl_lo = cl_lo < 0 ? f.cl_id : std::min(cl_lo, f.cl_id);
          cl_hi = std::max(cl_hi, f.cl_id);
          s += f.cl_len;
        } else {
          const bool plain = f.nH == 0 && f.nS == 0 && f.nK == f.nN && f.nK >= 1 && f.nK <= 2 &&
                             f.noff[1] == f.koff[1] && (f.nK == 1 || (f.noff[2] == f.koff[2] && f.noff[3] == f.koff[3]));
          if (!plain) { ok = false; break; }
          op.kind = f.nK == 1 ? kSvOpGate1 : kSvOpGate2;
          op.p0 = (int8_t)f.kloc[0];
          op.p1 = (int8_t)(f.nK == 2 ? f.kloc[1] : 0);
          op.conj = (int8_t)f.conj;
          op.gate = f.gate;
          op.slot = w.n_plain++;
          const int d = 1 << f.nK;
          for (int n = 0; n < d; ++n)
            for (int k = 0; k < d; ++k) op.idx[n * d + k] = (int8_t)(f.nB[n] + f.kB[k]);
          ++s;
        }
        ops.push_back(op);
      }
      if (!ok) break;
      w.n_ops = (int32_t)ops.size() - w.op_off;
      w.cl_first = cl_lo < 0 ? 0 : cl_lo;
      w.n_cl = cl_lo < 0 ? 0 : cl_hi - cl_lo + 1;
      for (int k = w.op_off; k < (int)ops.size(); ++k)
        if (ops[(size_t)k].kind == kSvOpCluster) ops[(size_t)k].slot -= w.cl_first;
      wins.push_back(w);
    }
    if (!ok) {
      wins.clear();
      ops.clear();
    }
  }
}


bool make_gemv_lanes(const BatchPlan& bp, GemvLanes& g) {
  const int nx = (int)bp.xT.size(), nk = (int)bp.lk.size();
  const int rows = 1 << (int)bp.xb.size();
  if (bp.doubled || bp.xb.size() > 1 || nk < 1 || nk > 12 || nx + nk < 6 || nx > 32) return false;
  if ((size_t)rows * ((size_t)8 << nk) > 32768) return false;          // V rows staged in LDS
  auto off = [](const SplitTable& t, int i) -> int64_t {
    return i < t.lo_bits ? t.lo[(size_t)1 << i] : t.hi[(size_t)1 << (i - t.lo_bits)];
  };
  struct Bit { int64_t toff, ooff; int kbit; bool is_k; };
  std::vector<Bit> bits;
  for (int i = 0; i < nx; ++i) bits.push_back({off(bp.t_x, i), off(bp.o_x, i), 0, false});
  for (int i = 0; i < nk; ++i) bits.push_back({off(bp.t_k, i), 0, 1 << i, true});
  std::sort(bits.begin(), bits.end(), [](const Bit& a, const Bit& b) { return a.toff < b.toff; });
  if (!bits[0].is_k) return false;
  int n_hx = 0, n_hk = 0;
  for (size_t q = 0; q < bits.size(); ++q) {
    const Bit& b = bits[q];
    if (q < 6) {
      g.lane_toff[q] = b.toff;
      g.lane_ooff[q] = b.is_k ? 0 : b.ooff;
      g.lane_kbit[q] = b.is_k ? b.kbit : 0;
      g.lane_is_k[q] = b.is_k ? 1 : 0;
    } else if (b.is_k) {
      g.hk_toff[n_hk] = b.toff;
      g.hk_kbit[n_hk] = b.kbit;
      ++n_hk;
    } else {
      g.hx_toff[n_hx] = b.toff;
      g.hx_ooff[n_hx] = b.ooff;
      ++n_hx;
    }
  }
  g.n_hx = n_hx;
  g.n_hk = n_hk;
  return n_hk <= 10;
}

bool make_gemv_tiling(const BatchPlan& bp, GemvTiling& g) {
  const int nx = (int)bp.xT.size();
  if (nx < 12 || nx - 12 > 32) return false;
  auto off = [](const SplitTable& t, int i) -> int64_t {
    return i < t.lo_bits ? t.lo[(size_t)1 << i] : t.hi[(size_t)1 << (i - t.lo_bits)];
  };
  std::vector<int64_t> to((size_t)nx), oo((size_t)nx);
  for (int i = 0; i < nx; ++i) {
    to[(size_t)i] = off(bp.t_x, i);
    oo[(size_t)i] = off(bp.o_x, i);
  }
  std::vector<int> by_t((size_t)nx), by_o((size_t)nx);
  std::iota(by_t.begin(), by_t.end(), 0);
  std::iota(by_o.begin(), by_o.end(), 0);
  std::sort(by_t.begin(), by_t.end(), [&](int a, int b) { return to[(size_t)a] < to[(size_t)b]; });
  std::sort(by_o.begin(), by_o.end(), [&](int a, int b) { return oo[(size_t)a] < oo[(size_t)b]; });
  // tile bits: the 6 x bits of smallest T offset, the 6 of smallest output offset
  // among the rest, then further bits by T offset until there are 12
  std::vector<char> in((size_t)nx, 0);
  int n_in = 0;
  for (int q = 0; q < 6; ++q) { in[(size_t)by_t[(size_t)q]] = 1; ++n_in; }
  for (int q = 0, c = 0; q < nx && c < 6; ++q)
    if (!in[(size_t)by_o[(size_t)q]]) { in[(size_t)by_o[(size_t)q]] = 1; ++n_in; ++c; }
  for (int q = 0; q < nx && n_in < 12; ++q)
    if (!in[(size_t)by_t[(size_t)q]]) { in[(size_t)by_t[(size_t)q]] = 1; ++n_in; }
  std::vector<int> rd, wr, hi;
  for (int i : by_t) if (in[(size_t)i]) rd.push_back(i); else hi.push_back(i);
  for (int i : by_o) if (in[(size_t)i]) wr.push_back(i);
  for (int s = 0; s < 12; ++s) {
    g.t_off[s] = to[(size_t)rd[(size_t)s]];
    g.o_read[s] = oo[(size_t)rd[(size_t)s]];
    g.w_of[s] = (int32_t)(std::find(wr.begin(), wr.end(), rd[(size_t)s]) - wr.begin());
    g.o_off[s] = oo[(size_t)wr[(size_t)s]];
  }
  g.n_hi = (int32_t)hi.size();
  for (size_t h = 0; h < hi.size(); ++h) {
    g.t_hi[h] = to[(size_t)hi[h]];
    g.o_hi[h] = oo[(size_t)hi[h]];
  }
  return true;
}

}  // namespace ptsbe
