"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: amplitudes 1e-5 L2-relative per element, marginals 1e-6 absolute on
the normalised conditionals, shots identical except CDF-boundary flips (their
exact per-draw probability is computed from both marginals), trajectory weights
1e-6 relative."""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import sampling, tn
from oracle import statevector as sv
from tests.gpu_helpers import (assert_shot_parity, flip_probability, oracle_shots_sv, oracle_states,
                               prefix_words, shots_to_ints, to_dev, torch_dev)

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _plan(circuit, bs, **kw):
    """method "network-lc": the network method with the light-cone option (doubled
    networks keep the gates in the measured qubits' light cone, non-unitary gates
    and their past); the oracle keeps every gate."""
    import paper_2604_08467_amd as P
    if kw.get("method") == "network-lc":
        kw = dict(kw, method="network", light_cone=True)
    return P.Plan(circuit, bs, **kw)


def _contract(plan, torch, dev, kraus_d, traj, prefixes, j, amp=False):
    import paper_2604_08467_amd as P
    et = to_dev(torch, dev, np.asarray(traj, dtype=np.int32))
    ep = to_dev(torch, dev, prefix_words(prefixes, plan.n_words))
    out, tot = plan.contract_batch(j, kraus_d, et, ep, P.OUT_AMPLITUDE if amp else P.OUT_POPULATION)
    torch.cuda.synchronize()
    return out.cpu().numpy(), (None if tot is None else tot.cpu().numpy())


METHODS = ["network", "statevector"]
METHODS_LC = METHODS + ["network-lc"]


# ------------------------------------------------------------------ config 1
@pytest.mark.parametrize("method", METHODS)
def test_chain10_d8_amplitudes_populations_and_weights(method):
    torch, dev = torch_dev()
    wl = W.chain10_d8()
    c = wl.circuit
    _say(f"chain10_d8 ({method}): plan + PTS")
    plan = _plan(c, wl.batch_sizes, method=method)
    assert plan.method == method
    kr, mult, lq, nd = plan.sample_trajectories(wl.pts_seed, wl.n_traj)
    E = len(kr)
    kd = to_dev(torch, dev, kr)
    psis = oracle_states(c, kr)
    amp, _ = _contract(plan, torch, dev, kd, range(E), [0] * E, 0, amp=True)
    pop, tot = _contract(plan, torch, dev, kd, range(E), [0] * E, 0)
    for i in range(E):
        ref = psis[i]
        rel = np.linalg.norm(amp[i] - ref) / np.linalg.norm(ref)
        assert rel <= 1e-5, (i, rel)
        pref = np.abs(ref) ** 2
        assert np.abs(pop[i] - pref).max() <= 1e-6, i
        Z = np.vdot(ref, ref).real
        assert abs(tot[i] - Z) <= 1e-6 * Z
    _say("chain10_d8: amplitudes/populations ok")


@pytest.mark.parametrize("method", METHODS)
def test_chain10_d8_shots_match_oracle_sampler(method):
    torch, dev = torch_dev()
    wl = W.chain10_d8()
    c = wl.circuit
    plan = _plan(c, wl.batch_sizes, method=method)
    kr, mult, lq, nd = plan.sample_trajectories(wl.pts_seed, wl.n_traj)
    E, m = len(kr), wl.shots_per_traj
    kd = to_dev(torch, dev, kr)
    md = to_dev(torch, dev, np.full(E, m, dtype=np.int64))
    multd = to_dev(torch, dev, mult)
    out = plan.sample_shots(kd, md, wl.shot_seed, mult_dev=multd)
    torch.cuda.synchronize()
    shots = shots_to_ints(out["shots"].cpu().numpy())
    straj = out["shot_traj"].cpu().numpy()
    assert np.array_equal(straj, np.repeat(np.arange(E), m))
    psis = oracle_states(c, kr)
    ref, _ = oracle_shots_sv(c, psis, wl.batch_sizes, m, wl.shot_seed)
    pop, _ = _contract(plan, torch, dev, kd, range(E), [0] * E, 0)
    mism, expect = 0, 0.0
    for i in range(E):
        got = shots[i * m:(i + 1) * m]
        mism += sum(1 for a, b in zip(got, ref[i]) if a != b)
        expect += m * flip_probability(pop[i], np.abs(psis[i]) ** 2)
    _say(f"chain10_d8 ({method}) shots: {mism} mismatches of {E * m}, expected flips {expect:.3g}")
    assert_shot_parity(mism, expect, E * m)
    # weights: W_i = mult_i Z_i / sum mult Z (Pauli noise: Z_i = 1 up to gate rounding)
    Z = np.array([np.vdot(p, p).real for p in psis])
    wref = sampling.trajectory_weights(Z, mult)
    np.testing.assert_allclose(out["weights"].cpu().numpy(), wref, rtol=1e-6)
    np.testing.assert_allclose(out["norms"].cpu().numpy(), Z, rtol=1e-6)
    assert list(out["elements_per_batch"]) == [E]


@pytest.mark.parametrize("method", METHODS)
def test_chain10_d8_pooled_shots_tvd(method):
    """Pooled shots vs the weighted mean of the per-trajectory oracle distributions."""
    torch, dev = torch_dev()
    wl = W.chain10_d8()
    c = wl.circuit
    plan = _plan(c, wl.batch_sizes, method=method)
    kr, mult, _, _ = plan.sample_trajectories(wl.pts_seed, wl.n_traj)
    E, m = len(kr), wl.shots_per_traj
    out = plan.sample_shots(to_dev(torch, dev, kr), to_dev(torch, dev, np.full(E, m, dtype=np.int64)),
                            wl.shot_seed)
    shots = np.array(shots_to_ints(out["shots"].cpu().numpy()))
    pbar = np.mean([np.abs(p) ** 2 for p in oracle_states(c, kr)], axis=0)
    M = E * m
    hist = np.bincount(shots, minlength=1024) / M
    tvd = 0.5 * np.abs(hist - pbar).sum()
    bound = 0.5 * math.sqrt(1024 / M) + math.sqrt(math.log(1e9) / (2 * M))
    assert tvd <= bound, (tvd, bound)
    for q in range(10):
        p1 = np.mean((shots >> q) & 1)
        ref = sum(pbar[x] for x in range(1024) if (x >> q) & 1)
        assert abs(p1 - ref) <= 0.5 * math.sqrt(2 / M) * 2 + math.sqrt(math.log(1e9) / (2 * M))


# ------------------------------------------------- multi-batch small circuits
def _small_cases():
    rng = np.random.default_rng(77)
    cases = []
    c = W.random_brickwork(12, 5, rng, 0.05)
    cases.append(("bw12", c, [4, 4, 4]))
    c = W.small_random_circuit(14, 40, rng, [W.depolarizing(0.1), W.amplitude_damping(0.2), W.depolarizing2(0.05)],
                               site_prob=0.6)
    cases.append(("rand14_ad", c, [3, 5, 6]))
    c = W.random_brickwork(16, 6, rng, 0.02, layout="2d")
    cases.append(("grid16", c, [5, 5, 6]))
    c = W.random_brickwork(13, 4, rng, 0.05)
    cases.append(("bw13_uneven", c, [1, 6, 2, 4]))
    return cases


@pytest.mark.parametrize("method", METHODS_LC)
@pytest.mark.parametrize("case", range(4))
def test_small_multibatch_marginals(case, method):
    torch, dev = torch_dev()
    name, c, bs = _small_cases()[case]
    _say(f"{name} ({method}): marginals b={bs}")
    plan = _plan(c, bs, method=method)
    kr, mult, _, _ = plan.sample_trajectories(11 + case, 8)
    kd = to_dev(torch, dev, kr)
    psis = oracle_states(c, kr)
    n = c.n_qubits
    starts = sampling.batch_starts(bs)
    rng = np.random.default_rng(case)
    for j, (a, b) in enumerate(zip(starts, bs)):
        traj = np.sort(rng.integers(0, len(kr), size=12))
        pre = [int(rng.integers(0, 2 ** a)) if a else 0 for _ in traj]
        pop, tot = _contract(plan, torch, dev, kd, traj, pre, j)
        for e, (i, p) in enumerate(zip(traj, pre)):
            ref = sampling.marginal_from_state(psis[i], n, a, b, p)
            Z = ref.sum()
            # network: relative to the element's own total (prefix-projected contraction),
            # at the amplitudes' relative tolerance, 1e-5: rounding depends on the
            # contraction path (on one amplitude-damping element with a prefix weight of
            # 1e-5, light-cone and full plans on different paths measured 4e-7 .. 4e-6);
            # statevector: 1e-6 absolute on joint marginals, scaled by the trajectory's
            # norm (the FP32 state's error is set by the whole state, not by the prefix)
            if method != "statevector":
                bound = 1e-5 * max(Z, 1e-30)
            else:
                bound = 1e-6 * np.vdot(psis[i], psis[i]).real
            assert np.abs(pop[e] - ref).max() <= bound + 1e-12, (name, j, e)
            assert abs(tot[e] - Z) <= 1e-5 * (Z if method != "statevector" else np.vdot(psis[i], psis[i]).real) + 1e-12
        if j == len(bs) - 1:
            amp, _ = _contract(plan, torch, dev, kd, traj, pre, j, amp=True)
            for e, (i, p) in enumerate(zip(traj, pre)):
                ref = sampling.amplitudes_from_state(psis[i], n, a, b, p)
                nr = np.linalg.norm(ref)
                if nr > 1e-12:
                    assert np.linalg.norm(amp[e] - ref) / nr <= 1e-5, (name, e)


@pytest.mark.parametrize("method", ["network", "network-lc"])
@pytest.mark.parametrize("case", [0, 1])
def test_right_part_sharing(case, method):
    """Trajectories that agree on the Kraus choices of a batch's per-trajectory part
    share its tensor: variants of each trajectory that change one site outside
    (shared right tensor, different left part) or inside (own right tensor) that set
    must each still give their own oracle marginals."""
    torch, dev = torch_dev()
    name, c, bs = _small_cases()[case]
    plan = _plan(c, bs, method=method)
    base, _, _, _ = plan.sample_trajectories(31 + case, 6)
    rng = np.random.default_rng(500 + case)
    n_kraus = [c.channels[ch].kraus.shape[0] for ch in c.site_channel]
    n, starts = c.n_qubits, sampling.batch_starts(bs)
    for j in range(1, len(bs)):
        inside = set(plan.right_sites(j).tolist())
        outside = [s for s in range(len(n_kraus)) if s not in inside and n_kraus[s] > 1]
        inside = [s for s in inside if n_kraus[s] > 1]
        rows = []
        for kr in base:
            rows.append(kr.copy())
            for pool in (outside, inside):
                if pool:
                    v = kr.copy()
                    s = int(rng.choice(pool))
                    v[s] = (v[s] + 1 + int(rng.integers(0, n_kraus[s] - 1))) % n_kraus[s]
                    rows.append(v)
        kr_all = np.stack(rows).astype(np.uint8)
        assert len(outside) > 0 and len(inside) > 0, (name, j)
        _say(f"{name}: batch {j}, {len(kr_all)} trajectories, {len(inside)} right-part sites")
        psis = oracle_states(c, kr_all)
        a, b = starts[j], bs[j]
        traj = np.arange(len(kr_all))
        pre = [int(rng.integers(0, 2 ** a)) for _ in traj]
        pop, tot = _contract(plan, torch, dev, to_dev(torch, dev, kr_all), traj, pre, j)
        for e, (i, p) in enumerate(zip(traj, pre)):
            ref = sampling.marginal_from_state(psis[i], n, a, b, p)
            Z = ref.sum()
            assert np.abs(pop[e] - ref).max() <= 1e-5 * max(Z, 1e-30) + 1e-12, (name, j, e)


@pytest.mark.parametrize("method", METHODS_LC)
@pytest.mark.parametrize("case", range(4))
def test_small_multibatch_shots(case, method):
    torch, dev = torch_dev()
    name, c, bs = _small_cases()[case]
    _say(f"{name} ({method}): NBS shots b={bs}")
    plan = _plan(c, bs, method=method)
    kr, mult, _, _ = plan.sample_trajectories(11 + case, 8)
    E, m = len(kr), 300
    kd = to_dev(torch, dev, kr)
    out = plan.sample_shots(kd, to_dev(torch, dev, np.full(E, m, dtype=np.int64)), 1234 + case,
                            mult_dev=to_dev(torch, dev, mult))
    shots = shots_to_ints(out["shots"].cpu().numpy())
    psis = oracle_states(c, kr)
    ref, distinct = oracle_shots_sv(c, psis, bs, m, 1234 + case)
    n = c.n_qubits
    starts = sampling.batch_starts(bs)
    mism = 0
    expect = 0.0
    for i in range(E):
        got = shots[i * m:(i + 1) * m]
        for t in range(m):
            if got[t] != ref[i][t]:
                mism += 1
        # expected flips: every batch of every oracle shot, from the GPU marginals
        prefixes = {}
        for t in range(m):
            for j in range(len(bs)):
                p = ref[i][t] & ((1 << starts[j]) - 1)
                prefixes[(j, p)] = prefixes.get((j, p), 0) + 1
        for (j, p), cnt in prefixes.items():
            g, _ = _contract(plan, torch, dev, kd, [i], [p], j)
            expect += cnt * flip_probability(g[0], sampling.marginal_from_state(psis[i], n, starts[j], bs[j], p))
    _say(f"{name}: {mism} mismatches / {E * m}, expected {expect:.3g}")
    assert_shot_parity(mism, expect, E * m)
    Z = np.array([np.vdot(p, p).real for p in psis])
    np.testing.assert_allclose(out["norms"].cpu().numpy(), Z, rtol=1e-5)
    np.testing.assert_allclose(out["weights"].cpu().numpy(), sampling.trajectory_weights(Z, mult), rtol=1e-5)
    if mism == 0:
        got_distinct = list(out["elements_per_batch"])
        want = [E] + [sum(d[j] for d in distinct) for j in range(1, len(bs))]
        assert got_distinct == want


# ------------------------------------------------------------------ config 2
BW50_LISTS = {"b10-full": ([10] * 5, False), "b10-light-cone": ([10] * 5, True),
              "b5-light-cone": ([5] * 10, True), "b4-light-cone": ([4] * 12 + [2], True),
              "b3-light-cone": ([3] * 16 + [2], True)}


@pytest.mark.parametrize("case", list(BW50_LISTS))
def test_brickwork50_d6_sampled_marginals_vs_tensor_network_oracle(case):
    """The benchmark circuit under the batch lists the benchmark may pick (its
    tuner chooses among uniform lists b = 3..10 by measured time): elements on the
    prefixes of real GPU shots at every batch against the explicit FP64 network."""
    bs, light_cone = BW50_LISTS[case]
    torch, dev = torch_dev()
    wl = W.brickwork50_d6()
    c = wl.circuit
    _say(f"brickwork50_d6 ({case}): plan + PTS(64)")
    plan = _plan(c, bs, light_cone=light_cone, hypersamples=8)
    kr, mult, _, _ = plan.sample_trajectories(wl.pts_seed, 64)
    kd = to_dev(torch, dev, kr)
    # realistic prefixes: from a short GPU sampling run on trajectories 0..3
    out = plan.sample_shots(kd[:4].contiguous(), to_dev(torch, dev, np.full(4, 4, dtype=np.int64)), 7)
    shots = shots_to_ints(out["shots"].cpu().numpy())
    starts = sampling.batch_starts(bs)
    f = len(bs)
    checks = [(0, 0, 0), (1, 0, 0)]
    for j in sorted({1, 2, f // 2, f - 2, f - 1}):
        r = (j * 5) % len(shots)
        checks.append((j, r // 4, shots[r] & ((1 << starts[j]) - 1)))
    for (j, i, p) in checks:
        kind = "ket" if j == f - 1 else "doubled"
        ref = tn.batch_network_value(c, kr[i], starts[j], bs[j], p, kind)
        if kind == "ket":
            amp, _ = _contract(plan, torch, dev, kd, [i], [p], j, amp=True)
            rel = np.linalg.norm(amp[0] - ref) / np.linalg.norm(ref)
            _say(f"brickwork50_d6 {case} j={j} traj={i}: amplitude rel err {rel:.3g}")
            assert rel <= 1e-5
            ref = np.abs(ref) ** 2
        pop, tot = _contract(plan, torch, dev, kd, [i], [p], j)
        Z = ref.sum()
        err = np.abs(pop[0] / tot[0] - ref / Z).max()
        _say(f"brickwork50_d6 {case} j={j} traj={i}: conditional max abs err {err:.3g}, Z rel {abs(tot[0] - Z) / Z:.3g}")
        assert err <= 1e-6
        assert abs(tot[0] - Z) <= 1e-5 * Z


@pytest.mark.parametrize("case", ["b10-full", "b5-light-cone"])
def test_brickwork50_d6_shots_of_one_trajectory_vs_oracle(case):
    bs, light_cone = BW50_LISTS[case]
    torch, dev = torch_dev()
    wl = W.brickwork50_d6()
    c = wl.circuit
    plan = _plan(c, bs, light_cone=light_cone)
    kr, mult, _, _ = plan.sample_trajectories(wl.pts_seed, 8)
    i, m = 5, 6
    kd = to_dev(torch, dev, kr)
    md = np.zeros(len(kr), dtype=np.int64)
    md[i] = m
    out = plan.sample_shots(kd, to_dev(torch, dev, md), wl.shot_seed)
    got = shots_to_ints(out["shots"].cpu().numpy())
    starts = sampling.batch_starts(bs)
    f = len(bs)

    used = {}

    def mfn(j, prefix):
        v = tn.batch_network_value(c, kr[i], starts[j], bs[j], prefix, "ket" if j == f - 1 else "doubled")
        used[(j, prefix)] = np.abs(v) ** 2 if j == f - 1 else v
        return used[(j, prefix)]

    ref, _ = sampling.sample_trajectory(mfn, i, 50, bs, m, wl.shot_seed)
    mism = sum(1 for a, b in zip(got, ref) if a != b)
    # expected CDF-boundary flips: every draw of every oracle shot, from the GPU marginals
    expect = 0.0
    for t in range(m):
        for j, a in enumerate(starts):
            p = ref[t] & ((1 << a) - 1)
            g, _ = _contract(plan, torch, dev, kd, [i], [p], j)
            expect += flip_probability(g[0], used[(j, p)])
    _say(f"brickwork50_d6 {case} traj {i}: {mism} mismatches of {m}, expected flips {expect:.3g}")
    assert_shot_parity(mism, expect, m)


def test_brickwork50_d6_full_size_properties():
    """512 trajectories x 1000 shots at full circuit size: deterministic shots,
    unit Pauli norms, normalised weights, and the chain rule Z(child) = pi_parent(x)."""
    torch, dev = torch_dev()
    wl = W.brickwork50_d6()
    c = wl.circuit
    plan = _plan(c, wl.batch_sizes)
    kr, mult, _, _ = plan.sample_trajectories(wl.pts_seed, 512)
    E, m = len(kr), 1000
    kd = to_dev(torch, dev, kr)
    md = to_dev(torch, dev, np.full(E, m, dtype=np.int64))
    ws = torch.empty(8 << 30, dtype=torch.uint8, device=dev)
    o1 = plan.sample_shots(kd, md, wl.shot_seed, mult_dev=to_dev(torch, dev, mult), workspace=ws)
    s1 = o1["shots"].clone()
    o2 = plan.sample_shots(kd, md, wl.shot_seed, mult_dev=to_dev(torch, dev, mult), workspace=ws)
    assert torch.equal(s1, o2["shots"])
    norms = o1["norms"].cpu().numpy()
    assert np.abs(norms - 1).max() < 2e-4
    w = o1["weights"].cpu().numpy()
    assert abs(w.sum() - 1) < 1e-12
    epb = list(o1["elements_per_batch"])
    _say(f"brickwork50_d6 512x1000 elements per batch {epb}")
    assert epb[0] == E and all(epb[j] <= E * m for j in range(5))
    # chain rule on a few (parent, child) pairs
    shots = shots_to_ints(s1[:2000].cpu().numpy())
    starts = sampling.batch_starts(wl.batch_sizes)
    for j in range(1, 4):
        traj, pre, chil = [], [], []
        for r in range(0, 2000, 250):
            traj.append(r // m)
            pre.append(shots[r] & ((1 << starts[j]) - 1))
            chil.append(shots[r] & ((1 << starts[j + 1]) - 1))
        pop, tot = _contract(plan, torch, dev, kd, traj, pre, j)
        _, tchild = _contract(plan, torch, dev, kd, traj, chil, j + 1) if j + 1 < 4 else (None, None)
        if tchild is None:
            continue
        for e in range(len(traj)):
            x = (chil[e] >> starts[j]) & 1023
            assert abs(tchild[e] - pop[e][x]) <= 1e-4 * pop[e][x] + 1e-30


# ------------------------------------------------------- split precision (BF16)
@pytest.mark.parametrize("prec", [1, 2], ids=["bf16", "f16"])
def test_brickwork50_d6_split_bf16_error_vs_fp64(prec):
    """The split-precision join (bf16, or fp16 with power-of-two scaling) against
    the FP64 explicit-network oracle on sampled elements, and against the complex64
    path on every element of a batch.  The error is stated (printed); the bound
    checked is a sanity bound."""
    torch, dev = torch_dev()
    wl = W.brickwork50_d6()
    c = wl.circuit
    plan64 = _plan(c, wl.batch_sizes)
    plan16 = _plan(c, wl.batch_sizes, precision=prec)
    tag = "split-bf16" if prec == 1 else "split-f16"
    kr, mult, _, _ = plan64.sample_trajectories(wl.pts_seed, 32)
    kd = to_dev(torch, dev, kr)
    out = plan64.sample_shots(kd, to_dev(torch, dev, np.full(len(kr), 40, dtype=np.int64)), 3)
    shots = shots_to_ints(out["shots"].cpu().numpy())
    starts = sampling.batch_starts(wl.batch_sizes)
    worst_fp64 = 0.0
    for j in (1, 2, 3):
        r = 41 * j
        i, p = r // 40, shots[r] & ((1 << starts[j]) - 1)
        ref = tn.batch_network_value(c, kr[i], starts[j], 10, p, "doubled")
        pop, tot = _contract(plan16, torch, dev, kd, [i], [p], j)
        err = np.abs(pop[0] / tot[0] - ref / ref.sum()).max()
        worst_fp64 = max(worst_fp64, err)
        _say(f"{tag} j={j}: conditional max abs error vs FP64 {err:.3g}")
    assert worst_fp64 < 1e-4
    # every element of batch 2 for all 32 trajectories: split vs complex64
    traj = np.repeat(np.arange(len(kr)), 40)
    pre = [shots[r] & ((1 << starts[2]) - 1) for r in range(len(shots))]
    p64, t64 = _contract(plan64, torch, dev, kd, traj, pre, 2)
    p16, t16 = _contract(plan16, torch, dev, kd, traj, pre, 2)
    d = np.abs(p16 / t16[:, None] - p64 / t64[:, None]).max()
    _say(f"{tag} vs complex64, batch 2, {len(traj)} elements: max abs conditional difference {d:.3g}")
    assert d < 1e-4
