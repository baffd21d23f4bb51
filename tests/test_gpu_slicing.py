"""Sliced last batch (plan option max_part_rank).

When the last batch's per-trajectory tensor would exceed max_part_rank, the
planner fixes the first crossing wires to each of their values in turn on both
parts (sliced legs read bits n.. of the jobs' prefix words) and the join's
amplitudes are summed over the slices: the sum over a contracted index split
into its terms (Sec. II-B's contraction of the batch network, reorganised).
Small circuits force slicing with a low cap and are held to the FP64 oracle;
the 100-qubit chain of the batch-size sweep (Sec. V-B) is checked at b = 22
(one sliced wire, rank-31 per-trajectory tensors) against the unsliced b = 20
plan of the same circuit: P(prefix, x_22) with x_22 = (two bits, x_20) must equal
P(prefix + two bits, x_20)."""
import numpy as np
import pytest

import workloads as W
from oracle import sampling, tn
from tests.gpu_helpers import (assert_shot_parity, flip_probability, oracle_shots_sv, oracle_states, prefix_words,
                               shots_to_ints, to_dev, torch_dev)

pytestmark = pytest.mark.gpu


def _contract(plan, torch, dev, kd, traj, prefixes, j, amp=False, workspace=None):
    import paper_2604_08467_amd as P
    et = to_dev(torch, dev, np.asarray(traj, dtype=np.int32))
    ep = to_dev(torch, dev, prefix_words(prefixes, plan.n_words))
    out, tot = plan.contract_batch(j, kd, et, ep, P.OUT_AMPLITUDE if amp else P.OUT_POPULATION,
                                   workspace=workspace)
    torch.cuda.synchronize()
    return out.cpu().numpy(), (None if tot is None else tot.cpu().numpy())


def _chain12():
    rng = np.random.default_rng(6060)
    c = W.Circuit(12)
    dep = c.add_channel(W.depolarizing(0.03))
    ad = c.add_channel(W.amplitude_damping(0.05))
    for layer in W.brickwork_1d(12, 8):
        for (q0, q1) in layer:
            g = c.add_gate((q0, q1), W.haar_su4(rng))
            c.add_site(g, (q0,), dep)
            c.add_site(g, (q1,), ad)
    return c.round_to_complex64()


@pytest.mark.parametrize("cap", [9, 7, 5])
def test_sliced_last_batch_vs_oracle(cap):
    """12-qubit chain of depth 8 with depolarising and amplitude damping, batches
    [3, 3, 6]: the last batch's per-trajectory tensor (rank 12 unsliced) capped at
    9, 7 and 5; amplitudes and populations of every prefix of two trajectories
    and a few of six more against the explicit FP64 network, and populations
    against the unsliced plan."""
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    c = _chain12()
    bs = [3, 3, 6]
    full = P.Plan(c, bs, method="network")
    sl = P.Plan(c, bs, method="network", max_part_rank=cap)
    bf, bsl = full.batch_info(2), sl.batch_info(2)
    assert bf["slice_bits"] == 0 and bsl["slice_bits"] > 0 and bsl["right_peak_rank"] <= cap
    kr, _, _, _ = sl.sample_trajectories(6061, 8)
    kd = to_dev(torch, dev, kr)
    rng = np.random.default_rng(6062)
    traj, pre = [], []
    for i in range(len(kr)):
        ps = range(64) if i < 2 else rng.integers(0, 64, size=3)
        for p in ps:
            traj.append(i)
            pre.append(int(p))
    amp, _ = _contract(sl, torch, dev, kd, traj, pre, 2, amp=True)
    pop, tot = _contract(sl, torch, dev, kd, traj, pre, 2)
    pop_f, _ = _contract(full, torch, dev, kd, traj, pre, 2)
    worst_a = worst_p = worst_f = 0.0
    for e, (i, p) in enumerate(zip(traj, pre)):
        ref = tn.batch_network_value(c, kr[i], 6, 6, p, "ket")
        nrm = max(np.linalg.norm(ref), 1e-30)
        worst_a = max(worst_a, np.linalg.norm(amp[e] - ref) / nrm)
        Z = max(float((np.abs(ref) ** 2).sum()), 1e-30)
        worst_p = max(worst_p, np.abs(pop[e] - np.abs(ref) ** 2).max() / Z)
        worst_f = max(worst_f, np.abs(pop[e] - pop_f[e]).max() / Z)
    print(f"chain12 cap {cap}: {bsl['slice_bits']} sliced wires, {len(traj)} elements; amplitude rel err "
          f"{worst_a:.3g}, population err {worst_p:.3g} (of Z), vs unsliced plan {worst_f:.3g}", flush=True)
    assert worst_a <= 1e-5 and worst_p <= 1e-6 and worst_f <= 1e-6


def test_sliced_shots_vs_oracle_sampler():
    """Proportional NBS through the sliced last batch (cap 7, resumed left part):
    8 trajectories x 300 shots against the FP64 oracle sampler, mismatches within
    the CDF-boundary flip bound."""
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    c = _chain12()
    bs = [3, 3, 6]
    plan = P.Plan(c, bs, method="network", max_part_rank=7)
    assert plan.batch_info(2)["slice_bits"] > 0
    kr, mult, _, _ = plan.sample_trajectories(6063, 8)
    E, m = len(kr), 300
    kd = to_dev(torch, dev, kr)
    out = plan.sample_shots(kd, to_dev(torch, dev, np.full(E, m, dtype=np.int64)), 6064,
                            mult_dev=to_dev(torch, dev, mult))
    shots = shots_to_ints(out["shots"].cpu().numpy())
    psis = oracle_states(c, kr)
    ref, _ = oracle_shots_sv(c, psis, bs, m, 6064)
    starts = sampling.batch_starts(bs)
    mism, expect = 0, 0.0
    for i in range(E):
        got = shots[i * m:(i + 1) * m]
        mism += sum(1 for a, b in zip(got, ref[i]) if a != b)
        prefixes = {}
        for t in range(m):
            for j in range(len(bs)):
                p = ref[i][t] & ((1 << starts[j]) - 1)
                prefixes[(j, p)] = prefixes.get((j, p), 0) + 1
        for (j, p), cnt in prefixes.items():
            g, _ = _contract(plan, torch, dev, kd, [i], [p], j)
            expect += cnt * flip_probability(g[0], sampling.marginal_from_state(psis[i], 12, starts[j], bs[j], p))
    print(f"chain12 sliced shots: {mism} mismatches of {E * m}, expected flips {expect:.3g}", flush=True)
    assert_shot_parity(mism, expect, E * m)
    Z = np.array([np.vdot(p, p).real for p in psis])
    np.testing.assert_allclose(out["norms"].cpu().numpy(), Z, rtol=1e-5)


def test_chain100_b22_sliced_against_b20():
    """The batch-size sweep's 100-qubit chain (594 Haar SU(4) gates, depth 12,
    depolarising 0.005): the last batch at b = 22 needs a rank-32 per-trajectory
    tensor, so one crossing wire is sliced (two rank-31 contractions summed);
    its populations for one trajectory and prefix must match the unsliced
    b = 20 plan at the four extensions of the prefix by qubits 78 and 79."""
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    rng = np.random.default_rng(5001)
    c = W.random_brickwork(100, 12, rng, 0.005).round_to_complex64()
    b22 = [10] * 7 + [8, 22]
    b20 = [10] * 8 + [20]
    p10 = P.Plan(c, [10] * 10, hypersamples=8, method="network")
    kr, _, _, _ = p10.sample_trajectories(5002, 4)
    kd = to_dev(torch, dev, kr)
    # a likely prefix: qubits 0..77 of one shot of trajectory 0 (batches of 10)
    m = np.zeros(len(kr), dtype=np.int64)
    m[0] = 1
    ws = torch.empty(200 << 30, dtype=torch.uint8, device=dev)
    shot = shots_to_ints(p10.sample_shots(kd, to_dev(torch, dev, m), 5003, workspace=ws)["shots"].cpu().numpy())[0]
    prefix = int(shot) & ((1 << 78) - 1)
    del p10
    p20 = P.Plan(c, b20, hypersamples=8, method="network")
    assert p20.batch_info(8)["slice_bits"] == 0
    ext = [prefix | (v << 78) for v in range(4)]
    pop20, _ = _contract(p20, torch, dev, kd, [0] * 4, ext, 8, workspace=ws)
    del p20
    p22 = P.Plan(c, b22, hypersamples=8, method="network")
    bi = p22.batch_info(8)
    assert bi["slice_bits"] >= 1 and bi["right_peak_rank"] <= 31
    pop22, tot22 = _contract(p22, torch, dev, kd, [0], [prefix], 8, workspace=ws)
    # x_22 bit 0 is qubit 78, bit 1 qubit 79, bits 2.. the b = 20 batch's x
    p22r = pop22[0].reshape(1 << 20, 4)
    Z = float(tot22[0])
    err = max(np.abs(p22r[:, v] - pop20[v]).max() for v in range(4)) / Z
    print(f"chain100 b22 ({bi['slice_bits']} sliced wires, rank {bi['right_peak_rank']}): P(prefix) {Z:.6g}, "
          f"max |P22 - P20| / P(prefix) = {err:.3g}", flush=True)
    assert err <= 1e-6


@pytest.mark.parametrize("bs", [[6, 14], [7, 13]], ids=["rows2", "rows1"])
@pytest.mark.parametrize("cap", [0, 20])
def test_gemv_join_with_many_crossing_wires_vs_oracle(bs, cap):
    """The last batch's GEMV join over T in its own layout with 2^11 crossing
    values (k staged in LDS chunks of 512), unsliced and with the tensor capped at
    rank 20 (sliced): a 20-qubit chain of depth 12, one element per trajectory,
    populations against the FP64 statevector marginals."""
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    rng = np.random.default_rng(7070)
    c = W.random_brickwork(20, 12, rng, 0.01).round_to_complex64()
    plan = P.Plan(c, bs, method="network", max_part_rank=cap)
    bi = plan.batch_info(1)
    assert bi["crossing"] > 6 and bs[1] - bi["join_rows_log2"] >= 12
    assert (bi["slice_bits"] > 0) == (cap > 0)
    kr, _, _, _ = plan.sample_trajectories(7071, 6)
    kd = to_dev(torch, dev, kr)
    psis = oracle_states(c, kr)
    pre = [int(p) for p in np.random.default_rng(7072).integers(0, 1 << bs[0], size=len(kr))]
    pop, tot = _contract(plan, torch, dev, kd, range(len(kr)), pre, 1)
    worst = 0.0
    for i, p in enumerate(pre):
        ref = sampling.marginal_from_state(psis[i], 20, bs[0], bs[1], p)
        Z = max(float(ref.sum()), 1e-30)
        worst = max(worst, np.abs(pop[i] - ref).max() / Z, abs(tot[i] - Z) / Z * 1e-1)
    print(f"chain20 {bs} cap {cap}: crossing {bi['crossing']}, {bi['slice_bits']} sliced; max population err "
          f"{worst:.3g} of Z", flush=True)
    assert worst <= 1e-6
