"""GPU parity of the statevector method (through the C ABI) against the FP64 oracle.

Marginals 1e-6 absolute on joint probabilities (per unit trajectory norm: the
FP32 state's rounding error is set by the whole state), norms 1e-5 relative,
shots identical except CDF-boundary flips.
The 25-qubit grid is checked against stored oracle values (tests/golden/
grid25_sv.json, written by tests/golden/make_grid25.py from oracle/ only)."""
import json
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import sampling
from tests.gpu_helpers import (assert_shot_parity, flip_probability, oracle_shots_sv, oracle_states,
                               prefix_words, shots_to_ints, to_dev, torch_dev)

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "grid25_sv.json")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _contract(plan, torch, dev, kraus_d, traj, prefixes, j, amp=False):
    import paper_2604_08467_amd as P
    et = to_dev(torch, dev, np.asarray(traj, dtype=np.int32))
    ep = to_dev(torch, dev, prefix_words(prefixes, plan.n_words))
    out, tot = plan.contract_batch(j, kraus_d, et, ep, P.OUT_AMPLITUDE if amp else P.OUT_POPULATION)
    torch.cuda.synchronize()
    return out.cpu().numpy(), (None if tot is None else tot.cpu().numpy())


def test_grid16_marginals_amplitudes_and_shots():
    """4x4 grid of the sqrt-gate / CZ family with depolarising + amplitude damping
    (non-unitary Kraus, importance weights); batches [6, 6, 4]."""
    torch, dev = torch_dev()
    import paper_2604_08467_amd as P
    c = W.sqrt_grid(4, 4, 8, np.random.default_rng(31), p=0.05, gamma=0.1)
    bs = [6, 6, 4]
    plan = P.Plan(c, bs)
    assert plan.method == "statevector"
    kr, mult, _, _ = plan.sample_trajectories(32, 12)
    E, m = len(kr), 200
    kd = to_dev(torch, dev, kr)
    psis = oracle_states(c, kr)
    n, starts = c.n_qubits, sampling.batch_starts(bs)
    rng = np.random.default_rng(5)
    for j, (a, b) in enumerate(zip(starts, bs)):
        traj = np.sort(rng.integers(0, E, size=10))
        pre = [int(rng.integers(0, 2 ** a)) if a else 0 for _ in traj]
        pop, tot = _contract(plan, torch, dev, kd, traj, pre, j)
        for e, (i, p) in enumerate(zip(traj, pre)):
            ref = sampling.marginal_from_state(psis[i], n, a, b, p)
            Zt = np.vdot(psis[i], psis[i]).real     # joint marginals, absolute, per unit trajectory norm
            assert np.abs(pop[e] - ref).max() <= 1e-6 * Zt + 1e-12, (j, e)
            assert abs(tot[e] - ref.sum()) <= 1e-5 * Zt + 1e-12
    amp, _ = _contract(plan, torch, dev, kd, traj, pre, len(bs) - 1, amp=True)
    for e, (i, p) in enumerate(zip(traj, pre)):
        ref = sampling.amplitudes_from_state(psis[i], n, starts[-1], bs[-1], p)
        nr = np.linalg.norm(ref)
        if nr > 1e-12:
            assert np.linalg.norm(amp[e] - ref) / nr <= 1e-5
    out = plan.sample_shots(kd, to_dev(torch, dev, np.full(E, m, dtype=np.int64)), 99,
                            mult_dev=to_dev(torch, dev, mult))
    shots = shots_to_ints(out["shots"].cpu().numpy())
    ref, _ = oracle_shots_sv(c, psis, bs, m, 99)
    mism, expect = 0, 0.0
    for i in range(E):
        got = shots[i * m:(i + 1) * m]
        mism += sum(1 for x, y in zip(got, ref[i]) if x != y)
        prefixes = {}
        for t in range(m):
            for j in range(len(bs)):
                p = ref[i][t] & ((1 << starts[j]) - 1)
                prefixes[(j, p)] = prefixes.get((j, p), 0) + 1
        for (j, p), cnt in prefixes.items():
            g, _ = _contract(plan, torch, dev, kd, [i], [p], j)
            expect += cnt * flip_probability(g[0], sampling.marginal_from_state(psis[i], n, starts[j], bs[j], p))
    _say(f"grid16: {mism} mismatches / {E * m}, expected {expect:.3g}")
    assert_shot_parity(mism, expect, E * m)
    Z = np.array([np.vdot(p, p).real for p in psis])
    np.testing.assert_allclose(out["norms"].cpu().numpy(), Z, rtol=1e-5)
    np.testing.assert_allclose(out["weights"].cpu().numpy(), sampling.trajectory_weights(Z, mult), rtol=1e-5)


def test_chunked_sampling_is_identical():
    """A workspace that forces many trajectory chunks gives bit-identical shots,
    norms and weights to a single chunk."""
    torch, dev = torch_dev()
    import paper_2604_08467_amd as P
    c = W.sqrt_grid(4, 5, 6, np.random.default_rng(8))
    plan = P.Plan(c, [8, 8, 4])
    kr, mult, _, _ = plan.sample_trajectories(9, 64)
    E = len(kr)
    kd = to_dev(torch, dev, kr)
    md = to_dev(torch, dev, np.random.default_rng(1).integers(0, 50, size=E).astype(np.int64))
    multd = to_dev(torch, dev, mult)
    big = torch.empty(2 << 30, dtype=torch.uint8, device=dev)
    o1 = plan.sample_shots(kd, md, 5, mult_dev=multd, workspace=big)
    s1, w1, n1 = o1["shots"].clone(), o1["weights"].clone(), o1["norms"].clone()
    small = torch.empty(96 << 20, dtype=torch.uint8, device=dev)   # a few 8 MB states per chunk
    o2 = plan.sample_shots(kd, md, 5, mult_dev=multd, workspace=small)
    assert torch.equal(s1, o2["shots"])
    assert torch.equal(w1, o2["weights"]) and torch.equal(n1, o2["norms"])
    assert list(o1["elements_per_batch"]) == list(o2["elements_per_batch"])


def test_methods_agree_on_a_chain():
    """A 22-qubit chain (depth 4) both methods can take: marginals of sampled
    elements and the shots of the two methods agree."""
    torch, dev = torch_dev()
    import paper_2604_08467_amd as P
    c = W.random_brickwork(22, 4, np.random.default_rng(12), 0.02)
    bs = [8, 8, 6]
    pn = P.Plan(c, bs, method="network")
    ps = P.Plan(c, bs, method="statevector")
    kr, mult, _, _ = pn.sample_trajectories(13, 16)
    E, m = len(kr), 64
    kd = to_dev(torch, dev, kr)
    md = to_dev(torch, dev, np.full(E, m, dtype=np.int64))
    on = pn.sample_shots(kd, md, 21)
    os_ = ps.sample_shots(kd, md, 21)
    sn, ss = shots_to_ints(on["shots"].cpu().numpy()), shots_to_ints(os_["shots"].cpu().numpy())
    mism = sum(1 for a, b in zip(sn, ss) if a != b)
    _say(f"chain22: network vs statevector shots differ in {mism} of {E * m}")
    assert mism <= 0.01 * E * m + 1
    np.testing.assert_allclose(on["norms"].cpu().numpy(), os_["norms"].cpu().numpy(), rtol=1e-5)
    starts = sampling.batch_starts(bs)
    for j in range(len(bs)):
        traj = list(range(0, E, 3))
        pre = [ss[i * m] & ((1 << starts[j]) - 1) for i in traj]
        a, ta = _contract(pn, torch, dev, kd, traj, pre, j)
        b, tb = _contract(ps, torch, dev, kd, traj, pre, j)
        assert np.abs(a - b).max() <= 2e-6   # joint marginals (Pauli noise: trajectory norm 1)


def test_grid25_against_stored_oracle_values():
    """Full 25-qubit grid (5x5, depth 8, depolarising + amplitude damping), batches
    [10, 10, 5]: marginals, norms and shots of two trajectories vs stored FP64
    oracle values."""
    torch, dev = torch_dev()
    import paper_2604_08467_amd as P
    with open(GOLDEN) as f:
        gold = json.load(f)
    wl = W.grid5x5_d8(tuple(gold["batch_sizes"]))
    c = wl.circuit
    plan = P.Plan(c, wl.batch_sizes)
    assert plan.method == "statevector"
    kr_host, _, _, _ = plan.sample_trajectories(gold["pts_seed"], len(gold["trajectories"]))
    kr = np.array([t["kraus"] for t in gold["trajectories"]], dtype=np.uint8)
    assert np.array_equal(kr, kr_host)
    E, m = len(kr), len(gold["trajectories"][0]["shots"])
    kd = to_dev(torch, dev, kr)
    out = plan.sample_shots(kd, to_dev(torch, dev, np.full(E, m, dtype=np.int64)), gold["shot_seed"])
    shots = shots_to_ints(out["shots"].cpu().numpy())
    norms = out["norms"].cpu().numpy()
    mism, expect = 0, 0.0
    for i, rec in enumerate(gold["trajectories"]):
        assert abs(norms[i] - rec["Z"]) <= 1e-5 * rec["Z"], (i, norms[i], rec["Z"])
        for mg in rec["marginals"]:
            ref = np.array(mg["pi"])
            pop, tot = _contract(plan, torch, dev, kd, [i], [mg["prefix"]], mg["j"])
            err = np.abs(pop[0] / tot[0] - ref / ref.sum()).max()
            _say(f"grid25 traj {i} j={mg['j']}: conditional max abs err {err:.3g}")
            assert err <= 1e-6
            if mg["j"] == 0:
                expect += m * flip_probability(pop[0], ref)
        mism += sum(1 for a, b in zip(shots[i * m:(i + 1) * m], rec["shots"]) if a != b)
    _say(f"grid25: {mism} shot mismatches of {E * m}")
    assert mism <= expect + 5 * np.sqrt(max(expect, 1e-12)) + 1


def test_grid25_full_size_properties():
    """2048 trajectories x 256 shots of the 25-qubit grid: deterministic shots,
    self-normalised weights, per-element totals consistent with contract_batch."""
    torch, dev = torch_dev()
    import paper_2604_08467_amd as P
    wl = W.grid5x5_d8((10, 10, 5))
    plan = P.Plan(wl.circuit, wl.batch_sizes)
    kr, mult, _, _ = plan.sample_trajectories(wl.pts_seed, 2048)
    E, m = len(kr), wl.shots_per_traj
    kd = to_dev(torch, dev, kr)
    md = to_dev(torch, dev, np.full(E, m, dtype=np.int64))
    ws = torch.empty(48 << 30, dtype=torch.uint8, device=dev)
    import time
    t = time.perf_counter()
    o1 = plan.sample_shots(kd, md, wl.shot_seed, mult_dev=to_dev(torch, dev, mult), workspace=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    s1 = o1["shots"].clone()
    _say(f"grid25 {E}x{m}: {dt:.2f} s, {E * m / dt:.3g} shots/s, elements {list(o1['elements_per_batch'])}")
    o2 = plan.sample_shots(kd, md, wl.shot_seed, mult_dev=to_dev(torch, dev, mult), workspace=ws)
    assert torch.equal(s1, o2["shots"])
    w = o1["weights"].cpu().numpy()
    norms = o1["norms"].cpu().numpy()
    assert abs(w.sum() - 1) < 1e-12 and np.all(w >= 0)
    # annihilated trajectories (amplitude damping's K1 twice around a CZ) have Z = 0 and weight 0
    assert np.all(np.isfinite(norms) & (norms >= 0))
    # Z_i = |psi_i|^2 with inserted operators K/sqrt(q) is unbiased: E_q[Z] = 1 (each
    # unique trajectory counted with its multiplicity); individual Z_i may exceed 1
    zbar = np.sum(mult * norms) / np.sum(mult)
    zsd = np.sqrt(np.sum(mult * (norms - zbar) ** 2) / np.sum(mult)) / np.sqrt(np.sum(mult))
    _say(f"grid25: weighted mean Z {zbar:.5f} +- {zsd:.5f}")
    assert abs(zbar - 1) <= 5 * zsd + 1e-3
    assert np.array_equal(w == 0, norms == 0)
    _say(f"grid25: {int(np.sum(norms == 0))} annihilated trajectories of {E}")
    traj = [0, 100, 2000]
    _, tot = _contract(plan, torch, dev, kd, traj, [0, 0, 0], 0)
    np.testing.assert_allclose(tot, norms[traj], rtol=1e-6)
