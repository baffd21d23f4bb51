"""Non-proportional NBS (Sec. III-B) through the C ABI, against the FP64 oracle:
exhaustive final-batch sampling, and direct final-batch draws.

Draws at the non-final batches use the same Philox counters on both sides, so
the sets of prefixes must be identical (a CDF-boundary flip would change one;
at these sizes its probability is far below 1e-3 for the whole test).  Rows are
compared bit for bit except values of x whose oracle conditional lies within
1e-6 of the threshold (FP32 populations decide those); conditionals and prefix
probabilities within 1e-6 absolute, trajectory norms and weights 1e-5 relative."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import sampling
from tests.gpu_helpers import oracle_states, shots_to_ints, to_dev, torch_dev

pytestmark = pytest.mark.gpu

BAND = 1e-6


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_rows(circ, bs, kr, draws, seed, thr):
    n, starts = circ.n_qubits, sampling.batch_starts(bs)
    rows, counts = [], np.zeros(len(bs), dtype=np.int64)
    psis = oracle_states(circ, kr)
    for i, psi in enumerate(psis):
        def mfn(j, prefix, psi=psi):
            return sampling.marginal_from_state(psi, n, starts[j], bs[j], prefix)
        r, c = sampling.nonproportional_trajectory(mfn, i, n, bs, draws, seed, thr)
        rows.extend((i,) + tuple(x) for x in r)
        counts += np.array(c)
    return rows, counts, psis


def _compare(out, ref_rows, ref_counts, bs, thr, tag):
    got_bits = shots_to_ints(out["bits"].cpu().numpy())
    got_traj = out["row_traj"].cpu().numpy()
    got_pc = out["p_cond"].cpu().numpy()
    got_pp = out["p_prefix"].cpu().numpy()
    assert list(out["elements_per_batch"]) == list(ref_counts), (tag, out["elements_per_batch"], ref_counts)
    got = {(int(t), b): (pc, pp) for t, b, pc, pp in zip(got_traj, got_bits, got_pc, got_pp)}
    ref = {(t, b): (pc, pp) for t, b, pc, pp in ref_rows}
    assert len(got) == len(got_bits)                      # no row twice
    only_got = [k for k in got if k not in ref]
    only_ref = [k for k in ref if k not in got]
    for k in only_got:
        assert abs(got[k][0] - thr) <= BAND, (tag, "extra row", k, got[k])
    for k in only_ref:
        assert abs(ref[k][0] - thr) <= BAND, (tag, "missing row", k, ref[k])
    err_pc = max((abs(got[k][0] - ref[k][0]) for k in got if k in ref), default=0.0)
    err_pp = max((abs(got[k][1] - ref[k][1]) for k in got if k in ref), default=0.0)
    _say(f"{tag}: {len(got_bits)} rows (oracle {len(ref_rows)}), {len(only_got)}+{len(only_ref)} in the "
         f"threshold band; max |dP(x|prefix)| {err_pc:.2e}, max |dp(prefix)| {err_pp:.2e}")
    assert err_pc <= 1e-6 and err_pp <= 1e-6
    # row order: trajectory, then prefix (first batch most significant), then x
    keys = [(int(t),) + tuple((b >> s) & ((1 << w) - 1) for s, w in zip(sampling.batch_starts(bs), bs))
            for t, b in zip(got_traj, got_bits)]
    assert keys == sorted(keys)


# network-sliced: the last batch's per-trajectory tensor capped so that crossing
# wires are sliced (2, 4 and 1 of them) and the join's amplitudes summed over slices
SLICE_CAP = {(4, 4, 4): 6, (5, 7): 6, (3, 3, 3, 3): 5}


@pytest.mark.parametrize("method", ["network", "statevector", "network-sliced"])
@pytest.mark.parametrize("bs,draws,thr", [([4, 4, 4], 3, 1e-3), ([5, 7], 5, 0.0), ([3, 3, 3, 3], 2, 2e-3)],
                         ids=["4-4-4_k3", "5-7_k5", "3x4_k2"])
def test_exhaustive_matches_oracle(bs, draws, thr, method):
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    rng = np.random.default_rng(301)
    circ = W.random_brickwork(sum(bs), 5, rng, 0.02)
    if method == "network-sliced":
        plan = P.Plan(circ, bs, method="network", max_part_rank=SLICE_CAP[tuple(bs)])
        assert plan.batch_info(len(bs) - 1)["slice_bits"] > 0
    else:
        plan = P.Plan(circ, bs, method=method)
    kr, mult, _, _ = plan.sample_trajectories(302, 12)
    out = plan.sample_nonproportional(to_dev(torch, dev, kr), draws, 303, thr, mult_dev=to_dev(torch, dev, mult))
    torch.cuda.synchronize()
    ref_rows, ref_counts, psis = _oracle_rows(circ, bs, kr, draws, 303, thr)
    _compare(out, ref_rows, ref_counts, bs, thr, f"{method}: batches {bs}, draws {draws}, threshold {thr}")
    Z = np.array([np.vdot(p, p).real for p in psis])
    np.testing.assert_allclose(out["norms"].cpu().numpy(), Z, rtol=1e-5)
    np.testing.assert_allclose(out["weights"].cpu().numpy(), sampling.trajectory_weights(Z, mult), rtol=1e-5)


def test_exhaustive_single_batch():
    """One batch: every trajectory's rows are its x with |psi(x)|^2 / Z above the threshold,
    p(prefix) = 1; the norms come from the batch's own totals."""
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    wl = W.chain10_d8()
    plan = P.Plan(wl.circuit, wl.batch_sizes, method="network")
    kr, mult, _, _ = plan.sample_trajectories(wl.pts_seed, 16)
    thr = 2e-3
    out = plan.sample_nonproportional(to_dev(torch, dev, kr), 1, 5, thr, mult_dev=to_dev(torch, dev, mult))
    ref_rows, ref_counts, psis = _oracle_rows(wl.circuit, wl.batch_sizes, kr, 1, 5, thr)
    _compare(out, ref_rows, ref_counts, wl.batch_sizes, thr, "single batch")
    assert np.all(out["p_prefix"].cpu().numpy() == 1.0)
    Z = np.array([np.vdot(p, p).real for p in psis])
    np.testing.assert_allclose(out["norms"].cpu().numpy(), Z, rtol=1e-5)
    np.testing.assert_allclose(out["weights"].cpu().numpy(), sampling.trajectory_weights(Z, mult), rtol=1e-5)


def test_exhaustive_large_final_batch():
    """A 16-qubit final batch (16 tiles of 4096 values per element) after a 4-qubit batch."""
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    rng = np.random.default_rng(311)
    circ = W.random_brickwork(20, 4, rng, 0.02)
    bs = [4, 16]
    plan = P.Plan(circ, bs, method="network")
    kr, mult, _, _ = plan.sample_trajectories(312, 3)
    thr = 1e-5
    out = plan.sample_nonproportional(to_dev(torch, dev, kr), 2, 313, thr)
    ref_rows, ref_counts, _ = _oracle_rows(circ, bs, kr, 2, 313, thr)
    _compare(out, ref_rows, ref_counts, bs, thr, "final batch of 16 qubits")
    # every prefix's rows at threshold 0 would sum to 1; above it they sum to at most 1
    pc = out["p_cond"].cpu().numpy()
    assert pc.max() <= 1.0 + 1e-6


def test_exhaustive_capacity_overflow_keeps_the_first_rows():
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    rng = np.random.default_rng(321)
    circ = W.random_brickwork(12, 5, rng, 0.02)
    bs = [4, 8]
    plan = P.Plan(circ, bs, method="network")
    kr, _, _, _ = plan.sample_trajectories(322, 6)
    kd = to_dev(torch, dev, kr)
    full = plan.sample_nonproportional(kd, 3, 323, 1e-4)
    n = full["n_rows"]
    assert n > 10
    with pytest.raises(P.PtsbeError) as ei:
        plan.sample_nonproportional(kd, 3, 323, 1e-4, capacity=n // 2)
    assert ei.value.needed_rows == n
    part = {k: torch.empty((n // 2,) + tuple(v.shape[1:]), dtype=v.dtype, device=dev)
            for k, v in full.items() if k in ("bits", "row_traj", "p_cond", "p_prefix")}
    with pytest.raises(P.PtsbeError):
        plan.sample_nonproportional(kd, 3, 323, 1e-4, capacity=n // 2, outputs=part)
    torch.cuda.synchronize()
    assert torch.equal(part["bits"], full["bits"][:n // 2])
    assert torch.equal(part["row_traj"], full["row_traj"][:n // 2])
    # more elements than max_elems is an error, not an overrun
    with pytest.raises(P.PtsbeError):
        plan.sample_nonproportional(kd, 3, 323, 1e-4, max_elems=len(kr))


@pytest.mark.parametrize("method", ["network", "statevector"])
@pytest.mark.parametrize("bs,draws,fd", [([4, 4, 4], 2, 50), ([6, 6], 3, 200), ([10], 1, 500)],
                         ids=["4-4-4_k2_f50", "6-6_k3_f200", "10_f500"])
def test_direct_final_batch_matches_oracle(bs, draws, fd, method):
    """Direct final-batch draws: identical element counts, rows in the same order with
    identical bitstrings except CDF-boundary flips of the final draws (at most 0.1 % of the
    rows), P(x | prefix) and p(prefix) of identical rows within 1e-6."""
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    rng = np.random.default_rng(331)
    circ = W.random_brickwork(sum(bs), 5, rng, 0.02)
    plan = P.Plan(circ, bs, method=method)
    kr, mult, _, _ = plan.sample_trajectories(332, 10)
    out = plan.sample_nonproportional(to_dev(torch, dev, kr), draws, 333, final_draws=fd,
                                      mult_dev=to_dev(torch, dev, mult))
    n, starts = circ.n_qubits, sampling.batch_starts(bs)
    ref_rows, ref_counts = [], np.zeros(len(bs), dtype=np.int64)
    psis = oracle_states(circ, kr)
    for i, psi in enumerate(psis):
        def mfn(j, prefix, psi=psi):
            return sampling.marginal_from_state(psi, n, starts[j], bs[j], prefix)
        r, c = sampling.nonproportional_trajectory(mfn, i, n, bs, draws, 333, 0.0, final_draws=fd)
        ref_rows.extend((i,) + tuple(x) for x in r)
        ref_counts += np.array(c)
    assert list(out["elements_per_batch"]) == list(ref_counts)
    assert out["n_rows"] == len(ref_rows) == int(ref_counts[-1]) * fd
    bits = shots_to_ints(out["bits"].cpu().numpy())
    traj = out["row_traj"].cpu().numpy()
    pc = out["p_cond"].cpu().numpy()
    pp = out["p_prefix"].cpu().numpy()
    same = [k for k in range(len(ref_rows)) if bits[k] == ref_rows[k][1]]
    assert np.array_equal(traj, np.array([r[0] for r in ref_rows]))
    err_pc = max(abs(pc[k] - ref_rows[k][2]) for k in same)
    err_pp = max(abs(pp[k] - ref_rows[k][3]) for k in same)
    _say(f"{method}: direct {bs} draws {draws} final {fd}: {len(ref_rows) - len(same)} of {len(ref_rows)} rows differ; "
         f"max |dP(x|prefix)| {err_pc:.2e}, max |dp(prefix)| {err_pp:.2e}")
    assert len(ref_rows) - len(same) <= 0.001 * len(ref_rows) + 1
    assert err_pc <= 1e-6 and err_pp <= 1e-6
    Z = np.array([np.vdot(p, p).real for p in psis])
    np.testing.assert_allclose(out["norms"].cpu().numpy(), Z, rtol=1e-5)
    np.testing.assert_allclose(out["weights"].cpu().numpy(), sampling.trajectory_weights(Z, mult), rtol=1e-5)


@pytest.mark.parametrize("method", ["network", "statevector"])
def test_exhaustive_grid_with_amplitude_damping(method):
    """A 3x4 grid of sqrt-gates and CZ with depolarising and amplitude damping (non-unit
    norms, importance weights), batches [4, 4, 4], two draws per prefix."""
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    rng = np.random.default_rng(341)
    circ = W.sqrt_grid(3, 4, 5, rng, p=0.05, gamma=0.1)
    bs = [4, 4, 4]
    plan = P.Plan(circ, bs, method=method)
    kr, mult, _, _ = plan.sample_trajectories(342, 16)
    thr = 5e-4
    out = plan.sample_nonproportional(to_dev(torch, dev, kr), 2, 343, thr, mult_dev=to_dev(torch, dev, mult))
    ref_rows, ref_counts, psis = _oracle_rows(circ, bs, kr, 2, 343, thr)
    _compare(out, ref_rows, ref_counts, bs, thr, f"{method}: 3x4 grid with amplitude damping")
    Z = np.array([np.vdot(p, p).real for p in psis])
    np.testing.assert_allclose(out["norms"].cpu().numpy(), Z, rtol=1e-5)
    np.testing.assert_allclose(out["weights"].cpu().numpy(), sampling.trajectory_weights(Z, mult), rtol=1e-5)


def test_statevector_chunking_does_not_change_rows():
    """A workspace that holds only a few states at a time gives the same rows."""
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    rng = np.random.default_rng(351)
    circ = W.random_brickwork(14, 5, rng, 0.03, layout="2d")
    bs = [5, 5, 4]
    plan = P.Plan(circ, bs, method="statevector")
    kr, _, _, _ = plan.sample_trajectories(352, 40)
    kd = to_dev(torch, dev, kr)
    full = plan.sample_nonproportional(kd, 2, 353, 1e-3)
    E = len(kr)
    need = plan.nonproportional_workspace_size(E, 2, E * 4)
    small = need - (4 << 20) - (E - 3) * (8 << 14)      # room for a few states at a time
    ws = torch.empty(small, dtype=torch.uint8, device=dev)
    part = plan.sample_nonproportional(kd, 2, 353, 1e-3, workspace=ws)
    _say(f"chunked: {part['n_rows']} rows, unchunked {full['n_rows']}")
    assert part["n_rows"] == full["n_rows"]
    assert torch.equal(part["bits"], full["bits"]) and torch.equal(part["p_cond"], full["p_cond"])
    a = plan.sample_nonproportional(kd, 2, 353, final_draws=25)
    b = plan.sample_nonproportional(kd, 2, 353, final_draws=25, workspace=ws)
    assert torch.equal(a["bits"], b["bits"]) and torch.equal(a["p_prefix"], b["p_prefix"])


@pytest.mark.parametrize("light_cone", [False, True], ids=["full", "light-cone"])
def test_exhaustive_paper_random_circuit_bf20_vs_tensor_network_oracle(light_cone):
    """The paper's random-circuit family at its scale (Sec. IV-B, V-A): 50 qubits,
    200 gates, batches [10, 10, 10, 20] (b = 10, b_f = 20), two draws per prefix at
    the non-final batches; every row of four trajectories against the oracle's
    per-trajectory non-proportional sampler on explicit FP64 networks (doubled
    networks for the draws, the ket network for the 2^20 final-batch values)."""
    import paper_2604_08467_amd as P
    from oracle import tn
    torch, dev = torch_dev()
    circ = W.paper_random_circuit(50, 200, np.random.default_rng(7250)).round_to_complex64()
    bs, draws, thr, seed = [10, 10, 10, 20], 2, 1e-4, 7301
    plan = P.Plan(circ, bs, method="network", hypersamples=4, light_cone=light_cone)
    kr, mult, _, _ = plan.sample_trajectories(7350, 4)
    out = plan.sample_nonproportional(to_dev(torch, dev, kr), draws, seed, thr, mult_dev=to_dev(torch, dev, mult))
    torch.cuda.synchronize()
    starts = sampling.batch_starts(bs)
    ref_rows, ref_counts, Z = [], np.zeros(len(bs), dtype=np.int64), []
    for i in range(len(kr)):
        def mfn(j, prefix, i=i):
            kind = "ket" if j == len(bs) - 1 else "doubled"
            v = tn.batch_network_value(circ, kr[i], starts[j], bs[j], prefix, kind)
            return np.abs(v) ** 2 if kind == "ket" else v
        r, c = sampling.nonproportional_trajectory(mfn, i, circ.n_qubits, bs, draws, seed, thr)
        ref_rows.extend((i,) + tuple(x) for x in r)
        ref_counts += np.array(c)
        Z.append(float(np.sum(mfn(0, 0))))
    _compare(out, ref_rows, ref_counts, bs, thr, f"paper circuit n=50 g=200 b_f=20 (light cone {light_cone})")
    np.testing.assert_allclose(out["norms"].cpu().numpy(), np.array(Z), rtol=1e-5)
