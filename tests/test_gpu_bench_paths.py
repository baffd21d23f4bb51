"""GPU parity of the doubled-network join at the shapes the benchmark runs it.

The benchmark's dominant kernel is the K = 32 slot GEMM of the doubled join
(32 crossing-wire values, >= 128 values of x per tile row), run over many row
tiles of one trajectory, several trajectories per grid, trajectories sharing a
per-trajectory tensor, and trajectory chunks when the workspace is small.  These
tests put every one of those paths against the FP64 oracle (Sec. II-B for the
batch-wise marginals, Sec. III-B for the shots):

* a 20-qubit depth-6 chain with batches [8, 8, 4]: every marginal the oracle's
  per-shot sampler uses, element by element (doubled batches: 1e-6 on the
  conditional; the last batch, contracted to amplitudes: 1e-5 L2-relative on the
  amplitudes and 1e-6 on the joint marginal), and all 64 x 1000 shots under the
  CDF-boundary flip bound, with a workspace that forces trajectory chunks;
* the 50-qubit benchmark circuit: 112 distinct batch-1 prefixes of one trajectory
  (224 join rows, four row tiles), plus a trajectory sharing its per-trajectory
  tensor and one with its own, in one call, against the explicit FP64 network.

Both run with and without the light-cone option (the oracle keeps every gate).

The oracle runs in spawned worker processes (numpy only)."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import sampling
from tests.gpu_helpers import (assert_shot_parity, flip_probability, oracle_pool, prefix_words, shots_to_ints,
                               sv_trajectory_job, tn_value_job, to_dev, torch_dev)

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _smallest_workspace(plan, call, E, count, j, want):
    """Smallest workspace (host query, no device work) whose chunks at batch j hold
    at least `want` trajectories while every batch holds at least one."""
    lo, hi = 1 << 16, 1 << 36
    while hi - lo > 4096:
        mid = (lo + hi) // 2
        caps = plan.chunking(call, E, count, mid)
        if caps[j] >= want and caps.min() >= 1:
            hi = mid
        else:
            lo = mid
    return hi


def _contract(plan, torch, dev, kd, traj, prefixes, j, ws=None, amp=False):
    import paper_2604_08467_amd as P
    et = to_dev(torch, dev, np.asarray(traj, dtype=np.int32))
    ep = to_dev(torch, dev, prefix_words(prefixes, plan.n_words))
    pop, tot = plan.contract_batch(j, kd, et, ep, P.OUT_AMPLITUDE if amp else P.OUT_POPULATION, workspace=ws)
    torch.cuda.synchronize()
    return pop.cpu().numpy(), (None if tot is None else tot.cpu().numpy())


@pytest.mark.parametrize("light_cone", [False, True], ids=["full", "light-cone"])
def test_chain20_k32_join_chunks_and_shared_tensors_vs_statevector_oracle(light_cone):
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    c = W.random_brickwork(20, 6, np.random.default_rng(2024), 0.005).round_to_complex64()
    bs, m, seed = [8, 8, 4], 1000, 2025
    plan = P.Plan(c, bs, method="network", light_cone=light_cone)
    bi = plan.batch_info(1)
    # K = 2^5 crossing wires and >= 128 values of x per row: the qform<32, 8> join
    assert bi["doubled"] and bi["crossing"] == 5 and bi["size"] - bi["join_rows_log2"] >= 7, bi
    kr, mult, _, _ = plan.sample_trajectories(2026, 64)
    E = len(kr)
    assert E == 64
    rs = plan.right_sites(1)
    n_pat = len({tuple(r[rs]) for r in kr})
    _say(f"chain20: {E} trajectories, {n_pat} distinct batch-1 per-trajectory tensors")
    ws_s = _smallest_workspace(plan, "sample", E, E * m, 1, 20)
    caps = plan.chunking("sample", E, E * m, ws_s)
    assert 20 <= caps[1] < E // 2, caps
    # trajectories of one chunk that agree on those sites share one tensor (one slot)
    t = int(caps[1])
    shared = [t1 - t0 - len({tuple(r[rs]) for r in kr[t0:t1]})
              for t0, t1 in ((a, min(E, a + t)) for a in range(0, E, t))]
    assert sum(1 for x in shared if x > 0) >= 2, shared
    _say(f"chain20: sampling workspace {ws_s / 2**20:.1f} MiB, trajectories per chunk {caps.tolist()}")

    with oracle_pool() as pool:
        futs = [pool.submit(sv_trajectory_job, c, kr[i], i, bs, m, seed) for i in range(E)]
        kd = to_dev(torch, dev, kr)
        ws = torch.empty(ws_s, dtype=torch.uint8, device=dev)
        out = plan.sample_shots(kd, to_dev(torch, dev, np.full(E, m, dtype=np.int64)), seed,
                                mult_dev=to_dev(torch, dev, mult), workspace=ws)
        torch.cuda.synchronize()
        got = shots_to_ints(out["shots"].cpu().numpy())
        del ws
        res = [f.result() for f in futs]
    _say("chain20: oracle done")
    ref_shots = [r[0] for r in res]
    used = [r[1] for r in res]
    Z = np.array([r[2] for r in res])
    last_amps = [r[3] for r in res]
    np.testing.assert_allclose(out["norms"].cpu().numpy(), Z, rtol=1e-6)

    # every marginal the oracle used, element by element, batch by batch
    starts = sampling.batch_starts(bs)
    gpu_marg = {}
    for j in range(len(bs)):
        traj, pre = [], []
        for i in range(E):
            for (jj, p) in sorted(used[i]):
                if jj == j:
                    traj.append(i)
                    pre.append(p)
        ws_c = None
        if j == 1:
            wb = _smallest_workspace(plan, "contract", E, len(traj), 1, 16)
            caps_c = plan.chunking("contract", E, len(traj), wb)
            assert caps_c[1] < E // 2, caps_c
            ws_c = torch.empty(wb, dtype=torch.uint8, device=dev)
            per = np.bincount(np.asarray(traj), minlength=E)
            assert (per >= 33).sum() >= 4, per      # >= 33 elements: row tiles beyond the first
            _say(f"chain20: batch 1, {len(traj)} elements, {per.min()}..{per.max()} per trajectory, "
                 f"{caps_c[1]} trajectories per chunk")
        pop, tot = _contract(plan, torch, dev, kd, traj, pre, j, ws_c)
        last = j == len(bs) - 1
        amp = _contract(plan, torch, dev, kd, traj, pre, j, ws_c, amp=True)[0] if last else None
        del ws_c
        worst, worst_joint, worst_amp = 0.0, 0.0, 0.0
        for e, (i, p) in enumerate(zip(traj, pre)):
            ref = used[i][(j, p)]
            Ze = ref.sum()
            err = np.abs(pop[e] - ref).max() / max(Ze, 1e-30)
            worst = max(worst, err)
            if last:
                # the last batch is contracted to amplitudes (Sec. II-B): 1e-5 L2-relative on
                # the element's amplitudes, 1e-6 absolute on its joint marginal p(prefix) P(x | prefix)
                ra = last_amps[i][p]
                rel = np.linalg.norm(amp[e] - ra) / np.linalg.norm(ra)
                joint = err * Ze / Z[i]
                worst_amp, worst_joint = max(worst_amp, rel), max(worst_joint, joint)
                assert rel <= 1e-5, (j, i, p, rel)
                assert joint <= 1e-6, (j, i, p, joint)
            else:
                assert err <= 1e-6, (j, i, p, err)
            assert abs(tot[e] - Ze) <= 1e-5 * Ze + 1e-30, (j, i, p)
            gpu_marg[(i, j, p)] = pop[e]
        _say(f"chain20: batch {j}, {len(traj)} elements, worst conditional error {worst:.3g}"
             + (f", worst amplitude L2-rel {worst_amp:.3g}, worst joint marginal {worst_joint:.3g}" if last else ""))

    # all shots against the oracle's per-shot sampler, under the flip bound
    mism, expect = 0, 0.0
    for i in range(E):
        g = got[i * m:(i + 1) * m]
        mism += sum(1 for a, b in zip(g, ref_shots[i]) if a != b)
        draws = {}                   # draws made from each marginal by the oracle's shots
        for t in range(m):
            for j, a in enumerate(starts):
                key = (j, ref_shots[i][t] & ((1 << a) - 1))
                draws[key] = draws.get(key, 0) + 1
        for (j, p), cnt in draws.items():
            expect += cnt * flip_probability(gpu_marg[(i, j, p)], used[i][(j, p)])
    _say(f"chain20: {mism} of {E * m} shots differ, expected boundary flips {expect:.3g}")
    assert_shot_parity(mism, expect, E * m)


@pytest.mark.parametrize("light_cone", [False, True], ids=["full", "light-cone"])
@pytest.mark.parametrize("bs,j", [([10] * 5, 1), ([5] * 10, 2)], ids=["b10", "b5"])
def test_brickwork50_bench_join_many_prefixes_vs_tensor_network_oracle(bs, j, light_cone):
    """The benchmark's plans (batch lists b = 10 and b = 5, the measured choice)
    at the batch that starts at qubit 10."""
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    wl = W.brickwork50_d6()
    c = wl.circuit
    plan = P.Plan(c, bs, hypersamples=8, light_cone=light_cone)      # the benchmark's plan
    bi = plan.batch_info(j)
    assert bi["doubled"] and bi["crossing"] == 5 and bi["start"] == 10, bi
    kr, _, _, _ = plan.sample_trajectories(wl.pts_seed, 64)
    rs = set(plan.right_sites(j).tolist())
    n_kraus = [c.channels[ch].kraus.shape[0] for ch in c.site_channel]
    # A: a trajectory with an error inside batch 1's per-trajectory part; A2: A with one
    # site outside that part changed (shares A's tensor); B: another trajectory
    a = next(i for i in range(len(kr)) if any(kr[i, s] for s in rs))
    outside = next(s for s in range(len(n_kraus)) if s not in rs and n_kraus[s] > 1 and kr[a, s] == 0)
    a2 = kr[a].copy()
    a2[outside] = 1
    b = next(i for i in range(len(kr)) if i != a and tuple(kr[i, sorted(rs)]) != tuple(kr[a, sorted(rs)]))
    rows = np.stack([kr[a], a2, kr[b]]).astype(np.uint8)
    rng = np.random.default_rng(7117)
    pre = [int(x) for x in rng.choice(1024, 112, replace=False)]
    pre += [int(x) for x in rng.choice(1024, 16, replace=False)]
    pre += [int(x) for x in rng.choice(1024, 16, replace=False)]
    traj = [0] * 112 + [1] * 16 + [2] * 16
    _say(f"brickwork50 {bs[0]}: 144 elements of batch {j} of 3 trajectories (A = {a}, B = {b}), oracle in workers")
    with oracle_pool() as pool:
        futs = [pool.submit(tn_value_job, c, rows[t], 10, bs[j], p, "doubled") for t, p in zip(traj, pre)]
        kd = to_dev(torch, dev, rows)
        pop, tot = _contract(plan, torch, dev, kd, traj, pre, j)
        refs = [f.result() for f in futs]
    worst = 0.0
    for e, ref in enumerate(refs):
        Ze = ref.sum()
        err = np.abs(pop[e] / tot[e] - ref / Ze).max()
        worst = max(worst, err)
        assert err <= 1e-6, (e, traj[e], pre[e], err)
        assert abs(tot[e] - Ze) <= 1e-5 * Ze, (e, tot[e], Ze)
    _say(f"brickwork50: 144 elements, worst conditional error vs FP64 {worst:.3g}")
