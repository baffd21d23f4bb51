"""Ragged sets (several circuits in shared persistent launches) through the C ABI.

Each job of a ragged set must give the shots, norms and weights of the same
plan sampled alone (same Philox counters), one job is also checked against the
FP64 oracle sampler, and graph replay, multi-wave splitting and the autotuner
must not change the results."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import sampling
from tests.gpu_helpers import (assert_shot_parity, flip_probability, oracle_states, shots_to_ints, to_dev,
                               torch_dev)

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mixed_jobs(torch, dev):
    import paper_2604_08467_amd as P
    rng = np.random.default_rng(404)
    specs = [
        (W.random_brickwork(12, 6, rng, 0.02), [10, 2], 24, 40),
        (W.random_brickwork(16, 5, rng, 0.02, layout="2d"), [6, 10], 10, 64),
        (W.sqrt_grid(3, 4, 6, rng, p=0.05, gamma=0.1), [5, 7], 16, 32),
        (W.random_brickwork(20, 4, rng, 0.01), [10, 10], 6, 100),
        (W.random_brickwork(14, 7, rng, 0.03, layout="2d"), [4, 4, 6], 12, 50),
        (W.small_random_circuit(9, 30, rng, [W.depolarizing(0.1), W.amplitude_damping(0.2)]), [9], 20, 30),
    ]
    jobs = []
    for k, (c, bs, E, m) in enumerate(specs):
        plan = P.Plan(c, bs, method="statevector")
        kr, mult, _, _ = plan.sample_trajectories(500 + k, E)
        ms = np.random.default_rng(k).integers(m // 2, m + 1, size=len(kr)).astype(np.int64)
        jobs.append({"plan": plan, "circuit": c, "batch_sizes": bs, "kraus_host": kr,
                     "kraus": to_dev(torch, dev, kr), "mult": to_dev(torch, dev, mult), "mult_host": mult,
                     "shots_per_traj": ms, "seed": 900 + k})
    return jobs


def _alone(torch, dev, jb):
    out = jb["plan"].sample_shots(jb["kraus"], to_dev(torch, dev, jb["shots_per_traj"]), jb["seed"],
                                  mult_dev=jb["mult"])
    return (shots_to_ints(out["shots"].cpu().numpy()), out["norms"].cpu().numpy(), out["weights"].cpu().numpy())


def _compare(torch, dev, jobs, outs, tag):
    for c, (jb, o) in enumerate(zip(jobs, outs)):
        s_alone, n_alone, w_alone = _alone(torch, dev, jb)
        got = shots_to_ints(o["shots"].cpu().numpy())
        mism = sum(1 for a, b in zip(got, s_alone) if a != b)
        _say(f"{tag} job {c} (n={jb['plan'].n_qubits}): {mism} of {len(got)} shots differ from the plan alone")
        assert len(got) == len(s_alone)
        assert mism <= 0.002 * len(got) + 1
        np.testing.assert_allclose(o["norms"].cpu().numpy(), n_alone, rtol=1e-6)
        np.testing.assert_allclose(o["weights"].cpu().numpy(), w_alone, rtol=1e-6)


def test_ragged_set_matches_each_plan_alone():
    torch, dev = torch_dev()
    from paper_2604_08467_amd.ragged import RaggedSet
    jobs = _mixed_jobs(torch, dev)
    rs = RaggedSet()
    outs, lat = rs.sample_shots(jobs)
    info = rs.info()
    _say(f"ragged: {info['n_waves']} wave(s), {info['launches']} launches, latency us {np.round(lat, 1)}")
    assert info["n_waves"] == 1
    assert np.all(lat > 0)
    _compare(torch, dev, jobs, outs, "one wave")


def test_ragged_job_against_oracle():
    """Two jobs of the set (one with amplitude damping) against the FP64 oracle sampler;
    expected CDF-boundary flips come from the plan's own first-batch marginals."""
    torch, dev = torch_dev()
    import paper_2604_08467_amd as P
    from paper_2604_08467_amd.ragged import RaggedSet
    from tests.gpu_helpers import prefix_words
    jobs = _mixed_jobs(torch, dev)
    outs, _ = RaggedSet().sample_shots(jobs)
    for c in (2, 5):
        jb = jobs[c]
        circ, bs, plan = jb["circuit"], jb["batch_sizes"], jb["plan"]
        psis = oracle_states(circ, jb["kraus_host"])
        got = shots_to_ints(outs[c]["shots"].cpu().numpy())
        n, starts = circ.n_qubits, sampling.batch_starts(bs)
        E = len(psis)
        et = to_dev(torch, dev, np.arange(E, dtype=np.int32))
        ep = to_dev(torch, dev, prefix_words([0] * E, plan.n_words))
        pop0, _ = plan.contract_batch(0, jb["kraus"], et, ep, P.OUT_POPULATION)
        pop0 = pop0.cpu().numpy()
        mism, expect, row = 0, 0.0, 0
        for i, psi in enumerate(psis):
            m = int(jb["shots_per_traj"][i])

            def mfn(j, prefix, psi=psi):
                return sampling.marginal_from_state(psi, n, starts[j], bs[j], prefix)

            ref, _ = sampling.sample_trajectory(mfn, i, n, bs, m, jb["seed"])
            mism += sum(1 for a, b in zip(got[row:row + m], ref) if a != b)
            row += m
            expect += m * flip_probability(pop0[i], mfn(0, 0))
        Z = np.array([np.vdot(p, p).real for p in psis])
        np.testing.assert_allclose(outs[c]["norms"].cpu().numpy(), Z, rtol=1e-5)
        np.testing.assert_allclose(outs[c]["weights"].cpu().numpy(),
                                   sampling.trajectory_weights(Z, jb["mult_host"]), rtol=1e-5)
        _say(f"ragged job {c} vs oracle: {mism} of {row} shots differ (expected first-batch flips {expect:.3g})")
        assert_shot_parity(mism, expect, row)


def test_ragged_graph_replay_and_waves():
    torch, dev = torch_dev()
    from paper_2604_08467_amd.ragged import RaggedSet
    jobs = _mixed_jobs(torch, dev)
    rs = RaggedSet()
    ref, _ = rs.sample_shots(jobs)
    ref_shots = [o["shots"].clone() for o in ref]
    stream = torch.cuda.Stream(dev)
    with torch.cuda.stream(stream):
        ws = torch.empty(rs.workspace_size(jobs), dtype=torch.uint8, device=dev)
        outs = None
        for k in range(3):
            if outs is not None:
                for o in outs:
                    o["shots"].fill_(-1)          # the replay must rewrite every row
            outs, lat = rs.sample_shots(jobs, graph=True, workspace=ws, stream=stream.cuda_stream, outputs=outs)
            info = rs.info()
            _say(f"graph call {k}: waves {info['n_waves']}, replayed {info['graphs_replayed']}")
            assert info["graphs_replayed"] == (0 if k == 0 else info["n_waves"])
            torch.cuda.synchronize()              # eager work and a synchronisation between replays
            for o, r in zip(outs, ref_shots):
                assert torch.equal(o["shots"], r)
    torch.cuda.synchronize()
    # a workspace that forces several waves gives the same shots
    small = torch.empty(48 << 20, dtype=torch.uint8, device=dev)
    outs2, _ = rs.sample_shots(jobs, workspace=small)
    info = rs.info()
    _say(f"small workspace: {info['n_waves']} waves")
    assert info["n_waves"] > 1
    for o, r in zip(outs2, ref_shots):
        assert torch.equal(o["shots"], r)


def test_ragged_autotune():
    torch, dev = torch_dev()
    from paper_2604_08467_amd.ragged import RaggedSet
    jobs = _mixed_jobs(torch, dev)
    rs = RaggedSet()
    best, ms = rs.autotune(jobs)
    _say(f"autotune windows {list(best)}; ms/traj {np.round(ms, 4).tolist()}")
    assert np.all((best >= 10) & (best <= 12))
    assert np.all(ms > 0)
    outs, _ = rs.sample_shots(jobs)
    _compare(torch, dev, jobs, outs, "autotuned")
