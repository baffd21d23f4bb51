"""Subtree reuse in the per-trajectory parts (plan option subtree_reuse, Sec. VI:
cached intermediates between error sets).  Jobs whose Kraus choices agree on the
sites absorbed so far share the running tensor and split at the launch that
absorbs a site they disagree on; every group runs on gates all its members
share, so populations and shots must be bit-identical to the plan without reuse
(which the other GPU tests hold to the FP64 oracle), and close to the oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import sampling, tn
from tests.gpu_helpers import prefix_words, shots_to_ints, to_dev, torch_dev

pytestmark = pytest.mark.gpu


def _contract(plan, torch, dev, kd, traj, prefixes, j):
    import paper_2604_08467_amd as P
    et = to_dev(torch, dev, np.asarray(traj, dtype=np.int32))
    ep = to_dev(torch, dev, prefix_words(prefixes, plan.n_words))
    pop, tot = plan.contract_batch(j, kd, et, ep, P.OUT_POPULATION)
    torch.cuda.synchronize()
    return pop.cpu().numpy(), tot.cpu().numpy()


@pytest.mark.parametrize("light_cone", [False, True], ids=["full", "light-cone"])
def test_brickwork50_populations_identical_with_and_without_reuse(light_cone):
    """64 trajectories (each with errors somewhere) at batches 1..3 of the 50-qubit
    brickwork; 3 prefixes per trajectory; the first trajectory also against the
    explicit FP64 network."""
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    wl = W.brickwork50_d6()
    c = wl.circuit
    on = P.Plan(c, wl.batch_sizes, hypersamples=8, light_cone=light_cone, subtree_reuse=True)
    off = P.Plan(c, wl.batch_sizes, hypersamples=8, light_cone=light_cone)
    assert on.subtree_reuse and not off.subtree_reuse
    kr, _, _, _ = on.sample_trajectories(wl.pts_seed, 64)
    kd = to_dev(torch, dev, kr)
    rng = np.random.default_rng(31)
    starts = sampling.batch_starts(wl.batch_sizes)
    for j in (1, 2, 3):
        traj = np.repeat(np.arange(len(kr)), 3)
        pre = [int(rng.integers(0, 1 << starts[j])) for _ in traj]
        on.profile_enable(1)
        off.profile_enable(1)
        a, ta = _contract(on, torch, dev, kd, traj, pre, j)
        b, tb = _contract(off, torch, dev, kd, traj, pre, j)
        s_on, s_off = on.profile_read_sweeps(), off.profile_read_sweeps()
        moved_on = s_on["step_bytes"] + s_on["fused_bytes"]
        moved_off = s_off["step_bytes"] + s_off["fused_bytes"]
        print(f"brickwork50 j={j}: per-trajectory part bytes {moved_on / 1e9:.3f} GB with reuse, "
              f"{moved_off / 1e9:.3f} GB without", flush=True)
        assert moved_on < moved_off
        assert np.array_equal(a, b) and np.array_equal(ta, tb), j
        ref = tn.batch_network_value(c, kr[0], starts[j], 10, pre[0], "doubled")
        err = np.abs(a[0] / ta[0] - ref / ref.sum()).max()
        print(f"brickwork50 j={j}: {len(traj)} elements identical with reuse; trajectory 0 vs FP64 {err:.3g}",
              flush=True)
        assert err <= 1e-6


def test_chain_with_amplitude_damping_shots_identical_with_and_without_reuse():
    """A 20-qubit chain with depolarising and amplitude damping, batches [8, 8, 4],
    48 trajectories x 200 shots: shots, weights and norms bit-identical."""
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    rng = np.random.default_rng(77)
    c = W.Circuit(20)
    dep = c.add_channel(W.depolarizing(0.02))
    ad = c.add_channel(W.amplitude_damping(0.05))
    for layer in W.brickwork_1d(20, 6):
        for (q0, q1) in layer:
            g = c.add_gate((q0, q1), W.haar_su4(rng))
            c.add_site(g, (q0,), dep)
            c.add_site(g, (q1,), ad)
    c = c.round_to_complex64()
    bs = [8, 8, 4]
    on = P.Plan(c, bs, method="network", subtree_reuse=True)
    off = P.Plan(c, bs, method="network")
    kr, mult, _, _ = on.sample_trajectories(78, 48)
    kd, md = to_dev(torch, dev, kr), to_dev(torch, dev, np.full(len(kr), 200, dtype=np.int64))
    multd = to_dev(torch, dev, mult)
    a = on.sample_shots(kd, md, 79, mult_dev=multd)
    b = off.sample_shots(kd, md, 79, mult_dev=multd)
    torch.cuda.synchronize()
    for k in ("shots", "weights", "norms"):
        assert torch.equal(a[k], b[k]), k
    assert list(a["elements_per_batch"]) == list(b["elements_per_batch"])
    print(f"chain20 ad: {len(kr)} trajectories, shots identical; elements {list(a['elements_per_batch'])}",
          flush=True)
