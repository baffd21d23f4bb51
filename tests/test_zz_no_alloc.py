"""The allocation-free contraction entry point (ptsbe_contract_batch_noalloc)
against ptsbe_contract_batch with a caller workspace: the same populations,
amplitudes and totals on two calls in a row (the second with fewer elements),
for both contraction methods; sizes beyond the static scratch are rejected with
an error before any device work."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import prefix_words, to_dev, torch_dev

pytestmark = pytest.mark.gpu


def _elements(rng, E, n_elems, start):
    traj = np.sort(rng.integers(0, E, size=n_elems)).astype(np.int32)
    pre = [int(rng.integers(0, 2 ** start)) if start else 0 for _ in traj]
    return traj, pre


@pytest.mark.parametrize("method", ["network", "statevector"])
def test_noalloc_matches_workspace_call(method):
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    c = W.random_brickwork(16, 6, np.random.default_rng(77), 0.02).round_to_complex64()
    bs = [6, 6, 4]
    plan = P.Plan(c, bs, method=method)
    kr, _, _, _ = plan.sample_trajectories(78, 24)
    E = len(kr)
    kd = to_dev(torch, dev, kr)
    rng = np.random.default_rng(79)
    starts = [0, 6, 12]
    for j in range(len(bs)):
        for n_elems in (40, 9):            # two calls in a row, the second smaller
            traj, pre = _elements(rng, E, n_elems, starts[j])
            et = to_dev(torch, dev, traj)
            ep = to_dev(torch, dev, prefix_words(pre, plan.n_words))
            ref, rtot = plan.contract_batch(j, kd, et, ep, P.OUT_POPULATION)
            out = torch.full((n_elems, 2 ** bs[j]), float("nan"), dtype=torch.float32, device=dev)
            tot = torch.full((n_elems,), float("nan"), dtype=torch.float64, device=dev)
            plan.contract_batch_noalloc(j, kd, et, ep, out, tot)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (method, j, n_elems)
            assert torch.equal(tot, rtot), (method, j, n_elems)
            if j == len(bs) - 1:
                aref, _ = plan.contract_batch(j, kd, et, ep, P.OUT_AMPLITUDE)
                amp = torch.full((n_elems, 2 ** bs[j], 2), float("nan"), dtype=torch.float32, device=dev)
                plan.contract_batch_noalloc(j, kd, et, ep, amp, None, out_kind=P.OUT_AMPLITUDE)
                torch.cuda.synchronize()
                assert torch.equal(torch.view_as_complex(amp), aref), (method, j, n_elems)


def test_noalloc_rejects_calls_beyond_the_scratch():
    """20 000 trajectories of the 50-qubit benchmark circuit need more merged gates
    than the static scratch holds: an error, no device work, and the entry point
    still works afterwards."""
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    wl = W.brickwork50_d6()
    plan = P.Plan(wl.circuit, wl.batch_sizes, hypersamples=2)
    kr, _, _, _ = plan.sample_trajectories(wl.pts_seed, 8)
    big = np.repeat(kr, 2500, axis=0)          # 20000 rows (merged gates alone: 20000 x 147 x 128 B)
    kd = to_dev(torch, dev, big)
    et = to_dev(torch, dev, np.zeros(1, dtype=np.int32))
    ep = to_dev(torch, dev, prefix_words([0], plan.n_words))
    out = torch.zeros((1, 1024), dtype=torch.float32, device=dev)
    with pytest.raises(P.PtsbeError) as ei:
        plan.contract_batch_noalloc(0, kd, et, ep, out)
    assert ei.value.status == 2 and "static scratch" in str(ei.value), str(ei.value)
    kd8 = to_dev(torch, dev, kr)
    ref, _ = plan.contract_batch(0, kd8, et, ep, P.OUT_POPULATION)
    plan.contract_batch_noalloc(0, kd8, et, ep, out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
