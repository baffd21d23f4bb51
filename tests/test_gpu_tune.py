"""Batch lists against measured time (ptsbe_tune_batches, Sec. V-B): every
candidate list is planned and sampled on the same trajectories and timed; lists
the sampler cannot run report -1; the fastest list is returned.  The shots of
each list are checked elsewhere (batch-wise sampling is exact for any list)."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import to_dev, torch_dev

pytestmark = pytest.mark.gpu


def test_tune_batches_times_every_candidate_and_returns_the_fastest():
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    c = W.random_brickwork(24, 6, np.random.default_rng(61), 0.01).round_to_complex64()
    kr, mult, _, _ = P.Plan(c, [8, 8, 8], device=0).sample_trajectories(62, 32)
    E = len(kr)
    cands = [[6, 6, 6, 6], [8, 8, 8], [12, 12], [4] * 6, [13, 11], [5, 5, 5, 5]]
    ws = torch.empty(4 << 30, dtype=torch.uint8, device=dev)
    times, best = P.tune_batches(c, cands, to_dev(torch, dev, kr), to_dev(torch, dev, np.full(E, 200, np.int64)),
                                 63, mult_dev=to_dev(torch, dev, mult), workspace=ws, method="network")
    print("tune:", dict(zip(map(str, cands), np.round(times, 3))), "best", cands[best], flush=True)
    assert times[4] == -1.0 and times[5] == -1.0          # a 13-qubit batch; sizes not summing to 24
    ok = [i for i in range(len(cands)) if i not in (4, 5)]
    assert all(times[i] > 0 for i in ok)
    assert best == min(ok, key=lambda i: times[i])
