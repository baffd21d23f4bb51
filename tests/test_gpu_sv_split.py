"""Split precision on the statevector method: the gate clusters of every window
(16 x 16 complex matrices, the dense contractions of that method) run on 16-bit
MFMA with hi + lo operands and three products, FP32 accumulation; every other
step stays complex64 and FP64 sums, CDFs and weights are unchanged.

The error against the FP64 oracle is measured and printed for every result and
held to a bound derived from the operand precision: a hi + lo pair of bf16
values carries 16 significant bits and of fp16 values 22 (with the per-column
power-of-two scaling that keeps them normal), against complex64's 24.  The
rounding error of the cluster products therefore grows by at most 2^(24 - 16)
= 256 (bf16) or 2^(24 - 22) = 4 (fp16) over that of the complex64 path, whose
tolerance on joint marginals is 1e-6 per unit trajectory norm: 2.56e-4 (bf16),
4e-6 (fp16).  Amplitudes (1e-5 L2-relative for complex64) scale the same way.
The complex64 form runs the same kernel with FP32 MFMA and keeps its own
tolerances."""
import json
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import sampling
from tests.gpu_helpers import oracle_states, prefix_words, to_dev, torch_dev

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "grid25_sv.json")
PREC = {"c64": 0, "bf16": 1, "f16": 2}
GROWTH = {"c64": 1.0, "bf16": 256.0, "f16": 4.0}     # 2^(24 - significant bits of the operands)


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


@pytest.mark.parametrize("prec", ["c64", "bf16", "f16"])
def test_grid16_split_clusters_error_vs_fp64(prec):
    """4x4 grid (sqrt gates, CZ, depolarising + amplitude damping), batches [6, 6, 4]:
    joint marginals of every batch and last-batch amplitudes of 12 trajectories
    against the FP64 statevector."""
    torch, dev = torch_dev()
    import paper_2604_08467_amd as P
    c = W.sqrt_grid(4, 4, 8, np.random.default_rng(31), p=0.05, gamma=0.1)
    bs = [6, 6, 4]
    plan = P.Plan(c, bs, precision=PREC[prec])
    assert plan.method == "statevector" and plan.precision == PREC[prec]
    assert plan.sv_clusters >= 1, "the windows hold no gate cluster: nothing runs in split precision"
    kr, _, _, _ = plan.sample_trajectories(32, 12)
    E = len(kr)
    kd = to_dev(torch, dev, kr)
    psis = oracle_states(c, kr)
    n, starts = c.n_qubits, sampling.batch_starts(bs)
    rng = np.random.default_rng(5)
    g = GROWTH[prec]
    worst_m, worst_a = 0.0, 0.0
    for j, (a, b) in enumerate(zip(starts, bs)):
        traj = np.repeat(np.arange(E), 3)
        pre = [int(rng.integers(0, 2 ** a)) if a else 0 for _ in traj]
        pop, tot = _contract(plan, torch, dev, kd, traj, pre, j)
        for e, (i, p) in enumerate(zip(traj, pre)):
            ref = sampling.marginal_from_state(psis[i], n, a, b, p)
            Zt = np.vdot(psis[i], psis[i]).real
            err = np.abs(pop[e] - ref).max() / max(Zt, 1e-30)
            worst_m = max(worst_m, err)
            assert err <= g * 1e-6 + 1e-12, (prec, j, e, err)
        if j == len(bs) - 1:
            amp, _ = _contract(plan, torch, dev, kd, traj, pre, j, amp=True)
            for e, (i, p) in enumerate(zip(traj, pre)):
                ref = sampling.amplitudes_from_state(psis[i], n, a, b, p)
                nr = np.linalg.norm(ref)
                if nr > 1e-6 * np.sqrt(np.vdot(psis[i], psis[i]).real):
                    rel = np.linalg.norm(amp[e] - ref) / nr
                    worst_a = max(worst_a, rel)
                    assert rel <= g * 1e-5, (prec, e, rel)
    _say(f"grid16 {prec}: {plan.sv_clusters} clusters ({plan.sv_cluster_steps} gates); max joint-marginal error "
         f"vs FP64 {worst_m:.3g} (bound {g * 1e-6:.3g}), max amplitude L2-rel {worst_a:.3g} (bound {g * 1e-5:.3g})")


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_grid25_split_against_stored_oracle_values(prec):
    """The 25-qubit 5x5 grid (depth 8, depolarising + amplitude damping), batches
    [10, 10, 5], in split precision: norms and the stored FP64 marginals of every
    batch (tests/golden/grid25_sv.json)."""
    torch, dev = torch_dev()
    import paper_2604_08467_amd as P
    with open(GOLDEN) as f:
        gold = json.load(f)
    wl = W.grid5x5_d8(tuple(gold["batch_sizes"]))
    plan = P.Plan(wl.circuit, wl.batch_sizes, precision=PREC[prec])
    assert plan.method == "statevector" and plan.sv_clusters >= plan.sv_windows
    kr = np.array([t["kraus"] for t in gold["trajectories"]], dtype=np.uint8)
    kd = to_dev(torch, dev, kr)
    g = GROWTH[prec]
    worst_c, worst_j = 0.0, 0.0
    for i, rec in enumerate(gold["trajectories"]):
        for mg in rec["marginals"]:
            ref = np.array(mg["pi"])
            pop, tot = _contract(plan, torch, dev, kd, [i], [mg["prefix"]], mg["j"])
            if mg["j"] == 0:
                assert abs(tot[0] - rec["Z"]) <= g * 1e-5 * rec["Z"], (i, tot[0], rec["Z"])
            joint = np.abs(pop[0] - ref).max() / rec["Z"]
            cond = np.abs(pop[0] / tot[0] - ref / ref.sum()).max()
            worst_c, worst_j = max(worst_c, cond), max(worst_j, joint)
            assert joint <= g * 1e-6, (prec, i, mg["j"], joint)
    _say(f"grid25 {prec}: max joint-marginal error vs FP64 {worst_j:.3g} (bound {g * 1e-6:.3g}), "
         f"max conditional error {worst_c:.3g}, over {len(gold['trajectories'])} trajectories x 3 batches")
