"""Lane-per-element sampling and element splitting (plan option sample_kernel).

Batches of at most 5 qubits whose elements carry few shots (the later batches of
proportional NBS, Sec. III-B) are sampled and split into children one lane per
element; elements with more shots go to one wavefront each inside the same
kernels.  The lane kernels repeat the wavefront kernel's FP64 partial sums,
chunk ends and binary search in the same order, so shots, weights, norms and
element counts must be bit-identical to the plan that samples every element with
a wavefront (which the other GPU tests hold to the FP64 oracle)."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import to_dev, torch_dev

pytestmark = pytest.mark.gpu


def _both(c, bs, kr, mult, shots_per_traj, seed, **kw):
    import paper_2604_08467_amd as P
    torch, dev = torch_dev()
    auto = P.Plan(c, bs, method="network", **kw)
    wave = P.Plan(c, bs, method="network", sample_kernel="wavefront", **kw)
    kd, md = to_dev(torch, dev, kr), to_dev(torch, dev, shots_per_traj)
    multd = to_dev(torch, dev, mult)
    a = auto.sample_shots(kd, md, seed, mult_dev=multd)
    b = wave.sample_shots(kd, md, seed, mult_dev=multd)
    torch.cuda.synchronize()
    return a, b


def _check(a, b, M, bs, name):
    for k in ("shots", "weights", "norms"):
        assert a[k].shape == b[k].shape and bool((a[k] == b[k]).all()), (name, k)
    ea, eb = [int(v) for v in a["elements_per_batch"]], [int(v) for v in b["elements_per_batch"]]
    assert ea == eb, name
    # the lane kernels ran: some batch of <= 5 qubits with at most 4 shots per element
    lanes = [j for j, (bj, u) in enumerate(zip(bs, ea)) if bj <= 5 and M <= 4 * u]
    print(f"{name}: {M} shots, elements per batch {ea}; lane kernels at batches {lanes}; identical", flush=True)
    assert lanes


def test_brickwork50_b5_skewed_shot_counts():
    """The benchmark circuit under its tuned list [5] * 10 with the light cone;
    256 trajectories, one with 2000 shots and one with 40 (elements with more than
    16 shots inside lane-kernel batches take the wavefront path), the rest 3."""
    torch_dev()          # torch initialises the GPU before the library does
    wl = W.brickwork50_d6()
    import paper_2604_08467_amd as P
    plan = P.Plan(wl.circuit, [5] * 10, hypersamples=8, light_cone=True, method="network")
    kr, mult, _, _ = plan.sample_trajectories(wl.pts_seed, 256)
    m = np.full(len(kr), 3, dtype=np.int64)
    m[0], m[1] = 2000, 40
    a, b = _both(wl.circuit, [5] * 10, kr, mult, m, wl.shot_seed, hypersamples=8, light_cone=True)
    _check(a, b, int(m.sum()), [5] * 10, "brickwork50 b5")


@pytest.mark.parametrize("bs", [[2, 3, 1, 4, 2], [5, 5, 2]], ids=["b1-4", "b5-2"])
def test_chain12_mixed_batch_sizes(bs):
    """A 12-qubit chain (depolarising and amplitude damping) under batch sizes 1..5,
    96 trajectories with 1..12 shots each."""
    torch_dev()
    rng = np.random.default_rng(5150)
    c = W.Circuit(12)
    dep = c.add_channel(W.depolarizing(0.03))
    ad = c.add_channel(W.amplitude_damping(0.05))
    for layer in W.brickwork_1d(12, 6):
        for (q0, q1) in layer:
            g = c.add_gate((q0, q1), W.haar_su4(rng))
            c.add_site(g, (q0,), dep)
            c.add_site(g, (q1,), ad)
    c = c.round_to_complex64()
    import paper_2604_08467_amd as P
    plan = P.Plan(c, bs, method="network")
    kr, mult, _, _ = plan.sample_trajectories(5151, 96)
    m = np.random.default_rng(5152).integers(1, 13, size=len(kr)).astype(np.int64)
    a, b = _both(c, bs, kr, mult, m, 5153)
    _check(a, b, int(m.sum()), bs, f"chain12 {bs}")

