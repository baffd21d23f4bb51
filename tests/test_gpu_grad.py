"""GPU adjoint contraction (through the C ABI) against the FP64 oracle gradients.

Bar: value 1e-5 relative, gradient 1e-4 relative L2 against the FP64 adjoint
gradient (which the CPU pins tie to parameter shift and central differences)."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import gradients as gr
from oracle import pts as opts_pts
from tests.gpu_helpers import to_dev, torch_dev

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _setup(n, layers, noise, E, seed):
    import paper_2604_08467_amd as P
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0, 2 * np.pi, size=2 * n * layers)
    c = W.hea(n, layers, theta, noise)
    gp, ga = W.rotation_spec(c)
    terms = W.zz_chain_terms(n)
    plan = P.Plan(c, [n])
    kr, mult, _, _ = plan.sample_trajectories(seed + 1, E)
    w = mult / mult.sum()
    return P, c, plan, kr, w, theta, gp, ga, terms


@pytest.mark.parametrize("noise,ck", [("depol", 1), ("depol", 7), ("ad", 5), ("ad", 1000)])
def test_small_hea_value_and_gradient(noise, ck):
    torch, dev = torch_dev()
    chans = [W.depolarizing(0.05)] if noise == "depol" else [W.depolarizing(0.05), W.amplitude_damping(0.1)]
    P, c, plan, kr, w, theta, gp, ga, terms = _setup(6, 3, chans, 8, 3)
    spec = P.GradSpec(len(theta), gp, ga, terms, checkpoint_every=ck)
    out = plan.expect_grad(spec, to_dev(torch, dev, kr), to_dev(torch, dev, w), to_dev(torch, dev, theta))
    torch.cuda.synchronize()
    f_ref = gr.value(c, kr, w, theta, gp, ga, terms)
    g_ref = gr.adjoint_gradient(c, kr, w, theta, gp, ga, terms)
    f = float(out["value"].item())
    g = out["grad"].cpu().numpy()
    tv = out["traj_values"].cpu().numpy()
    tv_ref = gr.trajectory_values(c, kr, theta, gp, ga, terms)
    _say(f"hea6 {noise} ck={ck}: f {f:.8f} ref {f_ref:.8f}; grad rel-L2 "
         f"{np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref):.3g}")
    assert abs(f - f_ref) <= 1e-5 * max(1.0, abs(f_ref))
    np.testing.assert_allclose(tv, tv_ref, rtol=1e-5, atol=1e-5)
    assert np.linalg.norm(g - g_ref) <= 1e-4 * np.linalg.norm(g_ref)


def test_small_hea_gradient_vs_central_difference():
    """The GPU gradient against FP64 central differences (h = 1e-3) of the oracle's f."""
    torch, dev = torch_dev()
    P, c, plan, kr, w, theta, gp, ga, terms = _setup(5, 2, [W.depolarizing(0.1)], 6, 11)
    spec = P.GradSpec(len(theta), gp, ga, terms, checkpoint_every=4)
    out = plan.expect_grad(spec, to_dev(torch, dev, kr), to_dev(torch, dev, w), to_dev(torch, dev, theta))
    g = out["grad"].cpu().numpy()
    for k in range(0, len(theta), 3):
        fd = gr.central_difference(c, kr, w, theta, gp, ga, terms, k, h=1e-3)
        assert abs(g[k] - fd) <= 2e-4 * max(1.0, abs(fd)), (k, g[k], fd)


def test_autograd_function_and_gradcheck():
    torch, dev = torch_dev()
    P, c, plan, kr, w, theta, gp, ga, terms = _setup(4, 2, [W.depolarizing(0.1)], 4, 5)
    spec = P.GradSpec(len(theta), gp, ga, terms, checkpoint_every=3)
    kd, wd = to_dev(torch, dev, kr), to_dev(torch, dev, w)
    th = torch.tensor(theta, dtype=torch.float64, device=dev, requires_grad=True)
    f = P.ExpectZZ.apply(th, plan, spec, kd, wd)
    (3.0 * f).backward()
    g_ref = gr.adjoint_gradient(c, kr, w, theta, gp, ga, terms)
    np.testing.assert_allclose(th.grad.cpu().numpy(), 3.0 * g_ref, rtol=1e-4, atol=1e-5)
    # numerical check of the autograd wiring (the forward runs in FP32 on the GPU)
    th2 = torch.tensor(theta, dtype=torch.float64, device=dev, requires_grad=True)
    assert torch.autograd.gradcheck(lambda t: P.ExpectZZ.apply(t, plan, spec, kd, wd), (th2,),
                                    eps=1e-2, atol=2e-3, rtol=1e-2)


def test_hea20_l10_full_size_gradient():
    """20-qubit HEA, 10 layers, 400 angles, 1024 trajectories on the GPU; the FP64
    adjoint gradient of trajectory 0 alone (weight 1) is the reference."""
    torch, dev = torch_dev()
    import paper_2604_08467_amd as P
    wl = W.hea20_l10()
    c = wl.circuit
    theta = W.hea20_angles().astype(np.float64)
    gp, ga = W.rotation_spec(c)
    terms = W.zz_chain_terms(20)
    plan = P.Plan(c, [20])
    kr, mult, _, _ = plan.sample_trajectories(wl.pts_seed, wl.n_traj)
    _say(f"hea20_l10: {len(kr)} trajectories")
    spec = P.GradSpec(400, gp, ga, terms, checkpoint_every=24)
    kd = to_dev(torch, dev, kr)
    w = mult / mult.sum()
    import time
    t = time.perf_counter()
    out = plan.expect_grad(spec, kd, to_dev(torch, dev, w), to_dev(torch, dev, theta))
    torch.cuda.synchronize()
    _say(f"hea20_l10: value {out['value'].item():.6f}, forward+adjoint {time.perf_counter() - t:.2f} s")
    g_all = out["grad"].cpu().numpy()
    assert np.all(np.isfinite(g_all))
    # trajectory 0 alone
    w1 = np.zeros(len(kr))
    w1[0] = 1.0
    out1 = plan.expect_grad(spec, kd, to_dev(torch, dev, w1), to_dev(torch, dev, theta))
    g1 = out1["grad"].cpu().numpy()
    g_ref = gr.adjoint_gradient(c, kr[:1], np.ones(1), theta, gp, ga, terms)
    f_ref = gr.value(c, kr[:1], np.ones(1), theta, gp, ga, terms)
    rel = np.linalg.norm(g1 - g_ref) / np.linalg.norm(g_ref)
    _say(f"hea20_l10 trajectory 0: f {out1['value'].item():.6f} ref {f_ref:.6f}, grad rel-L2 {rel:.3g}")
    assert abs(out1["value"].item() - f_ref) <= 1e-4 * max(1.0, abs(f_ref))
    assert rel <= 1e-4
