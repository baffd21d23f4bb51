"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
(closed forms, invariants, brute force on tiny inputs), never against itself."""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import philox, pts, sampling, statevector as sv, tn, upv


# ----------------------------------------------------------------- bit order
def _circuit(n, gates):
    c = W.Circuit(n)
    for qs, m in gates:
        c.add_gate(qs, m)
    return c


def test_cnot_truth_table_and_bit_order():
    # qubit q <-> bit q of the amplitude index; CNOT(q0 -> q1) index 2*x[q0] + x[q1]
    for ctrl, tgt in [(0, 1), (1, 0), (2, 0), (0, 2)]:
        for inp in range(8):
            c = W.Circuit(3)
            for q in range(3):
                if (inp >> q) & 1:
                    c.add_gate((q,), W.pauli_x)
            c.add_gate((ctrl, tgt), W.CNOT)
            psi = sv.ideal_state(c)
            out = inp ^ ((((inp >> ctrl) & 1)) << tgt)
            assert abs(psi[out] - 1) < 1e-15, (ctrl, tgt, inp)


def test_ghz_marginals_closed_form():
    n = 4
    gates = [((0,), W.HADAMARD)] + [((q, q + 1), W.CNOT) for q in range(n - 1)]
    psi = sv.ideal_state(_circuit(n, gates))
    assert abs(np.linalg.norm(psi) - 1) < 1e-14
    # batch 1 = qubits {0,1}: P(00) = P(11) = 1/2
    m = sampling.marginal_from_state(psi, n, 0, 2, 0)
    np.testing.assert_allclose(m, [0.5, 0, 0, 0.5], atol=1e-15)
    # given prefix 11 the last batch is fixed to 11; given 01 it has weight 0
    m = sampling.marginal_from_state(psi, n, 2, 2, 0b11)
    np.testing.assert_allclose(m, [0, 0, 0, 0.5], atol=1e-15)
    assert np.all(sampling.marginal_from_state(psi, n, 2, 2, 0b01) == 0)


def test_product_state_marginals_factorise():
    rng = np.random.default_rng(7)
    n = 5
    gates, probs = [], []
    for q in range(n):
        th = rng.uniform(0, np.pi)
        gates.append(((q,), W.ry(th)))
        probs.append(np.sin(th / 2) ** 2)        # P(x_q = 1) for RY(th)|0>
    psi = sv.ideal_state(_circuit(n, gates))
    m = sampling.marginal_from_state(psi, n, 1, 3, 1)
    want = np.zeros(8)
    for x in range(8):
        pr = probs[0]                            # prefix qubit 0 = 1
        for k in range(3):
            bit = (x >> k) & 1
            pr *= probs[1 + k] if bit else 1 - probs[1 + k]
        want[x] = pr
    np.testing.assert_allclose(m, want, atol=1e-14)


# ------------------------------------------------------------------- channels
@pytest.mark.parametrize("ch", [W.depolarizing(0.01), W.depolarizing(0.3), W.amplitude_damping(0.02),
                                W.amplitude_damping(0.7), W.depolarizing2(0.1)])
def test_channels_are_cptp(ch):
    d = ch.kraus.shape[1]
    s = sum(k.conj().T @ k for k in ch.kraus)
    np.testing.assert_allclose(s, np.eye(d), atol=1e-14)
    q = upv.proposal(ch)
    assert abs(q.sum() - 1) < 1e-14 and np.all(q > 0)


def test_pauli_inserted_operators_are_unitary():
    for ch in [W.depolarizing(0.2), W.depolarizing2(0.1)]:
        for k in range(len(ch.kraus)):
            op = upv.inserted_operator(ch, k)
            np.testing.assert_allclose(op.conj().T @ op, np.eye(op.shape[0]), atol=1e-14)


def test_haar_su4():
    rng = np.random.default_rng(3)
    for _ in range(20):
        u = W.haar_su4(rng)
        np.testing.assert_allclose(u.conj().T @ u, np.eye(4), atol=1e-13)
        assert abs(np.linalg.det(u) - 1) < 1e-12


def test_embed_matches_kron():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    np.testing.assert_allclose(upv.embed(a, (5,), (5, 9)), np.kron(a, np.eye(2)), atol=0)
    np.testing.assert_allclose(upv.embed(a, (9,), (5, 9)), np.kron(np.eye(2), a), atol=0)
    b = rng.standard_normal((4, 4))
    swap = np.eye(4)[[0, 2, 1, 3]]
    np.testing.assert_allclose(upv.embed(b, (9, 5), (5, 9)), swap @ b @ swap, atol=0)


# ------------------------------------------------------------------------ UPV
def _tiny_noisy(seed, n=4, gates=7, channels=None):
    rng = np.random.default_rng(seed)
    if channels is None:
        channels = [W.depolarizing(0.2), W.amplitude_damping(0.3)]
    return W.small_random_circuit(n, gates, rng, channels, site_prob=0.7)


def _random_rows(c, rng, count):
    qs = [upv.proposal(c.channels[ch]) for ch in c.site_channel]
    return [np.array([rng.integers(0, len(q)) for q in qs], dtype=np.uint8) for _ in range(count)]


def test_upv_merged_equals_explicit_insertion_statevector():
    rng = np.random.default_rng(11)
    for seed in range(4):
        c = _tiny_noisy(seed, n=4, gates=9)
        for row in _random_rows(c, rng, 5):
            a = sv.trajectory_state(c, row)
            b = sv.trajectory_state_explicit(c, row)
            np.testing.assert_allclose(a, b, atol=1e-13)


def test_upv_merged_network_equals_explicit_network():
    """The paper's central UPV claim: merging the error operators into their gates
    gives the same network value as inserting them as separate tensors."""
    rng = np.random.default_rng(12)
    c = _tiny_noisy(5, n=5, gates=10)
    for row in _random_rows(c, rng, 3):
        for (start, b, kind) in [(0, 2, "doubled"), (2, 2, "doubled"), (3, 2, "ket")]:
            prefix = int(rng.integers(0, 2 ** start)) if start else 0
            a = tn.batch_network_value(c, row, start, b, prefix, kind, explicit=False)
            e = tn.batch_network_value(c, row, start, b, prefix, kind, explicit=True)
            np.testing.assert_allclose(a, e, atol=1e-13)


# ------------------------------------------- trajectory average == density matrix
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_exact_enumeration_equals_density_matrix(seed):
    rng = np.random.default_rng(100 + seed)
    chans = [W.depolarizing(0.15), W.amplitude_damping(0.25)]
    c = W.small_random_circuit(3, 3, rng, chans, site_prob=1.0, two_qubit_frac=0.5)
    # keep at most 6 sites so that enumeration stays tiny
    keep = list(range(min(6, c.n_sites)))
    c.site_gate = [c.site_gate[i] for i in keep]
    c.site_qubits = [c.site_qubits[i] for i in keep]
    c.site_channel = [c.site_channel[i] for i in keep]
    rho = sv.density_matrix_diag(c)
    acc = np.zeros(2 ** c.n_qubits)
    for row, qk in sv.enumerate_trajectories(c):
        acc += qk * np.abs(sv.trajectory_state(c, row)) ** 2
    np.testing.assert_allclose(acc, rho, atol=1e-12)
    assert abs(rho.sum() - 1) < 1e-12


def test_pauli_trajectory_norm_is_one():
    rng = np.random.default_rng(21)
    c = W.random_brickwork(8, 4, rng, 0.3)          # unrounded FP64 gates
    for row in _random_rows(c, rng, 10):
        psi = sv.trajectory_state(c, row)
        assert abs(np.vdot(psi, psi).real - 1) < 1e-12


def test_monte_carlo_weighted_average_converges_to_density_matrix():
    """PTS draws + self-normalised importance weights (non-unitary amplitude
    damping) converge to the exact density-matrix diagonal within 5 sigma."""
    rng = np.random.default_rng(31)
    c = W.small_random_circuit(3, 4, rng, [W.depolarizing(0.2), W.amplitude_damping(0.4)], site_prob=1.0)
    rho = sv.density_matrix_diag(c)
    kr, mult, logq, nd = pts.presample(c, seed=77, n_unique=10 ** 6, max_draws=4000)
    Z = np.empty(len(kr))
    P = np.empty((len(kr), 2 ** c.n_qubits))
    for i, row in enumerate(kr):
        psi = sv.trajectory_state(c, row)
        Z[i] = np.vdot(psi, psi).real
        P[i] = np.abs(psi) ** 2 / Z[i]
    Wt = sampling.trajectory_weights(Z, mult)
    est = Wt @ P
    # per-draw values of the ratio estimator and their spread
    draws = np.repeat(np.arange(len(kr)), mult)
    num = (Z[:, None] * P)[draws]
    den = Z[draws]
    resid = num - est[None, :] * den[:, None]
    sigma = resid.std(axis=0) / den.mean() / math.sqrt(len(draws))
    assert nd == 4000
    assert np.all(np.abs(est - rho) <= 5 * sigma + 1e-12), (est, rho, sigma)


# ------------------------------------------------------------ path independence
def test_tn_orders_and_statevector_agree():
    rng = np.random.default_rng(41)
    c = W.random_brickwork(7, 4, rng, 0.2)
    row = _random_rows(c, rng, 1)[0]
    psi = sv.trajectory_state(c, row)
    n = 7
    for (start, b) in [(0, 3), (3, 2), (2, 5)]:
        kind = "ket" if start + b == n else "doubled"
        for prefix in range(min(2 ** start, 4)):
            if kind == "ket":
                want = sampling.amplitudes_from_state(psi, n, start, b, prefix)
            else:
                want = sampling.marginal_from_state(psi, n, start, b, prefix)
            for order in ("ltr", "rtl", "inward"):
                got = tn.batch_network_value(c, row, start, b, prefix, kind, order=order)
                np.testing.assert_allclose(got, want, atol=1e-12)


def test_chain_rule_of_marginals():
    rng = np.random.default_rng(51)
    c = W.random_brickwork(8, 5, rng, 0.1)
    psi = sv.trajectory_state(c, _random_rows(c, rng, 1)[0])
    n = 8
    p1 = sampling.marginal_from_state(psi, n, 0, 3, 0)
    assert abs(p1.sum() - 1) < 1e-12
    for x in range(8):
        p2 = sampling.marginal_from_state(psi, n, 3, 3, x)
        assert abs(p2.sum() - p1[x]) < 1e-13


# --------------------------------------------------------------------- sampling
def test_inverse_cdf_brute_force():
    pi = np.array([0.0, 0.25, 0.0, 0.5, 0.25, 0.0])
    # boundaries of the strict rule C(x) > u Z
    assert sampling.inverse_cdf(pi, 0.0) == 1
    assert sampling.inverse_cdf(pi, 0.2499999) == 1
    assert sampling.inverse_cdf(pi, 0.25) == 3
    assert sampling.inverse_cdf(pi, 0.7499999) == 3
    assert sampling.inverse_cdf(pi, 0.75) == 4
    assert sampling.inverse_cdf(pi, 1 - 2 ** -53) == 4
    # unnormalised input: the rule scales u by the total
    assert sampling.inverse_cdf(4 * pi, 0.75) == 4
    for u in np.linspace(0, 1 - 1e-12, 1001):
        assert pi[sampling.inverse_cdf(pi, u)] > 0


def test_shot_distribution_tvd_bound():
    """Per-shot sampler vs the exact distribution: TVD <= 1/2 sqrt(K/M) + sqrt(ln(1/d)/(2M))."""
    rng = np.random.default_rng(61)
    c = W.random_brickwork(6, 4, rng, 0.0)
    psi = sv.ideal_state(c)
    n, bs = 6, [2, 2, 2]
    starts = sampling.batch_starts(bs)

    def mfn(j, prefix):
        return sampling.marginal_from_state(psi, n, starts[j], bs[j], prefix)

    M = 20000
    shots, distinct = sampling.sample_trajectory(mfn, 0, n, bs, M, seed=5)
    hist = np.bincount(np.array(shots), minlength=64) / M
    tvd = 0.5 * np.abs(hist - np.abs(psi) ** 2).sum()
    bound = 0.5 * math.sqrt(64 / M) + math.sqrt(math.log(1e9) / (2 * M))
    assert tvd <= bound, (tvd, bound)
    assert distinct[0] == 1 and distinct[1] <= 4 and distinct[2] <= 16


def test_nbs_memo_matches_unmemoised_per_shot_sampling():
    rng = np.random.default_rng(62)
    c = W.random_brickwork(6, 3, rng, 0.0)
    psi = sv.ideal_state(c)
    n, bs = 6, [3, 3]
    starts = sampling.batch_starts(bs)
    calls = []

    def mfn(j, prefix):
        calls.append((j, prefix))
        return sampling.marginal_from_state(psi, n, starts[j], bs[j], prefix)

    shots, _ = sampling.sample_trajectory(mfn, 3, n, bs, 300, seed=9)
    # redo every shot independently, without memoisation
    for t in range(300):
        prefix = 0
        for j in range(2):
            u = sampling.shot_uniforms(9, 3, j, 300)[t]
            x = sampling.inverse_cdf(sampling.marginal_from_state(psi, n, starts[j], bs[j], prefix), u)
            prefix |= x << starts[j]
        assert prefix == shots[t]
    assert len(calls) == len(set(calls))        # each (batch, prefix) contracted once


# ------------------------------------------------------------------- Philox / PTS
def test_philox_uniform_chi_square_and_streams():
    t = np.arange(200000, dtype=np.uint64)
    u = philox.uniform(123, philox.TAG_SHOTS, t, 0, 0)
    assert u.min() >= 0 and u.max() < 1
    h = np.bincount((u * 100).astype(int), minlength=100)
    chi2 = ((h - 2000) ** 2 / 2000).sum()
    assert chi2 < 180        # 99 dof, p ~ 1e-6
    v = philox.uniform(123, philox.TAG_PTS, t, 0, 0)
    assert np.mean(u == v) < 1e-4
    w = philox.uniform(124, philox.TAG_SHOTS, t, 0, 0)
    assert np.mean(u == w) < 1e-4
    # counter words are not interchangeable
    x = philox.uniform(123, philox.TAG_SHOTS, 0, t, 0)
    assert np.mean(u == x) < 1e-4


def test_pts_properties():
    c = W.chain10_d8().circuit
    kr, mult, logq, nd = pts.presample(c, seed=1002, n_unique=64)
    assert kr.shape == (64, 72)
    assert len({r.tobytes() for r in kr}) == 64
    assert mult.sum() == nd and np.all(mult >= 1)
    q = upv.proposal(c.channels[0])
    for r, lq in zip(kr, logq):
        assert abs(lq - np.log(q[r]).sum()) < 1e-9
    # the error-free set is the most likely one (P ~ 0.485): present, largest multiplicity
    free = [i for i, r in enumerate(kr) if not r.any()]
    assert len(free) == 1 and mult[free[0]] == mult.max()
    assert abs(mult[free[0]] / nd - 0.99 ** 72) < 5 * math.sqrt(0.25 / nd)


def test_pts_site_frequencies():
    c = W.Circuit(1)
    g = c.add_gate((0,), np.eye(2))
    ch = c.add_channel(W.depolarizing(0.3))
    for _ in range(12):
        c.add_site(g, (0,), ch)
    kr, mult, _, nd = pts.presample(c, seed=5, n_unique=10 ** 6, max_draws=20000)
    assert nd == 20000 and mult.sum() == 20000
    counts = np.zeros(4)
    for r, m in zip(kr, mult):
        counts[r[0]] += m
    p = np.array([0.7, 0.1, 0.1, 0.1])
    sd = np.sqrt(20000 * p * (1 - p))
    assert np.all(np.abs(counts - 20000 * p) < 5 * sd)


def test_pts_stops_when_every_error_set_has_appeared():
    c = W.Circuit(1)
    g = c.add_gate((0,), np.eye(2))
    ch = c.add_channel(W.pauli_channel(W.pauli_x, 0.5))
    c.add_site(g, (0,), ch)
    c.add_site(g, (0,), ch)
    kr, mult, _, nd = pts.presample(c, seed=3, n_unique=10)
    assert len(kr) == 4 and mult.sum() == nd
    assert sorted(map(tuple, kr.tolist())) == [(0, 0), (0, 1), (1, 0), (1, 1)]


# ----------------------------------------------------------------- gradients
def _hea_case(noise, seed=0, n=4, layers=2, E=3):
    from oracle import gradients as gr
    rng = np.random.default_rng(seed)
    angles = rng.uniform(0, 2 * np.pi, size=2 * n * layers)
    c = W.hea(n, layers, angles, noise)
    gp, ga = W.rotation_spec(c)
    kr, mult, _, _ = pts.presample(c, seed + 10, E)
    w = mult / mult.sum()
    return gr, c, kr, w, angles, gp, ga, W.zz_chain_terms(n)


@pytest.mark.parametrize("noise", ["depol", "ad"])
def test_adjoint_gradient_equals_parameter_shift(noise):
    chans = [W.depolarizing(0.2)] if noise == "depol" else [W.depolarizing(0.1), W.amplitude_damping(0.3)]
    gr, c, kr, w, th, gp, ga, terms = _hea_case(chans)
    g = gr.adjoint_gradient(c, kr, w, th, gp, ga, terms)
    for k in range(len(th)):
        ps = gr.parameter_shift(c, kr, w, th, gp, ga, terms, k)
        assert abs(g[k] - ps) < 1e-10, (k, g[k], ps)


def test_adjoint_gradient_matches_central_difference():
    gr, c, kr, w, th, gp, ga, terms = _hea_case([W.depolarizing(0.2)], seed=3)
    g = gr.adjoint_gradient(c, kr, w, th, gp, ga, terms)
    # f is a + R cos(theta - theta0) in each angle with R <= ||O|| = 3: truncation <= h^2/6 R
    for k in range(0, len(th), 3):
        fd = gr.central_difference(c, kr, w, th, gp, ga, terms, k, h=1e-3)
        assert abs(fd - g[k]) < 1e-5


def test_gradient_value_matches_statevector_definition():
    gr, c, kr, w, th, gp, ga, terms = _hea_case([W.depolarizing(0.2)], seed=4)
    f = gr.value(c, kr, w, th, gp, ga, terms)
    psis = [sv.trajectory_state(c, row) for row in kr]      # gates built from the same angles
    o = gr.zz_diagonal(c.n_qubits, terms)
    ref = sum(wi * np.real(np.vdot(p, o * p)) for wi, p in zip(w, psis))
    assert abs(f - ref) < 1e-12


def test_diagonal_observable_gradient_matches_central_difference():
    """A general real diagonal observable with non-unitary Kraus (amplitude damping):
    the oracle's adjoint gradient against FP64 central differences of its value."""
    gr, c, kr, w, th, gp, ga, _ = _hea_case([W.depolarizing(0.1), W.amplitude_damping(0.2)], seed=5)
    o = np.random.default_rng(6).normal(size=2 ** c.n_qubits)
    g = gr.adjoint_gradient_obs(c, kr, w, th, gp, ga, o)
    h = 1e-5
    for k in range(len(th)):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (gr.value_obs(c, kr, w, tp, gp, ga, o) - gr.value_obs(c, kr, w, tm, gp, ga, o)) / (2 * h)
        assert abs(fd - g[k]) < 1e-8, (k, fd, g[k])


def test_gate_adjoint_matches_entrywise_finite_differences():
    """2 dL/d conj(U_g) of the oracle against central differences of L under a real
    (gives the real part) and an imaginary (the imaginary part) perturbation of
    single entries of a fixed two-qubit gate and of a rotation gate's matrix."""
    import copy
    gr, c, kr, w, th, gp, ga, terms = _hea_case([W.depolarizing(0.1), W.amplitude_damping(0.2)], seed=7)
    o = gr.zz_diagonal(c.n_qubits, terms)
    adj = gr.gate_adjoint(c, kr, w, th, gp, ga, o=o)
    fixed = [g for g in range(c.n_gates) if gp[g] < 0 and len(c.gate_qubits[g]) == 2][1]
    rot = [g for g in range(c.n_gates) if gp[g] >= 0][3]
    eps = 1e-6
    for g, entries in ((fixed, [(0, 0), (1, 3), (3, 2)]), (rot, [(0, 1), (1, 1)])):
        base = gr.rotation(ga[g], th[gp[g]]) if gp[g] >= 0 else c.gate_mats[g]
        for (a, b) in entries:
            for part in (1.0, 1j):
                vals = []
                for sgn in (1, -1):
                    cc = copy.deepcopy(c)
                    m = np.array(base, dtype=np.complex128)
                    m[a, b] += sgn * eps * part
                    cc.gate_mats[g] = m
                    gp2 = gp.copy()
                    gp2[g] = -1                  # the perturbed matrix replaces the rotation
                    vals.append(gr.value_obs(cc, kr, w, th, gp2, ga, o))
                fd = (vals[0] - vals[1]) / (2 * eps)
                pred = adj[g][a, b].real if part == 1.0 else adj[g][a, b].imag
                assert abs(fd - pred) < 1e-7, (g, a, b, part, fd, pred)


def test_seeded_gradient_of_a_linear_functional():
    """L = 2 Re sum_i <chi_i|psi_i> has psi-bar_i = chi_i: the oracle's seeded
    gradient against central differences of L."""
    gr, c, kr, w, th, gp, ga, _ = _hea_case([W.depolarizing(0.1)], seed=8)
    rng = np.random.default_rng(9)
    chis = [rng.normal(size=2 ** c.n_qubits) + 1j * rng.normal(size=2 ** c.n_qubits) for _ in kr]

    def L(t):
        tot = 0.0
        for row, chi in zip(kr, chis):
            psi = gr._forward_states(c, row, t, gp, ga)[3][-1]
            tot += 2.0 * np.real(np.vdot(chi, psi))
        return tot

    g = gr.seeded_gradient(c, kr, th, gp, ga, chis)
    h = 1e-5
    for k in range(0, len(th), 2):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        assert abs((L(tp) - L(tm)) / (2 * h) - g[k]) < 1e-7, k


def test_annihilated_trajectory_has_weight_zero_and_zero_shots():
    """Amplitude damping's K1 twice on a qubit with only a diagonal gate between
    maps every state to 0: Z = 0 exactly, the trajectory weight is 0, the
    all-zero marginal draws x = 0, and the exact enumeration identity still holds
    (the term contributes nothing).  K1 = [[0, sqrt(g)], [0, 0]], K1 K1 = 0."""
    g = 0.3
    c = W.Circuit(1)
    ad = c.add_channel(W.amplitude_damping(g))
    h = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2)
    g0 = c.add_gate((0,), h)
    c.add_site(g0, (0,), ad)
    g1 = c.add_gate((0,), np.diag([1, 1j]).astype(np.complex128))   # S: diagonal
    c.add_site(g1, (0,), ad)
    dead = np.array([1, 1], dtype=np.uint8)
    psi = sv.trajectory_state(c, dead)
    assert np.all(psi == 0)
    Z = np.array([np.vdot(sv.trajectory_state(c, np.array(k, dtype=np.uint8)),
                          sv.trajectory_state(c, np.array(k, dtype=np.uint8))).real
                  for k in ([0, 0], [0, 1], [1, 0], [1, 1])])
    assert Z[3] == 0.0 and np.all(Z[:3] > 0)
    w = sampling.trajectory_weights(Z, np.ones(4))
    assert w[3] == 0.0 and abs(w.sum() - 1) < 1e-15
    pi = sampling.marginal_from_state(psi, 1, 0, 1, 0)
    for u in (0.0, 0.5, 1 - 2 ** -53):
        assert sampling.inverse_cdf(pi, u) == 0
    shots, _ = sampling.sample_trajectory(lambda j, p: pi, 3, 1, [1], 5, 7)
    assert shots == [0] * 5
    # exact enumeration: sum_K q(K) |psi_K|^2 = diag rho (textbook channel application)
    q = {0: 1 - g / 2, 1: g / 2}
    diag = np.zeros(2)
    for k in itertools.product((0, 1), repeat=2):
        st = sv.trajectory_state(c, np.array(k, dtype=np.uint8))
        diag += q[k[0]] * q[k[1]] * np.abs(st) ** 2
    np.testing.assert_allclose(diag, sv.density_matrix_diag(c), atol=1e-14)


# ----------------------------------------------- non-proportional NBS, exhaustive final batch
def _sv_marginals(psi, n, bs):
    starts = sampling.batch_starts(bs)
    return lambda j, prefix: sampling.marginal_from_state(psi, n, starts[j], bs[j], prefix)


def test_nonproportional_ghz_closed_form():
    """GHZ on 4 qubits, batches [2, 2]: the first batch gives 00 or 11 with 1/2 each,
    and each fixes the last batch, so the exhaustive rows are (0000, 1, 1/2) and
    (1111, 1, 1/2); the strict threshold drops them at 1."""
    n = 4
    gates = [((0,), W.HADAMARD)] + [((q, q + 1), W.CNOT) for q in range(n - 1)]
    mfn = _sv_marginals(sv.ideal_state(_circuit(n, gates)), n, [2, 2])
    rows, counts = sampling.nonproportional_trajectory(mfn, 0, n, [2, 2], 64, 11, 0.5)
    assert counts == [1, 2]                      # both outcomes of 64 draws (miss probability 2^-63)
    assert [r[0] for r in rows] == [0b0000, 0b1111]
    for _, pc, pp in rows:
        assert abs(pc - 1) < 1e-14 and abs(pp - 0.5) < 1e-14
    rows1, _ = sampling.nonproportional_trajectory(mfn, 0, n, [2, 2], 1, 11, 0.5)
    assert len(rows1) == 1 and rows1[0][0] in (0b0000, 0b1111)
    assert sampling.nonproportional_trajectory(mfn, 0, n, [2, 2], 64, 11, 1.0)[0] == []


def test_nonproportional_rows_follow_the_chain_rule():
    """Every row's P(x | prefix) p(prefix) is the bitstring's probability |psi|^2 / Z
    (Sec. II-B chain rule), each reached prefix lists each of its bitstrings once at
    threshold -1, and every prefix whose conditionals at each level are >= 0.05 is
    reached by 200 draws (miss probability below 1e-4 per prefix)."""
    rng = np.random.default_rng(64)
    n, bs = 6, [2, 2, 2]
    psi = sv.ideal_state(W.random_brickwork(n, 4, rng, 0.0))
    p = np.abs(psi) ** 2 / np.vdot(psi, psi).real
    mfn = _sv_marginals(psi, n, bs)
    rows, counts = sampling.nonproportional_trajectory(mfn, 5, n, bs, 200, 12, -1.0)
    assert len(rows) == counts[-1] * 4
    bits = [r[0] for r in rows]
    assert len(set(bits)) == len(bits)
    for b, pc, pp in rows:
        assert abs(pc * pp - p[b]) < 1e-13, b
    reached = {b & 0xF for b in bits}
    assert counts == [1, len({b & 0x3 for b in bits}), len(reached)]
    p1 = np.array([p[[x for x in range(64) if x & 3 == a]].sum() for a in range(4)])
    p2 = np.array([p[[x for x in range(64) if x & 15 == a]].sum() for a in range(16)])
    for a in range(16):
        if p1[a & 3] >= 0.05 and p2[a] / p1[a & 3] >= 0.05:
            assert a in reached, a
    # thresholded rows are the subset with P(x | prefix) > threshold
    thr = 0.3
    rows_t, _ = sampling.nonproportional_trajectory(mfn, 5, n, bs, 200, 12, thr)
    assert rows_t == [r for r in rows if r[1] > thr]


def test_nonproportional_draws_follow_the_conditional():
    """One draw per prefix: over many trajectory ids (independent counters) the first
    batch's outcome follows the closed-form product-state marginal within the TVD
    bound, and every prefix has exactly one child."""
    n, bs = 4, [2, 2]
    th = [0.7, 2.1, 1.0, 0.4]
    psi = sv.ideal_state(_circuit(n, [((q,), W.ry(t)) for q, t in enumerate(th)]))
    pq = [np.sin(t / 2) ** 2 for t in th]
    want = np.array([(pq[0] if x & 1 else 1 - pq[0]) * (pq[1] if x & 2 else 1 - pq[1]) for x in range(4)])
    mfn = _sv_marginals(psi, n, bs)
    N = 4000
    hist = np.zeros(4)
    for t in range(N):
        rows, counts = sampling.nonproportional_trajectory(mfn, t, n, bs, 1, 21, -1.0)
        assert counts == [1, 1] and len(rows) == 4
        assert len({r[0] & 3 for r in rows}) == 1
        hist[rows[0][0] & 3] += 1
    assert sampling.nonproportional_trajectory(mfn, 0, n, bs, 1, 21, 2.0)[0] == []   # threshold above 1
    tvd = 0.5 * np.abs(hist / N - want).sum()
    assert tvd <= 0.5 * math.sqrt(4 / N) + math.sqrt(math.log(1e9) / (2 * N)), tvd


def test_nonproportional_children_bound_and_zero_weight():
    """A prefix has at most min(draws, 2^b) children; a trajectory of zero norm
    (amplitude damping's K1 twice) gives no rows."""
    rng = np.random.default_rng(65)
    n, bs = 6, [3, 2, 1]
    psi = sv.ideal_state(W.random_brickwork(n, 3, rng, 0.0))
    mfn = _sv_marginals(psi, n, bs)
    for k in (1, 3, 20):
        _, counts = sampling.nonproportional_trajectory(mfn, 2, n, bs, k, 13, 0.0)
        assert counts[1] <= min(k, 8) and counts[2] <= counts[1] * min(k, 4)
    zero = lambda j, prefix: np.zeros(2 ** bs[j])
    assert sampling.nonproportional_trajectory(zero, 0, n, bs, 4, 13, -1.0)[0] == []
    # direct final draws from a zero-weight trajectory: x = 0 rows with P = p(prefix) = 0
    rows, counts = sampling.nonproportional_trajectory(zero, 0, n, bs, 4, 13, 0.0, final_draws=3)
    assert counts == [1, 1, 1] and rows == [(0, 0.0, 0.0)] * 3


def test_nonproportional_direct_final_batch():
    """Direct final-batch sampling: GHZ rows repeat the prefix's forced completion with
    P = 1; on a random circuit every row obeys the chain rule; on a product state the
    final draws of one prefix follow the closed-form conditional within the TVD bound."""
    n = 4
    gates = [((0,), W.HADAMARD)] + [((q, q + 1), W.CNOT) for q in range(n - 1)]
    mfn = _sv_marginals(sv.ideal_state(_circuit(n, gates)), n, [2, 2])
    rows, counts = sampling.nonproportional_trajectory(mfn, 0, n, [2, 2], 64, 11, 0.0, final_draws=5)
    assert counts == [1, 2] and len(rows) == 10
    assert [r[0] for r in rows] == [0b0000] * 5 + [0b1111] * 5
    assert all(abs(pc - 1) < 1e-14 and abs(pp - 0.5) < 1e-14 for _, pc, pp in rows)
    rng = np.random.default_rng(66)
    n, bs = 6, [2, 2, 2]
    psi = sv.ideal_state(W.random_brickwork(n, 4, rng, 0.0))
    p = np.abs(psi) ** 2 / np.vdot(psi, psi).real
    rows, counts = sampling.nonproportional_trajectory(_sv_marginals(psi, n, bs), 1, n, bs, 3, 14, 0.0,
                                                       final_draws=7)
    assert len(rows) == 7 * counts[-1]
    for b, pc, pp in rows:
        assert abs(pc * pp - p[b]) < 1e-13 and pc > 0
    th = [0.9, 1.7, 2.4]
    psi = sv.ideal_state(_circuit(3, [((q,), W.ry(t)) for q, t in enumerate(th)]))
    pq = [np.sin(t / 2) ** 2 for t in th]
    want = np.array([(pq[1] if x & 1 else 1 - pq[1]) * (pq[2] if x & 2 else 1 - pq[2]) for x in range(4)])
    N = 4000
    rows, counts = sampling.nonproportional_trajectory(_sv_marginals(psi, 3, [1, 2]), 0, 3, [1, 2], 1, 15, 0.0,
                                                       final_draws=N)
    assert counts == [1, 1]
    hist = np.bincount([r[0] >> 1 for r in rows], minlength=4) / N
    assert 0.5 * np.abs(hist - want).sum() <= 0.5 * math.sqrt(4 / N) + math.sqrt(math.log(1e9) / (2 * N))


# ----------------------------------------------------------------- light cone
def _brickwork_cone_count(n, depth, e):
    """Kept gates of a brickwork chain (layer t pairs (q, q+1), q = t mod 2) for
    measured qubits [0, e), by the light-speed argument: going back one layer,
    the live prefix [0, r) grows by one qubit exactly when that layer has a gate
    on the pair (r-1, r); every gate of the layer with q < r touches it."""
    r, kept = e, 0
    for t in reversed(range(depth)):
        kept += sum(1 for q in range(t % 2, n - 1, 2) if q < r)
        if r < n and (r - 1) % 2 == t % 2:
            r += 1
    return kept


def test_light_cone_brickwork_count_closed_form():
    """Forward reachability over the dependency graph agrees with the geometric
    light cone of a brickwork chain (Pauli noise: every gate unitary)."""
    from oracle import lightcone
    rng = np.random.default_rng(3)
    for n, depth in [(12, 4), (16, 6), (13, 5)]:
        c = W.random_brickwork(n, depth, rng, 0.05)
        for e in range(1, n + 1):
            keep = lightcone.kept_gates(c, e)
            assert int(keep.sum()) == _brickwork_cone_count(n, depth, e), (n, depth, e)
            assert all(keep[g] for g in range(c.n_gates) if min(c.gate_qubits[g]) < e)


def test_light_cone_doubled_network_equals_full_for_unitary_trajectories():
    """Pauli channels: the pruned doubled network gives the full network's
    marginal for every prefix of several batches, whatever the Kraus choices."""
    rng = np.random.default_rng(5)
    n = 9
    c = W.random_brickwork(n, 5, rng, 0.3)
    c2 = W.small_random_circuit(n, 30, rng, [W.depolarizing(0.3)], two_qubit_frac=0.6)
    for circ in (c, c2):
        S = len(circ.site_gate)
        for trial in range(3):
            kr = rng.integers(0, 4, size=S).astype(np.uint8)
            for start, b in [(0, 3), (3, 2), (5, 2)]:
                for prefix in range(0, 1 << start, max(1, (1 << start) // 3)):
                    full = tn.batch_network_value(circ, kr, start, b, prefix, "doubled")
                    cut = tn.batch_network_value(circ, kr, start, b, prefix, "doubled", light_cone=True)
                    np.testing.assert_allclose(cut, full, rtol=0, atol=1e-12)


def test_light_cone_keeps_non_unitary_gates_and_their_past():
    """Amplitude damping on gates outside the measured qubits' light cone: keeping
    those gates and their past reproduces the full network; the plain light cone
    (a plausible mistake) does not."""
    from oracle import lightcone
    rng = np.random.default_rng(9)
    n = 8
    c = W.Circuit(n)
    dep = c.add_channel(W.depolarizing(0.2))
    ad = c.add_channel(W.amplitude_damping(0.6))
    for layer in W.brickwork_1d(n, 4):
        for (a, b2) in layer:
            g = c.add_gate((a, b2), W.haar_su4(rng))
            c.add_site(g, (a,), dep)
            if a >= 5:
                c.add_site(g, (b2,), ad)
    S = len(c.site_gate)
    start, b = 0, 2
    plain = lightcone.kept_gates(c, start + b, respect_non_unitary=False)
    full_keep = lightcone.kept_gates(c, start + b)
    assert full_keep.sum() > plain.sum()
    worst_plain = 0.0
    for trial in range(4):
        kr = np.zeros(S, dtype=np.uint8)
        for s in range(S):
            ch = c.site_channel[s]
            kr[s] = rng.integers(0, 4) if ch == dep else 1     # the decay operator everywhere
        full = tn.batch_network_value(c, kr, start, b, 0, "doubled")
        cut = tn.batch_network_value(c, kr, start, b, 0, "doubled", light_cone=True)
        np.testing.assert_allclose(cut, full, rtol=0, atol=1e-12)
        wrong = tn.batch_network_value(c, kr, start, b, 0, "doubled", keep=plain)
        worst_plain = max(worst_plain, float(np.abs(wrong - full).max()))
    assert worst_plain > 1e-3
