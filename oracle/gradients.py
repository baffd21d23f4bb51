"""FP64 gradients of a trajectory-averaged observable (test infrastructure).

    f(theta) = sum_i W_i <psi_i(theta)| O |psi_i(theta)>,   O = sum_t c_t Z_a Z_b,

with the error sets fixed (pre-sampled once) and psi_i built from the UPV-merged
gates (Sec. III-A) of a circuit whose rotation gates are exp(-i theta P / 2).

* ``value``            - f by dense statevectors.
* ``adjoint_gradient`` - reverse-mode gradient of f: with A_k the k-th merged gate,
  psi_k = A_k ... A_1 |0>, lambda_N = O psi_N and lambda_{k-1} = A_k^dag lambda_k,
  df/dtheta = sum_i W_i 2 Re <lambda_k | (dA_k/dtheta) psi_{k-1}> summed over the
  gates k that use theta (adjoint differentiation, Jones & Gacon, arXiv:2009.02823).
  The states psi_{k-1} are kept from the forward pass, so non-unitary A_k are fine.
* ``parameter_shift`` - exact for rotations: df/dtheta = [f(theta + pi/2) - f(theta - pi/2)] / 2
  for a parameter used by one gate.
* ``central_difference`` - [f(theta + h) - f(theta - h)] / (2 h).

The same quantities for a general real diagonal observable (``*_obs``, diagonal
``o`` over the 2^n basis states), for a caller's seed psi-bar_i = dL/d conj(psi_i)
(``seeded_gradient``: dL/dtheta = 2 Re sum_i <lambda_k|(dA_k/dtheta) psi_{k-1}>
with lambda_N = psi-bar_i), and the gate-tensor adjoints (``gate_adjoint``):
2 dL/d conj(U_g) = 2 sum_i (S_g^dag lambda_g) psi_{g-1}^dag reduced over the
qubits the gate does not touch, S_g the product of g's inserted operators (the
derivative of L = Re-linear functional of U_g's entries, torch's convention).
"""
import numpy as np

from .statevector import apply_gate, zero_state
from .upv import embed, inserted_operator

PAULI = [np.array([[0, 1], [1, 0]], dtype=np.complex128),
         np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
         np.array([[1, 0], [0, -1]], dtype=np.complex128)]


def rotation(axis: int, theta: float) -> np.ndarray:
    return np.cos(theta / 2) * np.eye(2) - 1j * np.sin(theta / 2) * PAULI[axis]


def rotation_derivative(axis: int, theta: float) -> np.ndarray:
    return -0.5 * np.sin(theta / 2) * np.eye(2) - 0.5j * np.cos(theta / 2) * PAULI[axis]


def _site_product(circuit, g, kraus_row):
    """Product of g's inserted operators (later sites on the left), gate space."""
    d = 2 ** len(circuit.gate_qubits[g])
    m = np.eye(d, dtype=np.complex128)
    for s, gg in enumerate(circuit.site_gate):
        if gg != g:
            continue
        ch = circuit.channels[circuit.site_channel[s]]
        m = embed(inserted_operator(ch, int(kraus_row[s])), circuit.site_qubits[s], circuit.gate_qubits[g]) @ m
    return m


def _gate_matrix(circuit, g, theta, gate_param, gate_axis):
    if gate_param[g] >= 0:
        return rotation(gate_axis[g], theta[gate_param[g]])
    return circuit.gate_mats[g]


def zz_diagonal(n, terms):
    x = np.arange(2 ** n)
    o = np.zeros(2 ** n)
    for (a, b), cf in terms:
        za = 1 - 2 * ((x >> a) & 1)
        zb = 1 - 2 * ((x >> b) & 1)
        o += cf * za * zb
    return o


def trajectory_values(circuit, kraus, theta, gate_param, gate_axis, terms):
    n = circuit.n_qubits
    o = zz_diagonal(n, terms)
    vals = []
    for row in kraus:
        psi = zero_state(n)
        for g in range(circuit.n_gates):
            A = _site_product(circuit, g, row) @ _gate_matrix(circuit, g, theta, gate_param, gate_axis)
            psi = apply_gate(psi, n, A, circuit.gate_qubits[g])
        vals.append(float(np.real(np.vdot(psi, o * psi))))
    return np.array(vals)


def value(circuit, kraus, weights, theta, gate_param, gate_axis, terms):
    return float(np.dot(weights, trajectory_values(circuit, kraus, theta, gate_param, gate_axis, terms)))


def adjoint_gradient(circuit, kraus, weights, theta, gate_param, gate_axis, terms):
    n = circuit.n_qubits
    o = zz_diagonal(n, terms)
    grad = np.zeros(len(theta))
    G = circuit.n_gates
    for w, row in zip(weights, kraus):
        K = [_site_product(circuit, g, row) for g in range(G)]
        A = [K[g] @ _gate_matrix(circuit, g, theta, gate_param, gate_axis) for g in range(G)]
        states = [zero_state(n)]
        for g in range(G):
            states.append(apply_gate(states[-1], n, A[g], circuit.gate_qubits[g]))
        lam = o * states[-1]
        for g in range(G - 1, -1, -1):
            if gate_param[g] >= 0:
                dA = K[g] @ rotation_derivative(gate_axis[g], theta[gate_param[g]])
                mu = apply_gate(states[g], n, dA, circuit.gate_qubits[g])
                grad[gate_param[g]] += w * 2.0 * np.real(np.vdot(lam, mu))
            lam = apply_gate(lam, n, A[g].conj().T, circuit.gate_qubits[g])
    return grad


def parameter_shift(circuit, kraus, weights, theta, gate_param, gate_axis, terms, k):
    tp = np.array(theta, dtype=np.float64).copy()
    tm = tp.copy()
    tp[k] += np.pi / 2
    tm[k] -= np.pi / 2
    return 0.5 * (value(circuit, kraus, weights, tp, gate_param, gate_axis, terms) -
                  value(circuit, kraus, weights, tm, gate_param, gate_axis, terms))


def central_difference(circuit, kraus, weights, theta, gate_param, gate_axis, terms, k, h=1e-3):
    tp = np.array(theta, dtype=np.float64).copy()
    tm = tp.copy()
    tp[k] += h
    tm[k] -= h
    return (value(circuit, kraus, weights, tp, gate_param, gate_axis, terms) -
            value(circuit, kraus, weights, tm, gate_param, gate_axis, terms)) / (2 * h)


def _forward_states(circuit, row, theta, gate_param, gate_axis):
    n = circuit.n_qubits
    G = circuit.n_gates
    K = [_site_product(circuit, g, row) for g in range(G)]
    U = [_gate_matrix(circuit, g, theta, gate_param, gate_axis) for g in range(G)]
    A = [K[g] @ U[g] for g in range(G)]
    states = [zero_state(n)]
    for g in range(G):
        states.append(apply_gate(states[-1], n, A[g], circuit.gate_qubits[g]))
    return K, U, A, states


def trajectory_values_obs(circuit, kraus, theta, gate_param, gate_axis, o):
    vals = []
    for row in kraus:
        psi = _forward_states(circuit, row, theta, gate_param, gate_axis)[3][-1]
        vals.append(float(np.real(np.vdot(psi, o * psi))))
    return np.array(vals)


def value_obs(circuit, kraus, weights, theta, gate_param, gate_axis, o):
    return float(np.dot(weights, trajectory_values_obs(circuit, kraus, theta, gate_param, gate_axis, o)))


def _reduce_outer(lam, psi, n, qubits):
    """sum over the other qubits of lam[., rest] conj(psi[., rest]) in the gate's
    index order (first listed qubit = high bit)."""
    t_l = lam.reshape([2] * n)
    t_p = psi.reshape([2] * n)
    axes = [n - 1 - q for q in qubits]
    other = [a for a in range(n) if a not in axes]
    l = np.transpose(t_l, axes + other).reshape(2 ** len(qubits), -1)
    p = np.transpose(t_p, axes + other).reshape(2 ** len(qubits), -1)
    return l @ p.conj().T


def _backward(circuit, row, theta, gate_param, gate_axis, lam, want_adj):
    """Reverse pass from lambda_N = lam: angle-gradient contributions and
    (want_adj) 2 (S^dag lambda_g) psi_{g-1}^dag per gate."""
    n = circuit.n_qubits
    K, U, A, states = _forward_states(circuit, row, theta, gate_param, gate_axis)
    grad = np.zeros(max([p for p in gate_param] + [-1]) + 1)
    adj = [None] * circuit.n_gates
    for g in range(circuit.n_gates - 1, -1, -1):
        qs = circuit.gate_qubits[g]
        if gate_param[g] >= 0:
            dA = K[g] @ rotation_derivative(gate_axis[g], theta[gate_param[g]])
            mu = apply_gate(states[g], n, dA, qs)
            grad[gate_param[g]] += 2.0 * np.real(np.vdot(lam, mu))
        if want_adj:
            adj[g] = 2.0 * K[g].conj().T @ _reduce_outer(lam, states[g], n, qs)
        lam = apply_gate(lam, n, A[g].conj().T, qs)
    return grad, adj


def adjoint_gradient_obs(circuit, kraus, weights, theta, gate_param, gate_axis, o):
    n_par = max([p for p in gate_param] + [-1]) + 1
    grad = np.zeros(n_par)
    for w, row in zip(weights, kraus):
        psi = _forward_states(circuit, row, theta, gate_param, gate_axis)[3][-1]
        grad += _backward(circuit, row, theta, gate_param, gate_axis, w * o * psi, False)[0]
    return grad


def seeded_gradient(circuit, kraus, theta, gate_param, gate_axis, psi_bars):
    n_par = max([p for p in gate_param] + [-1]) + 1
    grad = np.zeros(n_par)
    for row, pb in zip(kraus, psi_bars):
        grad += _backward(circuit, row, theta, gate_param, gate_axis, np.asarray(pb, dtype=np.complex128), False)[0]
    return grad


def gate_adjoint(circuit, kraus, weights, theta, gate_param, gate_axis, o=None, psi_bars=None):
    """[n_gates] list of d x d complex arrays: 2 dL/d conj(U_g) summed over the
    trajectories, for L = sum_i w_i <psi_i|O|psi_i> (o) or the seeds psi_bars."""
    total = None
    for i, row in enumerate(kraus):
        if psi_bars is None:
            psi = _forward_states(circuit, row, theta, gate_param, gate_axis)[3][-1]
            lam = weights[i] * o * psi
        else:
            lam = np.asarray(psi_bars[i], dtype=np.complex128)
        adj = _backward(circuit, row, theta, gate_param, gate_axis, lam, True)[1]
        total = adj if total is None else [a + b for a, b in zip(total, adj)]
    return total
