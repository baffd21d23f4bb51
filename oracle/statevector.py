"""Dense FP64 statevector of one trajectory (the definition the method reaches).

Index convention: amplitude index = sum_q x_q 2^q (qubit 0 is the lowest bit).
A two-qubit gate on (q0, q1) has matrix index 2*x[q0] + x[q1].

* ``trajectory_state``  - |psi~_i> = prod_l d'_l(i) |0^n> with UPV-merged gates
  (Sec. III-A); its squared norm is the trajectory's importance ratio.
* ``trajectory_state_explicit`` - the same trajectory with each inserted
  operator applied as its own operation after the gate (the traditional
  error-insertion network of Fig. 2b); used to pin the merge.
* ``density_matrix_diag`` - textbook density-matrix evolution rho -> sum_k K rho
  K^dag after every gate's sites (tiny n only); the exact quantity that the
  trajectory average estimates (Sec. II-B).
"""
import itertools

import numpy as np

from .upv import embed, inserted_operator, merged_gates, proposal, sites_of_gate


def apply_gate(psi: np.ndarray, n: int, mat: np.ndarray, qubits) -> np.ndarray:
    t = psi.reshape([2] * n)                      # axis a <-> qubit n-1-a
    axes = [n - 1 - q for q in qubits]
    k = len(qubits)
    g = mat.reshape([2] * (2 * k))                # (out..., in...)
    t = np.tensordot(g, t, axes=(list(range(k, 2 * k)), axes))
    # tensordot puts the gate's output axes first; move them back
    t = np.moveaxis(t, list(range(k)), axes)
    return t.reshape(-1)


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def trajectory_state(circuit, kraus_row) -> np.ndarray:
    n = circuit.n_qubits
    psi = zero_state(n)
    for g, m in enumerate(merged_gates(circuit, kraus_row)):
        psi = apply_gate(psi, n, m, circuit.gate_qubits[g])
    return psi


def trajectory_state_explicit(circuit, kraus_row) -> np.ndarray:
    n = circuit.n_qubits
    psi = zero_state(n)
    per = sites_of_gate(circuit)
    for g in range(circuit.n_gates):
        psi = apply_gate(psi, n, circuit.gate_mats[g], circuit.gate_qubits[g])
        for s in per[g]:
            ch = circuit.channels[circuit.site_channel[s]]
            psi = apply_gate(psi, n, inserted_operator(ch, int(kraus_row[s])), circuit.site_qubits[s])
    return psi


def ideal_state(circuit) -> np.ndarray:
    n = circuit.n_qubits
    psi = zero_state(n)
    for g in range(circuit.n_gates):
        psi = apply_gate(psi, n, circuit.gate_mats[g], circuit.gate_qubits[g])
    return psi


def _apply_left_right(rho, n, mat, qubits):
    """rho -> M rho M^dag for a 2^n x 2^n density matrix."""
    cols = np.stack([apply_gate(rho[:, c], n, mat, qubits) for c in range(rho.shape[1])], axis=1)
    rows = np.stack([apply_gate(cols[r, :].conj(), n, mat, qubits).conj() for r in range(rho.shape[0])], axis=0)
    return rows


def density_matrix_diag(circuit) -> np.ndarray:
    """Textbook noisy evolution: after gate l, each of its sites applies
    rho -> sum_k K_k rho K_k^dag with the channel's own Kraus operators."""
    n = circuit.n_qubits
    rho = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    rho[0, 0] = 1.0
    per = sites_of_gate(circuit)
    for g in range(circuit.n_gates):
        rho = _apply_left_right(rho, n, circuit.gate_mats[g], circuit.gate_qubits[g])
        for s in per[g]:
            ch = circuit.channels[circuit.site_channel[s]]
            rho = sum(_apply_left_right(rho, n, K, circuit.site_qubits[s]) for K in ch.kraus)
    return np.real(np.diag(rho)).copy()


def enumerate_trajectories(circuit):
    """Every Kraus sequence K with its proposal probability q(K) (tiny circuits)."""
    qs = [proposal(circuit.channels[c]) for c in circuit.site_channel]
    for row in itertools.product(*[range(len(q)) for q in qs]):
        qk = float(np.prod([qs[p][k] for p, k in enumerate(row)]))
        yield np.array(row, dtype=np.uint8), qk
