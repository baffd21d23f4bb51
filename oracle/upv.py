"""Noise proposal, inserted operators and the unified-path-variation merge.

Sec. II-C: error sets are pre-sampled by a user rule, "proportional with error
probabilities" being the example.  Reading used here: the proposal for Kraus
operator k of a channel is its given probability, else tr(K_k^dag K_k)/d (a
distribution because sum_k K_k^dag K_k = I).  The operator inserted into a
trajectory is K_k / sqrt(q_k): a unitary Pauli for mixed-unitary channels (norm
stays 1), and a rescaled Kraus operator otherwise, whose squared state norm is
then the trajectory's importance ratio.

Sec. III-A (UPV): each sampled operator is merged into the gate it follows, so
the merged tensor has the gate's shape and every trajectory's network has the
same structure:  d'_l = (product of the inserted operators of l's sites, later
sites on the left) . d_l, a one-qubit operator on a two-qubit gate being padded
with the identity on the other qubit.
"""
import numpy as np


def proposal(channel) -> np.ndarray:
    if channel.probs is not None:
        return np.asarray(channel.probs, dtype=np.float64)
    d = channel.kraus.shape[1]
    return np.array([np.trace(k.conj().T @ k).real / d for k in channel.kraus])


def inserted_operator(channel, k: int) -> np.ndarray:
    q = proposal(channel)[k]
    return channel.kraus[k] / np.sqrt(q)


def embed(op: np.ndarray, op_qubits, gate_qubits) -> np.ndarray:
    """Matrix of `op` (acting on op_qubits) on the space of gate_qubits, index
    convention: first listed qubit is the high bit.  Written as explicit loops
    over basis states."""
    G = list(gate_qubits)
    S = list(op_qubits)
    nG = len(G)
    out = np.zeros((2 ** nG, 2 ** nG), dtype=np.complex128)

    def bits(x, qs):
        return {q: (x >> (len(qs) - 1 - i)) & 1 for i, q in enumerate(qs)}

    for gx in range(2 ** nG):
        bx = bits(gx, G)
        for gy in range(2 ** nG):
            by = bits(gy, G)
            if any(bx[q] != by[q] for q in G if q not in S):
                continue
            sx = sum(bx[q] << (len(S) - 1 - i) for i, q in enumerate(S))
            sy = sum(by[q] << (len(S) - 1 - i) for i, q in enumerate(S))
            out[gx, gy] = op[sx, sy]
    return out


def sites_of_gate(circuit):
    per = [[] for _ in range(circuit.n_gates)]
    for s, g in enumerate(circuit.site_gate):
        per[g].append(s)
    return per


def merged_gate(circuit, g: int, kraus_row) -> np.ndarray:
    """d'_l for gate g given the trajectory's Kraus index per site (Sec. III-A)."""
    m = circuit.gate_mats[g].copy()
    for s, gg in enumerate(circuit.site_gate):
        if gg != g:
            continue
        ch = circuit.channels[circuit.site_channel[s]]
        op = inserted_operator(ch, int(kraus_row[s]))
        m = embed(op, circuit.site_qubits[s], circuit.gate_qubits[g]) @ m
    return m


def merged_gates(circuit, kraus_row):
    return [merged_gate(circuit, g, kraus_row) for g in range(circuit.n_gates)]
