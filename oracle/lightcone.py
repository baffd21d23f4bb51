"""Light-cone selection of the gates of a doubled (ket x bra) batch network.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. VI names light-cone simplification as something the unified path of UPV
does not yet allow.  The fact it rests on: in the doubled network of batch j,
rho = U rho0 U^dag with the qubits after the batch traced, a gate that no
measured output and no kept gate depends on meets its own conjugate copy under
the trace and contributes G^dag G.  For a trajectory the gate is the UPV-merged
one (Sec. III-A), the bare gate times the inserted operators K / sqrt(q) of its
sites; G^dag G = I for every trajectory exactly when the bare gate and every
operator its sites' channels can insert are unitary.  A gate that is not unitary
for some trajectory stays, and with it every gate it depends on.

``kept_gates`` therefore keeps a gate when, moving forward in time through gates
that share a qubit, it reaches a gate on a measured qubit or a non-unitary gate
(forward search from each gate over the gate dependency graph).  The set depends
on the channel types only, never on a trajectory's Kraus choices, which is what
lets one contraction path keep serving every error set.
"""
import numpy as np

from .upv import inserted_operator, sites_of_gate

UNITARY_TOL = 1e-6


def is_unitary(m, tol=UNITARY_TOL) -> bool:
    m = np.asarray(m, dtype=np.complex128)
    return bool(np.abs(m.conj().T @ m - np.eye(m.shape[0])).max() <= tol)


def gate_always_unitary(circuit, g: int, per_gate_sites=None) -> bool:
    """The merged gate g is unitary for every Kraus choice of its sites."""
    per = per_gate_sites if per_gate_sites is not None else sites_of_gate(circuit)
    if not is_unitary(circuit.gate_mats[g]):
        return False
    for s in per[g]:
        ch = circuit.channels[circuit.site_channel[s]]
        q = ch.probs if ch.probs is not None else None
        for k in range(len(ch.kraus)):
            if q is not None and not q[k] > 0:
                continue
            if not is_unitary(inserted_operator(ch, k)):
                return False
    return True


def successors(circuit):
    """For each gate, the next gate on each of its qubits (the dependency graph)."""
    nxt = [set() for _ in range(circuit.n_gates)]
    last = {}
    for g in range(circuit.n_gates):
        for q in circuit.gate_qubits[g]:
            if q in last:
                nxt[last[q]].add(g)
            last[q] = g
    return nxt


def kept_gates(circuit, e: int, respect_non_unitary: bool = True) -> np.ndarray:
    """Boolean mask over gates: the gates of the doubled network that measures
    qubits [0, e) (prefix and batch).  ``respect_non_unitary=False`` keeps only the
    measured qubits' past light cone, which is exact only when every gate is
    unitary for every trajectory."""
    per = sites_of_gate(circuit)
    source = []
    for g in range(circuit.n_gates):
        on_measured = any(q < e for q in circuit.gate_qubits[g])
        source.append(on_measured or (respect_non_unitary and not gate_always_unitary(circuit, g, per)))
    nxt = successors(circuit)
    keep = np.zeros(circuit.n_gates, dtype=bool)
    for g in range(circuit.n_gates):
        seen, stack = {g}, [g]
        while stack:
            h = stack.pop()
            if source[h]:
                keep[g] = True
                break
            for s in nxt[h]:
                if s not in seen:
                    seen.add(s)
                    stack.append(s)
    return keep
