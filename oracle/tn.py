"""Explicit tensor networks for one batch of the batch-wise sampler, contracted
pairwise with numpy einsum in FP64.

Network for trajectory i, batch [start, start+b) and prefix p (Sec. II-B with the
UPV-merged gates of Sec. III-A):

* ket network: |0> vector per qubit, then every (merged) gate as a tensor
  G[o0, o1, i0, i1] = M[2 o0 + o1, 2 i0 + i1];
* ``kind="doubled"`` (batches before the last): the ket network, its complex
  conjugate (bra) with its own wire labels, <s_q| on both output legs of every
  prefix qubit, ket and bra outputs of a batch qubit sharing one open label
  (diagonal), ket and bra outputs of a later qubit sharing one summed label
  (trace).  Result: pi_p(x) over the batch qubits.
* ``kind="ket"`` (the last batch): the ket network with <s_q| on the prefix
  outputs; result: amplitudes over the batch qubits.

The contraction order is the oracle's own sweep: tensors sorted by the highest
qubit they touch (ascending for ``order="ltr"``, descending for ``"rtl"``), then
by time, ket before bra; ``"inward"`` (default) sweeps the columns before the
batch and the columns after it separately and then absorbs the batch columns
between the two partial results.  ``light_cone=True`` (doubled networks only)
keeps only the gates of ``lightcone.kept_gates``: the others cancel against their
conjugate copies under the trace when they are unitary for every trajectory
(Sec. VI names light-cone simplification under UPV as open).
"""
import string

import numpy as np

from .lightcone import kept_gates
from .upv import embed, inserted_operator, merged_gates, sites_of_gate

LETTERS = string.ascii_letters


class _Net:
    def __init__(self):
        self.tensors = []      # (array, [labels], sort_key)
        self.next_label = 0

    def label(self):
        self.next_label += 1
        return self.next_label - 1

    def add(self, arr, labels, key):
        assert arr.ndim == len(labels)
        self.tensors.append((np.asarray(arr, dtype=np.complex128), list(labels), key))


def _ket_layer(net, n, ops, conj=False, key_shift=0):
    """Adds |0> vectors and the given operator list [(matrix, qubits)] in order.
    Returns the output label per qubit."""
    wire = []
    for q in range(n):
        L = net.label()
        net.add(np.array([1.0, 0.0]), [L], (q, -1, key_shift))
        wire.append(L)
    for t, (m, qs) in enumerate(ops):
        k = len(qs)
        arr = m.reshape([2] * (2 * k))
        if conj:
            arr = arr.conj()
        outs = [net.label() for _ in qs]
        ins = [wire[q] for q in qs]
        net.add(arr, outs + ins, (max(qs), t, key_shift))
        for q, L in zip(qs, outs):
            wire[q] = L
    return wire


def _absorb(items, remaining, out_set, cur=None, cur_labs=None):
    """Absorb tensors one at a time into a running tensor; a label is summed as
    soon as no unabsorbed tensor and not the output refers to it."""
    if cur is None:
        cur, cur_labs = np.array(1.0 + 0j), []
    for arr, labs in items:
        for L in labs:
            remaining[L] -= 1
        keep = []
        for L in cur_labs + labs:
            if L in keep:
                continue
            if L in out_set or remaining.get(L, 0) > 0:
                keep.append(L)
        uniq = sorted(set(cur_labs + labs + keep))
        m = {L: LETTERS[i] for i, L in enumerate(uniq)}
        spec = "".join(m[L] for L in cur_labs) + "," + "".join(m[L] for L in labs) + "->" + "".join(m[L] for L in keep)
        cur = np.einsum(spec, cur, arr)
        cur_labs = keep
    return cur, cur_labs


def _contract(net, out_labels, order="ltr", lo=0, hi=0):
    """order 'ltr' / 'rtl' / 'time': one running tensor in that sweep order.
    order 'inward': the columns below `lo` (left to right) and from `hi` up
    (right to left) are each contracted to one tensor first, then the columns in
    [lo, hi) are absorbed left to right between them."""
    ts = list(net.tensors)
    remaining = {}
    for _, labs, _ in ts:
        for L in labs:
            remaining[L] = remaining.get(L, 0) + 1
    out_set = set(out_labels)
    if order == "inward":
        left = sorted([t for t in ts if t[2][0] < lo], key=lambda x: (x[2][0], x[2][1], x[2][2]))
        right = sorted([t for t in ts if t[2][0] >= hi], key=lambda x: (-x[2][0], x[2][1], x[2][2]))
        mid = sorted([t for t in ts if lo <= t[2][0] < hi], key=lambda x: (x[2][0], x[2][1], x[2][2]))
        ta = _absorb([(a, l) for a, l, _ in left], remaining, out_set)
        tc = _absorb([(a, l) for a, l, _ in right], remaining, out_set)
        # the two partial results are absorbed like ordinary tensors
        for L in tc[1]:
            remaining[L] = remaining.get(L, 0) + 1
        cur, cur_labs = _absorb([(a, l) for a, l, _ in mid] + [tc], remaining, out_set, ta[0], ta[1])
    else:
        if order == "ltr":
            ts.sort(key=lambda x: (x[2][0], x[2][1], x[2][2]))
        elif order == "rtl":
            ts.sort(key=lambda x: (-x[2][0], x[2][1], x[2][2]))
        elif order == "time":
            ts.sort(key=lambda x: (x[2][1], x[2][0], x[2][2]))
        else:
            raise ValueError(order)
        cur, cur_labs = _absorb([(a, l) for a, l, _ in ts], remaining, out_set)
    m = {L: LETTERS[i] for i, L in enumerate(sorted(set(cur_labs)))}
    spec = "".join(m[L] for L in cur_labs) + "->" + "".join(m[L] for L in out_labels)
    return np.einsum(spec, cur)


def _ops_merged(circuit, kraus_row):
    return [(m, circuit.gate_qubits[g]) for g, m in enumerate(merged_gates(circuit, kraus_row))]


def _ops_explicit(circuit, kraus_row):
    """Traditional insertion: the gate, then each inserted operator as its own tensor."""
    ops = []
    per = sites_of_gate(circuit)
    for g in range(circuit.n_gates):
        ops.append((circuit.gate_mats[g], circuit.gate_qubits[g]))
        for s in per[g]:
            ch = circuit.channels[circuit.site_channel[s]]
            ops.append((inserted_operator(ch, int(kraus_row[s])), circuit.site_qubits[s]))
    return ops


def batch_network_value(circuit, kraus_row, start: int, b: int, prefix: int, kind: str,
                        order: str = "inward", explicit: bool = False, light_cone: bool = False,
                        keep=None) -> np.ndarray:
    """pi_p(x) (kind 'doubled') or amplitudes (kind 'ket') over the batch qubits,
    index x = sum_k x_{start+k} 2^k.  light_cone: drop the gates outside
    ``lightcone.kept_gates(circuit, start + b)`` from a doubled network (``keep``:
    a caller's own gate mask instead)."""
    n = circuit.n_qubits
    ops = _ops_explicit(circuit, kraus_row) if explicit else _ops_merged(circuit, kraus_row)
    if (light_cone or keep is not None) and kind == "doubled":
        assert not explicit, "the light cone selects merged gates"
        mask = keep if keep is not None else kept_gates(circuit, start + b)
        ops = [op for g, op in enumerate(ops) if mask[g]]
    net = _Net()
    ket_out = _ket_layer(net, n, ops, conj=False, key_shift=0)
    batch = list(range(start, start + b))
    if kind == "ket":
        assert start + b == n, "the ket-only network is used for the last batch"
        for q in range(start):
            s = (prefix >> q) & 1
            net.add(np.array([1.0 - s, float(s)]), [ket_out[q]], (q, 10 ** 9, 0))
        out = [ket_out[q] for q in reversed(batch)]
        return _contract(net, out, order, start, start + b).reshape(-1)
    assert kind == "doubled"
    sub = _Net()
    sub.next_label = net.next_label
    bra_out = _ket_layer(sub, n, ops, conj=True, key_shift=1)
    # relabel the bra outputs of batch and later qubits to the ket output labels
    ren = {}
    for q in range(start, n):
        ren[bra_out[q]] = ket_out[q]
    for arr, labs, key in sub.tensors:
        net.add(arr, [ren.get(L, L) for L in labs], key)
    net.next_label = sub.next_label
    for q in range(start):
        s = (prefix >> q) & 1
        v = np.array([1.0 - s, float(s)])
        net.add(v, [ket_out[q]], (q, 10 ** 9, 0))
        net.add(v, [bra_out[q]], (q, 10 ** 9, 1))
    out = [ket_out[q] for q in reversed(batch)]
    return np.real(_contract(net, out, order, start, start + b)).reshape(-1)
