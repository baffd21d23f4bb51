"""Seeded synthetic inputs for PTSBE: circuits, noise channels and workloads.

This module only *generates inputs*.  It holds none of the method's arithmetic
(no contraction, no trajectory sampling, no marginals, no shot sampling), so both
the FP64 oracle (``oracle/``) and the GPU library's tests and benchmark may draw
their circuits from it.

Conventions (shared by every consumer):

* A circuit is a list of gates applied in order to ``n_qubits`` qubits that all
  start in |0>.  A one-qubit gate is a 2x2 matrix, a two-qubit gate on
  ``(q0, q1)`` a 4x4 matrix whose row/column index is ``2*x[q0] + x[q1]``
  (first listed qubit = high bit); rows are outputs, columns inputs.
* A noise *site* attaches a channel to a gate (noise acts right after the gate,
  the reading of "errors are preceded or succeeded by a gate of the same size and
  location", Sec. III-A).  A gate's sites act in list order.
* A channel is a list of Kraus operators (2x2 or 4x4) plus, optionally, the
  probability with which trajectory pre-sampling picks each one; when omitted the
  proposal is ``tr(K^dag K)/d``.

The workload recipes follow the paper's random-circuit family (Sec. IV-B) at the
sizes of the five benchmark configurations: a 10-qubit chain, a 50-qubit chain, a
5x5 grid with amplitude damping, a ragged mix of 256 circuits and a 20-qubit
rotation-layer circuit for gradients.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Channel", "Circuit", "Workload", "haar_su4", "depolarizing", "amplitude_damping",
    "pauli_x", "pauli_y", "pauli_z", "brickwork_1d", "chain10_d8", "brickwork50_d6", "grid5x5_d8",
    "hea20_l10", "random_brickwork", "small_random_circuit", "grid_layers", "hea", "rotation_spec",
    "zz_chain_terms",
]

I2 = np.eye(2, dtype=np.complex128)
pauli_x = np.array([[0, 1], [1, 0]], dtype=np.complex128)
pauli_y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
pauli_z = np.array([[1, 0], [0, -1]], dtype=np.complex128)


@dataclass
class Channel:
    """A CPTP map given by Kraus operators ``kraus[k]`` (d x d, d = 2 or 4)."""
    kraus: np.ndarray                      # (K, d, d) complex128
    probs: Optional[np.ndarray] = None     # (K,) float64 or None

    @property
    def arity(self) -> int:
        return 1 if self.kraus.shape[1] == 2 else 2


@dataclass
class Circuit:
    n_qubits: int
    gate_qubits: List[Tuple[int, ...]] = field(default_factory=list)
    gate_mats: List[np.ndarray] = field(default_factory=list)
    channels: List[Channel] = field(default_factory=list)
    site_gate: List[int] = field(default_factory=list)
    site_qubits: List[Tuple[int, ...]] = field(default_factory=list)
    site_channel: List[int] = field(default_factory=list)
    # optional: per-gate parameter description for differentiable circuits
    gate_param: List[Optional[Tuple[str, int]]] = field(default_factory=list)

    @property
    def n_gates(self) -> int:
        return len(self.gate_qubits)

    @property
    def n_sites(self) -> int:
        return len(self.site_gate)

    def add_gate(self, qubits: Sequence[int], mat: np.ndarray, param=None) -> int:
        qubits = tuple(int(q) for q in qubits)
        assert mat.shape == (2 ** len(qubits),) * 2
        self.gate_qubits.append(qubits)
        self.gate_mats.append(np.asarray(mat, dtype=np.complex128))
        self.gate_param.append(param)
        return len(self.gate_qubits) - 1

    def add_channel(self, ch: Channel) -> int:
        self.channels.append(ch)
        return len(self.channels) - 1

    def add_site(self, gate: int, qubits: Sequence[int], channel: int) -> None:
        self.site_gate.append(int(gate))
        self.site_qubits.append(tuple(int(q) for q in qubits))
        self.site_channel.append(int(channel))

    def round_to_complex64(self) -> "Circuit":
        """Round every gate matrix to complex64 (values kept as complex128)."""
        self.gate_mats = [m.astype(np.complex64).astype(np.complex128) for m in self.gate_mats]
        return self


@dataclass
class Workload:
    name: str
    circuit: Circuit
    n_traj: int                    # unique (non-degenerate) error sets E
    shots_per_traj: int            # m_i (same for every trajectory)
    batch_sizes: List[int]         # b_j, contiguous ascending qubit batches
    pts_seed: int
    shot_seed: int
    max_draws: int = 1 << 40


# --------------------------------------------------------------------------- gates
def haar_su4(rng: np.random.Generator) -> np.ndarray:
    """Haar-random SU(4): QR of a complex Ginibre matrix with R's diagonal phases
    moved into Q (Mezzadri 2007), divided by the principal 4th root of det."""
    z = (rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    q = q * (d / np.abs(d))[None, :]
    det = np.linalg.det(q)
    return q / det ** 0.25


def _rot(pauli: np.ndarray, angle: float) -> np.ndarray:
    """exp(-i angle/2 P) for a Pauli-like P with P^2 = I."""
    return np.cos(angle / 2) * I2 - 1j * np.sin(angle / 2) * pauli


SQRT_X = _rot(pauli_x, np.pi / 2)
SQRT_Y = _rot(pauli_y, np.pi / 2)
SQRT_W = _rot((pauli_x + pauli_y) / np.sqrt(2.0), np.pi / 2)
CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)
CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128)
HADAMARD = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)


def ry(theta: float) -> np.ndarray:
    return _rot(pauli_y, theta)


def rz(phi: float) -> np.ndarray:
    return _rot(pauli_z, phi)


# ------------------------------------------------------------------------ channels
def depolarizing(p: float) -> Channel:
    """Single-qubit depolarising channel, Kraus {sqrt(1-p) I, sqrt(p/3) X, Y, Z}."""
    k = np.stack([np.sqrt(1 - p) * I2, np.sqrt(p / 3) * pauli_x,
                  np.sqrt(p / 3) * pauli_y, np.sqrt(p / 3) * pauli_z])
    return Channel(k, np.array([1 - p, p / 3, p / 3, p / 3]))


def depolarizing2(p: float) -> Channel:
    """Two-qubit depolarising channel: identity with prob 1-p, else one of the 15
    non-identity two-qubit Paulis with prob p/15."""
    paulis = [I2, pauli_x, pauli_y, pauli_z]
    ks, ps = [], []
    for a in range(4):
        for b in range(4):
            pr = (1 - p) if (a == 0 and b == 0) else p / 15
            ks.append(np.sqrt(pr) * np.kron(paulis[a], paulis[b]))
            ps.append(pr)
    return Channel(np.stack(ks), np.array(ps))


def pauli_channel(which: np.ndarray, p: float) -> Channel:
    """Single Pauli error channel {sqrt(1-p) I, sqrt(p) P}."""
    return Channel(np.stack([np.sqrt(1 - p) * I2, np.sqrt(p) * which]), np.array([1 - p, p]))


def amplitude_damping(gamma: float) -> Channel:
    """Amplitude damping, K0 = [[1,0],[0,sqrt(1-g)]], K1 = [[0,sqrt(g)],[0,0]].
    Non-unitary: no probabilities given, the proposal is tr(K^dag K)/2."""
    k0 = np.array([[1, 0], [0, np.sqrt(1 - gamma)]], dtype=np.complex128)
    k1 = np.array([[0, np.sqrt(gamma)], [0, 0]], dtype=np.complex128)
    return Channel(np.stack([k0, k1]), None)


# ------------------------------------------------------------------------ layouts
def brickwork_1d(n: int, depth: int) -> List[List[Tuple[int, int]]]:
    """Layers of nearest-neighbour pairs on an open chain; even layers first."""
    layers = []
    for d in range(depth):
        start = d % 2
        layers.append([(q, q + 1) for q in range(start, n - 1, 2)])
    return layers


def grid_layers(rows: int, cols: int, n: int) -> List[List[Tuple[int, int]]]:
    """The four nearest-neighbour pair patterns on a row-major grid (q = cols*r + c,
    only q < n exist): horizontal-even, vertical-even, horizontal-odd, vertical-odd."""
    def ok(q):
        return q < n
    pats = []
    for kind, par in (("h", 0), ("v", 0), ("h", 1), ("v", 1)):
        pairs = []
        for r in range(rows):
            for c in range(cols):
                if kind == "h" and c % 2 == par and c + 1 < cols:
                    a, b = cols * r + c, cols * r + c + 1
                elif kind == "v" and r % 2 == par and r + 1 < rows:
                    a, b = cols * r + c, cols * (r + 1) + c
                else:
                    continue
                if ok(a) and ok(b):
                    pairs.append((a, b))
        pats.append(pairs)
    return pats


def _noisy_pair_circuit(n: int, layers, rng, noise: Sequence[Channel], two_qubit_gate=None) -> Circuit:
    c = Circuit(n)
    ch_ids = [c.add_channel(ch) for ch in noise]
    for layer in layers:
        for (a, b) in layer:
            m = haar_su4(rng) if two_qubit_gate is None else two_qubit_gate
            g = c.add_gate((a, b), m)
            for q in (a, b):
                for cid in ch_ids:
                    c.add_site(g, (q,), cid)
    return c


def random_brickwork(n: int, depth: int, rng: np.random.Generator, p: float,
                     layout: str = "1d") -> Circuit:
    """Haar SU(4) brickwork (1D chain or 2D grid) with single-qubit depolarising
    noise of strength p on both qubits after every gate."""
    if layout == "1d":
        layers = brickwork_1d(n, depth)
    else:
        rows = int(np.floor(np.sqrt(n)))
        cols = int(np.ceil(n / rows))
        pats = grid_layers(rows, cols, n)
        layers = [pats[d % 4] for d in range(depth)]
    return _noisy_pair_circuit(n, layers, rng, [depolarizing(p)])


def small_random_circuit(n: int, n_gates: int, rng: np.random.Generator,
                         channels: Sequence[Channel], site_prob: float = 1.0,
                         two_qubit_frac: float = 0.5) -> Circuit:
    """Random small circuit for tests: random 1q (Haar U(2)) and nearest-neighbour
    2q (Haar SU(4)) gates; each listed channel is attached (with probability
    site_prob) to every qubit the gate touches; 2q channels attach to 2q gates."""
    c = Circuit(n)
    ids = [c.add_channel(ch) for ch in channels]
    for _ in range(n_gates):
        if n > 1 and rng.random() < two_qubit_frac:
            a = int(rng.integers(0, n - 1))
            qs = (a, a + 1) if rng.random() < 0.5 else (a + 1, a)
            m = haar_su4(rng)
        else:
            qs = (int(rng.integers(0, n)),)
            m = haar_su4(rng)[:2, :2]
            u, _, vh = np.linalg.svd(m)
            m = u @ vh
        g = c.add_gate(qs, m)
        for cid, ch in zip(ids, channels):
            if rng.random() >= site_prob:
                continue
            if ch.arity == 2:
                if len(qs) == 2:
                    c.add_site(g, qs, cid)
            else:
                for q in qs:
                    c.add_site(g, (q,), cid)
    return c


T_GATE = np.diag([1.0, np.exp(1j * np.pi / 4)]).astype(np.complex128)


def controlled(u: np.ndarray) -> np.ndarray:
    """Two-qubit controlled-u, control = first listed qubit (the high bit of the
    matrix index 2 x[q0] + x[q1])."""
    m = np.eye(4, dtype=np.complex128)
    m[2:, 2:] = u
    return m


def rx(theta: float) -> np.ndarray:
    return _rot(pauli_x, theta)


def paper_random_circuit(n: int, n_gates: int, rng: np.random.Generator, p_lo: float = 0.02,
                         p_hi: float = 0.2, two_qubit_frac: float = 0.2) -> Circuit:
    """The random-circuit family of the paper's experiments (Sec. IV-B): single-qubit
    gates H, X, Y, Z, T, Rx(theta) on a uniformly random qubit and nearest-neighbour
    controlled gates CX, CY, CZ, CH, CRx(theta) on a uniformly random adjacent pair
    (random control side), round(two_qubit_frac * n_gates) of the gates two-qubit,
    in random positions; theta ~ U[0, 2 pi).  Every gate carries its own noise
    channel with p ~ U[p_lo, p_hi]: after a single-qubit gate one Pauli error
    (X, Y or Z, drawn uniformly) with probability p, after a two-qubit gate the
    two-qubit depolarising channel of strength p (our reading of the noise model)."""
    c = Circuit(n)
    n2 = int(round(two_qubit_frac * n_gates))
    is2 = np.zeros(n_gates, dtype=bool)
    is2[rng.choice(n_gates, size=n2, replace=False)] = True
    one = ("h", "x", "y", "z", "t", "rx")
    two = ("cx", "cy", "cz", "ch", "crx")
    paulis = (pauli_x, pauli_y, pauli_z)
    for k in range(n_gates):
        p = float(rng.uniform(p_lo, p_hi))
        if is2[k] and n > 1:
            a = int(rng.integers(0, n - 1))
            qs = (a, a + 1) if rng.random() < 0.5 else (a + 1, a)
            kind = two[int(rng.integers(0, len(two)))]
            u = {"cx": pauli_x, "cy": pauli_y, "cz": pauli_z, "ch": HADAMARD}.get(kind)
            if u is None:
                u = rx(float(rng.uniform(0.0, 2 * np.pi)))
            g = c.add_gate(qs, controlled(u))
            c.add_site(g, qs, c.add_channel(depolarizing2(p)))
        else:
            q = int(rng.integers(0, n))
            kind = one[int(rng.integers(0, len(one)))]
            m = {"h": HADAMARD, "x": pauli_x, "y": pauli_y, "z": pauli_z, "t": T_GATE}.get(kind)
            if m is None:
                m = rx(float(rng.uniform(0.0, 2 * np.pi)))
            g = c.add_gate((q,), m)
            c.add_site(g, (q,), c.add_channel(pauli_channel(paulis[int(rng.integers(0, 3))], p)))
    return c


# ------------------------------------------------------------- benchmark workloads
def chain10_d8() -> Workload:
    """10-qubit open chain, 8 brickwork layers of Haar SU(4) (complex64-rounded),
    depolarising p=0.01 on both qubits after each gate, 64 unique trajectories x
    100 shots, one batch of 10 qubits."""
    rng = np.random.default_rng(1001)
    c = random_brickwork(10, 8, rng, 0.01).round_to_complex64()
    return Workload("chain10_d8", c, 64, 100, [10], pts_seed=1002, shot_seed=1003)


def brickwork50_d6() -> Workload:
    """50-qubit open chain, 6 brickwork layers of Haar SU(4) (complex64-rounded),
    depolarising p=0.005 per qubit after each gate, 4096 unique trajectories x
    1000 shots, batches of 10 qubits."""
    rng = np.random.default_rng(2001)
    c = random_brickwork(50, 6, rng, 0.005).round_to_complex64()
    return Workload("brickwork50_d6", c, 4096, 1000, [10] * 5, pts_seed=2002, shot_seed=2003)


def sqrt_grid(rows: int, cols: int, cycles: int, rng: np.random.Generator, p: float = 0.01,
              gamma: float = 0.02) -> Circuit:
    """rows x cols grid (q = cols*r + c): each cycle applies a random sqrt(X)/sqrt(Y)/
    sqrt(W) to every qubit, then a CZ layer (patterns H-even, V-even, H-odd, V-odd in
    turn); depolarising p then amplitude damping gamma after every gate on each qubit
    it touches."""
    n = rows * cols
    c = Circuit(n)
    dep = c.add_channel(depolarizing(p))
    ad = c.add_channel(amplitude_damping(gamma))
    pats = grid_layers(rows, cols, n)
    choices = [SQRT_X, SQRT_Y, SQRT_W]
    for cyc in range(cycles):
        for q in range(n):
            g = c.add_gate((q,), choices[int(rng.integers(0, 3))])
            c.add_site(g, (q,), dep)
            c.add_site(g, (q,), ad)
        for (a, b) in pats[cyc % 4]:
            g = c.add_gate((a, b), CZ)
            for q in (a, b):
                c.add_site(g, (q,), dep)
                c.add_site(g, (q,), ad)
    return c


def grid5x5_d8(batch_sizes=(25,)) -> Workload:
    """5x5 grid, 8 cycles of sqrt_grid (depolarising 0.01 + amplitude damping
    0.02); 16384 unique trajectories x 256 shots."""
    rng = np.random.default_rng(3001)
    c = sqrt_grid(5, 5, 8, rng)
    return Workload("grid5x5_d8", c, 16384, 256, list(batch_sizes), pts_seed=3002, shot_seed=3003)


def hea(n: int, layers: int, angles: np.ndarray, noise: Sequence[Channel]) -> Circuit:
    """Hardware-efficient ansatz: per layer RY on every qubit, RZ on every qubit,
    CNOT ladder 0->1 ... n-2->n-1; each listed channel after every gate on each
    qubit it touches.  Angle of layer L: RY uses 2nL + q, RZ uses 2nL + n + q."""
    angles = np.asarray(angles, dtype=np.float64)
    c = Circuit(n)
    ids = [c.add_channel(ch) for ch in noise]
    for L in range(layers):
        for q in range(n):
            k = 2 * n * L + q
            g = c.add_gate((q,), ry(angles[k]), param=("ry", k))
            for cid in ids:
                c.add_site(g, (q,), cid)
        for q in range(n):
            k = 2 * n * L + n + q
            g = c.add_gate((q,), rz(angles[k]), param=("rz", k))
            for cid in ids:
                c.add_site(g, (q,), cid)
        for q in range(n - 1):
            g = c.add_gate((q, q + 1), CNOT)
            for cid in ids:
                c.add_site(g, (q,), cid)
                c.add_site(g, (q + 1,), cid)
    return c


def rotation_spec(circuit: Circuit):
    """(gate_param, gate_axis) arrays: parameter index of every rotation gate (-1
    for fixed gates) and its axis (0 X, 1 Y, 2 Z)."""
    axis_of = {"rx": 0, "ry": 1, "rz": 2}
    gp = np.full(circuit.n_gates, -1, dtype=np.int32)
    ga = np.zeros(circuit.n_gates, dtype=np.int32)
    for g, prm in enumerate(circuit.gate_param):
        if prm is not None:
            gp[g] = prm[1]
            ga[g] = axis_of[prm[0]]
    return gp, ga


def zz_chain_terms(n: int):
    """O = sum_{q=0}^{n-2} Z_q Z_{q+1} as ((q, q+1), coefficient) pairs."""
    return [((q, q + 1), 1.0) for q in range(n - 1)]


def hea20_angles() -> np.ndarray:
    rng = np.random.default_rng(5005)
    return rng.uniform(0.0, 2 * np.pi, size=400).astype(np.float32)


def hea20_l10(angles: Optional[np.ndarray] = None) -> Workload:
    """20-qubit hardware-efficient ansatz: 10 layers of RY on all, RZ on all, CNOT
    ladder 0->1 ... 18->19; depolarising p=0.01 after each gate on each touched
    qubit; 1024 trajectories.  Angle k of layer L: RY uses 40L + q, RZ 40L + 20 + q."""
    if angles is None:
        angles = hea20_angles()
    c = hea(20, 10, angles, [depolarizing(0.01)])
    return Workload("hea20_l10", c, 1024, 0, [20], pts_seed=5002, shot_seed=5003)


def ragged_mix(n_circuits: int = 256, seed: int = 4001):
    """Ragged mix: n ~ U{12..40}, depth ~ U{4..10}, 1D or 2D brickwork (p = 1/2)
    of Haar SU(4) with depolarising p=0.005 after every gate, E_c =
    round(exp(U[ln 32, ln 2048])) unique trajectories and 100 shots each,
    batches of 10 qubits with the remainder last.  Returns a list of dicts
    (circuit, n_traj, shots_per_traj, batch_sizes, pts_seed, shot_seed, layout,
    depth)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_circuits):
        n = int(rng.integers(12, 41))
        depth = int(rng.integers(4, 11))
        layout = "2d" if rng.random() < 0.5 else "1d"
        E = int(round(float(np.exp(rng.uniform(np.log(32), np.log(2048))))))
        crng = np.random.default_rng([seed, k])
        c = random_brickwork(n, depth, crng, 0.005, layout).round_to_complex64()
        bs = [10] * (n // 10) + ([n % 10] if n % 10 else [])
        out.append({"circuit": c, "n_traj": E, "shots_per_traj": 100, "batch_sizes": bs,
                    "pts_seed": 4002 + 10 * k, "shot_seed": 4003 + 10 * k, "layout": layout, "depth": depth})
    return out
