"""Batch-wise conditional sampling, NBS bookkeeping and trajectory weights.

Sec. II-B: the n qubits are split into batches B_1..B_f; a shot is drawn batch by
batch, the bits already drawn (s_1..s_{j-1}) being projected into the network
before the marginal of batch j is contracted.  Readings of the paper used here:
batches are contiguous ascending qubit ranges; the marginal of batch j given the
prefix p is

    pi_p(x) = sum_y |psi~(p, x, y)|^2      (y: qubits after B_j)

unnormalised (its FP64 sum Z_p is the prefix's joint weight); a shot's draw at
batch j uses u = Philox(shot seed, tag 2; counter (trajectory, j, shot, 0)) and
takes x = min{x : C(x) > u * C(last)} with C the FP64 inclusive prefix sum in
index order (the largest x with pi(x) > 0 if rounding leaves no such x).

Sec. III-B (NBS, proportional mode): the same shots are produced while the
marginal is contracted once per distinct (trajectory, prefix); the oracle
memoises marginals per prefix, which changes no result.  Non-proportional mode
with exhaustive or direct final-batch sampling: nonproportional_trajectory.
"""
import numpy as np

from . import philox


def batch_starts(batch_sizes):
    starts = np.concatenate([[0], np.cumsum(batch_sizes)[:-1]]).astype(int)
    return [int(s) for s in starts]


def marginal_from_state(psi: np.ndarray, n: int, start: int, b: int, prefix: int) -> np.ndarray:
    """pi_p(x) for the batch [start, start+b) given prefix bits p of qubits < start."""
    t = psi.reshape(2 ** (n - start - b), 2 ** b, 2 ** start)   # (y, x, p) in C order
    a = t[:, :, prefix]
    return np.sum(np.abs(a) ** 2, axis=0)


def amplitudes_from_state(psi: np.ndarray, n: int, start: int, b: int, prefix: int) -> np.ndarray:
    """Amplitudes of the final batch (start + b == n) given the prefix."""
    assert start + b == n
    return psi.reshape(2 ** b, 2 ** start)[:, prefix].copy()


def inverse_cdf(pi: np.ndarray, u: float) -> int:
    """x = min{x : C(x) > u C(last)}; the largest x with pi(x) > 0 if rounding
    leaves none; 0 when pi is identically zero (a trajectory whose inserted
    operators annihilate the state: it has weight 0 and all-zero shots)."""
    c = np.cumsum(np.asarray(pi, dtype=np.float64))   # sequential, index order
    hit = np.nonzero(c > u * c[-1])[0]
    if hit.size:
        return int(hit[0])
    pos = np.nonzero(np.asarray(pi) > 0)[0]
    return int(pos[-1]) if pos.size else 0


def shot_uniforms(seed: int, traj: int, j: int, n_shots: int) -> np.ndarray:
    t = np.arange(n_shots, dtype=np.uint64)
    return philox.uniform(seed, philox.TAG_SHOTS, np.full_like(t, traj), np.full_like(t, j), t, 0)


def sample_trajectory(marginal_fn, traj: int, n_qubits: int, batch_sizes, n_shots: int, seed: int):
    """Traditional per-shot batch-wise sampling (Sec. II-B) with memoised
    marginals.  marginal_fn(j, prefix) -> pi (FP64, length 2^{b_j}).
    Returns (shots as python ints, number of distinct contractions per batch)."""
    starts = batch_starts(batch_sizes)
    us = [shot_uniforms(seed, traj, j, n_shots) for j in range(len(batch_sizes))]
    memo = {}
    shots = []
    for t in range(n_shots):
        prefix = 0
        for j, (a, b) in enumerate(zip(starts, batch_sizes)):
            key = (j, prefix)
            if key not in memo:
                memo[key] = marginal_fn(j, prefix)
            x = inverse_cdf(memo[key], float(us[j][t]))
            prefix |= x << a
        shots.append(prefix)
    distinct = [sum(1 for (jj, _) in memo if jj == j) for j in range(len(batch_sizes))]
    return shots, distinct


def pack_shots(shots, n_qubits: int) -> np.ndarray:
    nw = (n_qubits + 63) // 64
    out = np.zeros((len(shots), nw), dtype=np.uint64)
    for r, s in enumerate(shots):
        for w in range(nw):
            out[r, w] = np.uint64((s >> (64 * w)) & 0xFFFFFFFFFFFFFFFF)
    return out


def trajectory_weights(Z: np.ndarray, mult: np.ndarray) -> np.ndarray:
    """W_i = mult_i r_i / sum_k mult_k r_k with r_i = Z_i, the squared norm of the
    trajectory built from rescaled inserted operators (= 1 for Pauli channels)."""
    r = np.asarray(Z, dtype=np.float64) * np.asarray(mult, dtype=np.float64)
    return r / r.sum()


def extra_uniforms(seed: int, traj: int, j: int, t0: int, count: int) -> np.ndarray:
    """Uniforms of the non-proportional draws: tag 3, counter (trajectory, j, t, 0)."""
    t = np.arange(t0, t0 + count, dtype=np.uint64)
    return philox.uniform(seed, philox.TAG_EXTRA, np.full_like(t, traj), np.full_like(t, j), t, 0)


def nonproportional_trajectory(marginal_fn, traj: int, n_qubits: int, batch_sizes, draws: int, seed: int,
                               threshold: float, final_draws: int = 0):
    """Non-proportional NBS with exhaustive final-batch sampling (Sec. III-B).

    Non-final batches: every distinct prefix of the trajectory takes `draws`
    draws from its conditional marginal; the distinct outcomes x, in increasing
    order, extend it to the prefixes of the next batch.  Prefixes are visited in
    the order they were made (parent by parent, outcomes ascending), i.e.
    lexicographically with the first batch most significant; the r-th prefix of
    batch j draws with the counters t = r * draws + d, d < draws (tag 3).
    Final batch: for every prefix, every x whose conditional probability
    P(x | prefix) = pi(x) / sum(pi) is strictly above `threshold` gives one row
    (full bitstring, P(x | prefix), p(prefix) = sum(pi) / Z), in prefix order
    then x ascending; a prefix of zero weight gives no rows.
    final_draws > 0 selects direct final-batch sampling instead: the r-th prefix
    takes final_draws draws (counters r * final_draws + d, tag 3), one row per
    draw in draw order (repeats kept); a prefix of zero weight draws x = 0 with
    P(x | prefix) = p(prefix) = 0.
    Returns (rows, number of prefixes per batch)."""
    starts = batch_starts(batch_sizes)
    f = len(batch_sizes)
    Z = float(np.sum(marginal_fn(0, 0)))          # the trajectory's squared norm
    prefixes = [0]
    counts = []
    for j in range(f - 1):
        counts.append(len(prefixes))
        nxt = []
        for r, prefix in enumerate(prefixes):
            pi = marginal_fn(j, prefix)
            us = extra_uniforms(seed, traj, j, r * draws, draws)
            xs = sorted({inverse_cdf(pi, float(u)) for u in us})
            nxt.extend(prefix | (x << starts[j]) for x in xs)
        prefixes = nxt
    counts.append(len(prefixes))
    rows = []
    if final_draws > 0:
        for r, prefix in enumerate(prefixes):
            pi = np.asarray(marginal_fn(f - 1, prefix), dtype=np.float64)
            Ze = float(np.sum(pi))
            for u in extra_uniforms(seed, traj, f - 1, r * final_draws, final_draws):
                x = inverse_cdf(pi, float(u))
                pc, pp = (float(pi[x]) / Ze, Ze / Z) if Ze > 0.0 else (0.0, 0.0)
                rows.append((prefix | (x << starts[f - 1]), pc, pp))
        return rows, counts
    for prefix in prefixes:
        pi = np.asarray(marginal_fn(f - 1, prefix), dtype=np.float64)
        Ze = float(np.sum(pi))
        if not Ze > 0.0:
            continue
        p_prefix = Ze / Z
        for x in range(len(pi)):
            pc = float(pi[x]) / Ze
            if pc > threshold:
                rows.append((prefix | (x << starts[f - 1]), pc, p_prefix))
    return rows, counts
