"""Pre-trajectory sampling (Sec. II-C, first paragraph of the unoptimised PTSBE
description): E error sets are drawn before any network is built.

Draw d, site p: u = Philox(seed, tag 1; counter (lo32(d), p, hi32(d), 0)); the Kraus index is
the first k whose FP64 inclusive cumulative proposal exceeds u (if rounding
leaves none, the last k with non-zero proposal).  Draws are i.i.d.; sampling
stops as soon as n_unique distinct error sets have appeared, or every error set
that has non-zero probability has appeared, or max_draws draws were made.  Distinct sets are kept in order of first appearance with their
multiplicity among the draws made ("non-degenerate trajectories").
"""
import numpy as np

from . import philox
from .upv import proposal


def kraus_choice(u: float, cum: np.ndarray, q: np.ndarray) -> int:
    hit = np.nonzero(cum > u)[0]
    if hit.size:
        return int(hit[0])
    return int(np.nonzero(q > 0)[0][-1])


def presample(circuit, seed: int, n_unique: int, max_draws: int = 1 << 40, block: int = 2048):
    S = circuit.n_sites
    qs = [proposal(circuit.channels[c]) for c in circuit.site_channel]
    cums = [np.cumsum(q) for q in qs]
    # sampling also stops once every error set that can occur has appeared
    possible = 1
    for q in qs:
        possible *= int(np.count_nonzero(q > 0))
    n_unique = min(n_unique, possible)
    seen = {}
    rows, mult = [], []
    d0 = 0
    n_draws = 0
    while len(rows) < n_unique and d0 < max_draws:
        nb = int(min(block, max_draws - d0))
        dd = np.repeat(np.arange(d0, d0 + nb, dtype=np.uint64), S)
        pp = np.tile(np.arange(S, dtype=np.uint64), nb)
        u = philox.uniform(seed, philox.TAG_PTS, dd & np.uint64(0xFFFFFFFF), pp, dd >> np.uint64(32), 0).reshape(nb, S)
        ks = np.empty((nb, S), dtype=np.uint8)
        for p in range(S):
            # first k with cum[k] > u, i.e. searchsorted(..., side='right')
            k = np.searchsorted(cums[p], u[:, p], side="right")
            last = int(np.nonzero(qs[p] > 0)[0][-1])
            ks[:, p] = np.where(k >= len(qs[p]), last, k)
        for r in range(nb):
            row = ks[r]
            key = row.tobytes()
            n_draws += 1
            if key in seen:
                mult[seen[key]] += 1
            else:
                seen[key] = len(rows)
                rows.append(row.copy())
                mult.append(1)
                if len(rows) == n_unique:
                    break
        d0 += nb
    kraus = np.array(rows, dtype=np.uint8).reshape(len(rows), S)
    log_q = np.array([sum(np.log(qs[p][row[p]]) for p in range(S)) for row in rows])
    return kraus, np.array(mult, dtype=np.int64), log_q, n_draws
