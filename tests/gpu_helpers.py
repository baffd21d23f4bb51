"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import math

import numpy as np

from oracle import sampling
from oracle import statevector as sv


def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


def to_dev(torch, dev, arr, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(arr))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)


def prefix_words(prefixes, nw):
    out = np.zeros((len(prefixes), nw), dtype=np.uint64)
    for i, p in enumerate(prefixes):
        for w in range(nw):
            out[i, w] = np.uint64((int(p) >> (64 * w)) & 0xFFFFFFFFFFFFFFFF)
    return out.view(np.int64)


def shots_to_ints(shots_np):
    s = shots_np.view(np.uint64)
    vals = []
    for r in range(s.shape[0]):
        v = 0
        for w in range(s.shape[1]):
            v |= int(s[r, w]) << (64 * w)
        vals.append(v)
    return vals


def flip_probability(pi_gpu, pi_ref):
    """Probability that one uniform draw gives different x under the two CDFs:
    sum_x |C_gpu(x)/Z_gpu - C_ref(x)/Z_ref| (exact for the strict rule)."""
    cg = np.cumsum(np.asarray(pi_gpu, dtype=np.float64))
    cr = np.cumsum(np.asarray(pi_ref, dtype=np.float64))
    if cg[-1] == 0 or cr[-1] == 0:          # an annihilated trajectory: every draw gives x = 0
        return 0.0 if cg[-1] == cr[-1] else 1.0
    return float(np.abs(cg / cg[-1] - cr / cr[-1]).sum())


def assert_shot_parity(mismatch, expected_flips, n_shots):
    """Observed CDF-boundary flips must be <= expected + 5 sigma (Poisson-binomial
    upper bound), and at least 99 % of the shots identical."""
    bound = expected_flips + 5.0 * math.sqrt(max(expected_flips, 1e-12)) + 1.0
    assert mismatch <= bound, (mismatch, expected_flips)
    assert mismatch <= 0.01 * n_shots + 1, (mismatch, n_shots)


def oracle_states(circuit, kraus):
    return [sv.trajectory_state(circuit, row) for row in kraus]


def oracle_shots_sv(circuit, psis, batch_sizes, m, seed):
    n = circuit.n_qubits
    starts = sampling.batch_starts(batch_sizes)
    out, memos = [], []
    for i, psi in enumerate(psis):
        def mfn(j, prefix, psi=psi):
            return sampling.marginal_from_state(psi, n, starts[j], batch_sizes[j], prefix)
        shots, distinct = sampling.sample_trajectory(mfn, i, n, batch_sizes, m, seed)
        out.append(shots)
        memos.append(distinct)
    return out, memos


# ------------------------------------------------------- oracle in worker processes
# The FP64 oracle is slow on full-size circuits; the GPU tests run it in spawned
# worker processes (numpy only, one BLAS thread each), never in the process that
# holds the GPU.
_LIMITS = None


def _one_blas_thread():
    global _LIMITS
    from threadpoolctl import threadpool_limits
    _LIMITS = threadpool_limits(limits=1)


def oracle_pool(workers=None):
    """A process pool (spawn start method) for oracle work, sized to the host's cores."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os
    n = workers or max(1, min(16, len(os.sched_getaffinity(0))))
    return cf.ProcessPoolExecutor(max_workers=n, mp_context=mp.get_context("spawn"), initializer=_one_blas_thread)


def sv_trajectory_job(circuit, kraus_row, traj, batch_sizes, m, seed):
    """Oracle work for one trajectory: its statevector, its m shots from the
    per-shot batch-wise sampler, every marginal the sampler used
    ({(j, prefix): pi}), its squared norm, and the last batch's amplitudes of
    every prefix the sampler reached there ({prefix: amplitudes})."""
    psi = sv.trajectory_state(circuit, kraus_row)
    n = circuit.n_qubits
    starts = sampling.batch_starts(batch_sizes)
    f = len(batch_sizes)
    used, amps = {}, {}

    def mfn(j, prefix):
        pi = sampling.marginal_from_state(psi, n, starts[j], batch_sizes[j], prefix)
        used[(j, prefix)] = pi
        if j == f - 1:
            amps[prefix] = sampling.amplitudes_from_state(psi, n, starts[j], batch_sizes[j], prefix)
        return pi

    shots, _ = sampling.sample_trajectory(mfn, traj, n, batch_sizes, m, seed)
    return shots, used, float(np.vdot(psi, psi).real), amps


def tn_value_job(circuit, kraus_row, start, b, prefix, kind):
    """Oracle work for one element: the explicit-network value of one batch."""
    from oracle import tn
    return tn.batch_network_value(circuit, kraus_row, start, b, prefix, kind)
