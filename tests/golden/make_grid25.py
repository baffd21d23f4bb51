"""Writes grid25_sv.json: FP64 oracle values for the 25-qubit 5x5-grid workload
(sqrt(X)/sqrt(Y)/sqrt(W) layers and CZ layers, depolarising p=0.01 then amplitude
damping gamma=0.02 after every gate, batches [10, 10, 5]).

For the first eight unique trajectories of pre-trajectory sampling it stores
the Kraus indices, the squared norm Z, the first-batch marginal, the marginals
of the second and third batches at the prefix of the first oracle shot, and the
first 16 oracle shots (batch-wise conditional sampling with the shot stream).
Only oracle/ and the seeded generators are used; one trajectory state takes
about two minutes in FP64 (trajectories run in parallel worker processes).

    python tests/golden/make_grid25.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import pts, sampling  # noqa: E402
from oracle import statevector as sv  # noqa: E402

N_TRAJ, N_SHOTS = 8, 16


def trajectory_record(i, kraus_row, bs, shot_seed):
    from threadpoolctl import threadpool_limits
    wl = W.grid5x5_d8(tuple(bs))
    c = wl.circuit
    n = c.n_qubits
    starts = sampling.batch_starts(bs)
    with threadpool_limits(limits=1):
        psi = sv.trajectory_state(c, kraus_row)

        def mfn(j, prefix):
            return sampling.marginal_from_state(psi, n, starts[j], bs[j], prefix)

        shots, _ = sampling.sample_trajectory(mfn, i, n, bs, N_SHOTS, shot_seed)
        s0 = int(shots[0])
        rec = {"kraus": [int(x) for x in kraus_row], "Z": float(np.vdot(psi, psi).real),
               "shots": [int(s) for s in shots], "marginals": []}
        for j in range(len(bs)):
            p = s0 & ((1 << starts[j]) - 1)
            rec["marginals"].append({"j": j, "prefix": p, "pi": [float(v) for v in mfn(j, p)]})
    return rec


def main():
    import concurrent.futures as cf
    import multiprocessing as mp
    wl = W.grid5x5_d8((10, 10, 5))
    c = wl.circuit
    bs = list(wl.batch_sizes)
    kr, mult, _, _ = pts.presample(c, wl.pts_seed, N_TRAJ)
    out = {"workload": "5x5 grid, depth 8, depolarising 0.01 + amplitude damping 0.02, batches [10,10,5]",
           "pts_seed": wl.pts_seed, "shot_seed": wl.shot_seed, "batch_sizes": bs, "trajectories": []}
    workers = max(1, min(N_TRAJ, len(os.sched_getaffinity(0))))
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as pool:
        futs = [pool.submit(trajectory_record, i, kr[i], bs, wl.shot_seed) for i in range(N_TRAJ)]
        for i, fu in enumerate(futs):
            rec = fu.result()
            out["trajectories"].append(rec)
            print(f"trajectory {i}: Z = {rec['Z']:.12f}", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "grid25_sv.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
