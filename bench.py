"""Benchmark of the PTSBE hot path on one MI355X.

Workload: 50-qubit open-chain brickwork, depth 6 (147 Haar SU(4) gates rounded to
complex64), depolarising p=0.005 on both qubits after every gate (294 noise
sites), 4096 unique trajectories x 1000 shots, batches of 10 qubits.  One step is
one full non-degenerate batched sampling pass (all five batches: error injection,
contraction, FP64 CDFs, inverse-CDF draws, prefix deduplication, trajectory
weights) over all 4096 trajectories, inputs resident in HBM.  Path finding and
trajectory pre-sampling happen before the timed region.

Prints one JSON line (metric: sampled shots/s).
"""
import argparse
import glob
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
FP32_VECTOR_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0
# the join kernel version that profiles/join_traffic.txt must name to be used
SWEEP_KERNEL_TAG = "absorb_global_kernel<NK> single HBM sweep steps, 4 kept indices per thread"
JOIN_KERNEL_TAG = "qform_mfma_kernel<32,NC> bilinear slots"
# the LDS-sweep kernel version that profiles/lds_sweep_counters_brickwork50_b5.txt must name
VM_KERNEL_TAG = "part_vm_kernel 64-job groups, trajectory gate slots, product-order gates, last step to HBM"


def _oracle_shots_worker(circuit, kraus_row, traj, batch_sizes, seed, budget_s):
    """One worker of the CPU baseline: per-shot batch-wise sampling of one
    trajectory with memoised explicit-network FP64 marginals, until budget_s."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import sampling, tn

    starts = sampling.batch_starts(batch_sizes)
    f = len(batch_sizes)

    memo = {}    # marginals persist across calls: the call for m shots contracts only what shot m - 1 adds

    def mfn(j, p):
        if (j, p) not in memo:
            kind = "ket" if j == f - 1 else "doubled"
            v = tn.batch_network_value(circuit, kraus_row, starts[j], batch_sizes[j], p, kind)
            memo[(j, p)] = np.abs(v) ** 2 if kind == "ket" else v
        return memo[(j, p)]

    m = 0
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        while time.perf_counter() - t0 < budget_s:
            m += 1
            sampling.sample_trajectory(mfn, traj, circuit.n_qubits, batch_sizes, m, seed)
    return m, time.perf_counter() - t0


def _oracle_value_worker(circuit, kraus_row, start, b, prefix, kind):
    from threadpoolctl import threadpool_limits

    from oracle import tn
    with threadpool_limits(limits=1):
        return tn.batch_network_value(circuit, kraus_row, start, b, prefix, kind)


def _pool(n):
    import concurrent.futures as cf
    import multiprocessing as mp
    return cf.ProcessPoolExecutor(max_workers=n, mp_context=mp.get_context("spawn"))


def host_cores():
    return max(1, len(os.sched_getaffinity(0)))


def cpu_baseline(wl, kr, bs, budget_s=20.0):
    """The FP64 oracle, as it stands, on a bounded sample, one worker process per
    host core: worker w samples shots of trajectory w (per-shot batch-wise
    sampling with memoised explicit-network marginals) for budget_s seconds."""
    n = min(host_cores(), len(kr))
    t0 = time.perf_counter()
    with _pool(n) as pool:
        futs = [pool.submit(_oracle_shots_worker, wl.circuit, kr[w], w, bs, wl.shot_seed, budget_s)
                for w in range(n)]
        res = [f.result() for f in futs]
    dt = time.perf_counter() - t0
    shots = sum(r[0] for r in res)
    return {"value": shots / dt, "unit": "shots/s", "cores": n, "kind": "oracle",
            "sample": f"{shots} shots of trajectories 0..{n - 1} (one worker process per core, per-shot "
                      f"batch-wise sampling with memoised explicit FP64 networks, {dt:.1f} s wall)"}


def error_vs_fp64(plan, wl, kr, kd, shots_dev, bs, n_pick=8):
    """The run's own error against FP64: conditionals P(x | prefix) of the elements
    that n_pick of the step's shots passed through (every batch), from the GPU path
    (ptsbe_contract_batch on the same plan) and from the explicit FP64 network."""
    import numpy as np
    import torch

    import paper_2604_08467_amd as P
    from oracle import sampling

    c = wl.circuit
    starts = sampling.batch_starts(bs)
    f = len(bs)
    m = shots_dev.shape[0] // len(kr)
    rows = [int(r) for r in np.linspace(0, shots_dev.shape[0] - 1, n_pick).astype(np.int64)]
    sh = shots_dev[rows].cpu().numpy().view(np.uint64)
    picks = []
    for k, r in enumerate(rows):
        v = sum(int(sh[k, w]) << (64 * w) for w in range(sh.shape[1]))
        for j in range(f):
            picks.append((r // m, j, v & ((1 << starts[j]) - 1)))
    dev = kd.device
    with _pool(min(host_cores(), len(picks))) as pool:
        futs = [pool.submit(_oracle_value_worker, c, kr[t], starts[j], bs[j], p, "ket" if j == f - 1 else "doubled")
                for (t, j, p) in picks]
        gpu = []
        for (t, j, p) in picks:
            et = torch.tensor([t], dtype=torch.int32, device=dev)
            pw = np.array([[(p >> (64 * w)) & 0xFFFFFFFFFFFFFFFF for w in range(plan.n_words)]], dtype=np.uint64)
            ep = torch.from_numpy(pw.view(np.int64)).to(dev)
            pop, tot = plan.contract_batch(j, kd, et, ep, P.OUT_POPULATION)
            gpu.append((pop[0].double().cpu().numpy(), float(tot[0].item())))
        refs = [fu.result() for fu in futs]
    worst = {"doubled": 0.0, "ket": 0.0}
    for (t, j, p), (g, gt), ref in zip(picks, gpu, refs):
        kind = "ket" if j == f - 1 else "doubled"
        pr = np.abs(ref) ** 2 if kind == "ket" else np.asarray(ref)
        worst[kind] = max(worst[kind], float(np.abs(g / gt - pr / pr.sum()).max()))
    return {"max_abs_conditional_error": max(worst.values()),
            "doubled_batches": worst["doubled"], "last_batch": worst["ket"],
            "elements": len(picks), "reference": "explicit FP64 network of each element (oracle), "
                                                 "same complex64-rounded gates",
            "sample": f"the prefixes of {n_pick} of the step's shots, spread over its trajectories, at every batch"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--traj", type=int, default=4096)
    ap.add_argument("--shots", type=int, default=1000)
    ap.add_argument("--workspace-gb", type=float, default=64.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["c64", "bf16", "f16"], default="c64",
                    help="bf16 / f16: split-precision (16-bit hi+lo, three products) MFMA for the dense join")
    ap.add_argument("--traffic-file", default=os.path.join(ROOT, "profiles", "join_traffic.txt"))
    ap.add_argument("--final-batch", type=int, default=20, help="exhaustive workload: final batch size")
    ap.add_argument("--threshold", type=float, default=1e-6, help="exhaustive workload: P(x | prefix) threshold")
    ap.add_argument("--draws", type=int, default=1, help="exhaustive workload: draws per prefix")
    ap.add_argument("--points", default="50x200,50x400,100x600",
                    help="exhaustive-paper workload: n x g points of the paper's random-circuit family")
    ap.add_argument("--final-batches", default="20,24,28", help="exhaustive-paper workload: b_f values")
    ap.add_argument("--sweep-sizes", default="8,10,12,14,16,18,20,22,24", help="batch-sweep workload: final batch sizes")
    ap.add_argument("--workload", choices=["brickwork50", "ragged", "exhaustive", "batch-sweep", "grid5x5",
                                           "exhaustive-paper", "hea20", "batch-tune"],
                    default="brickwork50",
                    help="ragged: the ragged mix of circuits as one graph-captured ragged set; grid5x5: the 25-qubit "
                         "grid with amplitude damping, 16384 x 256 (statevector method, --precision c64|bf16|f16)")
    ap.add_argument("--batches", default="auto",
                    help="brickwork50: uniform batch size b (the remainder last), or auto: the fastest of b = 3..10 "
                         "measured by ptsbe_tune_batches before the timed region")
    ap.add_argument("--light-cone", choices=["on", "off"], default="on",
                    help="network method: doubled networks keep only the gates in the light cone of the measured "
                         "qubits (plus non-unitary gates and their past); off: full networks")
    ap.add_argument("--subtree-reuse", choices=["on", "off"], default="off",
                    help="network method: per-trajectory parts share partial sweeps between error sets that agree "
                         "on the sites absorbed so far (bit-identical results)")
    ap.add_argument("--ragged-max-qubits", type=int, default=26)
    ap.add_argument("--ragged-scope", choices=["statevector", "all"], default="statevector",
                    help="all: also the network-method plans of the mix, on a second stream")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the path shards over trajectories across GPUs by design, "
              "but this benchmark measures a single MI355X", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.workload == "ragged":
        bench_ragged(args)
        return
    if args.workload == "exhaustive":
        bench_exhaustive(args)
        return
    if args.workload == "batch-sweep":
        bench_batch_sweep(args)
        return
    if args.workload == "grid5x5":
        bench_grid(args)
        return
    if args.workload == "exhaustive-paper":
        bench_exhaustive_paper(args)
        return
    if args.workload == "hea20":
        bench_hea20(args)
        return
    if args.workload == "batch-tune":
        bench_batch_tune(args)
        return
    if args.copy_calibration:
        n = 1 << 30
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": n, "copy_bytes_written_per_launch": n, "launches": 3}))
        return

    import paper_2604_08467_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    wl = W.brickwork50_d6()
    c = wl.circuit
    lc = args.light_cone == "on"
    sr = args.subtree_reuse == "on"
    prec = {"c64": 0, "bf16": 1, "f16": 2}[args.precision]
    # error sets do not depend on the batch list: drawn once with any plan
    kr, mult, _, n_draws = P.Plan(c, wl.batch_sizes, device=-1).sample_trajectories(wl.pts_seed, args.traj)
    E = len(kr)
    kd = torch.from_numpy(kr).to(dev)
    md = torch.full((E,), args.shots, dtype=torch.int64, device=dev)
    multd = torch.from_numpy(mult).to(dev)
    M = E * args.shots
    ws = torch.empty(int(args.workspace_gb * (1 << 30)), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    tune = None
    if args.batches == "auto":
        # the batch list is chosen before the timed region by measured time (Sec. V-B),
        # like the path: uniform lists b = 3..10 on the first 512 trajectories
        cands = [_batch_list(c.n_qubits, b) for b in (3, 4, 5, 6, 8, 10)]
        ns = min(512, E)
        t_t = time.perf_counter()
        times, best = P.tune_batches(c, cands, kd[:ns].contiguous(), md[:ns].contiguous(), wl.shot_seed,
                                     mult_dev=multd[:ns].contiguous(), workspace=ws, hypersamples=8,
                                     precision=prec, light_cone=lc, subtree_reuse=sr)
        bs = cands[best]
        tune = {"candidates": cands, "candidate_ms": [round(float(t), 3) for t in times], "sample_trajectories": ns,
                "tune_s": round(time.perf_counter() - t_t, 3)}
        print(f"bench: batch lists {dict(zip(map(str, cands), tune['candidate_ms']))} -> {bs}", file=sys.stderr,
              flush=True)
    else:
        bs = _batch_list(c.n_qubits, int(args.batches))
    plan = P.Plan(c, bs, hypersamples=8, precision=prec, light_cone=lc, subtree_reuse=sr)

    def step():
        return plan.sample_shots(kd, md, wl.shot_seed, mult_dev=multd, workspace=ws, want_traj=True)

    for _ in range(args.warmup):
        out = step()
    torch.cuda.synchronize()
    plan.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = plan.profile_read()
    sw = plan.profile_read_sweeps()
    vm = plan.profile_read_lds_sweeps()
    plan.profile_enable(False)
    shots_per_s = M * args.steps / dt
    print(f"right-part sweeps, algorithmic bytes per step: single HBM steps {sw['step_bytes'] / args.steps / 1e9:.2f} "
          f"GB, fused in-place runs {sw['fused_bytes'] / args.steps / 1e9:.2f} GB", file=sys.stderr)
    epb = [int(x) for x in out["elements_per_batch"]]

    join_s = prof["join_ms"] / 1e3
    achieved = prof["join_flops"] / join_s / 1e12 if join_s > 0 else 0.0
    traffic = None
    for tf in [args.traffic_file] + sorted(glob.glob(os.path.join(ROOT, "profiles", "join_traffic_*.txt"))):
        if not os.path.exists(tf):
            continue
        # "bytes_per_launch: N" written from two rocprofv3 counter runs of this command;
        # used only when its "kernel:" line names the join kernel as it is now
        # and the batch list it was measured on is this run's
        kv = dict(ln.split(":", 1) for ln in open(tf) if ":" in ln and not ln.startswith("#"))
        if (kv.get("kernel", "").strip() == JOIN_KERNEL_TAG and "bytes_per_launch" in kv
                and kv.get("batches", "").strip() == str(bs)):
            traffic = float(kv["bytes_per_launch"])
    peak = FP32_MFMA_PEAK_TFLOPS if args.precision == "c64" else BF16_MFMA_PEAK_TFLOPS   # fp16 dense = bf16 dense
    roofline = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": traffic if args.precision == "c64" else None,
                "kernel": "qform_mfma_kernel<32,NC> (doubled-network join as a real GEMM over K^2 folded slots, "
                          "FP32 MFMA; NC = 16-column x groups per workgroup, 8 for b = 10, 1..2 for b = 5)"
                          if args.precision == "c64"
                          else f"qform_split_kernel<32,NC> (doubled-network join as the K^2-slot GEMM, "
                               f"{args.precision} hi+lo operands, three products on 16-bit MFMA, FP32 accumulate)",
                "flops": "real bilinear form over K^2 folded slots: 2K^2 per row and x (K=32: 2048; "
                         "the plain complex product would be 8320)",
                "launches": prof["join_launches"], "kernel_ms_per_step": prof["join_ms"] / args.steps}
    vm_rec = None
    if vm["ms"] > 0:
        # the per-element LDS sweeps: plain FP32 arithmetic in LDS, against the
        # chip's FP32 vector peak
        vm_rate = vm["flops"] / (vm["ms"] / 1e3) / 1e12 if vm["ms"] > 0 else 0.0
        vm_traffic = None
        vm_file = os.path.join(ROOT, "profiles", "lds_sweep_counters_brickwork50_b5.txt")
        if os.path.exists(vm_file) and vm["launches"] > 0:
            # HBM bytes per step from two counter runs (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0),
            # per launch; used only for the kernel version and batch list they were taken on
            kv = dict(ln.split(":", 1) for ln in open(vm_file) if ":" in ln and not ln.startswith("#"))
            if (kv.get("kernel_tag", "").strip() == VM_KERNEL_TAG and kv.get("batches", "").strip() == str(bs)
                    and "fetch_bytes_per_step" in kv and "write_bytes_per_step" in kv):
                per_step = float(kv["fetch_bytes_per_step"]) + float(kv["write_bytes_per_step"])
                vm_traffic = per_step / (vm["launches"] / args.steps)
        vm_rec = {"bound": "alu", "achieved": vm_rate, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                  "frac": vm_rate / FP32_VECTOR_PEAK_TFLOPS, "traffic": vm_traffic,
                  "kernel": "part_vm_kernel (whole per-element parts swept in LDS, one gate absorbed per step)",
                  "flops": "8 real flops per complex multiply-add of each absorbed gate",
                  "launches": vm["launches"], "kernel_ms_per_step": vm["ms"] / args.steps}
    # the kernel with the most event time is the roofline's; the other is reported beside it
    if vm_rec is not None and vm["ms"] > prof["join_ms"]:
        roofline = dict(vm_rec, join=roofline)
    elif vm_rec is not None:
        roofline = dict(roofline, lds_sweeps=vm_rec)
    line = {
        "metric": "sampled shots/sec", "value": shots_per_s, "unit": "shots/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"c64": "c64", "bf16": "c64+bf16x3", "f16": "c64+f16x3"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"50-qubit 1D brickwork depth 6, Haar SU(4) c64, depolarising p=0.005, "
                               f"{E} trajectories x {args.shots} shots, batches {bs}, proportional NBS",
                   "trajectories": E, "shots_per_traj": args.shots, "batch_sizes": bs, "batch_tuning": tune,
                   "light_cone": lc, "subtree_reuse": sr,
                   "kept_gates": [plan.batch_info(j)["kept_gates"] for j in range(len(bs))],
                   "pts_draws": int(n_draws), "elements_per_batch": epb,
                   "unique_bitstrings_last_step": int(torch.unique(out["shots"][:, 0]).numel())},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        print("bench: error vs FP64 on sampled elements", file=sys.stderr, flush=True)
        line["error_vs_fp64"] = error_vs_fp64(plan, wl, kr, kd, out["shots"], bs)
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(wl, kr, bs)
    print(json.dumps(line), flush=True)


def bench_exhaustive(args):
    """Non-proportional NBS with exhaustive final-batch sampling on the 50-qubit
    brickwork: batches [10, 10, 10, b_f] (b_f = --final-batch), --draws per prefix,
    every x with P(x | prefix) > --threshold returned with its probabilities.
    One step = one ptsbe_sample_nonproportional call (exhaustive final batch); value = rows (distinct labelled
    bitstrings) per second."""
    import torch

    import paper_2604_08467_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    wl = W.brickwork50_d6()
    bf = args.final_batch
    bs = [10, 10, 10, bf] if bf <= 20 else [10, 40 - bf, bf]
    assert sum(bs) == 50
    plan = P.Plan(wl.circuit, bs, hypersamples=8, method="network", light_cone=args.light_cone == "on")
    E_req = args.traj if args.traj != 4096 else 512
    kr, mult, _, _ = plan.sample_trajectories(wl.pts_seed, E_req)
    E = len(kr)
    kd = torch.from_numpy(kr).to(dev)
    multd = torch.from_numpy(mult).to(dev)
    max_elems = E * args.draws ** (len(bs) - 1)
    cap = max_elems << bf
    outs = {"bits": torch.empty((cap, plan.n_words), dtype=torch.int64, device=dev),
            "row_traj": torch.empty(cap, dtype=torch.int32, device=dev),
            "p_cond": torch.empty(cap, dtype=torch.float64, device=dev),
            "p_prefix": torch.empty(cap, dtype=torch.float64, device=dev)}
    ws = torch.empty(int(args.workspace_gb * (1 << 30)), dtype=torch.uint8, device=dev)
    print(f"exhaustive: E={E}, batches {bs}, capacity {cap} rows, workspace {args.workspace_gb} GB",
          file=sys.stderr, flush=True)

    def step():
        return plan.sample_nonproportional(kd, args.draws, wl.shot_seed, args.threshold, max_elems=max_elems,
                                      capacity=cap, mult_dev=multd, workspace=ws, outputs=outs)

    for k in range(args.warmup):
        out = step()
        torch.cuda.synchronize()
        print(f"exhaustive: warmup {k} done, {out['n_rows']} rows", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = step()
        torch.cuda.synchronize()
        print(f"exhaustive: step {k} done at {time.perf_counter() - t0:.2f} s", file=sys.stderr, flush=True)
    dt = time.perf_counter() - t0
    rows = out["n_rows"]
    # one more step with HIP events (recorded by the library on its launch stream)
    # around every single sweep step in HBM, the dominant kernel of this workload
    plan.profile_enable(2)
    step()
    torch.cuda.synchronize()
    sw = plan.profile_read_sweeps()
    plan.profile_enable(0)
    achieved = sw["step_bytes"] / (sw["step_ms"] / 1e3) / 1e9 if sw["step_ms"] > 0 else 0.0
    traffic = None
    tf = os.path.join(ROOT, "profiles", "absorb_global_traffic_exhaustive_n50.txt")
    if os.path.exists(tf) and bf == 20 and E == 512 and args.draws == 1:
        # HBM bytes per launch from two rocprofv3 counter runs of this workload, used only
        # while the file's "kernel:" line names the sweep-step kernel as it is now
        kv = dict(ln.split(":", 1) for ln in open(tf) if ":" in ln and not ln.startswith("#"))
        if kv.get("kernel", "").strip() == SWEEP_KERNEL_TAG and "bytes_per_launch" in kv:
            traffic = float(kv["bytes_per_launch"])
    # the row writer's algorithmic bytes: populations read (4 B per value of x) and the
    # rows written (8 B bits + 4 B trajectory + 8 B P(x|prefix) + 8 B p(prefix))
    n_final = int(out["elements_per_batch"][-1])
    line = {
        "metric": "distinct labelled bitstrings/sec (exhaustive non-proportional NBS)", "value": rows * args.steps / dt,
        "unit": "bitstrings/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"50-qubit 1D brickwork depth 6, Haar SU(4) c64, depolarising p=0.005, {E} "
                               f"trajectories, batches {bs}, {args.draws} draw(s) per prefix, exhaustive final "
                               f"batch above P(x|prefix) > {args.threshold}",
                   "trajectories": E, "batch_sizes": bs, "rows": rows, "final_elements": n_final,
                   "elements_per_batch": [int(x) for x in out["elements_per_batch"]],
                   "population_values_scanned": n_final << bf,
                   "row_bytes_written": rows * 28},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "absorb_global_kernel (single sweep steps of the per-trajectory part in HBM: each "
                               "job's input and output tensor once, 8 (2^rA + 2^rC) bytes)",
                     "launches": sw["step_launches"], "avg_us": sw["step_ms"] * 1e3 / max(sw["step_launches"], 1),
                     "bytes_per_step": sw["step_bytes"], "kernel_ms_per_step": sw["step_ms"]},
    }
    print(json.dumps(line), flush=True)


def _oracle_grid_worker(circuit, kraus_row, budget_s):
    """One worker of the grid's CPU baseline: the FP64 oracle statevector of one
    trajectory, gate by gate, until budget_s; returns (gates applied, seconds)."""
    from threadpoolctl import threadpool_limits

    from oracle import statevector as sv
    from oracle import upv
    n = circuit.n_qubits
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        mats = upv.merged_gates(circuit, kraus_row)
        psi = sv.zero_state(n)
        g = 0
        while g < len(mats) and time.perf_counter() - t0 < budget_s:
            psi = sv.apply_gate(psi, n, mats[g], circuit.gate_qubits[g])
            g += 1
        return g, time.perf_counter() - t0


def grid_error_vs_fp64(plan, torch, dev):
    """Marginals of the stored FP64 oracle trajectories (tests/golden/grid25_sv.json,
    written by tests/golden/make_grid25.py from the oracle) against the GPU path on
    the same plan: max joint-marginal error per unit trajectory norm and max
    conditional error, over every stored batch marginal."""
    import numpy as np

    import paper_2604_08467_amd as P
    with open(os.path.join(ROOT, "tests", "golden", "grid25_sv.json")) as f:
        gold = json.load(f)
    kr = np.array([t["kraus"] for t in gold["trajectories"]], dtype=np.uint8)
    kd = torch.from_numpy(kr).to(dev)
    worst_j, worst_c, n = 0.0, 0.0, 0
    for i, rec in enumerate(gold["trajectories"]):
        for mg in rec["marginals"]:
            ref = np.array(mg["pi"])
            et = torch.tensor([i], dtype=torch.int32, device=dev)
            ep = torch.tensor([[mg["prefix"]]], dtype=torch.int64, device=dev)
            pop, tot = plan.contract_batch(mg["j"], kd, et, ep, P.OUT_POPULATION)
            g = pop[0].double().cpu().numpy()
            worst_j = max(worst_j, float(np.abs(g - ref).max() / rec["Z"]))
            worst_c = max(worst_c, float(np.abs(g / float(tot[0].item()) - ref / ref.sum()).max()))
            n += 1
    return {"max_abs_joint_marginal_error": worst_j, "max_abs_conditional_error": worst_c, "marginals": n,
            "reference": "stored FP64 oracle statevector marginals (tests/golden/grid25_sv.json): "
                         f"{len(kr)} trajectories x {len(gold['batch_sizes'])} batches"}


def bench_grid(args):
    """The 25-qubit 5x5 grid (depth 8: random sqrt(X)/sqrt(Y)/sqrt(W) layers and CZ
    layers; depolarising 0.01 then amplitude damping 0.02 after every gate, 720
    noise sites), batches [10, 10, 5], 16384 trajectories x 256 shots, statevector
    method (one gate schedule of 12-qubit LDS windows shared by every trajectory).
    --precision bf16 / f16 runs the gate clusters of the windows with hi + lo 16-bit
    operands on MFMA.  One step = one ptsbe_sample_shots call over every trajectory."""
    import numpy as np
    import torch

    import paper_2604_08467_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    wl = W.grid5x5_d8((10, 10, 5))
    prec = {"c64": 0, "bf16": 1, "f16": 2}[args.precision]
    plan = P.Plan(wl.circuit, wl.batch_sizes, precision=prec)
    E_req = args.traj if args.traj != 4096 else wl.n_traj
    m = args.shots if args.shots != 1000 else wl.shots_per_traj
    kr, mult, _, n_draws = plan.sample_trajectories(wl.pts_seed, E_req)
    E = len(kr)
    kd = torch.from_numpy(kr).to(dev)
    md = torch.full((E,), m, dtype=torch.int64, device=dev)
    multd = torch.from_numpy(mult).to(dev)
    ws = torch.empty(int(args.workspace_gb * (1 << 30)), dtype=torch.uint8, device=dev)
    print(f"grid5x5: E={E} x {m} shots, precision {args.precision}, {plan.sv_windows} windows, "
          f"{plan.sv_clusters} clusters ({plan.sv_cluster_steps} of {plan.n_gates} gates)", file=sys.stderr, flush=True)

    def step():
        return plan.sample_shots(kd, md, wl.shot_seed, mult_dev=multd, workspace=ws)

    for k in range(args.warmup):
        t_w = time.perf_counter()
        out = step()
        torch.cuda.synchronize()
        print(f"grid5x5: warmup {k} {time.perf_counter() - t_w:.2f} s", file=sys.stderr, flush=True)
    plan.profile_enable(1)
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = step()
        torch.cuda.synchronize()
        print(f"grid5x5: step {k} done at {time.perf_counter() - t0:.2f} s", file=sys.stderr, flush=True)
    dt = time.perf_counter() - t0
    win = plan.profile_read_windows()
    plan.profile_enable(0)
    M = E * m
    achieved = win["bytes"] / (win["ms"] / 1e3) / 1e9 if win["ms"] > 0 else 0.0
    line = {
        "metric": "sampled shots/sec", "value": M * args.steps / dt, "unit": "shots/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"c64": "c64", "bf16": "c64+bf16x3", "f16": "c64+f16x3"}[args.precision], "data": "synthetic",
        "config": {"workload": f"5x5 grid depth 8 (sqrt(X)/sqrt(Y)/sqrt(W) + CZ layers), depolarising 0.01 + "
                               f"amplitude damping 0.02, {E} trajectories x {m} shots, batches [10, 10, 5], "
                               f"statevector method, proportional NBS",
                   "trajectories": E, "shots_per_traj": m, "batch_sizes": list(wl.batch_sizes),
                   "pts_draws": int(n_draws), "precision": args.precision,
                   "windows": plan.sv_windows, "clusters": plan.sv_clusters,
                   "elements_per_batch": [int(x) for x in out["elements_per_batch"]]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "sv_window_kernel (gate windows: every 2^12-amplitude tile read and written once "
                               "per window, gates and clusters applied in LDS)",
                     "launches": win["launches"], "avg_us": win["ms"] * 1e3 / max(win["launches"], 1),
                     "bytes_per_step": win["bytes"] / args.steps, "kernel_ms_per_step": win["ms"] / args.steps},
    }
    print("grid5x5: error vs FP64 on the stored oracle marginals", file=sys.stderr, flush=True)
    line["error_vs_fp64"] = grid_error_vs_fp64(plan, torch, dev)
    if not args.no_cpu_baseline:
        print("grid5x5: CPU oracle baseline", file=sys.stderr, flush=True)
        cores = min(host_cores(), E)
        budget = 20.0
        t_c = time.perf_counter()
        with _pool(cores) as pool:
            res = [f.result() for f in [pool.submit(_oracle_grid_worker, wl.circuit, kr[w], budget)
                                        for w in range(cores)]]
        wall = time.perf_counter() - t_c
        G = plan.n_gates
        per_traj_s = float(np.mean([t * G / max(g, 1) for g, t in res]))
        line["cpu_baseline"] = {
            "value": cores * m / per_traj_s, "unit": "shots/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle statevector of trajectories 0..{cores - 1}, one worker process per core, "
                      f"{budget:.0f} s each ({min(g for g, _ in res)}..{max(g for g, _ in res)} of {G} gates "
                      f"applied; {wall:.1f} s wall); time per trajectory extrapolated linearly to all {G} gates, "
                      f"{m} shots per trajectory (marginals and draws not counted)"}
    print(json.dumps(line), flush=True)


def _oracle_hea20_worker(kraus_row, theta, gp, ga, terms):
    """One trajectory of the 20-qubit ansatz through the FP64 oracle: the
    adjoint gradient of <sum Z_i Z_i+1> and the value, one thread."""
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import gradients as gr

    c = W.hea20_l10().circuit
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        g = gr.adjoint_gradient(c, [kraus_row], [1.0], theta, gp, ga, terms)
        f = gr.value(c, [kraus_row], [1.0], theta, gp, ga, terms)
    return g, f, time.perf_counter() - t0


def bench_hea20(args):
    """The 20-qubit hardware-efficient ansatz (10 layers of RY RZ on every qubit and
    a CNOT ladder, 400 angles in [0, 2 pi), depolarising 0.01 after every gate),
    1024 trajectories: one step = the trajectory-weighted value of sum_i Z_i Z_i+1
    and its gradient with respect to all 400 angles (ptsbe_expect_grad: windowed
    forward with checkpoints, adjoint seed, windowed backward)."""
    import numpy as np
    import torch

    import paper_2604_08467_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    wl = W.hea20_l10()
    c = wl.circuit
    theta = W.hea20_angles().astype(np.float64)
    gp, ga = W.rotation_spec(c)
    terms = W.zz_chain_terms(c.n_qubits)
    plan = P.Plan(c, [c.n_qubits])
    E_req = args.traj if args.traj != 4096 else wl.n_traj
    kr, mult, _, n_draws = plan.sample_trajectories(wl.pts_seed, E_req)
    E = len(kr)
    w = mult / mult.sum()
    spec = P.GradSpec(len(theta), gp, ga, terms)
    kd = torch.from_numpy(kr).to(dev)
    wd = torch.from_numpy(w).to(dev)
    td = torch.from_numpy(theta).to(dev)
    ws = torch.empty(int(args.workspace_gb * (1 << 30)), dtype=torch.uint8, device=dev)
    print(f"hea20: E={E}, {len(theta)} angles", file=sys.stderr, flush=True)

    def step():
        return plan.expect_grad(spec, kd, wd, td, want_grad=True, workspace=ws)

    for k in range(args.warmup):
        t_w = time.perf_counter()
        out = step()
        torch.cuda.synchronize()
        print(f"hea20: warmup {k} {time.perf_counter() - t_w:.2f} s", file=sys.stderr, flush=True)
    plan.profile_enable(1)
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = step()
        torch.cuda.synchronize()
        print(f"hea20: step {k} done at {time.perf_counter() - t0:.2f} s", file=sys.stderr, flush=True)
    dt = time.perf_counter() - t0
    win = plan.profile_read_windows()
    plan.profile_enable(0)
    t_v = time.perf_counter()
    plan.expect_grad(spec, kd, wd, td, want_grad=False, workspace=ws)
    torch.cuda.synchronize()
    value_only_ms = (time.perf_counter() - t_v) * 1e3
    achieved = win["bytes"] / (win["ms"] / 1e3) / 1e9 if win["ms"] > 0 else 0.0
    line = {
        "metric": "trajectory value+gradient evaluations/sec", "value": E * args.steps / dt,
        "unit": "trajectories/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"20-qubit hardware-efficient ansatz, 10 layers RY RZ + CNOT ladder, 400 angles, "
                               f"depolarising 0.01, {E} trajectories; weighted <sum Z_i Z_i+1> and its gradient "
                               f"(adjoint contraction)",
                   "trajectories": E, "angles": len(theta), "pts_draws": int(n_draws),
                   "value_only_ms": value_only_ms},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "adj_window_kernel (forward windows: checkpoint read, next written, 16 B per "
                               "amplitude; backward windows: state read, adjoint state read and written, 24 B)",
                     "launches": win["launches"], "avg_us": win["ms"] * 1e3 / max(win["launches"], 1),
                     "bytes_per_step": win["bytes"] / args.steps, "kernel_ms_per_step": win["ms"] / args.steps},
    }
    if not args.no_cpu_baseline:
        # the oracle on a bounded sample: trajectories 0.. (one worker process per
        # core); the same trajectories, with their multiplicities as weights, on the
        # GPU give the run's error against FP64
        cores = min(host_cores(), E)
        print(f"hea20: FP64 oracle on {cores} trajectories", file=sys.stderr, flush=True)
        pick = list(range(cores))
        wp = np.zeros(E)
        wp[pick] = mult[pick] / mult[pick].sum()
        t_c = time.perf_counter()
        with _pool(cores) as pool:
            futs = [pool.submit(_oracle_hea20_worker, kr[k], theta, gp, ga, terms) for k in pick]
            gpu = plan.expect_grad(spec, kd, torch.from_numpy(wp).to(dev), td, want_grad=True, workspace=ws)
            torch.cuda.synchronize()
            res = [f.result() for f in futs]
        wall = time.perf_counter() - t_c
        g_ref = sum(wp[k] * r[0] for k, r in zip(pick, res))
        f_ref = sum(wp[k] * r[1] for k, r in zip(pick, res))
        g = gpu["grad"].cpu().numpy()
        line["error_vs_fp64"] = {
            "value_abs_error": abs(float(gpu["value"].item()) - f_ref),
            "gradient_rel_l2_error": float(np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)),
            "gradient_max_abs_error": float(np.abs(g - g_ref).max()),
            "reference": f"FP64 oracle adjoint gradient of trajectories 0..{cores - 1}, weighted by multiplicity"}
        line["cpu_baseline"] = {
            "value": cores / wall, "unit": "trajectories/s", "cores": cores, "kind": "oracle",
            "sample": f"value and adjoint gradient of trajectories 0..{cores - 1}, one worker process per core "
                      f"({wall:.1f} s wall, {np.mean([r[2] for r in res]):.1f} s per trajectory)"}
    print(json.dumps(line), flush=True)


def bench_exhaustive_paper(args):
    """Non-proportional NBS with exhaustive final-batch sampling in the paper's own
    regime (Sec. IV-B, V-A): random circuits of its family (H, X, Y, Z, T, Rx and
    nearest-neighbour CX, CY, CZ, CH, CRx, 20 % two-qubit gates, a Pauli error after
    every single-qubit gate and two-qubit depolarising after every two-qubit gate,
    p ~ U[0.02, 0.2]; one seeded instance per point, complex64), non-final batches
    of 10 qubits with one draw each, final batch b_f, every x with
    P(x | prefix) > --threshold returned.  Per point: host path finding (timed,
    outside the loop), then --steps timed calls over --traj trajectories.  value =
    distinct labelled bitstrings per second over all points."""
    import numpy as np
    import torch

    import paper_2604_08467_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    E_req = args.traj if args.traj != 4096 else 16
    ws = torch.empty(int(args.workspace_gb * (1 << 30)), dtype=torch.uint8, device=dev)
    points = [tuple(int(v) for v in pt.split("x")) for pt in args.points.split(",")]
    bfs = [int(v) for v in args.final_batches.split(",")]
    table, tot_rows, tot_s = [], 0, 0.0
    for (n, g) in points:
        circ = W.paper_random_circuit(n, g, np.random.default_rng(7000 + n + g)).round_to_complex64()
        for bf in bfs:
            rest = n - bf
            bs = [10] * (rest // 10) + ([rest % 10] if rest % 10 else []) + [bf]
            row = {"n": n, "g": g, "b_f": bf, "batches": bs}
            try:
                t_p = time.perf_counter()
                plan = P.Plan(circ, bs, hypersamples=8, method="network", light_cone=args.light_cone == "on")
                row["plan_s"] = round(time.perf_counter() - t_p, 3)
                kr, mult, _, _ = plan.sample_trajectories(7100 + n + g, E_req)
                E = len(kr)
                kd = torch.from_numpy(kr).to(dev)
                multd = torch.from_numpy(mult).to(dev)
                # strict P(x | prefix) > threshold: at most 1 / threshold rows per final element
                per_elem = min(1 << bf, int(np.ceil(1.0 / args.threshold)) if args.threshold > 0 else 1 << bf)
                cap = E * per_elem
                outs = {"bits": torch.empty((cap, plan.n_words), dtype=torch.int64, device=dev),
                        "row_traj": torch.empty(cap, dtype=torch.int32, device=dev),
                        "p_cond": torch.empty(cap, dtype=torch.float64, device=dev),
                        "p_prefix": torch.empty(cap, dtype=torch.float64, device=dev)}

                def step():
                    return plan.sample_nonproportional(kd, 1, 7200 + n + g, args.threshold, max_elems=E,
                                                       capacity=cap, mult_dev=multd, workspace=ws, outputs=outs)

                out = step()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    out = step()
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / args.steps
                bi = plan.batch_info(len(bs) - 1)
                row.update({"trajectories": E, "rows": int(out["n_rows"]), "call_ms": round(dt * 1e3, 3),
                            "bitstrings_per_s": out["n_rows"] / dt, "final_right_rank": bi["right_rank"],
                            "final_crossing": bi["crossing"],
                            "final_contraction_ms_per_traj": round(dt * 1e3 / E, 3)})
                tot_rows += int(out["n_rows"])
                tot_s += dt
                del plan, outs, out
            except Exception as e:      # a point beyond the library's limits is reported, not fatal
                row["error"] = str(e)[:160]
            table.append(row)
            print(f"exhaustive-paper: {row}", file=sys.stderr, flush=True)
    line = {
        "metric": "distinct labelled bitstrings/sec (exhaustive non-proportional NBS)",
        "value": tot_rows / tot_s if tot_s > 0 else 0.0, "unit": "bitstrings/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": tot_s * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"paper random-circuit family (Sec. IV-B), points {args.points}, b = 10 with one "
                               f"draw per non-final batch, b_f in {args.final_batches}, threshold {args.threshold}, "
                               f"{E_req} trajectories per point", "table": table},
    }
    print(json.dumps(line), flush=True)


def _batch_list(n, b):
    """[b] * k with the remainder as the last batch."""
    k, r = divmod(n, b)
    bs = [b] * k
    if r:
        bs.append(r)
    return bs


def bench_batch_tune(args):
    """Batch lists chosen by measurement (Sec. V-B: the batch sizes are the
    interface's free parameter).  On the 50-qubit brickwork (depth 6, depolarising
    0.005, light cone per --light-cone) ptsbe_tune_batches times proportional NBS of
    a sample (the first 512 of the 4096 trajectories x 1000 shots) under the lists
    [b] * k + remainder for b = 5, 6, 7, 8, 10, 12; then the full workload runs
    --steps timed steps with the fastest list and with [10] * 5.  value = shots/s
    of the full workload with the chosen list."""
    import numpy as np
    import torch

    import paper_2604_08467_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    wl = W.brickwork50_d6()
    c = wl.circuit
    lc = args.light_cone == "on"
    plan0 = P.Plan(c, wl.batch_sizes, hypersamples=8, light_cone=lc)
    kr, mult, _, _ = plan0.sample_trajectories(wl.pts_seed, args.traj)
    E = len(kr)
    kd = torch.from_numpy(kr).to(dev)
    multd = torch.from_numpy(mult).to(dev)
    md = torch.full((E,), args.shots, dtype=torch.int64, device=dev)
    ws = torch.empty(int(args.workspace_gb * (1 << 30)), dtype=torch.uint8, device=dev)
    cands = [_batch_list(c.n_qubits, b) for b in (5, 6, 7, 8, 10, 12)]
    ns = min(512, E)
    t_t = time.perf_counter()
    times, best = P.tune_batches(c, cands, kd[:ns].contiguous(), md[:ns].contiguous(), wl.shot_seed,
                                 mult_dev=multd[:ns].contiguous(), workspace=ws, hypersamples=8, light_cone=lc)
    tune_s = time.perf_counter() - t_t
    print(f"batch-tune: {dict(zip(map(str, cands), np.round(times, 2)))} -> {cands[best]} ({tune_s:.1f} s)",
          file=sys.stderr, flush=True)
    res = {}
    for name, bs in (("tuned", cands[best]), ("default", list(wl.batch_sizes))):
        plan = P.Plan(c, bs, hypersamples=8, light_cone=lc)
        for _ in range(args.warmup):
            plan.sample_shots(kd, md, wl.shot_seed, mult_dev=multd, workspace=ws, want_traj=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = plan.sample_shots(kd, md, wl.shot_seed, mult_dev=multd, workspace=ws, want_traj=False)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[name] = {"batch_sizes": bs, "ms_per_step": dt * 1e3, "shots_per_s": E * args.shots / dt,
                     "elements_per_batch": [int(x) for x in out["elements_per_batch"]]}
        print(f"batch-tune: {name} {bs}: {dt * 1e3:.1f} ms per step", file=sys.stderr, flush=True)
    line = {
        "metric": "sampled shots/sec", "value": res["tuned"]["shots_per_s"], "unit": "shots/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["tuned"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"50-qubit 1D brickwork depth 6, Haar SU(4) c64, depolarising p=0.005, {E} "
                               f"trajectories x {args.shots} shots, proportional NBS, batch list chosen by "
                               f"ptsbe_tune_batches on {ns} trajectories", "light_cone": lc,
                   "candidates": cands, "candidate_ms": [round(float(t), 3) for t in times],
                   "tune_s": tune_s, "tuned": res["tuned"], "default": res["default"]},
    }
    print(json.dumps(line), flush=True)


def bench_batch_sweep(args):
    """Contraction time of the final batch against its size b (Sec. V-B), and the
    host path-finding time of each plan: a 100-qubit 1D brickwork of 594 Haar SU(4)
    gates (depth 12, depolarising p=0.005), batches [10, ..., remainder, b].  For each b
    the plan is built (timed on the host), 4 trajectories are drawn, and the final
    batch is contracted for them (one element each, empty prefix), timed with events
    on the launch stream after one untimed call.  From b = 22 the per-trajectory
    tensor would exceed rank 31: the plan slices crossing wires (slice_bits) and
    the part is contracted once per slice value (use --workspace-gb 200)."""
    import numpy as np
    import torch

    import paper_2604_08467_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(5001)
    circ = W.random_brickwork(100, 12, rng, 0.005).round_to_complex64()
    n_traj = 4
    ws = torch.empty(int(args.workspace_gb * (1 << 30)), dtype=torch.uint8, device=dev)
    table = []
    for b in [int(v) for v in args.sweep_sizes.split(",")]:
        rest = 100 - b
        bs = [10] * (rest // 10) + ([rest % 10] if rest % 10 else []) + [b]
        t0 = time.perf_counter()
        plan = P.Plan(circ, bs, hypersamples=8, method="network")
        t_plan = time.perf_counter() - t0
        kr, _, _, _ = plan.sample_trajectories(5002, n_traj)
        E = len(kr)
        kd = torch.from_numpy(kr).to(dev)
        et = torch.arange(E, dtype=torch.int32, device=dev)
        ep = torch.zeros((E, plan.n_words), dtype=torch.int64, device=dev)
        j = len(bs) - 1
        plan.contract_batch(j, kd, et, ep, P.OUT_POPULATION, workspace=ws)
        torch.cuda.synchronize()
        reps = 3
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            pop, tot = plan.contract_batch(j, kd, et, ep, P.OUT_POPULATION, workspace=ws)
        ev1.record()
        torch.cuda.synchronize()
        call_ms = ev0.elapsed_time(ev1) / reps
        # trajectories that agree on the Kraus choices of the per-trajectory part share its tensor
        sites = plan.right_sites(j)
        distinct = len({tuple(kr[t, sites]) for t in range(E)})
        bi = plan.batch_info(j)
        # a sliced last batch contracts its per-trajectory part once per slice value
        n_sl = 2 ** bi["slice_bits"]
        row = {"b": b, "batches": bs, "plan_s": round(t_plan, 3), "call_ms": round(call_ms, 3),
               "distinct_right_parts": distinct, "ms_per_right_part": round(call_ms / distinct, 3),
               "right_rank": bi["right_rank"], "crossing": bi["crossing"], "slice_bits": bi["slice_bits"],
               "alg_bytes_per_right_part": bi["bytes_per_traj"] * n_sl, "alg_flops_per_elem": bi["flops_per_elem"]}
        table.append(row)
        print(f"batch-sweep: b={b} plan {t_plan:.2f} s, {E} trajectories ({distinct} distinct right parts) in "
              f"{call_ms:.2f} ms", file=sys.stderr, flush=True)
        del plan, pop, tot
    last = table[-1]
    rate = last["alg_bytes_per_right_part"] / (last["ms_per_right_part"] / 1e3) / 1e9
    line = {
        "metric": "final-batch contraction time per distinct per-trajectory part at the largest batch size",
        "value": last["ms_per_right_part"], "unit": "ms", "n_gpus": 1, "steps": 3, "warmup": 1,
        "ms_per_step": last["call_ms"], "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": "100-qubit 1D brickwork depth 12 (594 Haar SU(4) gates, c64), depolarising "
                               "p=0.005, final batch of b qubits after batches of 10", "table": table},
        "roofline": {"bound": "hbm", "achieved": rate, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": rate / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole final-batch contraction (algorithmic sweep bytes of the distinct "
                               "per-trajectory parts over the call time; join and left parts included in the time)"},
    }
    print(json.dumps(line), flush=True)


def bench_ragged(args):
    """Ragged mix of circuits (n ~ U{12..40}, depth 4..10, 1D/2D, E log-uniform
    32..2048, 100 shots each).  Every circuit ptsbe_plan accepts runs in one step:
    the statevector-method plans (n <= --ragged-max-qubits) as one ragged set,
    graph-captured after one autotune pass, light circuits in the first waves;
    with --ragged-scope all, the network-method plans run at the same time on a
    second stream from a second host thread, lightest first, and the statevector
    plans beyond --ragged-max-qubits run one call each after the set (their
    states of up to 8.6 GB leave room for few trajectories per wave; they run
    in the timed steps only).  Circuits no method takes (2D beyond 30 qubits) are
    listed as excluded.  One step = every shot of
    every included circuit; latency = completion time of each circuit from the
    step's start (device stamps for the set, host clock for the network plans)."""
    import threading

    import numpy as np
    import torch

    import paper_2604_08467_amd as P
    import workloads as W
    from paper_2604_08467_amd.ragged import RaggedSet

    dev = torch.device("cuda:0")
    mix = W.ragged_mix()
    jobs, net_jobs, big_jobs, excluded = [], [], [], []
    t_plan = time.perf_counter()
    for k, c in enumerate(mix):
        n = c["circuit"].n_qubits
        try:
            plan = P.Plan(c["circuit"], c["batch_sizes"], hypersamples=2, light_cone=args.light_cone == "on")
        except P.PtsbeError as e:
            excluded.append({"n": n, "reason": str(e)[:120]})
            continue
        big = plan.method == "statevector" and n > args.ragged_max_qubits
        if big and args.ragged_scope != "all":
            excluded.append({"n": n, "reason": f"statevector plan beyond --ragged-max-qubits {args.ragged_max_qubits}"})
            continue
        if plan.method == "network" and args.ragged_scope != "all":
            excluded.append({"n": n, "reason": "network-method plan (--ragged-scope all runs it)"})
            continue
        kr, mult, _, _ = plan.sample_trajectories(c["pts_seed"], c["n_traj"])
        job = {"plan": plan, "kraus": torch.from_numpy(kr).to(dev), "mult": torch.from_numpy(mult).to(dev),
               "shots_per_traj": np.full(len(kr), c["shots_per_traj"], dtype=np.int64), "seed": c["shot_seed"],
               "n": n, "layout": c.get("layout", "")}
        (net_jobs if plan.method != "statevector" else (big_jobs if big else jobs)).append(job)
    t_plan = time.perf_counter() - t_plan
    print(f"ragged: {len(jobs)} statevector plans in the set, {len(net_jobs)} network plans, {len(big_jobs)} "
          f"statevector plans of more than {args.ragged_max_qubits} qubits, {len(excluded)} excluded; "
          f"plans + PTS {t_plan:.1f} s", file=sys.stderr, flush=True)
    net_ws_gb = min(48.0, args.workspace_gb / 3) if net_jobs else 0.0
    # network plans lightest first (per-trajectory right-part bytes x trajectories)
    def net_cost(j):
        p = j["plan"]
        return sum(p.batch_info(b)["bytes_per_traj"] for b in range(len(p.batch_sizes))) * j["kraus"].shape[0]
    net_jobs.sort(key=net_cost)
    rs = RaggedSet()
    stream = torch.cuda.Stream(dev)
    stream2 = torch.cuda.Stream(dev)
    with torch.cuda.stream(stream):
        ws = torch.empty(int((args.workspace_gb - net_ws_gb) * (1 << 30)), dtype=torch.uint8, device=dev)
    ws2 = torch.empty(int(net_ws_gb * (1 << 30)), dtype=torch.uint8, device=dev) if net_jobs else None
    net_md = [torch.from_numpy(j["shots_per_traj"]).to(dev) for j in net_jobs]

    def run_network(t0, out_lat):
        with torch.cuda.stream(stream2):
            for k, (j, md) in enumerate(zip(net_jobs, net_md)):
                j["plan"].sample_shots(j["kraus"], md, j["seed"], mult_dev=j["mult"], workspace=ws2,
                                       stream=stream2.cuda_stream)
                out_lat.append((time.perf_counter() - t0) * 1e3)
                print(f"ragged: network plan {k + 1}/{len(net_jobs)} (n={j['n']}, E={j['kraus'].shape[0]}) done "
                      f"at {out_lat[-1] / 1e3:.1f} s", file=sys.stderr, flush=True)

    # statevector plans too large for the set (states of up to 8.6 GB: a few
    # trajectories fill a wave): after the set, one sampling call per circuit,
    # lightest first
    big_jobs.sort(key=lambda j: j["kraus"].shape[0] * (2 ** j["n"]) * j["plan"].sv_windows)
    big_md = [torch.from_numpy(j["shots_per_traj"]).to(dev) for j in big_jobs]

    def run_big(t0, out_lat):
        for k, (j, md) in enumerate(zip(big_jobs, big_md)):
            j["plan"].sample_shots(j["kraus"], md, j["seed"], mult_dev=j["mult"], workspace=ws,
                                   stream=stream.cuda_stream, want_traj=False)
            stream.synchronize()
            out_lat.append((time.perf_counter() - t0) * 1e3)
            print(f"ragged: large statevector plan {k + 1}/{len(big_jobs)} (n={j['n']}, "
                  f"E={j['kraus'].shape[0]}) done at {out_lat[-1] / 1e3:.1f} s", file=sys.stderr, flush=True)

    with torch.cuda.stream(stream):
        t_tune = time.perf_counter()
        best, ms = rs.autotune(jobs, workspace=ws, stream=stream.cuda_stream)
        print(f"ragged: autotune {time.perf_counter() - t_tune:.1f} s, windows "
              f"{ {w: int(np.sum(best == w)) for w in (10, 11, 12)} }", file=sys.stderr, flush=True)
        outs = None
        for k in range(args.warmup):
            t_w = time.perf_counter()
            nl = []
            th = threading.Thread(target=run_network, args=(t_w, nl))
            th.start()
            outs, lat = rs.sample_shots(jobs, graph=True, workspace=ws, stream=stream.cuda_stream, outputs=outs)
            stream.synchronize()
            th.join()
            print(f"ragged: warmup {k} {time.perf_counter() - t_w:.1f} s, {rs.info()}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lats, nlats = [], []
        for k in range(args.steps):
            ts = time.perf_counter()
            nl = []
            th = threading.Thread(target=run_network, args=(ts, nl))
            th.start()
            outs, lat = rs.sample_shots(jobs, graph=True, workspace=ws, stream=stream.cuda_stream, outputs=outs)
            stream.synchronize()
            t_set = (time.perf_counter() - ts) * 1e3
            print(f"ragged: step {k} set done at {t_set / 1e3:.1f} s", file=sys.stderr, flush=True)
            bl = []
            run_big(ts, bl)
            th.join()
            lats.append(lat / 1e3)
            nlats.append(np.array(nl + bl))
            print(f"ragged: step {k} done at {time.perf_counter() - t0:.1f} s (set {t_set / 1e3:.1f} s)",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    info = rs.info()
    M = sum(int(np.sum(j["shots_per_traj"])) for j in jobs + net_jobs + big_jobs)
    lat_all = np.concatenate([np.concatenate([a, b]) for a, b in zip(lats, nlats)])   # ms
    lat_sv = np.concatenate(lats)
    # algorithmic bytes of the gate windows: read + write of every state once per window
    win_bytes = 0.0
    for jb, bw in zip(jobs, best):
        p = jb["plan"]
        win_bytes += float(jb["kraus"].shape[0]) * 16.0 * (2 ** p.n_qubits) * p.sv_windows_for(int(bw))
    n_all = [j["n"] for j in jobs + net_jobs + big_jobs]
    big_bytes = sum(float(j["kraus"].shape[0]) * 16.0 * (2 ** j["n"]) * j["plan"].sv_windows for j in big_jobs)
    line = {
        "metric": "sampled shots/sec", "value": M * args.steps / dt, "unit": "shots/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"ragged mix of {len(mix)} circuits (n 12..40, depth 4..10, 1D/2D Haar SU(4), "
                               f"depolarising 0.005, E log-uniform 32..2048, 100 shots): {len(jobs)} statevector "
                               f"plans as one graph-captured ragged set"
                               + (f" + {len(net_jobs)} network-method plans on a second stream" if net_jobs else "")
                               + (f" + {len(big_jobs)} statevector plans of more than {args.ragged_max_qubits} "
                                  "qubits, one call each after the set" if big_jobs else ""),
                   "circuits": len(jobs) + len(net_jobs) + len(big_jobs), "ragged_set_circuits": len(jobs),
                   "network_circuits": len(net_jobs), "large_statevector_circuits": len(big_jobs),
                   "excluded_circuits": len(excluded),
                   "excluded_reasons": sorted({e["reason"] for e in excluded}),
                   "qubits_range": [int(min(n_all)), int(max(n_all))] if n_all else None,
                   "trajectories": int(sum(j["kraus"].shape[0] for j in jobs + net_jobs + big_jobs)), "shots": M,
                   "waves": info["n_waves"], "graphs_replayed": info["graphs_replayed"],
                   "latency_ms_p50": float(np.percentile(lat_all, 50)), "latency_ms_p99": float(np.percentile(lat_all, 99)),
                   "latency_ms_min": float(np.min(lat_all)),
                   "ragged_set_latency_ms_p50": float(np.percentile(lat_sv, 50)),
                   "ragged_set_latency_ms_p99": float(np.percentile(lat_sv, 99)),
                   "autotuned_windows": {str(w): int(np.sum(best == w)) for w in (10, 11, 12)},
                   "plan_and_pts_s": t_plan},
        "roofline": {"bound": "hbm", "achieved": (win_bytes + big_bytes) / (dt / args.steps) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (win_bytes + big_bytes) / (dt / args.steps) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "gate windows of the statevector plans (rg_window_kernel in the set, sv_window_kernel "
                               "for the large plans; state read+write per window), over the whole step time"},
    }
    print(json.dumps(line), flush=True)

if __name__ == "__main__":
    main()
