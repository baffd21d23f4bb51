"""MI355X-native PTSBE hot path: Python binding of the C ABI in include/ptsbe.h.

Every step of the path runs in the HIP library ``libptsbe.so``; this module only
marshals arguments.  PyTorch provides device memory and the stream.

    plan = Plan(circuit, batch_sizes=[10] * 5)
    kraus, mult, log_q, n_draws = plan.sample_trajectories(seed, n_unique)
    out = plan.sample_shots(kraus_dev, shots_per_traj_dev, seed=...)          # proportional NBS
    rows = plan.sample_nonproportional(kraus_dev, draws=1, seed=..., threshold=1e-6)   # exhaustive
    rows = plan.sample_nonproportional(kraus_dev, draws=1, seed=..., final_draws=100)  # direct
"""
import ctypes as C

import numpy as np

from . import _lib
from ._lib import PtsbeError

__all__ = ["Plan", "PtsbeError", "GradSpec", "AdjointSpec", "ExpectZZ", "load_library", "OUT_POPULATION", "OUT_AMPLITUDE"]

OUT_POPULATION = 0
OUT_AMPLITUDE = 1


def load_library():
    return _lib.load()


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _tptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


class _CircuitArrays:
    """Packs a circuit (workloads.Circuit-like object) into ptsbe_circuit_t."""

    def __init__(self, c):
        G = len(c.gate_qubits)
        self.gate_arity = np.array([len(q) for q in c.gate_qubits], dtype=np.int32)
        gq = np.full((max(G, 1), 2), -1, dtype=np.int32)
        for g, qs in enumerate(c.gate_qubits):
            gq[g, :len(qs)] = qs
        self.gate_qubits = gq
        self.gate_mats = np.concatenate(
            [np.asarray(m, dtype=np.complex128).reshape(-1).view(np.float64) for m in c.gate_mats]
            or [np.zeros(2)])
        ch = c.channels
        self.ch_arity = np.array([1 if k.kraus.shape[1] == 2 else 2 for k in ch] or [0], dtype=np.int32)
        self.ch_nkraus = np.array([k.kraus.shape[0] for k in ch] or [0], dtype=np.int32)
        self.ch_kraus = np.concatenate(
            [np.asarray(k.kraus, dtype=np.complex128).reshape(-1).view(np.float64) for k in ch] or [np.zeros(2)])
        probs = []
        for k in ch:
            if k.probs is None:
                probs.append(-np.ones(k.kraus.shape[0]))
            else:
                probs.append(np.asarray(k.probs, dtype=np.float64))
        self.ch_prob = np.concatenate(probs or [np.zeros(1)])
        S = len(c.site_gate)
        self.site_gate = np.array(c.site_gate or [0], dtype=np.int32)
        sq = np.full((max(S, 1), 2), -1, dtype=np.int32)
        for s, qs in enumerate(c.site_qubits):
            sq[s, :len(qs)] = qs
        self.site_qubits = sq
        self.site_channel = np.array(c.site_channel or [0], dtype=np.int32)
        self.struct = _lib.Circuit_t(
            c.n_qubits, G, _ptr(self.gate_arity, C.c_int32), _ptr(self.gate_qubits, C.c_int32),
            _ptr(self.gate_mats, C.c_double), len(ch), _ptr(self.ch_arity, C.c_int32),
            _ptr(self.ch_nkraus, C.c_int32), _ptr(self.ch_kraus, C.c_double), _ptr(self.ch_prob, C.c_double),
            S, _ptr(self.site_gate, C.c_int32), _ptr(self.site_qubits, C.c_int32),
            _ptr(self.site_channel, C.c_int32))


class AdjointSpec:
    """Rotation gates and a diagonal observable for Plan.contract_adjoint
    (ptsbe_adjoint_spec_t): ZZ terms [(a, b), coef], or obs_diag, a float64 device
    tensor of 2^n entries (kept alive by this object)."""

    def __init__(self, n_params, gate_param, gate_axis, terms=(), obs_diag=None):
        self.n_params = int(n_params)
        self.gate_param = np.ascontiguousarray(gate_param, dtype=np.int32)
        self.gate_axis = np.ascontiguousarray(gate_axis, dtype=np.int32)
        terms = list(terms)
        self.zz_qubits = np.ascontiguousarray([q for (q, _c) in terms] or [(0, 0)], dtype=np.int32).reshape(-1)
        self.zz_coef = np.ascontiguousarray([cf for (_q, cf) in terms] or [0.0], dtype=np.float64)
        self.obs_diag = obs_diag
        self.struct = _lib.AdjointSpec_t(self.n_params, _ptr(self.gate_param, C.c_int32),
                                         _ptr(self.gate_axis, C.c_int32), len(terms),
                                         _ptr(self.zz_qubits, C.c_int32), _ptr(self.zz_coef, C.c_double),
                                         _tptr(obs_diag))


class GradSpec:
    """Rotation gates and ZZ observable for Plan.expect_grad (ptsbe_grad_spec_t)."""

    def __init__(self, n_params, gate_param, gate_axis, terms, checkpoint_every=16):
        self.n_params = int(n_params)
        self.gate_param = np.ascontiguousarray(gate_param, dtype=np.int32)
        self.gate_axis = np.ascontiguousarray(gate_axis, dtype=np.int32)
        self.zz_qubits = np.ascontiguousarray([q for (q, _c) in terms] or [(0, 0)], dtype=np.int32).reshape(-1)
        self.zz_coef = np.ascontiguousarray([cf for (_q, cf) in terms] or [0.0], dtype=np.float64)
        self.struct = _lib.GradSpec_t(self.n_params, _ptr(self.gate_param, C.c_int32), _ptr(self.gate_axis, C.c_int32),
                                      len(terms), _ptr(self.zz_qubits, C.c_int32), _ptr(self.zz_coef, C.c_double),
                                      int(checkpoint_every))


# contraction method of a plan: the sweep over each batch's network, or the
# statevector of each trajectory (n <= 30); "auto" lets the planner choose
METHODS = {"auto": 0, "network": 1, "statevector": 2}
# sampling and element-splitting kernels: "auto" takes one lane per element for
# batches of <= 5 qubits with few shots per element, "wavefront" one wavefront
# per element always (the same shots bit for bit)
SAMPLE_KERNELS = {"auto": 0, "wavefront": 1}


class Plan:
    """ptsbe_plan: the unified contraction path of every batch (host, once).

    Options (ptsbe_plan_opts_t in include/ptsbe.h): light_cone prunes the doubled
    networks to the measured qubits' past light cone; subtree_reuse shares partial
    per-trajectory sweeps between error sets; sample_kernel "wavefront" forces one
    wavefront per element in sampling and splitting (the default "auto" takes one
    lane per element for small batches, with the same draws); max_part_rank caps the
    last batch's per-trajectory tensor rank (0: 31), slicing crossing wires beyond it."""

    def __init__(self, circuit, batch_sizes, hypersamples=4, path_seed=0, device=0, precision=0,
                 device_budget_bytes=0, method="auto", light_cone=False, subtree_reuse=False,
                 sample_kernel="auto", max_part_rank=0):
        self._lib = _lib.load()
        self.n_qubits = circuit.n_qubits
        self.n_sites = len(circuit.site_gate)
        self.batch_sizes = list(batch_sizes)
        arrs = _CircuitArrays(circuit)
        bs = np.array(self.batch_sizes, dtype=np.int32)
        if method not in METHODS:
            raise ValueError(f"method must be one of {sorted(METHODS)}")
        if sample_kernel not in SAMPLE_KERNELS:
            raise ValueError(f"sample_kernel must be one of {sorted(SAMPLE_KERNELS)}")
        opts = _lib.PlanOpts_t(len(bs), _ptr(bs, C.c_int32), int(hypersamples), int(path_seed), int(precision),
                               int(device), int(device_budget_bytes), METHODS[method], int(light_cone),
                               int(subtree_reuse), SAMPLE_KERNELS[sample_kernel], int(max_part_rank))
        h = C.c_void_p()
        _lib.check(self._lib.ptsbe_plan(C.byref(arrs.struct), C.byref(opts), C.byref(h)))
        self._h = h
        self.device = device
        info = _lib.PlanInfo_t()
        _lib.check(self._lib.ptsbe_plan_query(self._h, C.byref(info)))
        self.n_words = info.n_words
        self.n_gates = info.n_gates
        self.plan_device_bytes = info.plan_device_bytes
        self.method = {v: k for k, v in METHODS.items()}[info.method]
        self.sv_windows = info.sv_windows
        self._sv_windows_by_size = list(info.sv_windows_by_size)
        self.sv_clusters = info.sv_clusters
        self.sv_cluster_steps = info.sv_cluster_steps
        self.precision = info.precision
        self.light_cone = bool(info.light_cone)
        self.subtree_reuse = bool(info.subtree_reuse)

    def sv_windows_for(self, window_qubits):
        """Gate windows (state passes) of the statevector schedule for windows of
        10, 11 or 12 qubits."""
        return self._sv_windows_by_size[int(window_qubits) - 10]

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ptsbe_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def join_tiling(self, j):
        """ptsbe_plan_join_tiling: the GEMV join's tiling of batch j over x (dict of arrays)."""
        a = {k: np.zeros(n, dtype=np.int64) for k, n in
             (("t_read", 12), ("o_read", 12), ("o_write", 12), ("t_hi", 32), ("o_hi", 32), ("x_t", 32), ("x_o", 32))}
        w = np.zeros(12, dtype=np.int32)
        nh, nx = C.c_int32(), C.c_int32()
        ptr = lambda v: v.ctypes.data_as(C.c_void_p)
        _lib.check(self._lib.ptsbe_plan_join_tiling(self._h, int(j), ptr(a["t_read"]), ptr(a["o_read"]), ptr(w),
                                                    ptr(a["o_write"]), ptr(a["t_hi"]), ptr(a["o_hi"]), C.byref(nh),
                                                    ptr(a["x_t"]), ptr(a["x_o"]), C.byref(nx)))
        a["w_of"] = w
        a["t_hi"], a["o_hi"] = a["t_hi"][:nh.value], a["o_hi"][:nh.value]
        a["x_t"], a["x_o"] = a["x_t"][:nx.value], a["x_o"][:nx.value]
        return a

    def right_sites(self, j):
        """ptsbe_plan_right_sites: sites whose Kraus choices enter batch j's per-trajectory part."""
        buf = np.zeros(max(self.n_sites, 1), dtype=np.int32)
        n = C.c_int32()
        _lib.check(self._lib.ptsbe_plan_right_sites(self._h, int(j), buf.ctypes.data_as(C.c_void_p), C.byref(n)))
        return buf[:n.value].copy()

    def sv_schedule(self, window_qubits=12):
        """ptsbe_plan_sv_schedule: (gate order, window offsets, window qubit lists)."""
        G = self.n_gates
        order = np.zeros(G, dtype=np.int32)
        first = np.zeros(G + 1, dtype=np.int32)
        wq = np.full((G, 12), -1, dtype=np.int32)
        nw = C.c_int32()
        _lib.check(self._lib.ptsbe_plan_sv_schedule(self._h, int(window_qubits), order.ctypes.data_as(C.c_void_p),
                                                     first.ctypes.data_as(C.c_void_p), wq.ctypes.data_as(C.c_void_p),
                                                     C.byref(nw)))
        k = nw.value
        return order, first[:k + 1], [list(q[q >= 0]) for q in wq[:k]]

    def batch_info(self, j):
        bi = _lib.BatchInfo_t()
        _lib.check(self._lib.ptsbe_plan_batch_info(self._h, int(j), C.byref(bi)))
        return {f: getattr(bi, f) for f, _ in bi._fields_}

    # ----------------------------------------------------------------- host PTS
    def sample_trajectories(self, seed, n_unique, max_draws=1 << 40):
        S = self.n_sites
        kr = np.zeros((n_unique, max(S, 1)), dtype=np.uint8)
        mult = np.zeros(n_unique, dtype=np.int64)
        lq = np.zeros(n_unique, dtype=np.float64)
        nu, nd = C.c_int64(), C.c_int64()
        _lib.check(self._lib.ptsbe_sample_trajectories(
            self._h, int(seed), int(n_unique), int(max_draws), kr.ctypes.data_as(C.c_void_p),
            mult.ctypes.data_as(C.c_void_p), lq.ctypes.data_as(C.c_void_p), C.byref(nu), C.byref(nd)))
        k = nu.value
        return kr[:k, :S].copy(), mult[:k].copy(), lq[:k].copy(), nd.value

    # --------------------------------------------------------------- device calls
    def contract_workspace_size(self, j, E, n_elems):
        b = C.c_size_t()
        _lib.check(self._lib.ptsbe_contract_workspace_size(self._h, int(j), int(E), int(n_elems), C.byref(b)))
        return b.value

    def sample_workspace_size(self, E, total_shots):
        b = C.c_size_t()
        _lib.check(self._lib.ptsbe_sample_workspace_size(self._h, int(E), int(total_shots), C.byref(b)))
        return b.value

    def chunking(self, call, E, count, workspace_bytes):
        """ptsbe_plan_chunking: trajectories per chunk at every batch for a workspace of
        workspace_bytes; call "contract" (count = elements) or "sample" (count = shots)."""
        out = np.zeros(len(self.batch_sizes), dtype=np.int64)
        _lib.check(self._lib.ptsbe_plan_chunking(self._h, {"contract": 0, "sample": 1}[call], int(E), int(count),
                                                 int(workspace_bytes), out.ctypes.data_as(C.c_void_p)))
        return out

    def contract_batch(self, j, kraus_dev, elem_traj_dev, elem_prefix_dev, out_kind=OUT_POPULATION,
                       workspace=None, stream=None):
        """ptsbe_contract_batch on torch device tensors; returns (out, totals)."""
        import torch
        E = kraus_dev.shape[0]
        U = elem_traj_dev.shape[0]
        b = self.batch_sizes[j]
        dev = kraus_dev.device
        if out_kind == OUT_AMPLITUDE:
            out = torch.empty((U, 2 ** b, 2), dtype=torch.float32, device=dev)
            totals = None
        else:
            out = torch.empty((U, 2 ** b), dtype=torch.float32, device=dev)
            totals = torch.empty(U, dtype=torch.float64, device=dev)
        if workspace is None:
            workspace = torch.empty(self.contract_workspace_size(j, E, U), dtype=torch.uint8, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev).cuda_stream
        _lib.check(self._lib.ptsbe_contract_batch(
            self._h, int(j), _tptr(kraus_dev), int(E), _tptr(elem_traj_dev), _tptr(elem_prefix_dev), int(U),
            int(out_kind), _tptr(out), _tptr(totals), _tptr(workspace), int(workspace.numel()),
            C.c_void_p(stream)))
        if out_kind == OUT_AMPLITUDE:
            out = torch.view_as_complex(out)
        return out, totals

    def contract_batch_noalloc(self, j, kraus_dev, elem_traj_dev, elem_prefix_dev, out, totals=None,
                               out_kind=OUT_POPULATION, stream=None):
        """ptsbe_contract_batch_noalloc: the same contraction into caller-given
        outputs (out: float32 [n_elems][2^b] populations, or float32 [n_elems][2^b][2]
        amplitudes; totals: float64 [n_elems] or None), with the library's static
        device scratch as the workspace (no device allocation by the library)."""
        import torch
        E = kraus_dev.shape[0]
        U = elem_traj_dev.shape[0]
        if stream is None:
            stream = torch.cuda.current_stream(kraus_dev.device).cuda_stream
        _lib.check(self._lib.ptsbe_contract_batch_noalloc(
            self._h, int(j), _tptr(kraus_dev), int(E), _tptr(elem_traj_dev), _tptr(elem_prefix_dev), int(U),
            int(out_kind), _tptr(out), _tptr(totals), C.c_void_p(stream)))

    def sample_shots(self, kraus_dev, shots_per_traj_dev, seed, mult_dev=None, workspace=None, stream=None,
                     want_traj=True):
        """ptsbe_sample_shots (proportional NBS); returns a dict of device tensors."""
        import torch
        E = kraus_dev.shape[0]
        dev = kraus_dev.device
        M = int(shots_per_traj_dev.sum().item())
        shots = torch.empty((max(M, 1), self.n_words), dtype=torch.int64, device=dev)
        shot_traj = torch.empty(max(M, 1), dtype=torch.int32, device=dev) if want_traj else None
        weights = torch.empty(E, dtype=torch.float64, device=dev)
        norms = torch.empty(E, dtype=torch.float64, device=dev)
        stats = np.zeros(len(self.batch_sizes), dtype=np.int64)
        if workspace is None:
            workspace = torch.empty(self.sample_workspace_size(E, M), dtype=torch.uint8, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev).cuda_stream
        _lib.check(self._lib.ptsbe_sample_shots(
            self._h, _tptr(kraus_dev), int(E), _tptr(mult_dev), _tptr(shots_per_traj_dev), 0, int(seed),
            _tptr(shots), _tptr(shot_traj), _tptr(weights), _tptr(norms),
            stats.ctypes.data_as(C.c_void_p), _tptr(workspace), int(workspace.numel()), C.c_void_p(stream)))
        return {"shots": shots[:M], "shot_traj": None if shot_traj is None else shot_traj[:M],
                "weights": weights, "norms": norms, "elements_per_batch": stats}

    def nonproportional_workspace_size(self, E, draws, max_elems, final_draws=0):
        b = C.c_size_t()
        _lib.check(self._lib.ptsbe_nonproportional_workspace_size(self._h, int(E), int(draws), int(final_draws),
                                                                  int(max_elems), C.byref(b)))
        return b.value

    def sample_nonproportional(self, kraus_dev, draws, seed, threshold=0.0, final_draws=0, max_elems=None,
                               capacity=None, mult_dev=None, workspace=None, stream=None, outputs=None):
        """ptsbe_sample_nonproportional (non-proportional NBS; exhaustive final batch when
        final_draws == 0, direct draws otherwise); returns a dict of device tensors trimmed to
        the rows found.  When the rows exceed capacity it raises PtsbeError (status
        OUT_OF_MEMORY) with `needed_rows` set."""
        import torch
        E = kraus_dev.shape[0]
        dev = kraus_dev.device
        if max_elems is None:
            max_elems = E * int(draws) ** max(len(self.batch_sizes) - 1, 0)
        if capacity is None:
            capacity = max_elems * final_draws if final_draws > 0 else min(max_elems << self.batch_sizes[-1], 1 << 24)
        if outputs is None:
            outputs = {"bits": torch.empty((max(capacity, 1), self.n_words), dtype=torch.int64, device=dev),
                       "row_traj": torch.empty(max(capacity, 1), dtype=torch.int32, device=dev),
                       "p_cond": torch.empty(max(capacity, 1), dtype=torch.float64, device=dev),
                       "p_prefix": torch.empty(max(capacity, 1), dtype=torch.float64, device=dev)}
        weights = torch.empty(E, dtype=torch.float64, device=dev)
        norms = torch.empty(E, dtype=torch.float64, device=dev)
        stats = np.zeros(len(self.batch_sizes), dtype=np.int64)
        n_rows = C.c_int64(0)
        if workspace is None:
            workspace = torch.empty(self.nonproportional_workspace_size(E, draws, max_elems, final_draws),
                                    dtype=torch.uint8, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev).cuda_stream
        st = self._lib.ptsbe_sample_nonproportional(
            self._h, _tptr(kraus_dev), int(E), _tptr(mult_dev), int(draws), int(final_draws), int(max_elems),
            int(seed), float(threshold), _tptr(outputs["bits"]), _tptr(outputs.get("row_traj")),
            _tptr(outputs.get("p_cond")), _tptr(outputs.get("p_prefix")), int(capacity), C.byref(n_rows),
            _tptr(weights), _tptr(norms), stats.ctypes.data_as(C.c_void_p), _tptr(workspace),
            int(workspace.numel()), C.c_void_p(stream))
        try:
            _lib.check(st)
        except _lib.PtsbeError as e:
            e.needed_rows = n_rows.value
            raise
        M = n_rows.value
        out = {k: (None if v is None else v[:M]) for k, v in outputs.items()}
        out.update({"n_rows": M, "weights": weights, "norms": norms, "elements_per_batch": stats})
        return out

    def expect_grad(self, spec, kraus_dev, weights_dev, theta_dev, want_grad=True, workspace=None, stream=None):
        """ptsbe_expect_grad: value, per-trajectory values and (optionally) the gradient."""
        import torch
        E = kraus_dev.shape[0]
        dev = kraus_dev.device
        value = torch.empty(1, dtype=torch.float64, device=dev)
        traj = torch.empty(E, dtype=torch.float64, device=dev)
        grad = torch.empty(max(spec.n_params, 1), dtype=torch.float64, device=dev) if want_grad else None
        if workspace is None:
            b = C.c_size_t()
            _lib.check(self._lib.ptsbe_expect_workspace_size(self._h, C.byref(spec.struct), int(E), C.byref(b)))
            workspace = torch.empty(b.value, dtype=torch.uint8, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev).cuda_stream
        _lib.check(self._lib.ptsbe_expect_grad(
            self._h, C.byref(spec.struct), _tptr(kraus_dev), int(E), _tptr(weights_dev), _tptr(theta_dev),
            _tptr(traj), _tptr(value), _tptr(grad), _tptr(workspace), int(workspace.numel()), C.c_void_p(stream)))
        return {"value": value[0], "traj_values": traj, "grad": None if grad is None else grad[:spec.n_params]}

    def contract_adjoint(self, spec, kraus_dev, weights_dev, theta_dev=None, psi_bar=None, want_grad=True,
                         want_gate_adj=False, want_values=True, workspace=None, stream=None):
        """ptsbe_contract_adjoint: values (with an observable), the angle gradient and
        (want_gate_adj) the gate-tensor adjoints 2 dL/d conj(U_g), complex128 [n_gates][16].
        psi_bar: complex64 device tensor [E][2^n], the seed dL/d conj(psi_i)."""
        import torch
        E = kraus_dev.shape[0]
        dev = kraus_dev.device
        value = torch.empty(1, dtype=torch.float64, device=dev) if want_values else None
        traj = torch.empty(E, dtype=torch.float64, device=dev) if want_values else None
        grad = torch.empty(max(spec.n_params, 1), dtype=torch.float64, device=dev) if want_grad else None
        gadj = torch.empty((self.n_gates, 16, 2), dtype=torch.float64, device=dev) if want_gate_adj else None
        if theta_dev is None:
            theta_dev = torch.zeros(max(spec.n_params, 1), dtype=torch.float64, device=dev)
        if psi_bar is not None:
            psi_bar = torch.view_as_real(psi_bar.to(torch.complex64).contiguous()).contiguous()
        if workspace is None:
            b = C.c_size_t()
            _lib.check(self._lib.ptsbe_adjoint_workspace_size(self._h, C.byref(spec.struct), int(E), C.byref(b)))
            workspace = torch.empty(b.value, dtype=torch.uint8, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev).cuda_stream
        _lib.check(self._lib.ptsbe_contract_adjoint(
            self._h, C.byref(spec.struct), _tptr(kraus_dev), int(E), _tptr(weights_dev), _tptr(theta_dev),
            _tptr(psi_bar), _tptr(traj), _tptr(value), _tptr(grad), _tptr(gadj), _tptr(workspace),
            int(workspace.numel()), C.c_void_p(stream)))
        return {"value": None if value is None else value[0], "traj_values": traj,
                "grad": None if grad is None else grad[:spec.n_params],
                "gate_adj": None if gadj is None else torch.view_as_complex(gadj)}

    # -------------------------------------------------------------- measurement
    def profile_enable(self, on=True):
        """on: False/0 off, True/1 join timing, 2 join and single HBM sweep-step timing."""
        _lib.check(self._lib.ptsbe_profile_enable(self._h, int(on)))

    def profile_read_windows(self):
        """ptsbe_profile_read_windows: statevector gate windows (ms, launches, algorithmic bytes)."""
        ms, n, b = C.c_double(), C.c_int64(), C.c_double()
        _lib.check(self._lib.ptsbe_profile_read_windows(self._h, C.byref(ms), C.byref(n), C.byref(b)))
        return {"ms": ms.value, "launches": n.value, "bytes": b.value}

    def profile_read_lds_sweeps(self):
        """ptsbe_profile_read_lds_sweeps: parts swept whole in LDS (ms, launches, flops)."""
        ms, n, fl = C.c_double(), C.c_int64(), C.c_double()
        _lib.check(self._lib.ptsbe_profile_read_lds_sweeps(self._h, C.byref(ms), C.byref(n), C.byref(fl)))
        return {"ms": ms.value, "launches": n.value, "flops": fl.value}

    def profile_read_sweeps(self):
        ms, b, fb = C.c_double(), C.c_double(), C.c_double()
        n = C.c_int64()
        _lib.check(self._lib.ptsbe_profile_read_sweeps(self._h, C.byref(ms), C.byref(n), C.byref(b), C.byref(fb)))
        return {"step_ms": ms.value, "step_launches": n.value, "step_bytes": b.value, "fused_bytes": fb.value}

    def profile_read(self):
        a, c, d, e = C.c_double(), C.c_double(), C.c_double(), C.c_double()
        b = C.c_int64()
        _lib.check(self._lib.ptsbe_profile_read(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d),
                                                C.byref(e)))
        return {"join_ms": a.value, "join_launches": b.value, "join_flops": c.value, "sweep_ms": d.value,
                "sweep_bytes": e.value}


def tune_batches(circuit, candidates, kraus_dev, shots_per_traj_dev, seed, mult_dev=None, workspace=None,
                 hypersamples=4, path_seed=0, device=0, precision=0, method="auto", light_cone=False,
                 subtree_reuse=False, stream=None):
    """ptsbe_tune_batches: time proportional sampling of the given trajectories under
    each candidate batch list (list of lists); returns (times_ms array, best index)."""
    import torch
    lib = _lib.load()
    arrs = _CircuitArrays(circuit)
    offs = np.zeros(len(candidates) + 1, dtype=np.int32)
    for c, bs in enumerate(candidates):
        offs[c + 1] = offs[c] + len(bs)
    sizes = np.array([b for bs in candidates for b in bs], dtype=np.int32)
    opts = _lib.PlanOpts_t(0, None, int(hypersamples), int(path_seed), int(precision), int(device), 0,
                           METHODS[method], int(light_cone), int(bool(subtree_reuse)))
    dev = kraus_dev.device
    E = kraus_dev.shape[0]
    M = int(shots_per_traj_dev.sum().item())
    words = (circuit.n_qubits + 63) // 64
    shots = torch.empty((max(M, 1), words), dtype=torch.int64, device=dev)
    if workspace is None:
        raise ValueError("tune_batches needs a workspace (device uint8 tensor)")
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    times = np.zeros(len(candidates), dtype=np.float64)
    best = C.c_int32()
    _lib.check(lib.ptsbe_tune_batches(
        C.byref(arrs.struct), C.byref(opts), len(candidates), _ptr(offs, C.c_int32), _ptr(sizes, C.c_int32),
        _tptr(kraus_dev), int(E), _tptr(mult_dev), _tptr(shots_per_traj_dev), int(seed), _tptr(shots),
        _tptr(workspace), int(workspace.numel()), C.c_void_p(stream), times.ctypes.data_as(C.c_void_p),
        C.byref(best)))
    return times, best.value


def _expect_zz_function():
    import torch

    class ExpectZZ(torch.autograd.Function):
        """f(theta) = sum_i w_i <psi_i(theta)|O|psi_i(theta)> through the HIP library.
        forward runs the forward contraction only (the value); backward runs the
        adjoint contraction (forward windows with their checkpoints, then the
        reverse pass seeded by grad_out w_i O psi_i) and returns the angle gradient."""

        @staticmethod
        def forward(ctx, theta, plan, spec, kraus_dev, weights_dev):
            th = theta.detach().to(torch.float64).contiguous()
            out = plan.expect_grad(spec, kraus_dev, weights_dev, th, want_grad=False)
            ctx.plan, ctx.spec, ctx.kraus, ctx.weights = plan, spec, kraus_dev, weights_dev
            ctx.save_for_backward(th)
            ctx.out_dtype = theta.dtype
            return out["value"].to(theta.dtype)

        @staticmethod
        def backward(ctx, gout):
            (th,) = ctx.saved_tensors
            w = ctx.weights * gout.to(torch.float64)
            out = ctx.plan.expect_grad(ctx.spec, ctx.kraus, w, th, want_grad=True)
            return out["grad"].to(ctx.out_dtype), None, None, None, None

    return ExpectZZ


class _Lazy:
    _cls = None

    def __getattr__(self, name):
        if _Lazy._cls is None:
            _Lazy._cls = _expect_zz_function()
        return getattr(_Lazy._cls, name)


ExpectZZ = _Lazy()
