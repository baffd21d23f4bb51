"""Binding of the ragged-set calls of include/ptsbe.h (argument marshalling only).

    rs = RaggedSet()
    rs.autotune(jobs)                       # optional: tile size per plan
    out = rs.sample_shots(jobs, graph=True)

A job is a dict with keys plan (statevector-method Plan), kraus (device uint8
tensor [E][S]), shots_per_traj (host int64 array [E]), seed, and optionally mult
(device int64 tensor [E]).
"""
import ctypes as C

import numpy as np

from . import _lib

GRAPH = 1


class RaggedJob_t(C.Structure):
    _fields_ = [
        ("plan", C.c_void_p), ("d_kraus_idx", C.c_void_p), ("E", C.c_int64), ("shots_per_traj", C.c_void_p),
        ("d_mult", C.c_void_p), ("seed", C.c_uint64), ("d_shots", C.c_void_p), ("d_traj_weight", C.c_void_p),
        ("d_traj_norm", C.c_void_p),
    ]


class RaggedInfo_t(C.Structure):
    _fields_ = [("n_waves", C.c_int32), ("graphs_replayed", C.c_int32), ("launches", C.c_int64),
                ("wall_clock_khz", C.c_double)]


def _setup(lib):
    if getattr(lib, "_ragged_ready", False):
        return lib
    P, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
    lib.ptsbe_ragged_create.argtypes = [i32, C.POINTER(P)]
    lib.ptsbe_ragged_destroy.argtypes = [P]
    lib.ptsbe_ragged_destroy.restype = None
    lib.ptsbe_ragged_info.argtypes = [P, C.POINTER(RaggedInfo_t)]
    lib.ptsbe_ragged_workspace_size.argtypes = [P, C.POINTER(RaggedJob_t), i32, C.POINTER(sz)]
    lib.ptsbe_ragged_autotune.argtypes = [P, C.POINTER(RaggedJob_t), i32, P, P, P, sz, P]
    lib.ptsbe_ragged_sample_shots.argtypes = [P, C.POINTER(RaggedJob_t), i32, i32, P, P, sz, P]
    for name in ("ptsbe_ragged_create", "ptsbe_ragged_info", "ptsbe_ragged_workspace_size",
                 "ptsbe_ragged_autotune", "ptsbe_ragged_sample_shots"):
        getattr(lib, name).restype = C.c_int
    lib._ragged_ready = True
    return lib


def _dptr(t):
    return None if t is None else t.data_ptr()


class RaggedSet:
    """ptsbe_ragged_*: several statevector-method plans sampled in shared launches."""

    def __init__(self, device=0):
        self._lib = _setup(_lib.load())
        h = C.c_void_p()
        _lib.check(self._lib.ptsbe_ragged_create(int(device), C.byref(h)))
        self._h = h
        self.device = device
        self._keep = []

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ptsbe_ragged_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _jobs(self, jobs, outputs=None):
        arr = (RaggedJob_t * len(jobs))()
        keep = []
        for c, jb in enumerate(jobs):
            m = np.ascontiguousarray(jb["shots_per_traj"], dtype=np.int64)
            keep.append(m)
            o = outputs[c] if outputs else {}
            arr[c] = RaggedJob_t(jb["plan"]._h.value, _dptr(jb["kraus"]), int(jb["kraus"].shape[0]),
                                 m.ctypes.data, _dptr(jb.get("mult")), int(jb["seed"]), _dptr(o.get("shots")),
                                 _dptr(o.get("weights")), _dptr(o.get("norms")))
        return arr, keep

    def workspace_size(self, jobs):
        arr, keep = self._jobs(jobs, [{"shots": _Fake()} for _ in jobs])
        n = C.c_size_t()
        _lib.check(self._lib.ptsbe_ragged_workspace_size(self._h, arr, len(jobs), C.byref(n)))
        return n.value

    def autotune(self, jobs, workspace=None, stream=None):
        """ptsbe_ragged_autotune: returns (window qubits per job, ms per trajectory [n_jobs][3])."""
        import torch
        dev = torch.device("cuda", self.device)
        arr, keep = self._jobs(jobs, [{"shots": _Fake()} for _ in jobs])
        best = np.zeros(len(jobs), dtype=np.int32)
        ms = np.zeros((len(jobs), 3), dtype=np.float32)
        if workspace is None:
            need = max(4 * (8 << jb["plan"].n_qubits) + 4 * 128 * jb["plan"].n_gates for jb in jobs) + (1 << 20)
            workspace = torch.empty(need, dtype=torch.uint8, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev).cuda_stream
        _lib.check(self._lib.ptsbe_ragged_autotune(self._h, arr, len(jobs), best.ctypes.data, ms.ctypes.data,
                                                   C.c_void_p(workspace.data_ptr()), int(workspace.numel()),
                                                   C.c_void_p(stream)))
        return best, ms

    def sample_shots(self, jobs, graph=False, workspace=None, stream=None, outputs=None, stamps=True):
        """ptsbe_ragged_sample_shots; returns per-job dicts (shots, weights, norms) and the
        completion stamps in microseconds after the start (one per job)."""
        import torch
        dev = torch.device("cuda", self.device)
        if outputs is None:
            outputs = []
            for jb in jobs:
                M = int(np.sum(jb["shots_per_traj"]))
                E = int(jb["kraus"].shape[0])
                outputs.append({"shots": torch.empty((max(M, 1), 1), dtype=torch.int64, device=dev),
                                "weights": torch.empty(E, dtype=torch.float64, device=dev),
                                "norms": torch.empty(E, dtype=torch.float64, device=dev), "M": M})
        arr, keep = self._jobs(jobs, outputs)
        if workspace is None:
            n = C.c_size_t()
            _lib.check(self._lib.ptsbe_ragged_workspace_size(self._h, arr, len(jobs), C.byref(n)))
            workspace = torch.empty(n.value, dtype=torch.uint8, device=dev)
        done = None
        if stamps:   # kept across calls: its address is part of a captured graph
            if getattr(self, "_done", None) is None or self._done.numel() != len(jobs) + 1:
                self._done = torch.zeros(len(jobs) + 1, dtype=torch.int64, device=dev)
            done = self._done
        if stream is None:
            stream = torch.cuda.current_stream(dev).cuda_stream
        _lib.check(self._lib.ptsbe_ragged_sample_shots(self._h, arr, len(jobs), GRAPH if graph else 0,
                                                       None if done is None else C.c_void_p(done.data_ptr()),
                                                       C.c_void_p(workspace.data_ptr()), int(workspace.numel()),
                                                       C.c_void_p(stream)))
        info = self.info()
        lat = None
        if done is not None:
            d = done.cpu().numpy().astype(np.float64)
            lat = (d[:-1] - d[-1]) / info["wall_clock_khz"] * 1e3   # ticks -> microseconds
        for o in outputs:
            o["shots"] = o["shots"][:o.get("M", o["shots"].shape[0])]
        return outputs, lat

    def info(self):
        inf = RaggedInfo_t()
        _lib.check(self._lib.ptsbe_ragged_info(self._h, C.byref(inf)))
        return {f: getattr(inf, f) for f, _ in inf._fields_}


class _Fake:
    """Stands in for an output tensor where a call only reads the job layout."""

    def data_ptr(self):
        return 1
