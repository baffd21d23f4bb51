"""ctypes binding of libptsbe.so (argument marshalling only).

The structures mirror include/ptsbe.h.  Loading fails loudly when the built
library is missing: there is no fallback path.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libptsbe.so")

PTSBE_OK = 0
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "OUT_OF_MEMORY", 4: "DEVICE", 5: "NUMERIC"}
EXPORTS = [
    "ptsbe_plan", "ptsbe_plan_query", "ptsbe_plan_batch_info", "ptsbe_plan_destroy", "ptsbe_last_error",
    "ptsbe_sample_trajectories", "ptsbe_contract_workspace_size", "ptsbe_sample_workspace_size",
    "ptsbe_contract_batch", "ptsbe_sample_shots", "ptsbe_profile_enable", "ptsbe_profile_read",
    "ptsbe_expect_workspace_size", "ptsbe_expect_grad",
    "ptsbe_ragged_create", "ptsbe_ragged_destroy", "ptsbe_ragged_info", "ptsbe_ragged_workspace_size",
    "ptsbe_ragged_autotune", "ptsbe_ragged_sample_shots", "ptsbe_plan_sv_schedule", "ptsbe_plan_right_sites",
    "ptsbe_nonproportional_workspace_size", "ptsbe_sample_nonproportional", "ptsbe_profile_read_sweeps",
    "ptsbe_plan_join_tiling", "ptsbe_plan_chunking", "ptsbe_contract_batch_noalloc",
    "ptsbe_profile_read_windows", "ptsbe_adjoint_workspace_size", "ptsbe_contract_adjoint",
    "ptsbe_tune_batches", "ptsbe_profile_read_lds_sweeps",
]


class PtsbeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ptsbe {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Circuit_t(C.Structure):
    _fields_ = [
        ("n_qubits", C.c_int32), ("n_gates", C.c_int32),
        ("gate_arity", C.POINTER(C.c_int32)), ("gate_qubits", C.POINTER(C.c_int32)),
        ("gate_mats", C.POINTER(C.c_double)),
        ("n_channels", C.c_int32), ("ch_arity", C.POINTER(C.c_int32)), ("ch_nkraus", C.POINTER(C.c_int32)),
        ("ch_kraus", C.POINTER(C.c_double)), ("ch_prob", C.POINTER(C.c_double)),
        ("n_sites", C.c_int32), ("site_gate", C.POINTER(C.c_int32)), ("site_qubits", C.POINTER(C.c_int32)),
        ("site_channel", C.POINTER(C.c_int32)),
    ]


class PlanOpts_t(C.Structure):
    _fields_ = [
        ("n_batches", C.c_int32), ("batch_sizes", C.POINTER(C.c_int32)), ("hypersamples", C.c_int32),
        ("path_seed", C.c_uint64), ("precision", C.c_int32), ("device", C.c_int32),
        ("device_budget_bytes", C.c_size_t), ("method", C.c_int32), ("light_cone", C.c_int32),
        ("subtree_reuse", C.c_int32), ("sample_kernel", C.c_int32), ("max_part_rank", C.c_int32),
    ]


class PlanInfo_t(C.Structure):
    _fields_ = [
        ("n_qubits", C.c_int32), ("n_gates", C.c_int32), ("n_sites", C.c_int32), ("n_batches", C.c_int32),
        ("n_words", C.c_int32), ("max_kraus", C.c_int32), ("plan_device_bytes", C.c_int64),
        ("method", C.c_int32), ("sv_windows", C.c_int32), ("sv_windows_by_size", C.c_int32 * 3),
        ("sv_clusters", C.c_int32), ("sv_cluster_steps", C.c_int32), ("precision", C.c_int32),
        ("light_cone", C.c_int32), ("subtree_reuse", C.c_int32),
    ]


class BatchInfo_t(C.Structure):
    _fields_ = [
        ("start", C.c_int32), ("size", C.c_int32), ("doubled", C.c_int32),
        ("n_left_steps", C.c_int32), ("n_right_steps", C.c_int32), ("n_resume_steps", C.c_int32),
        ("left_rank", C.c_int32), ("right_rank", C.c_int32),
        ("left_peak_rank", C.c_int32), ("right_peak_rank", C.c_int32),
        ("join_rows_log2", C.c_int32), ("crossing", C.c_int32),
        ("flops_per_traj", C.c_double), ("flops_per_elem", C.c_double),
        ("join_flops_per_elem", C.c_double), ("bytes_per_traj", C.c_double),
        ("n_right_launches", C.c_int32), ("n_right_fused_steps", C.c_int32), ("right_longest_run", C.c_int32),
        ("kept_gates", C.c_int32), ("slice_bits", C.c_int32),
    ]


class GradSpec_t(C.Structure):
    _fields_ = [
        ("n_params", C.c_int32), ("gate_param", C.POINTER(C.c_int32)), ("gate_axis", C.POINTER(C.c_int32)),
        ("n_terms", C.c_int32), ("zz_qubits", C.POINTER(C.c_int32)), ("zz_coef", C.POINTER(C.c_double)),
        ("checkpoint_every", C.c_int32),
    ]


class AdjointSpec_t(C.Structure):
    _fields_ = [
        ("n_params", C.c_int32), ("gate_param", C.POINTER(C.c_int32)), ("gate_axis", C.POINTER(C.c_int32)),
        ("n_terms", C.c_int32), ("zz_qubits", C.POINTER(C.c_int32)), ("zz_coef", C.POINTER(C.c_double)),
        ("d_obs_diag", C.c_void_p),
    ]


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "or python -m paper_2604_08467_amd.build")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    i32, i64, u64, sz = C.c_int32, C.c_int64, C.c_uint64, C.c_size_t
    lib.ptsbe_last_error.restype = C.c_char_p
    lib.ptsbe_plan.argtypes = [C.POINTER(Circuit_t), C.POINTER(PlanOpts_t), C.POINTER(P)]
    lib.ptsbe_plan_query.argtypes = [P, C.POINTER(PlanInfo_t)]
    lib.ptsbe_plan_batch_info.argtypes = [P, i32, C.POINTER(BatchInfo_t)]
    lib.ptsbe_plan_sv_schedule.argtypes = [P, i32, P, P, P, C.POINTER(i32)]
    lib.ptsbe_plan_right_sites.argtypes = [P, i32, P, C.POINTER(i32)]
    lib.ptsbe_plan_join_tiling.argtypes = [P, i32, P, P, P, P, P, P, C.POINTER(i32), P, P, C.POINTER(i32)]
    lib.ptsbe_plan_destroy.argtypes = [P]
    lib.ptsbe_plan_destroy.restype = None
    lib.ptsbe_sample_trajectories.argtypes = [P, u64, i64, i64, P, P, P, C.POINTER(i64), C.POINTER(i64)]
    lib.ptsbe_contract_workspace_size.argtypes = [P, i32, i64, i64, C.POINTER(sz)]
    lib.ptsbe_sample_workspace_size.argtypes = [P, i64, i64, C.POINTER(sz)]
    lib.ptsbe_plan_chunking.argtypes = [P, i32, i64, i64, sz, P]
    lib.ptsbe_contract_batch.argtypes = [P, i32, P, i64, P, P, i64, i32, P, P, P, sz, P]
    lib.ptsbe_contract_batch_noalloc.argtypes = [P, i32, P, i64, P, P, i64, i32, P, P, P]
    lib.ptsbe_sample_shots.argtypes = [P, P, i64, P, P, i32, u64, P, P, P, P, P, P, sz, P]
    lib.ptsbe_nonproportional_workspace_size.argtypes = [P, i64, i32, i32, i64, C.POINTER(sz)]
    lib.ptsbe_sample_nonproportional.argtypes = [P, P, i64, P, i32, i32, i64, u64, C.c_double, P, P, P, P, i64,
                                                 C.POINTER(i64), P, P, P, P, sz, P]
    lib.ptsbe_tune_batches.argtypes = [C.POINTER(Circuit_t), C.POINTER(PlanOpts_t), i32, P, P, P, i64, P, P, u64, P,
                                       P, sz, P, P, C.POINTER(i32)]
    lib.ptsbe_profile_read_lds_sweeps.argtypes = [P, C.POINTER(C.c_double), C.POINTER(i64), C.POINTER(C.c_double)]
    lib.ptsbe_profile_enable.argtypes = [P, i32]
    lib.ptsbe_profile_read_windows.argtypes = [P, C.POINTER(C.c_double), C.POINTER(i64), C.POINTER(C.c_double)]
    lib.ptsbe_profile_read_sweeps.argtypes = [P, C.POINTER(C.c_double), C.POINTER(i64), C.POINTER(C.c_double),
                                              C.POINTER(C.c_double)]
    lib.ptsbe_profile_read.argtypes = [P, C.POINTER(C.c_double), C.POINTER(i64), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.ptsbe_expect_workspace_size.argtypes = [P, C.POINTER(GradSpec_t), i64, C.POINTER(sz)]
    lib.ptsbe_expect_grad.argtypes = [P, C.POINTER(GradSpec_t), P, i64, P, P, P, P, P, P, sz, P]
    lib.ptsbe_adjoint_workspace_size.argtypes = [P, C.POINTER(AdjointSpec_t), i64, C.POINTER(sz)]
    lib.ptsbe_contract_adjoint.argtypes = [P, C.POINTER(AdjointSpec_t), P, i64, P, P, P, P, P, P, P, P, sz, P]
    for name in EXPORTS:
        f = getattr(lib, name)
        if name not in ("ptsbe_last_error", "ptsbe_plan_destroy", "ptsbe_ragged_destroy"):
            f.restype = C.c_int
    _lib = lib
    return lib


def check(status):
    if status != PTSBE_OK:
        msg = load().ptsbe_last_error().decode(errors="replace")
        raise PtsbeError(status, msg)
