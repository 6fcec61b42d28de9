"""ctypes declarations of the C ABI in ``include/mwu.h`` (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmwu.so")

# error codes
MWU_OK = 0
ERRORS = {
    -1: "MWU_ERR_INVALID_ARG", -2: "MWU_ERR_NEGATIVE_ENTRY", -3: "MWU_ERR_NONFINITE",
    -4: "MWU_ERR_BAD_RHS", -5: "MWU_ERR_GRAPH", -6: "MWU_ERR_TOO_LARGE", -7: "MWU_ERR_OOM",
    -8: "MWU_ERR_DEVICE", -9: "MWU_ERR_UNBOUNDED", -10: "MWU_ERR_STATE",
}
# outcomes
CERTIFIED, FEASIBLE_UNCERTIFIED, INFEASIBLE, MAX_ITER, FEASIBLE_POINT = 0, 1, 2, 3, 4
PROBE_RUNNING, PROBE_FEASIBLE, PROBE_INFEASIBLE, PROBE_MAX_ITER = 0, 1, 2, 3
PACKING, COVERING, MIXED, MIXED_MAX, MIXED_MIN = 0, 1, 2, 3, 4
MAT_CSR, MAT_INCIDENCE, MAT_INCIDENCE_T, MAT_EDGE_PAIR, MAT_INTERWEAVE = 0, 1, 2, 3, 4
STEP_STD, STEP_BIN, STEP_BIN_WARM, STEP_NEWTON = 0, 1, 2, 3
FP64, MIXED_FP32_FP64 = 0, 1
FLAG_NO_FACTOR2, FLAG_GENERIC, FLAG_NO_TUNE, FLAG_REUSE, FLAG_DROP_SATISFIED = 1, 2, 4, 8, 16
FLAG_KEEP_ORDER, FLAG_LOCALITY_ORDER, FLAG_TUNE = 32, 64, 128
LAYOUT_DEFAULT, LAYOUT_TUNED, LAYOUT_CACHED, LAYOUT_SET = 0, 1, 2, 3

EXPORTED = [
    "mwu_default_options", "mwu_create", "mwu_create_batch", "mwu_solve", "mwu_destroy",
    "mwu_status_string", "mwu_num_variables", "mwu_probe_sizes", "mwu_probe_begin",
    "mwu_probe_run", "mwu_probe_direction", "mwu_probe_read", "mwu_probe_eval_steps",
    "mwu_probe_eval_newton",
    "mwu_potential_forward", "mwu_potential_backward", "mwu_potential_backward_noalloc", "mwu_time_pass",
    "mwu_batch_get_layout", "mwu_batch_set_layout", "mwu_batch_probe_run", "mwu_batch_probe_read",
]


class MwuError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {ERRORS.get(code, code)}")


class Matrix(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("values", ctypes.c_void_p), ("num_vertices", ctypes.c_int64),
                ("num_edges", ctypes.c_int64), ("edge_u", ctypes.c_void_p),
                ("edge_v", ctypes.c_void_p)]


class Problem(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int), ("P", Matrix), ("C", Matrix), ("b_P", ctypes.c_void_p),
                ("b_C", ctypes.c_void_p), ("c", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("max_probes", ctypes.c_int32), ("step_rule", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("iters_per_launch", ctypes.c_int32),
                ("device", ctypes.c_int32), ("hip_stream", ctypes.c_void_p),
                ("mixed_fixed_lambda", ctypes.c_double), ("flags", ctypes.c_uint64),
                ("tune_cache", ctypes.c_char_p)]


class BatchLayout(ctypes.Structure):
    _fields_ = [("tile_edges", ctypes.c_int32), ("tile_vertices", ctypes.c_int32),
                ("workgroups_per_cu", ctypes.c_int32), ("search_launches", ctypes.c_int32),
                ("source", ctypes.c_int32), ("candidates_timed", ctypes.c_int32),
                ("edge_iters_per_sec", ctypes.c_double)]


class ResultInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("objective", ctypes.c_double),
                ("lower_bound", ctypes.c_double), ("upper_bound", ctypes.c_double),
                ("total_iterations", ctypes.c_int64), ("final_probe_iterations", ctypes.c_int64),
                ("search_passes", ctypes.c_int64), ("probes", ctypes.c_int64),
                ("max_violation", ctypes.c_double), ("seconds_solve", ctypes.c_double),
                ("evaluations", ctypes.c_int64)]


class Sizes(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m_P", ctypes.c_int64), ("m_C", ctypes.c_int64),
                ("eta", ctypes.c_double)]


class ProbeInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int64),
                ("search_passes", ctypes.c_int64), ("alpha", ctypes.c_double),
                ("L_P", ctypes.c_double), ("L_C", ctypes.c_double),
                ("pack_bound", ctypes.c_double), ("cover_bound", ctypes.c_double),
                ("evaluations", ctypes.c_int64)]


_lib = None


def _open_torch_device_first() -> None:
    """PyTorch ships its own HIP runtime, separate from the /opt/rocm runtime
    libmwu.so links.  When both use the GPU in one process, torch's runtime
    has to open the device first: opened after this library's runtime has
    created its streams, it can find no device.  So on a machine where torch
    sees a GPU its runtime is initialized before the library is loaded."""
    try:
        import torch
    except ImportError:
        return
    try:
        if torch.cuda.is_available():
            torch.cuda.init()
    except RuntimeError:
        pass


def load() -> ctypes.CDLL:
    """Load libmwu.so; raises if the library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2307_03307_amd.build` (hipcc, gfx950)")
    _open_torch_device_first()
    L = ctypes.CDLL(LIB_PATH)
    vp, P = ctypes.c_void_p, ctypes.POINTER
    L.mwu_default_options.argtypes = [P(Options)]
    L.mwu_default_options.restype = None
    L.mwu_create.argtypes = [P(Problem), P(Options), P(vp)]
    L.mwu_create_batch.argtypes = [P(Problem), ctypes.c_int32, P(Options), P(vp)]
    L.mwu_solve.argtypes = [vp, vp, vp, vp, vp]
    L.mwu_destroy.argtypes = [vp]
    L.mwu_destroy.restype = None
    L.mwu_status_string.argtypes = [ctypes.c_int32]
    L.mwu_status_string.restype = ctypes.c_char_p
    L.mwu_num_variables.argtypes = [vp]
    L.mwu_num_variables.restype = ctypes.c_int64
    L.mwu_probe_sizes.argtypes = [vp, P(Sizes)]
    L.mwu_probe_begin.argtypes = [vp, ctypes.c_double, vp]
    L.mwu_probe_run.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, P(ProbeInfo)]
    L.mwu_probe_direction.argtypes = [vp]
    L.mwu_probe_read.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int64]
    L.mwu_probe_eval_steps.argtypes = [vp, vp, ctypes.c_int32, vp, vp, vp]
    L.mwu_probe_eval_newton.argtypes = [vp, ctypes.c_double, vp, vp, vp, vp]
    L.mwu_potential_forward.argtypes = [vp, vp, vp, vp]
    L.mwu_potential_backward.argtypes = [vp, vp, ctypes.c_double, vp, vp]
    L.mwu_potential_backward_noalloc.argtypes = [vp, vp, ctypes.c_double, vp, vp, vp]
    L.mwu_batch_probe_run.argtypes = [vp, vp, ctypes.c_int32, vp]
    L.mwu_batch_probe_read.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int64]
    L.mwu_time_pass.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
    L.mwu_batch_get_layout.argtypes = [vp, P(BatchLayout)]
    L.mwu_batch_set_layout.argtypes = [vp, P(BatchLayout)]
    for name in EXPORTED:
        fn = getattr(L, name)
        if fn.restype is ctypes.c_int:  # default restype
            fn.restype = ctypes.c_int32
    _lib = L
    return L


def check(code: int, where: str) -> None:
    if code != MWU_OK:
        raise MwuError(code, where)
