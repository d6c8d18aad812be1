"""ctypes declarations of the C ABI in include/cnmf.h (argument marshalling only).

Loading fails loudly when libcnmf.so has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcnmf.so")

CNMF_OK, CNMF_EINVAL, CNMF_ENOMEM, CNMF_EDEVICE, CNMF_EBREAKDOWN, CNMF_ENOTSUP, CNMF_EBUSY = 0, -1, -2, -3, -4, -5, -6
CNMF_F64, CNMF_F32, CNMF_BF16, CNMF_FP8_E4M3 = 0, 1, 2, 3
CNMF_LEFT, CNMF_RIGHT, CNMF_BOTH = 1, 2, 3
CNMF_ADMM, CNMF_MU, CNMF_ADMM_FULL, CNMF_MU_FULL, CNMF_ANLS, CNMF_ANLS_FULL = 0, 1, 2, 3, 4, 5
CNMF_SERVER_GRAPHS, CNMF_SERVER_ONE_STEP = 1, 2
CNMF_DENSE, CNMF_DENSE_HOST, CNMF_CSR = 0, 1, 2
CNMF_TEST_GAUSSIAN, CNMF_TEST_SRHT = 0, 1

STATUS_NAMES = {0: "CNMF_OK", -1: "CNMF_EINVAL", -2: "CNMF_ENOMEM", -3: "CNMF_EDEVICE",
                -4: "CNMF_EBREAKDOWN", -5: "CNMF_ENOTSUP", -6: "CNMF_EBUSY"}

# every symbol include/cnmf.h declares (checked by the CPU test-suite)
EXPORTED = [
    "cnmf_create", "cnmf_destroy", "cnmf_last_error", "cnmf_status_string", "cnmf_version",
    "cnmf_sketch", "cnmf_factorize", "snmf_select", "cnmf_spa", "cnmf_workspace_bytes",
    "cnmf_factorize_capture", "cnmf_graph_launch", "cnmf_graph_destroy",
    "cnmf_set_timing", "cnmf_stage_ms", "cnmf_range_product", "cnmf_stage_flops", "cnmf_stage_launches",
    "cnmf_range_product_lowp", "cnmf_synchronize", "cnmf_gaussian", "cnmf_srht", "cnmf_spa_noalloc", "snmf_nnls",
    "cnmf_server_start", "cnmf_server_submit", "cnmf_server_poll", "cnmf_server_release",
    "cnmf_server_get_stats", "cnmf_server_stop", "cnmf_server_last_error", "cnmf_server_simulate",
]


class cnmf_input(C.Structure):
    _fields_ = [("data_dev", C.c_void_p), ("dtype", C.c_int), ("m", C.c_int64), ("n", C.c_int64),
                ("lda", C.c_int64), ("format", C.c_int32), ("reserved", C.c_int32), ("rowptr_dev", C.c_void_p),
                ("colind_dev", C.c_void_p), ("nnz", C.c_int64), ("block_rows", C.c_int64)]


class cnmf_sketch_desc(C.Structure):
    _fields_ = [("r", C.c_int32), ("k", C.c_int32), ("q", C.c_int32), ("sides", C.c_int32),
                ("pass_dtype", C.c_int), ("final_dtype", C.c_int), ("seed", C.c_uint64),
                ("omega_left_dev", C.c_void_p), ("omega_right_dev", C.c_void_p), ("test_matrix", C.c_int32),
                ("reserved", C.c_int32)]


class cnmf_sketch_out(C.Structure):
    _fields_ = [("L_dev", C.c_void_p), ("R_dev", C.c_void_p), ("B_dev", C.c_void_p),
                ("At_dev", C.c_void_p), ("Ac_dev", C.c_void_p), ("stats_dev", C.c_void_p)]


class cnmf_factorize_desc(C.Structure):
    _fields_ = [("sk", cnmf_sketch_desc), ("method", C.c_int32), ("iters", C.c_int32),
                ("lambda_", C.c_double), ("phi", C.c_double), ("xi", C.c_double), ("mu_eps", C.c_double),
                ("U0_dev", C.c_void_p), ("V0_dev", C.c_void_p)]


class cnmf_factorize_out(C.Structure):
    _fields_ = [("U_dev", C.c_void_p), ("V_dev", C.c_void_p), ("rel_residual_dev", C.c_void_p),
                ("sk_out", cnmf_sketch_out)]


class cnmf_server_config(C.Structure):
    _fields_ = [("device", C.c_int32), ("max_batch", C.c_int32), ("workers", C.c_int32), ("flags", C.c_int32),
                ("hbm_budget_bytes", C.c_uint64)]


class cnmf_ticket_info(C.Structure):
    _fields_ = [("state", C.c_int32), ("done", C.c_int32), ("status", C.c_int), ("reserved", C.c_int32),
                ("queue_ms", C.c_double), ("total_ms", C.c_double), ("message", C.c_char * 192)]


class cnmf_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("batch_steps", C.c_int64), ("batched_iterations", C.c_int64), ("max_batch_seen", C.c_int64),
                ("graph_replays", C.c_int64), ("graphs_built", C.c_int64),
                ("queued", C.c_int64), ("in_flight", C.c_int64), ("arena_bytes", C.c_uint64),
                ("arena_free_bytes", C.c_uint64), ("peak_arena_bytes", C.c_uint64)]


class CnmfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libcnmf.so (once).  Raises FileNotFoundError if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with `python -m paper_1505_04650_amd.build` "
            "(there is no non-HIP fallback)")
    lib = C.CDLL(path)
    vp, i32, i64, st = C.c_void_p, C.c_int32, C.c_int64, C.c_int
    lib.cnmf_create.argtypes = [C.c_int, vp, C.c_size_t, C.POINTER(vp)]
    lib.cnmf_create.restype = st
    lib.cnmf_destroy.argtypes = [vp]
    lib.cnmf_destroy.restype = st
    lib.cnmf_last_error.argtypes = [vp]
    lib.cnmf_last_error.restype = C.c_char_p
    lib.cnmf_status_string.argtypes = [st]
    lib.cnmf_status_string.restype = C.c_char_p
    lib.cnmf_version.argtypes = []
    lib.cnmf_version.restype = C.c_char_p
    lib.cnmf_synchronize.argtypes = [vp]
    lib.cnmf_synchronize.restype = st
    lib.cnmf_gaussian.argtypes = [vp, C.c_uint64, i32, i64, i32, vp, i64]
    lib.cnmf_gaussian.restype = st
    lib.cnmf_srht.argtypes = [vp, C.c_uint64, i32, i64, i32, vp, i64]
    lib.cnmf_srht.restype = st
    lib.cnmf_sketch.argtypes = [vp, C.POINTER(cnmf_input), C.POINTER(cnmf_sketch_desc), C.POINTER(cnmf_sketch_out)]
    lib.cnmf_sketch.restype = st
    lib.cnmf_factorize.argtypes = [vp, C.POINTER(cnmf_input), C.POINTER(cnmf_factorize_desc),
                                   C.POINTER(cnmf_factorize_out)]
    lib.cnmf_factorize.restype = st
    lib.cnmf_factorize_capture.argtypes = [vp, C.POINTER(cnmf_input), C.POINTER(cnmf_factorize_desc),
                                           C.POINTER(cnmf_factorize_out), C.POINTER(vp)]
    lib.cnmf_factorize_capture.restype = st
    lib.cnmf_graph_launch.argtypes = [vp]
    lib.cnmf_graph_launch.restype = st
    lib.cnmf_graph_destroy.argtypes = [vp]
    lib.cnmf_graph_destroy.restype = st
    lib.snmf_select.argtypes = [vp, C.POINTER(cnmf_input), C.POINTER(cnmf_sketch_desc), vp, vp, vp]
    lib.snmf_select.restype = st
    lib.cnmf_spa.argtypes = [vp, vp, st, i64, i64, i64, i32, vp, vp]
    lib.cnmf_spa.restype = st
    lib.cnmf_spa_noalloc.argtypes = [vp, vp, st, i64, i64, i64, i32, vp, vp]
    lib.cnmf_spa_noalloc.restype = st
    lib.snmf_nnls.argtypes = [vp, vp, st, i64, i64, i64, i32, vp, vp, i64, vp]
    lib.snmf_nnls.restype = st
    lib.cnmf_workspace_bytes.argtypes = [i64, i64, C.POINTER(cnmf_factorize_desc), C.POINTER(C.c_size_t)]
    lib.cnmf_workspace_bytes.restype = st
    lib.cnmf_range_product.argtypes = [vp, C.POINTER(cnmf_input), C.c_int, vp, i32, vp]
    lib.cnmf_range_product.restype = st
    lib.cnmf_range_product_lowp.argtypes = [vp, C.POINTER(cnmf_input), C.c_int, C.c_int, vp, i32, vp]
    lib.cnmf_range_product_lowp.restype = st
    lib.cnmf_set_timing.argtypes = [vp, C.c_int]
    lib.cnmf_set_timing.restype = st
    lib.cnmf_stage_ms.argtypes = [vp, C.c_int]
    lib.cnmf_stage_ms.restype = C.c_double
    lib.cnmf_stage_flops.argtypes = [vp, C.c_int]
    lib.cnmf_stage_flops.restype = C.c_double
    lib.cnmf_stage_launches.argtypes = [vp, C.c_int]
    lib.cnmf_stage_launches.restype = C.c_int
    lib.cnmf_server_start.argtypes = [C.POINTER(cnmf_server_config), C.POINTER(vp)]
    lib.cnmf_server_start.restype = st
    lib.cnmf_server_submit.argtypes = [vp, C.POINTER(cnmf_input), C.POINTER(cnmf_factorize_desc),
                                       C.POINTER(cnmf_factorize_out), vp, C.POINTER(C.c_uint64)]
    lib.cnmf_server_submit.restype = st
    lib.cnmf_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(cnmf_ticket_info)]
    lib.cnmf_server_poll.restype = st
    lib.cnmf_server_release.argtypes = [vp, C.c_uint64]
    lib.cnmf_server_release.restype = st
    lib.cnmf_server_get_stats.argtypes = [vp, C.POINTER(cnmf_server_stats)]
    lib.cnmf_server_get_stats.restype = st
    lib.cnmf_server_stop.argtypes = [vp]
    lib.cnmf_server_stop.restype = st
    lib.cnmf_server_last_error.argtypes = []
    lib.cnmf_server_last_error.restype = C.c_char_p
    dp, u64p = C.POINTER(C.c_double), C.POINTER(C.c_uint64)
    lib.cnmf_server_simulate.argtypes = [i32, dp, u64p, dp, C.c_uint64, i32, dp, dp, u64p]
    lib.cnmf_server_simulate.restype = st
    _lib = lib
    return lib


def check(status: int, handle=None):
    if status != CNMF_OK:
        msg = load().cnmf_last_error(handle).decode()
        raise CnmfError(status, msg)


def check_server(status: int):
    if status != CNMF_OK:
        raise CnmfError(status, load().cnmf_server_last_error().decode())
