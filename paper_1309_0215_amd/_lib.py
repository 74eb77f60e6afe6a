"""ctypes declarations of the C ABI in include/mr.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmr.so")

MR_OK = 0
MR_ERR_INVALID_ARG = -1
MR_ERR_CAPACITY = -2
MR_ERR_OVERFLOW = -3
MR_ERR_HIP = -4
MR_ERR_UNSUPPORTED = -5
MR_ERR_NO_DEVICE = -6

MAP_WORDS, MAP_U32_KEYS, MAP_U32_KV, MAP_RGB_HIST, MAP_KMEANS, MAP_BLOOM, MAP_LINKS = range(7)
REDUCE_COUNT, REDUCE_SUM, REDUCE_MIN, REDUCE_MAX = range(4)
STRAT_RULE, STRAT_LEARNED, STRAT_LDS_ARRAY, STRAT_GLOBAL_ARRAY, STRAT_HASH, STRAT_SORT = range(6)

N_FEATURES = 12
N_STRATS = 4
MLP_PARAMS = 5252

EXPORTS = [
    "mr_status_str", "mr_last_error", "mr_job_create", "mr_job_destroy", "mr_run", "mr_batch_run",
    "mr_job_features", "mr_selector_set", "mr_selector_predict", "mr_mlp_forward", "mr_mlp_loss_backward",
    "mr_mlp_adam", "mr_tune_set", "mr_rgb_hist_static", "mr_workspace_bytes", "mr_selector_load",
    "mr_selector_train", "mr_hash_words",
]


class JobConfig(C.Structure):
    _fields_ = [
        ("device", C.c_int32),
        ("stream", C.c_void_p),
        ("strategy", C.c_int),
        ("lds_slots", C.c_uint32),
        ("max_load_pct", C.c_uint32),
        ("tile_bytes", C.c_uint32),
        ("debug_hash", C.c_uint32),
        ("table_slots", C.c_uint64),
        ("timing", C.c_uint32),
        ("km_d", C.c_uint32),
        ("km_k", C.c_uint32),
        ("km_centroids", C.c_void_p),
        ("bloom_k", C.c_uint32),
        ("bloom_hashes", C.c_uint32),
        ("wave_combine", C.c_uint32),
        ("workspace", C.c_void_p),
        ("workspace_bytes", C.c_uint64),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("strategy_used", C.c_uint32),
        ("retries", C.c_uint32),
        ("table_slots", C.c_uint64),
        ("n_items", C.c_uint64),
        ("gpu_ms", C.c_float),
        ("map_ms", C.c_float),
        ("km_rechecked", C.c_uint32),
        ("selector_used", C.c_uint32),
        ("device_allocs", C.c_uint32),
        ("sort_spills", C.c_uint32),
        ("workspace_needed", C.c_uint64),
    ]


class Output(C.Structure):
    _fields_ = [
        ("keys", C.c_void_p),
        ("key_bytes", C.c_void_p),
        ("key_offsets", C.c_void_p),
        ("values", C.c_void_p),
        ("assign", C.c_void_p),
        ("sums", C.c_void_p),
        ("counts", C.c_void_p),
        ("centroids", C.c_void_p),
        ("cap_keys", C.c_uint64),
        ("cap_key_bytes", C.c_uint64),
        ("n_keys", C.c_uint64),
        ("key_bytes_used", C.c_uint64),
        ("status", C.c_int32),
        ("stats", Stats),
        ("list_offsets", C.c_void_p),
        ("list_ids", C.c_void_p),
        ("cap_list_ids", C.c_uint64),
        ("n_list_ids", C.c_uint64),
    ]


class TuneEntry(C.Structure):
    _fields_ = [
        ("kind", C.c_int),
        ("bytes_lo", C.c_uint64),
        ("bytes_hi", C.c_uint64),
        ("lds_slots", C.c_uint32),
        ("max_load_pct", C.c_uint32),
        ("map_grid_pct", C.c_uint32),
        ("lds_array_bytes", C.c_uint32),
    ]


class TrainConfig(C.Structure):
    _fields_ = [
        ("epochs", C.c_uint32),
        ("batch", C.c_uint32),
        ("lr", C.c_float),
        ("beta1", C.c_float),
        ("beta2", C.c_float),
        ("eps", C.c_float),
        ("seed", C.c_uint64),
    ]


class BatchItem(C.Structure):
    _fields_ = [
        ("kind", C.c_int),
        ("op", C.c_int),
        ("d_input", C.c_void_p),
        ("input_bytes", C.c_uint64),
        ("d_record_offsets", C.c_void_p),
        ("n_records", C.c_uint64),
        ("key_range", C.c_uint64),
    ]


_lib = None


def load(required: bool = True):
    """Load libmr.so. Raises when it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if required:
            raise RuntimeError(f"{LIB_PATH} is not built: run python -m paper_1309_0215_amd.build")
        return None
    lib = C.CDLL(LIB_PATH)
    P, U32, U64, I32, F = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32, C.c_float
    lib.mr_status_str.restype = C.c_char_p
    lib.mr_status_str.argtypes = [I32]
    lib.mr_last_error.restype = C.c_char_p
    lib.mr_last_error.argtypes = []
    lib.mr_job_create.restype = I32
    lib.mr_job_create.argtypes = [C.POINTER(JobConfig), C.POINTER(P)]
    lib.mr_job_destroy.restype = I32
    lib.mr_job_destroy.argtypes = [P]
    lib.mr_run.restype = I32
    lib.mr_run.argtypes = [P, C.c_int, C.c_int, P, U64, P, U64, U64, C.POINTER(Output)]
    lib.mr_batch_run.restype = I32
    lib.mr_batch_run.argtypes = [P, C.POINTER(BatchItem), U32, C.POINTER(Output)]
    lib.mr_tune_set.restype = I32
    lib.mr_tune_set.argtypes = [P, C.POINTER(TuneEntry), U32]
    lib.mr_rgb_hist_static.restype = I32
    lib.mr_rgb_hist_static.argtypes = [P, P, U64, P]
    lib.mr_workspace_bytes.restype = I32
    lib.mr_workspace_bytes.argtypes = [C.POINTER(JobConfig), C.c_int, U64, U64, C.POINTER(U64)]
    lib.mr_selector_load.restype = I32
    lib.mr_selector_load.argtypes = [P, C.c_char_p]
    lib.mr_hash_words.restype = I32
    lib.mr_hash_words.argtypes = [P, P, U64, U32, U32, U32, P, P, U64, C.POINTER(U64), C.POINTER(C.c_float)]
    lib.mr_selector_train.restype = I32
    lib.mr_selector_train.argtypes = [P, P, P, P, U32, C.POINTER(TrainConfig), P, C.c_char_p]
    if hasattr(lib, "mr_job_features"):
        lib.mr_job_features.restype = I32
        lib.mr_job_features.argtypes = [P, C.c_int, C.c_int, P, U64, U64, P]
        lib.mr_selector_set.restype = I32
        lib.mr_selector_set.argtypes = [P, P, P, P, P, P]
        lib.mr_selector_predict.restype = I32
        lib.mr_selector_predict.argtypes = [P, P, P]
        lib.mr_mlp_forward.restype = I32
        lib.mr_mlp_forward.argtypes = [P, P, P, U32, P, P, P]
        lib.mr_mlp_loss_backward.restype = I32
        lib.mr_mlp_loss_backward.argtypes = [P, P, P, P, P, P, P, P, U32, P, P]
        lib.mr_mlp_adam.restype = I32
        lib.mr_mlp_adam.argtypes = [P, P, P, P, P, U32, F, F, F, F]
    _lib = lib
    return lib


class MRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} ({status})")
        self.status = status


def check(status: int, what: str = ""):
    if status != MR_OK:
        lib = load()
        raise MRError(status, f"{what}: {lib.mr_status_str(status).decode()}: {lib.mr_last_error().decode()}")
