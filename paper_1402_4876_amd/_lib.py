"""ctypes declarations of the C ABI in include/mica_dp.h.

The shared library is built in-tree (libmica_dp.so next to this file).  There
is no fallback: importing the binding without the built library raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# MICA_LIB_PATH selects another build of the library (e.g. a variant being timed)
LIB_PATH = os.environ.get("MICA_LIB_PATH") or os.path.join(HERE, "libmica_dp.so")

OK = 0
STATUS_NAMES = {0: "MICA_OK", -1: "MICA_ERR_INVALID_ARG", -2: "MICA_ERR_LIMIT",
                -3: "MICA_ERR_OUT_OF_MEMORY", -4: "MICA_ERR_HIP", -5: "MICA_ERR_BUSY"}

MODE_SEMIGLOBAL = 0
MODE_LOCAL = 1
MODE_EXTEND = 2
OUT_START = 1 << 0
OUT_CIGAR = 1 << 1
FORCE_INT32 = 1 << 8
PLAIN_LAUNCH = 1 << 9
NO_GRAPH = 1 << 10
SERVE_FIFO = 1 << 16

ST_SATURATED = 1 << 0
ST_CIGAR_TRUNC = 1 << 1
ST_LEN_LIMIT = 1 << 2
ST_WIN_OOB = 1 << 3
ST_READ_OOB = 1 << 4
ST_INTERNAL = 1 << 5
ST_REPETITIVE = 1 << 6

MAX_READ_LEN = 1024
MAX_WIN_LEN = 8192
NOALLOC_MAX_PAIRS = 1 << 22
NOALLOC_SCRATCH_BYTES = 256 << 20

EXPORTS = ("mica_ctx_create", "mica_ctx_destroy", "mica_dp_align_batch", "mica_pack_2bit",
           "mica_ctx_set_plan", "mica_ctx_last_stats", "mica_ctx_set_timing", "mica_ctx_read_timing",
           "mica_ctx_autotune", "mica_ctx_save_plan", "mica_ctx_load_plan", "mica_server_create",
           "mica_server_now", "mica_server_submit", "mica_server_poll", "mica_server_fetch", "mica_server_stats",
           "mica_server_reset_stats", "mica_server_destroy", "mica_last_error", "mica_fm_suffix_array",
           "mica_fm_create", "mica_fm_destroy", "mica_fm_info", "mica_fm_search", "mica_pipe_create",
           "mica_pipe_run", "mica_pipe_destroy", "mica_dp_align_batch_noalloc", "mica_measure_valu_peak",
           "mica_server_replay", "mica_server_replay_wait", "mica_server_load_plan")


class Scoring(ctypes.Structure):
    _fields_ = [("match", ctypes.c_int32), ("mismatch", ctypes.c_int32),
                ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32)]


class Batch(ctypes.Structure):
    _fields_ = [
        ("ref2b", ctypes.c_void_p), ("ref_len", ctypes.c_uint64),
        ("win_off", ctypes.c_void_p), ("win_len", ctypes.c_void_p),
        ("reads2b", ctypes.c_void_p), ("reads_len", ctypes.c_uint64),
        ("read_off", ctypes.c_void_p), ("read_len", ctypes.c_void_p),
        ("mode", ctypes.c_void_p), ("default_mode", ctypes.c_int32),
        ("n_pairs", ctypes.c_int64),
        ("max_read_len", ctypes.c_int32), ("max_win_len", ctypes.c_int32),
        ("score", ctypes.c_void_p), ("read_end", ctypes.c_void_p), ("ref_end", ctypes.c_void_p),
        ("read_start", ctypes.c_void_p), ("ref_start", ctypes.c_void_p),
        ("cigar", ctypes.c_void_p), ("cigar_cap", ctypes.c_int32),
        ("n_cigar", ctypes.c_void_p), ("status", ctypes.c_void_p),
        ("ext_h0", ctypes.c_void_p), ("ext_default_h0", ctypes.c_int32), ("ext_clip", ctypes.c_int32),
        ("mode_mask", ctypes.c_int32), ("min_read_len", ctypes.c_int32), ("max_ext_h0", ctypes.c_int32),
    ]


class BatchStats(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int64), ("n_items", ctypes.c_int64),
                ("n_saturated", ctypes.c_int64), ("n_waves", ctypes.c_int64),
                ("scratch_bytes", ctypes.c_int64), ("n_fallback", ctypes.c_int64),
                ("n_deferred", ctypes.c_int64)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("m_lo", ctypes.c_int32), ("m_hi", ctypes.c_int32), ("lanes", ctypes.c_int32),
                ("rows", ctypes.c_int32), ("n_pairs", ctypes.c_int32), ("n_candidates", ctypes.c_int32),
                ("n_rejected", ctypes.c_int32), ("pad_", ctypes.c_int32), ("ms", ctypes.c_double),
                ("default_ms", ctypes.c_double)]


_lib = None


class FmBatch(ctypes.Structure):
    """mica_fm_batch_t of include/mica_fm.h."""
    _fields_ = [
        ("reads2b", ctypes.c_void_p), ("reads_len", ctypes.c_uint64), ("read_off", ctypes.c_void_p),
        ("read_len", ctypes.c_void_p), ("n_reads", ctypes.c_int64), ("k", ctypes.c_int32),
        ("max_occ", ctypes.c_int32), ("best_mm", ctypes.c_void_p), ("n_best", ctypes.c_void_p),
        ("n_hits", ctypes.c_void_p), ("pos", ctypes.c_void_p), ("status", ctypes.c_void_p),
        ("cand", ctypes.c_void_p),
    ]


class PipeParams(ctypes.Structure):
    """mica_pipe_params_t of include/mica_pipe.h."""
    _fields_ = [("k", ctypes.c_int32), ("max_occ", ctypes.c_int32), ("band", ctypes.c_int32),
                ("min_score", ctypes.c_int32), ("batch_reads", ctypes.c_int32), ("format_threads", ctypes.c_int32),
                ("scoring", Scoring)]


class PipeStats(ctypes.Structure):
    """mica_pipe_stats_t of include/mica_pipe.h."""
    _fields_ = [("reads", ctypes.c_int64), ("batches", ctypes.c_int64), ("mapped_search", ctypes.c_int64),
                ("mapped_dp", ctypes.c_int64), ("unmapped", ctypes.c_int64), ("non_acgt", ctypes.c_int64),
                ("repetitive", ctypes.c_int64), ("seconds", ctypes.c_double), ("parse_seconds", ctypes.c_double),
                ("gpu_seconds", ctypes.c_double), ("format_seconds", ctypes.c_double)]


def load():
    """Load libmica_dp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmica_dp.so is not built (%s); run __graft_entry__.build() "
                          "or python -m paper_1402_4876_amd.build" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
    lib.mica_ctx_create.argtypes = [ctypes.c_int, sz, ctypes.POINTER(P)]
    lib.mica_ctx_create.restype = ctypes.c_int
    lib.mica_ctx_destroy.argtypes = [P]
    lib.mica_ctx_destroy.restype = ctypes.c_int
    lib.mica_dp_align_batch.argtypes = [P, ctypes.POINTER(Batch), ctypes.POINTER(Scoring), u32, P]
    lib.mica_dp_align_batch.restype = ctypes.c_int
    lib.mica_dp_align_batch_noalloc.argtypes = [ctypes.POINTER(Batch), ctypes.POINTER(Scoring), u32, P]
    lib.mica_dp_align_batch_noalloc.restype = ctypes.c_int
    lib.mica_measure_valu_peak.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double)]
    lib.mica_measure_valu_peak.restype = ctypes.c_int
    lib.mica_pack_2bit.argtypes = [P, i64, P, P]
    lib.mica_pack_2bit.restype = ctypes.c_int
    lib.mica_ctx_set_plan.argtypes = [P, i32, i32, i32, i32]
    lib.mica_ctx_set_plan.restype = ctypes.c_int
    lib.mica_ctx_last_stats.argtypes = [P, P, ctypes.POINTER(BatchStats)]
    lib.mica_ctx_last_stats.restype = ctypes.c_int
    lib.mica_ctx_set_timing.argtypes = [P, ctypes.c_int]
    lib.mica_ctx_set_timing.restype = ctypes.c_int
    lib.mica_ctx_read_timing.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.mica_ctx_read_timing.restype = ctypes.c_int
    lib.mica_ctx_autotune.argtypes = [P, ctypes.POINTER(Batch), ctypes.POINTER(Scoring), u32, P, i32,
                                       ctypes.POINTER(TuneEntry), i32, ctypes.POINTER(i32)]
    lib.mica_ctx_autotune.restype = ctypes.c_int
    lib.mica_ctx_save_plan.argtypes = [P, ctypes.c_char_p]
    lib.mica_ctx_save_plan.restype = ctypes.c_int
    lib.mica_ctx_load_plan.argtypes = [P, ctypes.c_char_p]
    lib.mica_ctx_load_plan.restype = ctypes.c_int
    D = ctypes.POINTER(ctypes.c_double)
    lib.mica_server_create.argtypes = [ctypes.c_int, P, ctypes.c_uint64, sz, ctypes.c_int, ctypes.POINTER(Scoring),
                                       u32, ctypes.POINTER(P)]
    lib.mica_server_now.argtypes = [P, D]
    lib.mica_server_submit.argtypes = [P, ctypes.c_uint64, P, P, P, P, P, P, i64, ctypes.c_double]
    lib.mica_server_replay.argtypes = [P, P, P, P, P, P, P, P, P, P, i64, ctypes.c_uint64]
    lib.mica_server_replay_wait.argtypes = [P, D]
    lib.mica_server_load_plan.argtypes = [P, ctypes.c_char_p]
    lib.mica_server_poll.argtypes = [P, P, i64, ctypes.POINTER(i64)]
    lib.mica_server_fetch.argtypes = [P, ctypes.c_uint64, P, P, P, P, P, P, i32, P, P]
    lib.mica_server_stats.argtypes = [P, D, D, D]
    lib.mica_server_reset_stats.argtypes = [P]
    lib.mica_server_destroy.argtypes = [P]
    for f in ("create", "now", "submit", "poll", "fetch", "stats", "reset_stats", "destroy"):
        getattr(lib, "mica_server_" + f).restype = ctypes.c_int
    lib.mica_fm_suffix_array.argtypes = [P, ctypes.c_uint64, P]
    lib.mica_fm_create.argtypes = [ctypes.c_int, P, ctypes.c_uint64, ctypes.POINTER(P)]
    lib.mica_fm_destroy.argtypes = [P]
    lib.mica_fm_info.argtypes = [P, ctypes.POINTER(ctypes.c_uint64), D]
    lib.mica_fm_search.argtypes = [P, ctypes.POINTER(FmBatch), P]
    for f in ("suffix_array", "create", "destroy", "info", "search"):
        getattr(lib, "mica_fm_" + f).restype = ctypes.c_int
    lib.mica_pipe_create.argtypes = [ctypes.c_int, P, ctypes.c_uint64, ctypes.c_char_p, ctypes.POINTER(PipeParams),
                                     ctypes.POINTER(P)]
    lib.mica_pipe_run.argtypes = [P, ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(PipeStats)]
    lib.mica_pipe_destroy.argtypes = [P]
    for f in ("create", "run", "destroy"):
        getattr(lib, "mica_pipe_" + f).restype = ctypes.c_int
    lib.mica_last_error.argtypes = []
    lib.mica_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


class MicaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def check(status):
    if status != OK:
        raise MicaError(status, load().mica_last_error().decode(errors="replace"))
