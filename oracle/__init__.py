"""CPU oracle for affine-gap read alignment and few-mismatch search -- test
infrastructure only.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.  ``gotoh.c`` holds the DP arithmetic (full int32 H,
D and I matrices, best cell, traceback); ``kmm.c`` the few-mismatch search
as its definition (every placement of every read, brute force).  This
module only compiles them with gcc and marshals numpy arrays through
ctypes.

Parity status: pinned (exhaustive enumeration, closed forms, library
routines and invariants; see ``tests/test_oracle_*.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, f) for f in ("gotoh.c", "kmm.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

ST_CIGAR_TRUNC = 1 << 1
ST_LEN_LIMIT = 1 << 2
ST_WIN_OOB = 1 << 3
ST_READ_OOB = 1 << 4
ST_REPETITIVE = 1 << 6

SEMIGLOBAL = 0
LOCAL = 1
EXTEND = 2

DEFAULT_SCORING = (1, -4, 6, 1)  # match, mismatch, gap open, gap extend


def build(force: bool = False) -> str:
    """Compile gotoh.c and kmm.c into liboracle.so with gcc -O2 (plain C, no intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(s) for s in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-pthread"] + _SRCS + ["-o", tmp]
        )
        os.replace(tmp, _LIB)
    return _LIB


def bind(lib):
    """Declare the C entry points of a loaded oracle library (also used by tests
    that load modified builds)."""
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int32
    lib.oracle_align_batch.restype = ctypes.c_int
    lib.oracle_align_batch.argtypes = [
        P, i64, P, P, P, i64, P, P, P, i32, i64,
        i32, i32, i32, i32, i32, i32,
        P, P, P, P, P, P, P, P, i32,
    ]
    lib.oracle_align_batch_ext.restype = ctypes.c_int
    lib.oracle_align_batch_ext.argtypes = [
        P, i64, P, P, P, i64, P, P, P, i32, P, i32, i32, i64,
        i32, i32, i32, i32, i32, i32,
        P, P, P, P, P, P, P, P, i32,
    ]
    if hasattr(lib, "oracle_kmm_search"):
        lib.oracle_kmm_search.restype = ctypes.c_int
        lib.oracle_kmm_search.argtypes = [P, i64, P, i64, P, P, i64, i32, i32, P, P, P, P, P, i32]
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            _lib = bind(ctypes.CDLL(_LIB))
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def align_batch(ref, win_off, win_len, reads, read_off, read_len, mode=None,
                scoring=DEFAULT_SCORING, trace=False, cigar_cap=64, default_mode=SEMIGLOBAL,
                threads=None, h0=None, default_h0=0, clip=0):
    """Align every (read, window) pair exactly.

    ``ref`` and ``reads`` hold one base code (A0 C1 G2 T3) per byte.  Pair p
    aligns ``reads[read_off[p]:read_off[p]+read_len[p]]`` against
    ``ref[win_off[p]:win_off[p]+win_len[p]]``.  Returns a dict of numpy arrays:
    score, read_end, ref_end, status and, with ``trace``, read_start,
    ref_start, cigar (n_pairs x cigar_cap words ``len<<4 | op``; M=0, I=1,
    D=2) and n_cigar.  Coordinates are 0-based, half-open, window-relative.
    Extension pairs (mode 2) start from score ``h0[p]`` (or ``default_h0``)
    and are clipped unless aligning the whole read scores within ``clip`` of
    the best early end.
    """
    lib = _load()
    ref = np.ascontiguousarray(ref, dtype=np.uint8)
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    win_off = np.ascontiguousarray(win_off, dtype=np.int64)
    win_len = np.ascontiguousarray(win_len, dtype=np.int32)
    read_off = np.ascontiguousarray(read_off, dtype=np.int64)
    read_len = np.ascontiguousarray(read_len, dtype=np.int32)
    n = len(win_off)
    assert len(win_len) == n and len(read_off) == n and len(read_len) == n
    if mode is not None:
        mode = np.ascontiguousarray(mode, dtype=np.uint8)
        assert len(mode) == n
    if h0 is not None:
        h0 = np.ascontiguousarray(h0, dtype=np.int32)
        assert len(h0) == n
    a, b, o, e = (int(x) for x in scoring)
    out = {
        "score": np.zeros(n, np.int32),
        "read_end": np.zeros(n, np.int32),
        "ref_end": np.zeros(n, np.int32),
        "status": np.zeros(n, np.uint32),
    }
    if trace:
        out["read_start"] = np.zeros(n, np.int32)
        out["ref_start"] = np.zeros(n, np.int32)
        out["cigar"] = np.zeros((n, max(cigar_cap, 0)), np.uint32)
        out["n_cigar"] = np.zeros(n, np.int32)
    if threads is None:
        threads = os.cpu_count() or 1
    rc = lib.oracle_align_batch_ext(
        _ptr(ref), len(ref), _ptr(win_off), _ptr(win_len), _ptr(reads), len(reads),
        _ptr(read_off), _ptr(read_len), _ptr(mode), int(default_mode), _ptr(h0), int(default_h0), int(clip), n,
        a, b, o, e, 1 if trace else 0, int(cigar_cap),
        _ptr(out["score"]), _ptr(out.get("read_start")), _ptr(out["read_end"]),
        _ptr(out.get("ref_start")), _ptr(out["ref_end"]), _ptr(out.get("cigar")),
        _ptr(out.get("n_cigar")), _ptr(out["status"]), int(threads),
    )
    if rc != 0:
        raise ValueError("oracle rejected the scoring or batch arguments")
    return out


def align_pairs(pairs, mode=SEMIGLOBAL, scoring=DEFAULT_SCORING, trace=True, cigar_cap=4096,
                threads=1, h0=None, default_h0=0, clip=0):
    """Convenience wrapper: ``pairs`` is a list of (read_codes, window_codes)."""
    reads = [np.asarray(q, np.uint8) for q, _ in pairs]
    wins = [np.asarray(r, np.uint8) for _, r in pairs]
    read_len = np.array([len(q) for q in reads], np.int32)
    win_len = np.array([len(r) for r in wins], np.int32)
    read_off = np.concatenate([[0], np.cumsum(read_len)[:-1]]).astype(np.int64) if pairs else np.zeros(0, np.int64)
    win_off = np.concatenate([[0], np.cumsum(win_len)[:-1]]).astype(np.int64) if pairs else np.zeros(0, np.int64)
    R = np.concatenate(reads) if reads else np.zeros(0, np.uint8)
    W = np.concatenate(wins) if wins else np.zeros(0, np.uint8)
    modes = np.full(len(pairs), mode, np.uint8) if np.isscalar(mode) else np.asarray(mode, np.uint8)
    return align_batch(W, win_off, win_len, R, read_off, read_len, modes, scoring, trace,
                       cigar_cap, threads=threads, h0=h0, default_h0=default_h0, clip=clip)


def decode_cigar(words, n):
    """CIGAR words -> string such as '4M1D4M' (test helper)."""
    return "".join("%d%s" % (int(w) >> 4, "MID"[int(w) & 15]) for w in words[:n])


def kmm_search(ref, reads, read_off, read_len, k=2, max_occ=64, threads=None):
    """Few-mismatch search by its definition: for every read, every position
    p <= L - m whose placement has at most ``k`` mismatches.

    ``ref`` and ``reads`` hold one base code per byte.  Returns a dict of
    numpy arrays: best_mm (smallest mismatch count, -1 without hits),
    n_best (hits with that count), n_hits (all hits), pos (leftmost hit with
    the smallest count, -1 without) and status (ST_LEN_LIMIT, ST_READ_OOB,
    ST_REPETITIVE when one of the k + 1 parts occurs more than ``max_occ``
    times).
    """
    lib = _load()
    ref = np.ascontiguousarray(ref, dtype=np.uint8)
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    read_off = np.ascontiguousarray(read_off, dtype=np.int64)
    read_len = np.ascontiguousarray(read_len, dtype=np.int32)
    n = len(read_off)
    assert len(read_len) == n
    out = {"best_mm": np.zeros(n, np.int32), "n_best": np.zeros(n, np.int32), "n_hits": np.zeros(n, np.int32),
           "pos": np.zeros(n, np.int64), "status": np.zeros(n, np.uint32)}
    if threads is None:
        threads = os.cpu_count() or 1
    rc = lib.oracle_kmm_search(_ptr(ref), len(ref), _ptr(reads), len(reads), _ptr(read_off), _ptr(read_len), n,
                               int(k), int(max_occ), _ptr(out["best_mm"]), _ptr(out["n_best"]),
                               _ptr(out["n_hits"]), _ptr(out["pos"]), _ptr(out["status"]), int(threads))
    if rc != 0:
        raise ValueError("oracle rejected k or max_occ")
    return out
