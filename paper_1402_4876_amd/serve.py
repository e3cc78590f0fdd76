"""Python binding of the serving loop (mica_server_* in include/mica_dp.h).

Argument marshalling only: the server, its batching and its statistics live in
libmica_dp.so.  Inputs are host numpy arrays (copied by the library on
submit); outputs come back as numpy arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _lib


def _arr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


class Server:
    """A resident-reference DP server on one GPU.

    ref_words: uint32 2-bit packed reference (ref_len bases); slots: in-flight
    batches; fifo: one request per batch (the no-batching baseline).
    """

    def __init__(self, ref_words, ref_len, device=0, hbm_budget_bytes=0, slots=4, scoring=(1, -4, 6, 1),
                 out_cigar=True, fifo=False):
        lib = _lib.load()
        self._ref, rp = _arr(ref_words, np.uint32)
        sc = _lib.Scoring(*(int(x) for x in scoring))
        flags = (_lib.OUT_CIGAR | _lib.OUT_START if out_cigar else 0) | (_lib.SERVE_FIFO if fifo else 0)
        h = ctypes.c_void_p()
        _lib.check(lib.mica_server_create(int(device), rp, int(ref_len), int(hbm_budget_bytes), int(slots),
                                          ctypes.byref(sc), flags, ctypes.byref(h)))
        self._h = h
        self.out_cigar = out_cigar
        self._n = {}

    def now(self):
        t = ctypes.c_double()
        _lib.check(_lib.load().mica_server_now(self._h, ctypes.byref(t)))
        return t.value

    def submit(self, request_id, reads_words, read_off, read_len, win_off, win_len, mode=None, arrival=-1.0):
        n = len(read_len)
        rw, rwp = _arr(reads_words, np.uint32)
        ro, rop = _arr(read_off, np.uint64)
        rl, rlp = _arr(read_len, np.int32)
        wo, wop = _arr(win_off, np.uint64)
        wl, wlp = _arr(win_len, np.int32)
        mp = None
        if mode is not None:
            md, mp = _arr(mode, np.uint8)
        _lib.check(_lib.load().mica_server_submit(self._h, int(request_id), rwp, rop, rlp, wop, wlp, mp, n,
                                                  float(arrival)))
        self._n[int(request_id)] = n

    def replay(self, reads_words, read_off, read_len, win_off, win_len, req_first, req_count, arrival,
               first_id=0, mode=None):
        """Start the library's replay thread: request r is reads req_first[r] ..
        + req_count[r] of the arrays, id first_id + r, submitted at server time
        arrival[r].  The arrays are kept alive until replay_wait()."""
        keep = [_arr(reads_words, np.uint32), _arr(read_off, np.uint64), _arr(read_len, np.int32),
                _arr(win_off, np.uint64), _arr(win_len, np.int32), _arr(req_first, np.int64),
                _arr(req_count, np.int64), _arr(arrival, np.float64)]
        mp = None
        if mode is not None:
            md = _arr(mode, np.uint8)
            keep.append(md)
            mp = md[1]
        n = len(keep[5][0])
        _lib.check(_lib.load().mica_server_replay(self._h, keep[0][1], keep[1][1], keep[2][1], keep[3][1], keep[4][1],
                                                  mp, keep[5][1], keep[6][1], keep[7][1], n, int(first_id)))
        self._replay_keep = keep
        for r in range(n):
            self._n[int(first_id) + r] = int(keep[6][0][r])

    def replay_wait(self):
        """Wait for the replay thread; returns how far (seconds) the latest
        submission ran behind its scheduled time."""
        lag = ctypes.c_double()
        try:
            _lib.check(_lib.load().mica_server_replay_wait(self._h, ctypes.byref(lag)))
        finally:
            self._replay_keep = None
        return lag.value

    def load_plan(self, path):
        """Give every slot the kernel plan in `path` (Context.save_plan); waits
        for the queued and running batches, holds submissions meanwhile."""
        _lib.check(_lib.load().mica_server_load_plan(self._h, os.fsencode(path)))

    def poll(self, cap=4096):
        ids = np.zeros(cap, np.uint64)
        k = ctypes.c_int64()
        _lib.check(_lib.load().mica_server_poll(self._h, ids.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(k)))
        return [int(x) for x in ids[:k.value]]

    def fetch(self, request_id, cigar_cap=64, out=None):
        """Outputs of a finished request as numpy arrays.  ``out`` may hold
        preallocated arrays (at least n entries each, cigar rows of cigar_cap
        words) to fill instead of new ones; CIGAR words past a read's runs are
        left as they were."""
        n = self._n.get(int(request_id), 0)  # unknown ids: the library reports the error
        keys = ("score", "read_start", "read_end", "ref_start", "ref_end", "n_cigar", "status")
        cap = cigar_cap if self.out_cigar else 0
        if out is None:
            out = {k: np.empty(n, np.int32) for k in keys}
            out["cigar"] = np.zeros((n, max(cap, 1)), np.uint32)
        else:
            out = {k: out[k][:n] for k in keys + ("cigar",)}
            if out["cigar"].shape[1] != max(cap, 1):
                raise ValueError("out['cigar'] rows must have cigar_cap words")
        p = {k: v.ctypes.data_as(ctypes.c_void_p) for k, v in out.items()}
        _lib.check(_lib.load().mica_server_fetch(self._h, int(request_id), p["score"], p["read_start"],
                                                 p["read_end"], p["ref_start"], p["ref_end"], p["cigar"], cap,
                                                 p["n_cigar"], p["status"]))
        self._n.pop(int(request_id), None)
        out["status"] = out["status"].view(np.uint32)
        if not self.out_cigar:
            del out["cigar"]
        return out

    def forget(self, request_id):
        """Drop a finished request's outputs without copying them."""
        _lib.check(_lib.load().mica_server_fetch(self._h, int(request_id), None, None, None, None, None, None, 0,
                                                 None, None))
        self._n.pop(int(request_id), None)

    def stats(self):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _lib.check(_lib.load().mica_server_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"p50_s": a.value, "p99_s": b.value, "gcups": c.value}

    def reset_stats(self):
        _lib.check(_lib.load().mica_server_reset_stats(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().mica_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
