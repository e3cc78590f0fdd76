"""Binding of the few-mismatch search phase (include/mica_fm.h): argument
marshalling only; the index build runs in the library's host code and the
search in its HIP kernel.

    ix = FmIndex(ref_words_host, ref_len)          # build + upload, once
    out = ix.search(reads2b, read_off, read_len, k=2, max_occ=64)
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib


def suffix_array(codes):
    """Suffix array (host, uint32, len(codes) + 1 entries) of a uint8 code
    array followed by a sentinel, by the library's SA-IS."""
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    sa = np.empty(len(codes) + 1, np.uint32)
    _lib.check(_lib.load().mica_fm_suffix_array(codes.ctypes.data if len(codes) else None, len(codes),
                                                sa.ctypes.data))
    return sa


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != dtype or not t.is_contiguous():
        raise TypeError("%s must be a contiguous %s CUDA tensor" % (name, dtype))
    return t


class FmIndex:
    """FM index of a reference on one GPU (suffix array, BWT occurrence
    blocks, padded 2-bit reference)."""

    def __init__(self, ref_words, ref_len, device=0):
        words = np.ascontiguousarray(ref_words, dtype=np.uint32)
        if len(words) * 16 < ref_len:
            raise ValueError("ref_words holds fewer than ref_len bases")
        h = ctypes.c_void_p()
        _lib.check(_lib.load().mica_fm_create(int(device), words.ctypes.data, int(ref_len), ctypes.byref(h)))
        self._h = h
        self.ref_len = int(ref_len)
        self.device = device

    def info(self):
        b = ctypes.c_uint64()
        s = ctypes.c_double()
        _lib.check(_lib.load().mica_fm_info(self._h, ctypes.byref(b), ctypes.byref(s)))
        return {"device_bytes": b.value, "build_seconds": s.value}

    def search(self, reads2b, read_off, read_len, k=2, max_occ=64, reads_len=None, out=None, stream=None,
               cand=False):
        """Search every read with at most ``k`` mismatches; returns a dict of
        tensors best_mm, n_best, n_hits (int32), pos (int64), status (int32
        bits).  Asynchronous on ``stream``."""
        reads2b = _dev(reads2b, torch.int32, "reads2b")
        read_off = _dev(read_off, torch.int64, "read_off")
        read_len = _dev(read_len, torch.int32, "read_len")
        n = read_off.numel()
        if read_len.numel() != n:
            raise ValueError("read_off and read_len differ in length")
        if out is None:
            out = {key: torch.empty(n, dtype=torch.int32, device=reads2b.device)
                   for key in ("best_mm", "n_best", "n_hits", "status")}
            out["pos"] = torch.empty(n, dtype=torch.int64, device=reads2b.device)
        if cand and "cand" not in out:
            out["cand"] = torch.empty((n, 3), dtype=torch.int64, device=reads2b.device)
        b = _lib.FmBatch()
        b.reads2b = reads2b.data_ptr()
        b.reads_len = int(reads_len) if reads_len is not None else reads2b.numel() * 16
        b.read_off = read_off.data_ptr()
        b.read_len = read_len.data_ptr()
        b.n_reads = n
        b.k = int(k)
        b.max_occ = int(max_occ)
        for key in ("best_mm", "n_best", "n_hits", "pos", "status"):
            setattr(b, key, out[key].data_ptr())
        b.cand = out["cand"].data_ptr() if "cand" in out else None
        s = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        if stream is None:
            s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        _lib.check(_lib.load().mica_fm_search(self._h, ctypes.byref(b), s))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().mica_fm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
