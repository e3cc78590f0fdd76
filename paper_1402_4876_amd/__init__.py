"""MI355X-native DP phase of short-read alignment (MICA, Methods / DP section).

Thin Python binding of the C ABI (include/mica_dp.h): argument marshalling
only.  Every step of the alignment runs in the HIP kernels of libmica_dp.so;
PyTorch provides device memory and streams.

    ctx = Context()
    out = align(ctx, ref2b, win_off, win_len, reads2b, read_off, read_len,
                mode=mode, out_cigar=True, max_read_len=150, max_win_len=400)
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (FORCE_INT32, MAX_READ_LEN, MAX_WIN_LEN, MODE_EXTEND, MODE_LOCAL, MODE_SEMIGLOBAL, NO_GRAPH,
                   OUT_CIGAR, OUT_START, PLAIN_LAUNCH, ST_CIGAR_TRUNC, ST_LEN_LIMIT, ST_READ_OOB,
                   ST_REPETITIVE, ST_SATURATED, ST_WIN_OOB, MicaError)
from .fm import FmIndex, suffix_array
from .pack import pack_codes, unpack_words
from .pipe import Pipeline
from .serve import Server

__all__ = ["Context", "Server", "align", "align_noalloc", "measure_valu_peak", "pack_2bit", "pack_codes", "unpack_words", "MicaError", "FORCE_INT32",
           "PLAIN_LAUNCH", "NO_GRAPH", "OUT_START", "OUT_CIGAR", "MODE_LOCAL", "MODE_SEMIGLOBAL", "MODE_EXTEND", "ST_SATURATED",
           "ST_CIGAR_TRUNC", "ST_LEN_LIMIT", "ST_WIN_OOB", "ST_READ_OOB", "ST_REPETITIVE", "MAX_READ_LEN",
           "MAX_WIN_LEN", "FmIndex", "suffix_array", "Pipeline"]


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


class Context:
    """A library context (workspace, plan table) on one GPU."""

    def __init__(self, device=None, workspace_bytes=0):
        lib = _lib.load()
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = ctypes.c_void_p()
        _lib.check(lib.mica_ctx_create(self.device, int(workspace_bytes), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def set_plan(self, m_lo, m_hi, lanes, rows):
        _lib.check(_lib.load().mica_ctx_set_plan(self._h, int(m_lo), int(m_hi), int(lanes), int(rows)))

    def last_stats(self, stream=None):
        st = _lib.BatchStats()
        _lib.check(_lib.load().mica_ctx_last_stats(self._h, _stream_handle(stream), ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def set_timing(self, enable=True):
        """Record HIP events around the fill launches of every later batch."""
        _lib.check(_lib.load().mica_ctx_set_timing(self._h, 1 if enable else 0))

    def read_timing(self):
        """(summed fill milliseconds, number of timed batches) since the last read."""
        ms = ctypes.c_double()
        nb = ctypes.c_int64()
        _lib.check(_lib.load().mica_ctx_read_timing(self._h, ctypes.byref(ms), ctypes.byref(nb)))
        return ms.value, nb.value

    def autotune(self, ref2b, win_off, win_len, reads2b, read_off, read_len, mode=None,
                 scoring=(1, -4, 6, 1), out_start=False, out_cigar=False, cigar_cap=64, force_int32=False,
                 default_mode=MODE_SEMIGLOBAL, max_read_len=None, max_win_len=None, ref_len=None,
                 reads_len=None, reps=3, stream=None):
        """Tune the plan on a sample batch (same arguments as align); returns one dict per
        tuned read-length range.  The context keeps the chosen plan."""
        b, sc, flags, _ = _make_batch(ref2b, win_off, win_len, reads2b, read_off, read_len, mode, scoring,
                                      out_start, out_cigar, cigar_cap, force_int32, False, True,
                                      default_mode, max_read_len, max_win_len, ref_len, reads_len, None,
                                      outputs=False)
        cap = 64
        entries = (_lib.TuneEntry * cap)()
        n_out = ctypes.c_int32()
        _lib.check(_lib.load().mica_ctx_autotune(self._h, ctypes.byref(b), ctypes.byref(sc), flags,
                                                 _stream_handle(stream), int(reps), entries, cap,
                                                 ctypes.byref(n_out)))
        return [{f: getattr(entries[i], f) for f, _ in _lib.TuneEntry._fields_ if f != "pad_"}
                for i in range(n_out.value)]

    def save_plan(self, path):
        _lib.check(_lib.load().mica_ctx_save_plan(self._h, str(path).encode()))

    def load_plan(self, path):
        _lib.check(_lib.load().mica_ctx_load_plan(self._h, str(path).encode()))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().mica_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def measure_valu_peak(device=0):
    """Measured integer VALU throughput (TOP/s): (packed 16-bit, 32-bit)."""
    a, b = ctypes.c_double(), ctypes.c_double()
    _lib.check(_lib.load().mica_measure_valu_peak(int(device), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def pack_2bit(codes, stream=None):
    """Pack a uint8 tensor of base codes (A0 C1 G2 T3) on the GPU into int32 words."""
    codes = _dev(codes, torch.uint8, "codes")
    words = torch.empty((codes.numel() + 15) // 16, dtype=torch.int32, device=codes.device)
    _lib.check(_lib.load().mica_pack_2bit(_ptr(codes), codes.numel(), _ptr(words), _stream_handle(stream)))
    return words


def _make_batch(ref2b, win_off, win_len, reads2b, read_off, read_len, mode, scoring, out_start, out_cigar,
                cigar_cap, force_int32, plain, graph, default_mode, max_read_len, max_win_len, ref_len,
                reads_len, out, outputs=True, ext_h0=None, ext_default_h0=0, ext_clip=0, mode_mask=0,
                min_read_len=0, max_ext_h0=0):
    ref2b = _dev(ref2b, torch.int32, "ref2b")
    reads2b = _dev(reads2b, torch.int32, "reads2b")
    win_off = _dev(win_off, torch.int64, "win_off")
    win_len = _dev(win_len, torch.int32, "win_len")
    read_off = _dev(read_off, torch.int64, "read_off")
    read_len = _dev(read_len, torch.int32, "read_len")
    n = win_off.numel()
    if not (win_len.numel() == n and read_off.numel() == n and read_len.numel() == n):
        raise ValueError("per-pair arrays must have equal lengths")
    if mode is not None:
        mode = _dev(mode, torch.uint8, "mode")
        if mode.numel() != n:
            raise ValueError("mode must have one entry per pair")
    if ext_h0 is not None:
        ext_h0 = _dev(ext_h0, torch.int32, "ext_h0")
        if ext_h0.numel() != n:
            raise ValueError("ext_h0 must have one entry per pair")
    if max_read_len is None:
        max_read_len = int(read_len.max().item()) if n else 0
    if max_win_len is None:
        max_win_len = int(win_len.max().item()) if n else 0
    dev = win_off.device
    want_start = out_start or out_cigar
    if out is None and outputs:
        out = {
            "score": torch.empty(n, dtype=torch.int32, device=dev),
            "read_end": torch.empty(n, dtype=torch.int32, device=dev),
            "ref_end": torch.empty(n, dtype=torch.int32, device=dev),
            "status": torch.empty(n, dtype=torch.int32, device=dev),
        }
        if want_start:
            out["read_start"] = torch.empty(n, dtype=torch.int32, device=dev)
            out["ref_start"] = torch.empty(n, dtype=torch.int32, device=dev)
        if out_cigar:
            out["cigar"] = torch.empty((n, cigar_cap), dtype=torch.int32, device=dev)
            out["n_cigar"] = torch.empty(n, dtype=torch.int32, device=dev)
    out = out if out is not None else {}
    b = _lib.Batch()
    b.ref2b = _ptr(ref2b)
    b.ref_len = int(ref_len) if ref_len is not None else ref2b.numel() * 16
    b.win_off = _ptr(win_off)
    b.win_len = _ptr(win_len)
    b.reads2b = _ptr(reads2b)
    b.reads_len = int(reads_len) if reads_len is not None else reads2b.numel() * 16
    b.read_off = _ptr(read_off)
    b.read_len = _ptr(read_len)
    b.mode = _ptr(mode)
    b.default_mode = int(default_mode)
    b.n_pairs = n
    b.max_read_len = int(max_read_len)
    b.max_win_len = int(max_win_len)
    b.score = _ptr(out.get("score"))
    b.read_end = _ptr(out.get("read_end"))
    b.ref_end = _ptr(out.get("ref_end"))
    b.read_start = _ptr(out.get("read_start"))
    b.ref_start = _ptr(out.get("ref_start"))
    b.cigar = _ptr(out.get("cigar"))
    b.cigar_cap = int(cigar_cap) if out_cigar else 0
    b.n_cigar = _ptr(out.get("n_cigar"))
    b.status = _ptr(out.get("status"))
    b.ext_h0 = _ptr(ext_h0)
    b.ext_default_h0 = int(ext_default_h0)
    b.ext_clip = int(ext_clip)
    b.mode_mask = int(mode_mask)
    b.min_read_len = int(min_read_len)
    b.max_ext_h0 = int(max_ext_h0)
    a_, b_, o_, e_ = (int(x) for x in scoring)
    sc = _lib.Scoring(a_, b_, o_, e_)
    flags = (OUT_START if out_start else 0) | (OUT_CIGAR if out_cigar else 0) | \
        (FORCE_INT32 if force_int32 else 0) | (PLAIN_LAUNCH if plain else 0) | (0 if graph else NO_GRAPH)
    return b, sc, flags, out


def align_noalloc(ref2b, win_off, win_len, reads2b, read_off, read_len, mode=None, scoring=(1, -4, 6, 1),
                  out_start=False, out_cigar=False, cigar_cap=64, force_int32=False, plain=False,
                  default_mode=MODE_SEMIGLOBAL, max_read_len=None, max_win_len=None, ref_len=None,
                  reads_len=None, out=None, stream=None, ext_h0=None, ext_default_h0=0, ext_clip=0,
                  mode_mask=0, min_read_len=0, max_ext_h0=0):
    """The allocation-free call (mica_dp_align_batch_noalloc): same arguments
    and results as align() without a context; the library's workspace is one
    fixed device array per GPU, so overlapping calls on one GPU race.  Pass
    ``out`` (preallocated tensors) when the caller must not allocate either."""
    b, sc, flags, out = _make_batch(ref2b, win_off, win_len, reads2b, read_off, read_len, mode, scoring,
                                    out_start, out_cigar, cigar_cap, force_int32, plain, False, default_mode,
                                    max_read_len, max_win_len, ref_len, reads_len, out, ext_h0=ext_h0,
                                    ext_default_h0=ext_default_h0, ext_clip=ext_clip, mode_mask=mode_mask,
                                    min_read_len=min_read_len, max_ext_h0=max_ext_h0)
    _lib.check(_lib.load().mica_dp_align_batch_noalloc(ctypes.byref(b), ctypes.byref(sc), flags,
                                                       _stream_handle(stream)))
    return out


def align(ctx, ref2b, win_off, win_len, reads2b, read_off, read_len, mode=None, scoring=(1, -4, 6, 1),
          out_start=False, out_cigar=False, cigar_cap=64, force_int32=False, plain=False, graph=True,
          default_mode=MODE_SEMIGLOBAL, max_read_len=None, max_win_len=None, ref_len=None,
          reads_len=None, out=None, stream=None, ext_h0=None, ext_default_h0=0, ext_clip=0,
          mode_mask=0, min_read_len=0, max_ext_h0=0):
    """Align every (read, window) pair on the GPU; returns a dict of tensors.

    ref2b / reads2b: int32 tensors of 2-bit packed bases; win_off / read_off:
    int64 base offsets; win_len / read_len: int32 lengths; mode: optional uint8
    per pair (0 semi-global, 1 local).  Outputs: score, read_end, ref_end,
    status and, when requested, read_start, ref_start, cigar, n_cigar.
    ``max_read_len`` / ``max_win_len`` default to the batch maxima (one host
    synchronisation).  ``graph=False`` enqueues the kernels one by one
    instead of as one HIP graph.  Extension pairs (mode 2) start from
    ``ext_h0`` (int32 per pair) or ``ext_default_h0`` and are clipped unless
    the whole read scores within ``ext_clip`` of the best early end.
    ``mode_mask`` (bit per mode, 0 = all) names the modes a ``mode`` array
    may hold, so kernels of absent modes are not launched; ``min_read_len``
    (with ``max_read_len``) bounds the read lengths, so a batch of one
    length class runs that class's own kernel; ``max_ext_h0`` (0 = none)
    bounds the extension start scores, so a batch whose extensions provably
    fit 16-bit scores launches no saturation-checking kernels.  The
    call is asynchronous on ``stream``.
    """
    b, sc, flags, out = _make_batch(ref2b, win_off, win_len, reads2b, read_off, read_len, mode, scoring,
                                    out_start, out_cigar, cigar_cap, force_int32, plain, graph, default_mode,
                                    max_read_len, max_win_len, ref_len, reads_len, out, ext_h0=ext_h0,
                                    ext_default_h0=ext_default_h0, ext_clip=ext_clip, mode_mask=mode_mask,
                                    min_read_len=min_read_len, max_ext_h0=max_ext_h0)
    _lib.check(_lib.load().mica_dp_align_batch(ctx.handle, ctypes.byref(b), ctypes.byref(sc), flags,
                                               _stream_handle(stream)))
    return out


def to_device(batch, device="cuda"):
    """Upload a synth.Batch-like object (numpy arrays) as the tensors align() takes."""
    ref = batch.ref if batch.ref_packed else pack_codes(batch.ref)
    reads = pack_codes(batch.reads)
    ref_len = len(batch.ref) * 16 if batch.ref_packed else len(batch.ref)
    t = {
        "ref2b": torch.from_numpy(ref.view(np.int32)).to(device),
        "reads2b": torch.from_numpy(reads.view(np.int32)).to(device),
        "win_off": torch.from_numpy(batch.win_off.astype(np.int64)).to(device),
        "win_len": torch.from_numpy(batch.win_len.astype(np.int32)).to(device),
        "read_off": torch.from_numpy(batch.read_off.astype(np.int64)).to(device),
        "read_len": torch.from_numpy(batch.read_len.astype(np.int32)).to(device),
        "mode": torch.from_numpy(batch.mode.astype(np.uint8)).to(device),
        "ref_len": ref_len,
        "reads_len": len(batch.reads),
    }
    return t
