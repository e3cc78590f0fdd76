"""Binding of the host pipeline (include/mica_pipe.h): FASTQ in, SAM out,
the few-mismatch search and the DP phase on the GPU.  Argument marshalling
only; parsing, batching, the GPU work and SAM formatting run in the library.

    pipe = Pipeline(ref_words, ref_len, "chr1")
    stats = pipe.run("reads.fq", "out.sam")
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib


class Pipeline:
    def __init__(self, ref_words, ref_len, ref_name="ref", k=2, max_occ=64, band=32, min_score=0,
                 batch_reads=1 << 20, format_threads=8, scoring=(1, -4, 6, 1), device=0):
        words = np.ascontiguousarray(ref_words, dtype=np.uint32)
        if len(words) * 16 < ref_len:
            raise ValueError("ref_words holds fewer than ref_len bases")
        prm = _lib.PipeParams()
        prm.k, prm.max_occ, prm.band, prm.min_score = int(k), int(max_occ), int(band), int(min_score)
        prm.batch_reads, prm.format_threads = int(batch_reads), int(format_threads)
        prm.scoring = _lib.Scoring(*(int(x) for x in scoring))
        h = ctypes.c_void_p()
        _lib.check(_lib.load().mica_pipe_create(int(device), words.ctypes.data, int(ref_len), ref_name.encode(),
                                                ctypes.byref(prm), ctypes.byref(h)))
        self._h = h
        self.params = {"k": k, "max_occ": max_occ, "band": band, "min_score": min_score, "scoring": tuple(scoring)}

    def run(self, fastq_path, sam_path):
        """Align a FASTQ file into a SAM file; returns the run's statistics."""
        st = _lib.PipeStats()
        _lib.check(_lib.load().mica_pipe_run(self._h, str(fastq_path).encode(), str(sam_path).encode(),
                                             ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in _lib.PipeStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().mica_pipe_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
