"""Host-side 2-bit packing of base codes (the library's sequence layout).

Base codes A=0 C=1 G=2 T=3; base k of a buffer sits at bits 2*(k % 16) of
32-bit word k // 16.  ``mica_pack_2bit`` does the same on the GPU.
"""
from __future__ import annotations

import numpy as np

_SHIFTS = (2 * np.arange(16, dtype=np.uint32))


def pack_codes(codes):
    """uint8 codes (values 0..3) -> uint32 words, 16 bases per word."""
    codes = np.asarray(codes, dtype=np.uint8)
    n = len(codes)
    nw = (n + 15) // 16
    padded = np.zeros(nw * 16, dtype=np.uint32)
    padded[:n] = codes & 3
    return np.bitwise_or.reduce(padded.reshape(nw, 16) << _SHIFTS, axis=1).astype(np.uint32)


def unpack_words(words, n):
    """uint32 words -> the first n base codes (uint8)."""
    words = np.asarray(words).view(np.uint32)
    out = ((words[:, None] >> _SHIFTS) & 3).astype(np.uint8).reshape(-1)
    return out[:n]
