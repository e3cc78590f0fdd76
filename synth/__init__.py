"""Seeded synthetic inputs shaped like the paper's short-read workloads.

This module only draws random data: references, windows, reads with
planted substitutions and indels, modes and request streams.  It holds none
of the alignment arithmetic.  Both the GPU tests / benchmark and the CPU
oracle read their inputs from here, so the two sides see identical data.

The paper measures on real Illumina paired-end data (150 bp and 100 bp reads
of the YH genome, 1000 Genomes lanes), which is not available; i.i.d.
uniform references and simulated reads of the same lengths stand in for it.

Layout shared by every batch (all numpy):
  ref       uint8 codes A0 C1 G2 T3 (or, for the 3 Gbp serving reference,
            packed uint32 words: base k at bits 2*(k % 16) of word k // 16)
  win_off   int64 window start in the reference, win_len int32
  reads     uint8 codes; every read starts at a multiple of 16 bases so the
            same offsets address the 2-bit packed copy
  read_off  int64, read_len int32, mode uint8 (0 semi-global, 1 local)
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

SEED = 14024876
SCORING = (1, -4, 6, 1)  # match, mismatch, gap open, gap extend


def rng_for(key, *more):
    return np.random.default_rng(np.random.SeedSequence([SEED, key, *more]))


@dataclasses.dataclass
class Batch:
    ref: np.ndarray
    win_off: np.ndarray
    win_len: np.ndarray
    reads: np.ndarray
    read_off: np.ndarray
    read_len: np.ndarray
    mode: np.ndarray
    name: str = ""
    planted_start: np.ndarray | None = None  # window-relative start of the planted copy
    planted_end: np.ndarray | None = None
    planted_ops: list | None = None  # per read: list of (op, len), op in "MID"
    ref_packed: bool = False
    h0: np.ndarray | None = None  # extension pairs: score of the anchor (int32 per pair)

    @property
    def n_pairs(self):
        return len(self.win_off)

    def cells(self):
        return int(np.dot(self.read_len.astype(np.int64), self.win_len.astype(np.int64)))

    def digest(self):
        h = hashlib.sha256()
        for a in (self.ref, self.win_off, self.win_len, self.reads, self.read_off, self.read_len, self.mode):
            h.update(np.ascontiguousarray(a).view(np.uint8).tobytes() if a.size < (1 << 27) else a[:1 << 20].tobytes())
        return h.hexdigest()[:16]

    def subset(self, idx):
        """Pairs idx (reads and reference shared, offsets kept)."""
        idx = np.asarray(idx)
        return dataclasses.replace(
            self, win_off=self.win_off[idx], win_len=self.win_len[idx], read_off=self.read_off[idx],
            read_len=self.read_len[idx], mode=self.mode[idx],
            planted_start=None if self.planted_start is None else self.planted_start[idx],
            planted_end=None if self.planted_end is None else self.planted_end[idx],
            planted_ops=None if self.planted_ops is None else [self.planted_ops[i] for i in idx],
            h0=None if self.h0 is None else self.h0[idx])

    def window_codes(self, p):
        o, n = int(self.win_off[p]), int(self.win_len[p])
        if self.ref_packed:
            return base_at_packed(self.ref, np.arange(o, o + n, dtype=np.int64))
        return self.ref[o:o + n]

    def read_codes(self, p):
        o = int(self.read_off[p])
        return self.reads[o:o + int(self.read_len[p])]


def random_ref(rng, n):
    return rng.integers(0, 4, n, dtype=np.uint8)


def random_packed_ref(rng, n_bases):
    """i.i.d. uniform bases drawn directly as packed words (16 bases per uint32)."""
    assert n_bases % 16 == 0
    return rng.integers(0, 1 << 32, n_bases // 16, dtype=np.uint64).astype(np.uint32)


def base_at_packed(words, pos):
    pos = np.asarray(pos, np.int64)
    return ((words[pos >> 4] >> ((pos & 15) * 2).astype(np.uint32)) & 3).astype(np.uint8)


def _indel_lengths(rng, kind, k):
    if kind == "u123":
        return rng.integers(1, 4, k)
    if kind == "geom":  # Geometric(1/2) on {1, 2, ...}: mean 2
        return rng.geometric(0.5, k)
    raise ValueError(kind)


def simulate_reads(rng, base_at, start, limit, m, p_sub, p_indel, indel_kind, record=False):
    """Copy reads of lengths m from the reference starting at ``start``.

    Walk a pointer p from start; per step draw u ~ U[0,1): below p_indel an
    indel of length L (insertion of L random bases, truncated at m, or a
    deletion p += L, each with probability 1/2); below p_indel + p_sub a
    substituted base (one of the three others); else the reference base.
    A read whose pointer reaches ``limit`` before it is complete fails.
    Returns (codes (N, max m) uint8, ok bool, end pointer, ops or None).
    """
    N = len(start)
    Mx = int(m.max()) if N else 0
    out = np.zeros((N, Mx), np.uint8)
    p = start.astype(np.int64).copy()
    ln = np.zeros(N, np.int64)
    ok = np.ones(N, bool)
    active = (ln < m) & ok
    ev = [] if record else None
    while True:
        idx = np.nonzero(active)[0]
        if len(idx) == 0:
            break
        u = rng.random(len(idx))
        is_indel = u < p_indel
        is_sub = (~is_indel) & (u < p_indel + p_sub)
        is_base = ~is_indel
        # indels
        ii = idx[is_indel]
        if len(ii):
            L = _indel_lengths(rng, indel_kind, len(ii))
            ins = rng.random(len(ii)) < 0.5
            di = ii[~ins]
            p[di] += L[~ins]
            ii_ins, L_ins = ii[ins], L[ins]
            if len(ii_ins):
                rnd = rng.integers(0, 4, (len(ii_ins), int(L_ins.max())), dtype=np.uint8)
                for t in range(int(L_ins.max())):
                    w = (t < L_ins) & (ln[ii_ins] < m[ii_ins])
                    out[ii_ins[w], ln[ii_ins[w]]] = rnd[w, t]
                    ln[ii_ins[w]] += 1
            if record:
                ev.append(("indel", ii.copy(), L.copy(), ins.copy()))
        # aligned bases (match or substitution)
        bi = idx[is_base]
        if len(bi):
            past = p[bi] >= limit[bi]
            ok[bi[past]] = False
            bi2 = bi[~past]
            sub = is_sub[is_base][~past]
            ref_b = base_at(p[bi2])
            shift = rng.integers(1, 4, len(bi2)).astype(np.uint8)
            b = np.where(sub, (ref_b + shift) % 4, ref_b).astype(np.uint8)
            out[bi2, ln[bi2]] = b
            ln[bi2] += 1
            p[bi2] += 1
            if record:
                ev.append(("base", bi2.copy(), sub.copy()))
        active = (ln < m) & ok
    ops = None
    if record:
        ops = [[] for _ in range(N)]

        def push(k, op, L):
            if ops[k] and ops[k][-1][0] == op:
                ops[k][-1] = (op, ops[k][-1][1] + L)
            else:
                ops[k].append((op, L))
        cnt = np.zeros(N, np.int64)
        for e in ev:
            if e[0] == "base":
                for k in e[1]:
                    push(k, "M", 1)
                    cnt[k] += 1
            else:
                for k, L, isin in zip(e[1], e[2], e[3]):
                    if isin:
                        L = int(min(L, m[k] - cnt[k]))
                        if L > 0:
                            push(k, "I", L)
                            cnt[k] += L
                    else:
                        push(k, "D", int(L))
    return out, ok, p, ops


def _draw_reads(rng, base_at, lo, hi, m, limit_fn, p_sub, p_indel, indel_kind, record):
    """Draw start offsets in [lo, hi] (absolute) and simulate; redraw failures."""
    N = len(m)
    codes = np.zeros((N, int(m.max()) if N else 0), np.uint8)
    start = np.zeros(N, np.int64)
    end = np.zeros(N, np.int64)
    ops = [None] * N if record else None
    todo = np.arange(N)
    while len(todo):
        s = rng.integers(lo[todo], hi[todo] + 1)
        c, ok, p, o = simulate_reads(rng, base_at, s, limit_fn(todo), m[todo], p_sub, p_indel, indel_kind, record)
        good = todo[ok]
        codes[good, :c.shape[1]] = c[ok]
        start[good] = s[ok]
        end[good] = p[ok]
        if record:
            for k, g in enumerate(todo):
                if ok[k]:
                    ops[g] = o[k]
        todo = todo[~ok]
    return codes, start, end, ops


def pack_reads_layout(codes, m):
    """Concatenate reads, each starting at a multiple of 16 bases (zero padded)."""
    N = len(m)
    slot = ((m.astype(np.int64) + 15) // 16) * 16
    off = np.zeros(N, np.int64)
    if N:
        off[1:] = np.cumsum(slot)[:-1]
    total = int(slot.sum()) if N else 0
    flat = np.zeros(max(total, 16), np.uint8)
    for L in np.unique(m):
        sel = np.nonzero(m == L)[0]
        if L == 0 or len(sel) == 0:
            continue
        cols = off[sel][:, None] + np.arange(L)[None, :]
        flat[cols] = codes[sel, :L]
    return flat, off


def _finish(name, ref, win_off, win_len, codes, m, mode, pstart=None, pend=None, ops=None, packed=False):
    reads, read_off = pack_reads_layout(codes, m)
    return Batch(ref=ref, win_off=win_off.astype(np.int64), win_len=win_len.astype(np.int32),
                 reads=reads, read_off=read_off, read_len=m.astype(np.int32), mode=mode.astype(np.uint8),
                 name=name, planted_start=pstart, planted_end=pend, planted_ops=ops, ref_packed=packed)


def config0(n_pairs=1000, record=False):
    """1,000 reads of 150 bp, each against its own 200 bp window of i.i.d. bases.

    Read copied at a uniform window offset in [0, 50] with 1% substitutions and
    0.2% indels of length 1-3; semi-global, int32 scores, score + end only."""
    rng = rng_for(0)
    n, m = 200, 150
    ref = random_ref(rng, n * n_pairs)
    win_off = np.arange(n_pairs, dtype=np.int64) * n
    mm = np.full(n_pairs, m, np.int32)
    codes, s, e, ops = _draw_reads(rng, lambda pos: ref[pos], win_off, win_off + 50, mm,
                                   lambda idx: win_off[idx] + n, 0.01, 0.002, "u123", record)
    return _finish("c0", ref, win_off, np.full(n_pairs, n), codes, mm, np.zeros(n_pairs),
                   s - win_off, e - win_off, ops)


def config1(n_pairs=1_000_000, ref_len=100_000_000, record=False):
    """150 bp reads against 400 bp windows of a 100 Mbp reference (semi-global).

    Window start uniform over the reference, read offset in the window U{0..200},
    1% substitutions, 0.3% indels with Geometric(1/2) lengths (mean 2)."""
    rng = rng_for(1)
    n, m = 400, 150
    ref = random_ref(rng, ref_len)
    win_off = rng.integers(0, ref_len - n + 1, n_pairs).astype(np.int64)
    mm = np.full(n_pairs, m, np.int32)
    codes, s, e, ops = _draw_reads(rng, lambda pos: ref[pos], win_off, win_off + 200, mm,
                                   lambda idx: win_off[idx] + n, 0.01, 0.003, "geom", record)
    return _finish("c1", ref, win_off, np.full(n_pairs, n), codes, mm, np.zeros(n_pairs),
                   s - win_off, e - win_off, ops)


def config2(n_pairs=500_000, ref_len=100_000_000, record=False):
    """Mate rescue: 150 bp partners against 1,000 bp windows, local alignment.

    Anchor start A uniform; insert size round(N(500, 50)); the partner starts at
    A + I - 150; the window starts at A - 75 (1 kbp centred on the expected
    partner).  2% substitutions, 0.5% indels (Geometric(1/2) lengths); a seeded
    10% of partners are replaced by 150 uniform random bases."""
    rng = rng_for(2)
    n, m = 1000, 150
    ref = random_ref(rng, ref_len)
    A = rng.integers(1000, ref_len - 2000, n_pairs).astype(np.int64)
    ins = np.rint(rng.normal(500.0, 50.0, n_pairs)).astype(np.int64)
    pstart = A + ins - 150
    mm = np.full(n_pairs, m, np.int32)
    codes, s, e, ops = _draw_reads(rng, lambda pos: ref[pos], pstart, pstart, mm,
                                   lambda idx: np.full(len(idx), ref_len), 0.02, 0.005, "geom", record)
    rand = rng.random(n_pairs) < 0.10
    codes[rand] = rng.integers(0, 4, (int(rand.sum()), m), dtype=np.uint8)
    win_off = A - 75
    b = _finish("c2", ref, win_off, np.full(n_pairs, n), codes, mm, np.ones(n_pairs),
                s - win_off, e - win_off, ops)
    b.random_partner = rand
    return b


def config3(n_pairs=2_000_000, ref_len=100_000_000, record=False):
    """Uneven lengths: m ~ U{50..250}, windows of floor(1.5 m) + 64, half local.

    Read offset in the window U{0..n-m-8}; errors as config 1; the mode of each
    pair is a seeded coin flip; pairs come shuffled."""
    rng = rng_for(3)
    ref = random_ref(rng, ref_len)
    mm = rng.integers(50, 251, n_pairs).astype(np.int32)
    nn = (3 * mm) // 2 + 64
    win_off = (rng.random(n_pairs) * (ref_len - nn + 1)).astype(np.int64)
    codes, s, e, ops = _draw_reads(rng, lambda pos: ref[pos], win_off, win_off + nn - mm - 8, mm,
                                   lambda idx: win_off[idx] + nn[idx], 0.01, 0.003, "geom", record)
    mode = (rng.random(n_pairs) < 0.5).astype(np.uint8)
    return _finish("c3", ref, win_off, nn, codes, mm, mode, s - win_off, e - win_off, ops)


SERVE_LENGTHS = (100, 150, 250)


def serving_reference(ref_len=3_000_000_000):
    """3 Gbp reference as packed words (750 MB), i.i.d. uniform bases."""
    return random_packed_ref(rng_for(4), ref_len)


def serving_request(ref_words, ref_len, req_id, n_reads=None, max_reads=10_000):
    """One request: 1..10,000 reads of {100, 150, 250} bp, windows of 1.5 m + 64.

    Window start uniform over the reference, the read planted inside it with
    config-1 errors; semi-global."""
    rng = rng_for(4, 1, req_id)
    k = int(rng.integers(1, max_reads + 1)) if n_reads is None else int(n_reads)
    mm = rng.choice(np.array(SERVE_LENGTHS, np.int32), k)
    nn = (3 * mm) // 2 + 64
    win_off = (rng.random(k) * (ref_len - nn.astype(np.int64) + 1)).astype(np.int64)
    codes, s, e, _ = _draw_reads(rng, lambda pos: base_at_packed(ref_words, pos), win_off,
                                 win_off + nn - mm - 8, mm, lambda idx: win_off[idx] + nn[idx],
                                 0.01, 0.003, "geom", False)
    return _finish("c4req%d" % req_id, ref_words, win_off, nn, codes, mm, np.zeros(k), s - win_off,
                   e - win_off, None, packed=True)


def serving_pool(ref_words, ref_len, n_reads, seed=0):
    """A pool of planted serving reads ({100, 150, 250} bp, windows 1.5 m + 64
    anywhere in the packed reference, config-1 errors, semi-global) from
    which requests are cut as contiguous ranges."""
    return serving_request(ref_words, ref_len, 1_000_000 + seed, n_reads=n_reads)


def request_schedule(n_pool, n_req, seed_key, max_reads=10_000):
    """Requests as distinct ranges of a read pool: sizes U{1..max_reads},
    starts uniform over the pool.  Returns (first, count) int64 arrays."""
    rng = rng_for(4, 3, seed_key)
    count = rng.integers(1, max_reads + 1, n_req).astype(np.int64)
    first = (rng.random(n_req) * (n_pool - count + 1)).astype(np.int64)
    return first, count


def poisson_arrivals(rate, n, seed_key=0):
    """Open-loop arrival times (seconds) of n requests at the given rate."""
    rng = rng_for(4, 2, seed_key)
    return np.cumsum(rng.exponential(1.0 / rate, n))


def tiny_random(n_pairs, m_max, n_max, seed, mode=None, related=0.5):
    """Small mixed batch for parity tests: random lengths, some related pairs."""
    rng = rng_for(10, seed)
    m = rng.integers(0, m_max + 1, n_pairs).astype(np.int32)
    n = rng.integers(0, n_max + 1, n_pairs).astype(np.int32)
    ref_len = int(n.sum()) + 16
    ref = random_ref(rng, ref_len)
    win_off = np.concatenate([[0], np.cumsum(n.astype(np.int64))[:-1]]) if n_pairs else np.zeros(0, np.int64)
    codes = rng.integers(0, 4, (n_pairs, max(int(m.max()) if n_pairs else 0, 1)), dtype=np.uint8)
    rel = rng.random(n_pairs) < related
    for k in np.nonzero(rel & (n >= m) & (m > 0))[0]:
        s = int(rng.integers(0, n[k] - m[k] + 1))
        codes[k, :m[k]] = ref[win_off[k] + s: win_off[k] + s + m[k]]
        nmut = int(rng.integers(0, 4))
        for _ in range(nmut):
            codes[k, int(rng.integers(0, m[k]))] = rng.integers(0, 4)
    if mode is None:
        md = rng.integers(0, 2, n_pairs).astype(np.uint8)
    else:
        md = np.full(n_pairs, mode, np.uint8)
    return _finish("tiny", ref, win_off, n, codes, m, md)


def extension_like(n_pairs, seed=0, m_max=150, band=32, ref_len=4_000_000, p_junk=0.2):
    """Seed-extension pairs: the part of a read beyond an exact seed hit
    against the reference that follows the hit.

    Tail length m ~ U{0..m_max}; window = the m + band reference bases after
    the hit; the tail is copied from the window start with 1% substitutions
    and 0.3% indels (Geometric(1/2) lengths); a seeded fraction p_junk of
    tails turn into uniform random bases from a point U{0..m-1} on (adapter
    or chimeric ends, where clipping decides).  Anchor score h0 ~ U{19..60}
    (the score of an exact seed of that many bases at match score 1).
    Every pair has mode 2."""
    rng = rng_for(11, seed)
    m = rng.integers(0, m_max + 1, n_pairs).astype(np.int32)
    n = (m + band).astype(np.int32)
    ref = random_ref(rng, ref_len)
    win_off = rng.integers(0, ref_len - int(n.max()) + 1, n_pairs).astype(np.int64)
    codes, s, e, _ = _draw_reads(rng, lambda pos: ref[pos], win_off, win_off, m,
                                 lambda idx: win_off[idx] + n[idx], 0.01, 0.003, "geom", False)
    junk = (rng.random(n_pairs) < p_junk) & (m > 0)
    for k in np.nonzero(junk)[0]:
        c = int(rng.integers(0, m[k]))
        codes[k, c:m[k]] = rng.integers(0, 4, int(m[k]) - c, dtype=np.uint8)
    b = _finish("ext", ref, win_off, n, codes, m, np.full(n_pairs, 2))
    b.h0 = rng.integers(19, 61, n_pairs).astype(np.int32)
    b.junk = junk
    return b


def serving_like(n_pairs, ref_len=4_000_000, seed=0):
    """Config-4-shaped pairs ({100, 150, 250} bp reads, windows 1.5 m + 64) on a
    small unpacked reference, for parity tests of the serving read mix."""
    rng = rng_for(5, seed)
    ref = random_ref(rng, ref_len)
    mm = rng.choice(np.array(SERVE_LENGTHS, np.int32), n_pairs)
    nn = (3 * mm) // 2 + 64
    win_off = (rng.random(n_pairs) * (ref_len - nn + 1)).astype(np.int64)
    codes, s, e, _ = _draw_reads(rng, lambda pos: ref[pos], win_off, win_off + nn - mm - 8, mm,
                                 lambda idx: win_off[idx] + nn[idx], 0.01, 0.003, "geom", False)
    return _finish("c4like", ref, win_off, nn, codes, mm, np.zeros(n_pairs), s - win_off, e - win_off)


def pack_reads_unaligned(rng, codes, m):
    """Concatenate reads with 0..15 random filler bases before each one, so
    read offsets take every residue mod 16 (a word boundary anywhere in a
    read).  Returns (flat codes, offsets)."""
    N = len(m)
    gap = rng.integers(0, 16, N).astype(np.int64)
    off = np.zeros(N, np.int64)
    pos = 0
    for k in range(N):
        pos += int(gap[k])
        off[k] = pos
        pos += int(m[k])
    flat = rng.integers(0, 4, max(pos, 1) + 16, dtype=np.uint8)
    for k in range(N):
        flat[off[k]:off[k] + m[k]] = codes[k, :m[k]]
    return flat, off


LONG_REF_LEN = (1 << 32) + (1 << 26)  # 4.36 Gbp: window offsets past 2^31 and 2^32


def long_reference_batch(n_pairs=4000, ref_len=LONG_REF_LEN, hot_len=1 << 16, seed=0, modes=(0, 1, 2)):
    """Pairs whose windows sit past base 2^31 and 2^32 of a reference longer
    than 2^32 bases, for parity at the offsets a 3 Gbp resident reference
    reaches.

    The packed reference is zero words (all A) except for stretches of
    hot_len i.i.d. bases that start just below 2^31, straddle 2^31, straddle
    2^32, end at the last base, and start at 0; every window lies inside one
    stretch.  Reads of U{1..260} bases (windows 1.5 m + 64) are planted with
    config-1 errors; modes cycle over `modes` (extension pairs get h0 U{19..60});
    reads sit at unaligned offsets (pack_reads_unaligned).
    Returns (batch with ref = packed words and absolute win_off, stretch starts)."""
    assert ref_len % 16 == 0 and ref_len > (1 << 32) + 2 * hot_len
    rng = rng_for(12, seed)
    words = np.zeros(ref_len // 16, np.uint32)
    starts = np.array([(1 << 31) - hot_len, (1 << 31) - hot_len // 2, (1 << 32) - hot_len // 2,
                       ref_len - hot_len, 0], np.int64)
    for s in starts:
        words[s // 16:(s + hot_len) // 16] = random_packed_ref(rng, hot_len)
    m = rng.integers(1, 261, n_pairs).astype(np.int32)
    n = (3 * m) // 2 + 64
    region = starts[rng.integers(0, len(starts), n_pairs)]
    win_off = region + rng.integers(0, hot_len - n + 1).astype(np.int64)
    # every tenth window straddles 2^31, the next 2^32; the next ends at the last base
    k = np.arange(n_pairs)
    for r, edge in ((0, 1 << 31), (1, 1 << 32)):
        sel = k % 10 == r
        win_off[sel] = edge - rng.integers(1, n[sel]).astype(np.int64)
    win_off[k % 10 == 2] = ref_len - n[k % 10 == 2].astype(np.int64)
    codes, s, e, _ = _draw_reads(rng, lambda pos: base_at_packed(words, pos), win_off, win_off + n - m - 8, m,
                                 lambda idx: win_off[idx] + n[idx], 0.01, 0.003, "geom", False)
    # a fifth of the reads are random (low scores, long local tracebacks)
    junk = rng.random(n_pairs) < 0.2
    codes[junk] = rng.integers(0, 4, (int(junk.sum()), codes.shape[1]), dtype=np.uint8)
    reads, read_off = pack_reads_unaligned(rng, codes, m)
    mode = np.asarray(modes, np.uint8)[np.arange(n_pairs) % len(modes)]
    b = Batch(ref=words, win_off=win_off, win_len=n.astype(np.int32), reads=reads, read_off=read_off,
              read_len=m, mode=mode, name="longref", ref_packed=True)
    b.h0 = np.where(mode == 2, rng.integers(19, 61, n_pairs), 0).astype(np.int32)
    return b, starts


def rebase_windows(batch):
    """The same pairs with every window copied out of the (packed) reference
    into a small code array (windows back to back, offsets rebased); reads,
    modes and h0 unchanged.  The oracle aligns this copy."""
    n = batch.win_len.astype(np.int64)
    off = np.zeros(batch.n_pairs, np.int64)
    if batch.n_pairs:
        off[1:] = np.cumsum(n)[:-1]
    pos = np.concatenate([batch.win_off[p] + np.arange(n[p], dtype=np.int64) for p in range(batch.n_pairs)]
                         + [np.zeros(0, np.int64)])
    ref = base_at_packed(batch.ref, pos) if batch.ref_packed else batch.ref[pos]
    ref = np.concatenate([ref, np.zeros(16, np.uint8)])
    return dataclasses.replace(batch, ref=ref, win_off=off, ref_packed=False)


def band_mix(n_pairs, mode, seed=0):
    """Pairs of one mode whose alignments drift from their end diagonal by
    anything from nothing to far more than the banded traceback takes:
    reads of 60-150 bases copied from a window with 0-16 substitutions and
    0-2 indels of 1-10 bases each; a tenth of the reads are unrelated random
    bases.  Semi-global windows hold the copy with 0-24 extra bases on each
    side; local reads also carry random flanks of 0-20 bases; extension
    windows start at the copy and run 32 bases past the read's length, with
    anchor scores U{19..60}."""
    rng = rng_for(17, mode, seed)
    m = rng.integers(60, 151, n_pairs).astype(np.int32)
    pad = rng.integers(0, 25, n_pairs) if mode != 2 else np.zeros(n_pairs, np.int64)
    src_len = m + 64  # source stretch per pair, longer than any read drawn from it
    n = (m + 32 if mode == 2 else src_len + 2 * pad).astype(np.int32)
    win_off = np.concatenate([[0], np.cumsum(n.astype(np.int64))[:-1]])
    ref = random_ref(rng, int(n.sum()) + 16)
    codes = np.zeros((n_pairs, 250), np.uint8)
    lens = np.zeros(n_pairs, np.int32)
    for p in range(n_pairs):
        start = int(win_off[p] + pad[p])
        src = ref[start: start + int(src_len[p])].copy() if mode != 2 else ref[start: start + int(n[p])].copy()
        if rng.random() < 0.1:
            core = rng.integers(0, 4, int(m[p]), dtype=np.uint8)
        else:
            core = list(src[: int(m[p])])
            for _ in range(int(rng.integers(0, 3))):  # indels
                at = int(rng.integers(1, max(2, len(core) - 1)))
                ln = int(rng.integers(1, 11))
                if rng.random() < 0.5:
                    del core[at: at + ln]
                else:
                    core[at:at] = list(rng.integers(0, 4, ln, dtype=np.uint8))
            core = np.asarray(core[: int(m[p])], np.uint8)
            for _ in range(int(rng.integers(0, 17))):  # substitutions
                i = int(rng.integers(0, len(core)))
                core[i] = (core[i] + rng.integers(1, 4)) % 4
        if mode == 1:
            lf, rf = rng.integers(0, 21, 2)
            core = np.concatenate([rng.integers(0, 4, lf, dtype=np.uint8), core,
                                   rng.integers(0, 4, rf, dtype=np.uint8)])[:150]
        lens[p] = len(core)
        codes[p, : len(core)] = core
    if mode == 2:
        n = (lens + 32).astype(np.int32)
    b = _finish("band_mix", ref, win_off, n, codes[:, : max(int(lens.max()), 1)], lens, np.full(n_pairs, mode))
    if mode == 2:
        b.h0 = rng.integers(19, 61, n_pairs).astype(np.int32)
    return b
