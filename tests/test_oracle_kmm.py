"""Pins of the few-mismatch search oracle (oracle/kmm.c).

The oracle is the definition written out (every placement of every read).
It is pinned to things other than itself:
- exact search (k = 0) against Python's own substring search;
- a different construction of the hit set: every string within Hamming
  distance k of the read, each searched exactly with ``bytes.find``;
- planted reads with a known number of substitutions at a known position;
- the repetitive rule against overlapping-match counts from ``re``;
- invariants (complementing or reversing both sequences, growth with k).
Plausible mistakes planted in copies of kmm.c must fail these pins.
"""
import ctypes
import itertools
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(os.path.dirname(oracle.__file__), "kmm.c")


def _layout(reads):
    """One flat code array and offsets for a list of reads."""
    off = np.zeros(len(reads), np.int64)
    if reads:
        off[1:] = np.cumsum([len(r) for r in reads])[:-1]
    flat = np.concatenate([np.asarray(r, np.uint8) for r in reads] + [np.zeros(1, np.uint8)])
    return flat, off, np.array([len(r) for r in reads], np.int32)


def _run(search, ref, reads, k, max_occ=1 << 30):
    flat, off, ln = _layout(reads)
    return search(ref, flat, off, ln, k=k, max_occ=max_occ)


def _find_all(hay, needle):
    """Start positions of needle in hay (overlapping), by bytes.find."""
    out, s = [], hay.find(needle)
    while s >= 0:
        out.append(s)
        s = hay.find(needle, s + 1)
    return out


def _neighbourhood_hits(ref, read, k):
    """{position: mismatches} from every string within Hamming distance k of
    the read, each searched exactly."""
    hay = bytes(ref.tolist())
    m = len(read)
    hits = {}
    for d in range(k + 1):
        for where in itertools.combinations(range(m), d):
            for subs in itertools.product((1, 2, 3), repeat=d):
                s = list(read)
                for w, x in zip(where, subs):
                    s[w] = (s[w] + x) % 4
                for p in _find_all(hay, bytes(s)):
                    hits[p] = d
    return hits


def pin_exact_search(search):
    rng = np.random.default_rng(1)
    ref = rng.integers(0, 4, 3000, dtype=np.uint8)
    ref[1000:1040] = ref[200:240]  # a repeated stretch
    reads = [ref[200:230].copy(), ref[2970:3000].copy(), ref[0:25].copy(), rng.integers(0, 4, 40, dtype=np.uint8),
             ref[1005:1012].copy(), ref[10:11].copy()]
    o = _run(search, ref, reads, 0)
    hay = bytes(ref.tolist())
    for r, q in enumerate(reads):
        pos = _find_all(hay, bytes(q.tolist()))
        assert o["n_hits"][r] == len(pos), r
        assert o["n_best"][r] == len(pos)
        assert o["best_mm"][r] == (0 if pos else -1)
        assert o["pos"][r] == (pos[0] if pos else -1)


def pin_neighbourhood(search):
    rng = np.random.default_rng(2)
    for trial in range(6):
        ref = rng.integers(0, 4, 400, dtype=np.uint8)
        ref[100:160] = ref[300:360]
        reads = []
        for t in range(12):
            m = int(rng.integers(3, 10))
            p = int(rng.integers(0, len(ref) - m))
            q = ref[p:p + m].copy()
            for w in rng.choice(m, int(rng.integers(0, 3)), replace=False):
                q[w] = (q[w] + rng.integers(1, 4)) % 4
            reads.append(q)
        for k in (0, 1, 2):
            o = _run(search, ref, reads, k)
            for r, q in enumerate(reads):
                if len(q) < k + 1:
                    continue
                hits = _neighbourhood_hits(ref, q.tolist(), k)
                assert o["n_hits"][r] == len(hits), (trial, k, r)
                if hits:
                    best = min(hits.values())
                    bests = sorted(p for p, d in hits.items() if d == best)
                    assert o["best_mm"][r] == best
                    assert o["n_best"][r] == len(bests)
                    assert o["pos"][r] == bests[0]
                else:
                    assert o["best_mm"][r] == -1 and o["pos"][r] == -1


def pin_planted(search):
    rng = np.random.default_rng(3)
    ref = rng.integers(0, 4, 200_000, dtype=np.uint8)
    reads, want = [], []
    for t in range(60):
        m = int(rng.integers(30, 151))
        p = int(rng.integers(0, len(ref) - m + 1)) if t % 10 else len(ref) - m  # some at the very end
        d = t % 4
        q = ref[p:p + m].copy()
        for w in rng.choice(m, d, replace=False):
            q[w] = (q[w] + rng.integers(1, 4)) % 4
        reads.append(q)
        want.append((p, d))
    o = _run(search, ref, reads, 2)
    for r, (p, d) in enumerate(want):
        if d <= 2:
            assert (o["best_mm"][r], o["n_best"][r], o["n_hits"][r], o["pos"][r]) == (d, 1, 1, p), r
        else:
            assert (o["best_mm"][r], o["n_hits"][r], o["pos"][r]) == (-1, 0, -1), r


def pin_repetitive(search):
    rng = np.random.default_rng(4)
    unit = rng.integers(0, 4, 7, dtype=np.uint8)
    ref = np.concatenate([rng.integers(0, 4, 500, dtype=np.uint8), np.tile(unit, 30),
                          rng.integers(0, 4, 500, dtype=np.uint8)])
    hay = bytes(ref.tolist())
    read = np.tile(unit, 6)[:30]  # every part lies in the tandem repeat
    parts = [read[j * 30 // 3:(j + 1) * 30 // 3] for j in range(3)]
    occ = [len(re.findall(b"(?=" + re.escape(bytes(p.tolist())) + b")", hay)) for p in parts]
    lim = min(occ)
    o = _run(search, ref, [read], 2, max_occ=lim - 1)
    assert o["status"][0] == oracle.ST_REPETITIVE and o["best_mm"][0] == -1 and o["n_hits"][0] == 0
    o = _run(search, ref, [read], 2, max_occ=max(occ))
    assert o["status"][0] == 0 and o["best_mm"][0] == 0
    assert o["n_best"][0] == len(_find_all(hay, bytes(read.tolist())))
    assert o["n_hits"][0] == len(_neighbourhood_hits(ref, read.tolist(), 2))
    # the threshold is strict: max_occ equal to the largest count searches
    o = _run(search, ref, [read], 2, max_occ=max(occ) - 1)
    assert o["status"][0] == oracle.ST_REPETITIVE


def pin_invariants(search):
    rng = np.random.default_rng(5)
    ref = rng.integers(0, 4, 5000, dtype=np.uint8)
    ref[3000:3100] = ref[1000:1100]
    reads = []
    for t in range(30):
        m = int(rng.integers(8, 40))
        p = int(rng.integers(0, len(ref) - m))
        q = ref[p:p + m].copy()
        q[rng.integers(0, m, int(rng.integers(0, 3)))] = rng.integers(0, 4)
        reads.append(q)
    for k in (0, 1, 2):
        a = _run(search, ref, reads, k)
        c = _run(search, 3 - ref, [3 - q for q in reads], k)
        for key in ("best_mm", "n_best", "n_hits", "pos"):
            assert np.array_equal(a[key], c[key]), (k, key)
        rv = _run(search, ref[::-1].copy(), [q[::-1].copy() for q in reads], k)
        for key in ("best_mm", "n_best", "n_hits"):
            assert np.array_equal(a[key], rv[key]), (k, key)
        one = a["n_best"] == 1
        ln = np.array([len(q) for q in reads])
        assert np.array_equal(rv["pos"][one], len(ref) - ln[one] - a["pos"][one])
        if k < 2:
            b = _run(search, ref, reads, k + 1)
            assert (b["n_hits"] >= a["n_hits"]).all()
            has = a["best_mm"] >= 0
            assert np.array_equal(a["best_mm"][has], b["best_mm"][has])


def pin_length_rules(search):
    rng = np.random.default_rng(6)
    ref = rng.integers(0, 4, 300, dtype=np.uint8)
    reads = [ref[:2].copy(), ref[:3].copy(), rng.integers(0, 4, 400, dtype=np.uint8)]
    o = _run(search, ref, reads, 2)
    assert o["status"][0] == oracle.ST_LEN_LIMIT
    assert o["status"][1] == 0 and o["best_mm"][1] == 0
    assert o["status"][2] == 0 and o["best_mm"][2] == -1  # longer than the reference: no placement


PINS = [pin_exact_search, pin_neighbourhood, pin_planted, pin_repetitive, pin_invariants, pin_length_rules]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_oracle_pin(pin):
    pin(oracle.kmm_search)


# ---- planted mistakes ---------------------------------------------------------

MUTANTS = {
    "last_position_missed": ("for (int64_t p = 0; p + m <= J->ref_len; p++) {",
                             "for (int64_t p = 0; p + m < J->ref_len; p++) {"),
    "mismatch_bound_off_by_one": ("if (d > k) continue;", "if (d >= k) continue;"),
    "rightmost_best": ("} else if (d == best) {\n      nb++;", "} else if (d == best) {\n      nb++;\n      bp = p;"),
    "parts_cut_into_k": ("const int32_t a = (int32_t)((int64_t)j * m / (k + 1));\n    const int32_t b = (int32_t)((int64_t)(j + 1) * m / (k + 1));",
                         "const int32_t a = (int32_t)((int64_t)j * m / (k + 2));\n    const int32_t b = (int32_t)((int64_t)(j + 1) * m / (k + 2));"),
    "repetitive_not_strict": ("if (count_exact(J->ref, J->ref_len, q + a, b - a, J->max_occ) > J->max_occ) {",
                              "if (count_exact(J->ref, J->ref_len, q + a, b - a, J->max_occ) >= J->max_occ) {"),
    "hits_count_only_best": ("    nh++;\n", ""),
    "empty_part_allowed": ("if (m < k + 1 || m > KMM_MAX_M) {", "if (m < 1 || m > KMM_MAX_M) {"),
}


def _build_mutant(name, tmp):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, name
    src = os.path.join(tmp, "kmm_mut.c")
    lib = os.path.join(tmp, "libkmm_mut.so")
    with open(src, "w") as f:
        f.write(text.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", src, "-o", lib])
    return lib


def _searcher(libpath):
    lib = ctypes.CDLL(libpath)
    P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.oracle_kmm_search.restype = ctypes.c_int
    lib.oracle_kmm_search.argtypes = [P, i64, P, i64, P, P, i64, i32, i32, P, P, P, P, P, i32]

    def search(ref, reads, read_off, read_len, k=2, max_occ=64):
        ref = np.ascontiguousarray(ref, np.uint8)
        reads = np.ascontiguousarray(reads, np.uint8)
        read_off = np.ascontiguousarray(read_off, np.int64)
        read_len = np.ascontiguousarray(read_len, np.int32)
        n = len(read_off)
        out = {"best_mm": np.zeros(n, np.int32), "n_best": np.zeros(n, np.int32),
               "n_hits": np.zeros(n, np.int32), "pos": np.zeros(n, np.int64), "status": np.zeros(n, np.uint32)}
        p = lambda a: a.ctypes.data  # noqa: E731
        assert lib.oracle_kmm_search(p(ref), len(ref), p(reads), len(reads), p(read_off), p(read_len), n, k,
                                     max_occ, p(out["best_mm"]), p(out["n_best"]), p(out["n_hits"]),
                                     p(out["pos"]), p(out["status"]), 4) == 0
        return out
    return search


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_kmm_mutant_is_caught(name):
    os.makedirs(os.path.join(ROOT, "_build"), exist_ok=True)
    with tempfile.TemporaryDirectory(dir=os.path.join(ROOT, "_build")) as tmp:
        search = _searcher(_build_mutant(name, tmp))
        caught = []
        for pin in PINS:
            try:
                pin(search)
            except AssertionError:
                caught.append(pin.__name__)
        assert caught, "mutant %s passed every pin" % name
