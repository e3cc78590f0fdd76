"""Pins of the oracle's extension mode (seed-anchored DP with clipping) against
exhaustive enumeration, closed forms and invariants -- no DP recurrence on the
checking side."""
import itertools

import numpy as np
import pytest

import brute
import oracle

SCORINGS = [(1, -4, 6, 1), (3, 0, 2, 1), (2, -3, 5, 2), (1, -1, 0, 1)]


def _run(pairs, sc, h0, clip):
    return oracle.align_pairs(pairs, mode=2, scoring=sc, trace=True, default_h0=h0, clip=clip)


def _check(pairs, sc, h0, clip):
    got = _run(pairs, sc, h0, clip)
    for p, (q, r) in enumerate(pairs):
        score, (ei, ej), cig = brute.canonical_ext(q, r, sc, h0, clip)
        assert (got["score"][p], got["read_end"][p], got["ref_end"][p]) == (score, ei, ej), (q, r, sc, h0, clip)
        assert (got["read_start"][p], got["ref_start"][p]) == (0, 0)
        assert oracle.decode_cigar(got["cigar"][p], got["n_cigar"][p]) == "".join(cig), (q, r, sc, h0, clip)
        assert got["status"][p] == 0


@pytest.mark.parametrize("sc", SCORINGS)
def test_extension_all_small_pairs(sc):
    """Every pair with m, n <= 2 (and a sample up to 3), several start scores and penalties."""
    seqs = [tuple(s) for L in range(3) for s in itertools.product(range(4), repeat=L)]
    pairs = [(q, r) for q in seqs for r in seqs]
    rng = np.random.default_rng(11)
    pairs += [(tuple(rng.integers(0, 4, rng.integers(0, 4))), tuple(rng.integers(0, 4, rng.integers(0, 4))))
              for _ in range(150)]
    for h0, clip in ((0, 0), (5, 0), (5, 3), (12, 100)):
        _check(pairs, sc, h0, clip)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_extension_random_pairs(seed):
    rng = np.random.default_rng(seed)
    for sc in SCORINGS:
        pairs = []
        for _ in range(60):
            m, n = int(rng.integers(0, 6)), int(rng.integers(0, 6))
            r = rng.integers(0, 4, n)
            q = rng.integers(0, 4, m)
            if n and m and rng.random() < 0.5:  # a related read
                q[: min(m, n)] = r[: min(m, n)]
                q[rng.integers(0, m)] = rng.integers(0, 4)
            pairs.append((tuple(q), tuple(r)))
        h0 = int(rng.integers(0, 15))
        clip = int(rng.integers(0, 8))
        _check(pairs, sc, h0, clip)


def test_extension_closed_forms():
    sc = (1, -4, 6, 1)
    rng = np.random.default_rng(4)
    r = rng.integers(0, 4, 40)
    # identical read: whole read aligned, score h0 + m*a
    out = _run([(r[:30], r[:35])], sc, 20, 0)
    assert (out["score"][0], out["read_end"][0], out["ref_end"][0]) == (50, 30, 30)
    assert oracle.decode_cigar(out["cigar"][0], out["n_cigar"][0]) == "30M"
    # a read whose last 10 bases are all mismatches: the early end after 20
    # bases scores h0 + 20; the end-to-end alignment at best h0 + 20 - (6 + 10)
    q = r[:30].copy()
    q[20:] = (r[20:30] + 1) % 4
    small = _run([(q, r[:30])], sc, 20, 5)   # 16 > 5: clipped
    assert (small["score"][0], small["read_end"][0], small["ref_end"][0]) == (40, 20, 20)
    large = _run([(q, r[:30])], sc, 20, 16)  # within the penalty: end to end
    assert (large["score"][0], large["read_end"][0]) == (24, 30)
    assert oracle.decode_cigar(large["cigar"][0], large["n_cigar"][0]) == "20M10I"
    # empty read or window
    e1 = _run([((), r[:5])], sc, 7, 0)
    assert (e1["score"][0], e1["read_end"][0], e1["ref_end"][0], e1["n_cigar"][0]) == (7, 0, 0, 0)
    e2 = _run([(r[:3], ())], sc, 7, 100)  # end to end: 3 insertions at the anchor
    assert (e2["score"][0], e2["read_end"][0], e2["ref_end"][0]) == (7 - 9, 3, 0)
    assert oracle.decode_cigar(e2["cigar"][0], e2["n_cigar"][0]) == "3I"


def test_extension_invariants():
    rng = np.random.default_rng(9)
    sc = (1, -4, 6, 1)
    pairs = [(rng.integers(0, 4, int(rng.integers(1, 40))), rng.integers(0, 4, int(rng.integers(1, 60))))
             for _ in range(200)]
    base = _run(pairs, sc, 10, 3)
    # the empty extension is a candidate: never below h0 - clip
    assert (base["score"] >= 10 - 3).all()
    # start score shifts every score and keeps every coordinate
    shifted = _run(pairs, sc, 25, 3)
    assert np.array_equal(shifted["score"] - base["score"], np.full(len(pairs), 15))
    for k in ("read_end", "ref_end", "n_cigar"):
        assert np.array_equal(shifted[k], base[k])
    # a clipping penalty of 0 never prefers a lower end-to-end score; a huge
    # one always aligns the whole read
    full = _run(pairs, sc, 10, 1 << 19)
    assert all(full["read_end"][p] == len(q) for p, (q, _) in enumerate(pairs))
    # the CIGAR starts at the anchor and spans exactly the reported ends
    for p, (q, r) in enumerate(pairs):
        ops = [(int(w) >> 4, int(w) & 15) for w in base["cigar"][p][: base["n_cigar"][p]]]
        total, i, j = brute.rescore(q, r, 0, 0, ops, sc)
        assert (i, j) == (base["read_end"][p], base["ref_end"][p])
        assert total + 10 == base["score"][p]
