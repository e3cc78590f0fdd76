"""Pin the oracle with hand examples, closed forms and invariants (CPU only)."""
import os

import numpy as np
import pytest

import brute
import oracle

SC = (1, -4, 6, 1)
CODE = {"A": 0, "C": 1, "G": 2, "T": 3}
HERE = os.path.dirname(os.path.abspath(__file__))


def enc(s):
    return np.array([CODE[c] for c in s if c != "-"], np.uint8)


def load_hand_examples():
    rows = []
    with open(os.path.join(HERE, "golden", "hand_examples.tsv")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            mode, q, r, score, rs, re_, fs, fe, cig, _ = line.rstrip("\n").split("\t")
            rows.append((0 if mode == "sg" else 1, enc(q), enc(r), int(score),
                         (int(rs), int(re_), int(fs), int(fe)), "" if cig == "-" else cig))
    return rows


HAND = load_hand_examples()


@pytest.mark.parametrize("row", HAND, ids=[str(i) for i in range(len(HAND))])
def test_hand_example(row):
    mode, q, r, score, coords, cig = row
    # re-derive the expected row by exhaustive search (every alignment scoring at
    # least the stated score), independent of the oracle
    bscore, (ei, ej), (si, sj), bcig = brute.canonical_at_least(q, r, mode, SC, score)
    assert (bscore, si, ei, sj, ej, "".join(bcig)) == (score, *coords, cig)
    got = oracle.align_pairs([(q, r)], mode=mode, scoring=SC)
    assert got["score"][0] == score
    assert (got["read_start"][0], got["read_end"][0], got["ref_start"][0], got["ref_end"][0]) == coords
    assert oracle.decode_cigar(got["cigar"][0], got["n_cigar"][0]) == cig


def rand_seq(rng, n):
    return rng.integers(0, 4, n, dtype=np.uint8)


def test_closed_forms():
    """Planted edits in long random sequences: the optimum equals the planted score."""
    rng = np.random.default_rng(7)
    a, b, o, e = SC
    for trial in range(40):
        m = int(rng.integers(60, 160))
        read = rand_seq(rng, m)
        pad_l, pad_r = rand_seq(rng, 30), rand_seq(rng, 30)
        # identical read
        win = np.concatenate([pad_l, read, pad_r])
        for mode in (0, 1):
            got = oracle.align_pairs([(read, win)], mode=mode, scoring=SC)
            assert got["score"][0] == m * a
            assert (got["ref_start"][0], got["ref_end"][0]) == (30, 30 + m)
        # one substitution in the middle
        k = m // 2
        mut = read.copy()
        mut[k] = (mut[k] + 1 + rng.integers(0, 3)) % 4
        got = oracle.align_pairs([(mut, win)], mode=0, scoring=SC)
        assert got["score"][0] == (m - 1) * a + b
        assert oracle.decode_cigar(got["cigar"][0], got["n_cigar"][0]) == "%dM" % m
        # semi-global deletion of L window bases (read skips them)
        L = int(rng.integers(1, 6))
        cut = np.concatenate([read[:k], read[k + L:]])
        got = oracle.align_pairs([(cut, win)], mode=0, scoring=SC)
        assert got["score"][0] == (m - L) * a - (o + L * e)
        # semi-global insertion of L read bases absent from the window
        ins = np.concatenate([read[:k], rand_seq(rng, L), read[k:]])
        got = oracle.align_pairs([(ins, win)], mode=0, scoring=SC)
        assert got["score"][0] == m * a - (o + L * e)


def cig_ops(words, n):
    return [(int(w) >> 4, int(w) & 15) for w in words[:n]]


def test_cigar_rescores_to_score_and_spans_coordinates():
    rng = np.random.default_rng(11)
    for _ in range(300):
        m = int(rng.integers(0, 40))
        n = int(rng.integers(0, 60))
        q, r = rand_seq(rng, m), rand_seq(rng, n)
        if rng.random() < 0.5 and n >= m > 0:  # related pair
            s = int(rng.integers(0, n - m + 1))
            q = r[s:s + m].copy()
            for _ in range(int(rng.integers(0, 4))):
                q[int(rng.integers(0, m))] = rng.integers(0, 4)
        for mode in (0, 1):
            got = oracle.align_pairs([(q, r)], mode=mode, scoring=SC)
            ops = cig_ops(got["cigar"][0], got["n_cigar"][0])
            tot, ie, je = brute.rescore(q, r, got["read_start"][0], got["ref_start"][0], ops, SC)
            assert tot == got["score"][0]
            assert (ie, je) == (got["read_end"][0], got["ref_end"][0])
            if mode == 0:
                assert got["read_start"][0] == 0 and got["read_end"][0] == m


def test_invariants():
    rng = np.random.default_rng(12)
    for _ in range(150):
        m = int(rng.integers(1, 50))
        n = int(rng.integers(1, 80))
        q, r = rand_seq(rng, m), rand_seq(rng, n)
        sg = oracle.align_pairs([(q, r)], mode=0, scoring=SC)
        lo = oracle.align_pairs([(q, r)], mode=1, scoring=SC)
        assert lo["score"][0] >= sg["score"][0]
        assert lo["score"][0] >= 0
        # a base permutation applied to both sequences changes nothing
        perm = rng.permutation(4).astype(np.uint8)
        for mode, ref in ((0, sg), (1, lo)):
            got = oracle.align_pairs([(perm[q], perm[r])], mode=mode, scoring=SC)
            for k in ("score", "read_start", "read_end", "ref_start", "ref_end", "n_cigar"):
                assert got[k][0] == ref[k][0]
            assert np.array_equal(got["cigar"][0], ref["cigar"][0])
        # scaling every parameter by k scales the score, keeps coordinates and CIGAR
        kk = int(rng.integers(2, 40))
        sck = tuple(kk * x for x in SC)
        for mode, ref in ((0, sg), (1, lo)):
            got = oracle.align_pairs([(q, r)], mode=mode, scoring=sck)
            assert got["score"][0] == kk * ref["score"][0]
            for k in ("read_start", "read_end", "ref_start", "ref_end", "n_cigar"):
                assert got[k][0] == ref[k][0]
            assert np.array_equal(got["cigar"][0], ref["cigar"][0])
        # reversing both sequences keeps the score
        for mode, ref in ((0, sg), (1, lo)):
            got = oracle.align_pairs([(q[::-1], r[::-1])], mode=mode, scoring=SC)
            assert got["score"][0] == ref["score"][0]
        # local alignment is symmetric in its two sequences
        sw = oracle.align_pairs([(r, q)], mode=1, scoring=SC)
        assert sw["score"][0] == lo["score"][0]


def test_batch_order_and_threads_do_not_matter():
    rng = np.random.default_rng(13)
    pairs = [(rand_seq(rng, int(rng.integers(0, 70))), rand_seq(rng, int(rng.integers(0, 90))))
             for _ in range(500)]
    modes = rng.integers(0, 2, len(pairs)).astype(np.uint8)
    ref = oracle.align_pairs(pairs, mode=modes, scoring=SC, threads=1)
    perm = rng.permutation(len(pairs))
    got = oracle.align_pairs([pairs[i] for i in perm], mode=modes[perm], scoring=SC, threads=8)
    for k in ref:
        assert np.array_equal(got[k], ref[k][perm]), k


def test_edge_cases_and_status():
    a, b, o, e = SC
    # SG with an empty read: score 0 at ref [0, 0); empty window: all insertion
    got = oracle.align_pairs([(enc(""), enc("ACGT")), (enc("ACG"), enc(""))], mode=0, scoring=SC)
    assert list(got["score"]) == [0, -(o + 3 * e)]
    assert oracle.decode_cigar(got["cigar"][1], got["n_cigar"][1]) == "3I"
    # local with nothing positive
    got = oracle.align_pairs([(enc("AAAA"), enc("CCCC"))], mode=1, scoring=SC)
    assert got["score"][0] == 0 and got["n_cigar"][0] == 0
    # CIGAR capacity: an alternating alignment needs many ops
    q = enc("ACGTACGTACGTACGTACGT")
    r = enc("ACGATCGAACGTTCGTAAGT")
    full = oracle.align_pairs([(q, r)], mode=0, scoring=(1, -4, 0, 1), cigar_cap=4096)
    need = full["n_cigar"][0]
    assert need > 3
    cut = oracle.align_pairs([(q, r)], mode=0, scoring=(1, -4, 0, 1), cigar_cap=3)
    assert cut["status"][0] & oracle.ST_CIGAR_TRUNC
    assert cut["n_cigar"][0] == -need
    assert np.array_equal(cut["cigar"][0], full["cigar"][0][:3])
    # pair-level limits: read too long, window outside the reference, read outside the buffer
    R = np.zeros(3000, np.uint8)
    W = np.zeros(100, np.uint8)
    res = oracle.align_batch(W, np.array([0, 90, 0], np.int64), np.array([10, 20, 10], np.int32),
                             R, np.array([0, 0, 2995], np.int64), np.array([1025, 5, 10], np.int32),
                             None, SC, trace=True)
    assert list(res["status"]) == [oracle.ST_LEN_LIMIT, oracle.ST_WIN_OOB, oracle.ST_READ_OOB]
    assert not res["score"].any()
    with pytest.raises(ValueError):
        oracle.align_pairs([(q, r)], scoring=(0, -4, 6, 1))


def load_tie_cases():
    rows = []
    with open(os.path.join(HERE, "golden", "tie_cases.tsv")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            mode, sc, q, r = line.split()
            rows.append((0 if mode == "sg" else 1, tuple(int(x) for x in sc.split(",")), enc(q), enc(r)))
    return rows


TIES = load_tie_cases()


@pytest.mark.parametrize("row", TIES, ids=[str(i) for i in range(len(TIES))])
def test_gap_open_extend_tie_case(row):
    """Inputs where 'open beats extend' decides the traceback; expected by enumeration."""
    mode, sc, q, r = row
    score, (ei, ej), (si, sj), cig = brute.canonical(q, r, mode, sc)
    got = oracle.align_pairs([(q, r)], mode=mode, scoring=sc)
    assert (got["score"][0], got["read_end"][0], got["ref_end"][0]) == (score, ei, ej)
    assert (got["read_start"][0], got["ref_start"][0]) == (si, sj)
    assert oracle.decode_cigar(got["cigar"][0], got["n_cigar"][0]) == "".join(cig)
