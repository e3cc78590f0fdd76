"""Pin the oracle to exhaustive enumeration of alignments (CPU only).

Score and tie-broken end cell: every pair of sequences with m, n <= 4 in
both modes, plus 20,000 random pairs with m, n <= 6.  Start cell and CIGAR:
the canonical alignment (backward priorities stop > M > D > I, open >
extend) for every pair with m, n <= 3 and for random pairs up to 6, under
several scoring schemes, including ones with many ties.
"""
import itertools

import numpy as np
import pytest

import brute
import oracle

SCORINGS = [(1, -4, 6, 1), (2, -3, 5, 2), (1, -1, 1, 1), (3, 0, 2, 1), (1, -2, 0, 1)]


def all_seqs(k):
    if k == 0:
        return np.zeros((1, 0), np.uint8)
    return np.array(list(itertools.product(range(4), repeat=k)), np.uint8)


def run_oracle(Q, R, mode, sc, trace=False):
    N, m = Q.shape
    n = R.shape[1]
    return oracle.align_batch(
        R.reshape(-1), np.arange(N, dtype=np.int64) * n, np.full(N, n, np.int32),
        Q.reshape(-1), np.arange(N, dtype=np.int64) * m, np.full(N, m, np.int32),
        np.full(N, mode, np.uint8), sc, trace=trace, cigar_cap=64)


def brute_chunked(Q, R, mode, sc, chunk=4096):
    outs = [brute.best_batch(Q[k:k + chunk], R[k:k + chunk], mode, sc) for k in range(0, len(Q), chunk)]
    return tuple(np.concatenate([o[i] for o in outs]) for i in range(3))


@pytest.mark.parametrize("mode", [0, 1])
def test_exhaustive_score_and_end_cell_upto_4(mode):
    sc = (1, -4, 6, 1)
    for m in range(0, 5):
        for n in range(0, 5):
            qs, rs = all_seqs(m), all_seqs(n)
            Q = np.repeat(qs, len(rs), axis=0)
            R = np.tile(rs, (len(qs), 1))
            got = run_oracle(Q, R, mode, sc)
            s, bi, bj = brute_chunked(Q, R, mode, sc)
            assert np.array_equal(got["score"], s), (m, n)
            assert np.array_equal(got["read_end"], bi), (m, n)
            assert np.array_equal(got["ref_end"], bj), (m, n)
            assert not got["status"].any()


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("sc", SCORINGS)
def test_random_score_and_end_cell_upto_6(mode, sc):
    rng = np.random.default_rng(1402 + 10 * mode + SCORINGS.index(sc))
    total = 0
    for m in range(1, 7):
        for n in range(1, 7):
            N = 2000 // 36 + 1 if sc != (1, -4, 6, 1) else 20000 // 36 + 1
            Q = rng.integers(0, 4, (N, m), dtype=np.uint8)
            R = rng.integers(0, 4, (N, n), dtype=np.uint8)
            got = run_oracle(Q, R, mode, sc)
            s, bi, bj = brute_chunked(Q, R, mode, sc)
            assert np.array_equal(got["score"], s), (m, n)
            assert np.array_equal(got["read_end"], bi), (m, n)
            assert np.array_equal(got["ref_end"], bj), (m, n)
            total += N
    assert total >= (20000 if sc == (1, -4, 6, 1) else 2000)


def _check_canonical(q, r, mode, sc, got, p):
    score, (ei, ej), (si, sj), cig = brute.canonical(q, r, mode, sc)
    assert got["score"][p] == score
    assert (got["read_end"][p], got["ref_end"][p]) == (ei, ej)
    assert (got["read_start"][p], got["ref_start"][p]) == (si, sj), (q, r, mode, sc)
    nc = got["n_cigar"][p]
    assert oracle.decode_cigar(got["cigar"][p], nc) == "".join(cig), (q, r, mode, sc)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("sc", [(1, -4, 6, 1), (3, 0, 2, 1), (1, -1, 1, 1)])
def test_exhaustive_traceback_upto_3(mode, sc):
    for m in range(0, 4):
        for n in range(0, 4):
            qs, rs = all_seqs(m), all_seqs(n)
            Q = np.repeat(qs, len(rs), axis=0)
            R = np.tile(rs, (len(qs), 1))
            got = run_oracle(Q, R, mode, sc, trace=True)
            for p in range(len(Q)):
                _check_canonical(Q[p], R[p], mode, sc, got, p)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("sc", SCORINGS[:4])
def test_random_traceback_upto_6(mode, sc):
    rng = np.random.default_rng(4876 + mode + 7 * SCORINGS.index(sc))
    for _ in range(120):
        m = int(rng.integers(1, 7))
        n = int(rng.integers(1, 7))
        q = rng.integers(0, 4, m, dtype=np.uint8)
        r = rng.integers(0, 4, n, dtype=np.uint8)
        got = run_oracle(q[None], r[None], mode, sc, trace=True)
        _check_canonical(q, r, mode, sc, got, 0)


def test_tie_breaks_listed_by_enumeration():
    """The end cell is the lexicographic minimum of (-score, j, i) over every optimal end."""
    rng = np.random.default_rng(99)
    for mode in (0, 1):
        for _ in range(300):
            m = int(rng.integers(1, 6))
            n = int(rng.integers(1, 6))
            q = rng.integers(0, 2, m, dtype=np.uint8)  # two letters: many ties
            r = rng.integers(0, 2, n, dtype=np.uint8)
            score, cells = brute.optimal_end_cells(q, r, mode, (1, -1, 1, 1))
            want = min(cells, key=lambda c: (c[1], c[0]))
            got = run_oracle(q[None], r[None], mode, (1, -1, 1, 1))
            assert got["score"][0] == score
            assert (got["read_end"][0], got["ref_end"][0]) == want
