"""The seeded input generators: shapes, planted alignments, rates, determinism."""
import numpy as np

import oracle
import synth


def test_config0_shape_and_planted_copy():
    b = synth.config0(record=True)
    assert b.n_pairs == 1000 and b.cells() == 3 * 10 ** 7
    assert (b.read_len == 150).all() and (b.win_len == 200).all()
    assert (b.planted_start >= 0).all() and (b.planted_start <= 50).all()
    assert (b.planted_end <= 200).all()
    assert (b.read_off % 16 == 0).all()
    for p in range(200):
        q, w = b.read_codes(p), b.window_codes(p)
        i, j = 0, int(b.planted_start[p])
        ins = 0
        for op, L in b.planted_ops[p]:
            if op == "M":
                i += L
                j += L
            elif op == "I":
                i += L
                ins += L
            else:
                j += L
        assert i == 150 and j == b.planted_end[p]


def test_planted_alignment_bounds_the_optimum():
    """The semi-global optimum is at least the planted alignment's score."""
    b = synth.config1(n_pairs=300, ref_len=200_000, record=True)
    o = oracle.align_batch(b.ref, b.win_off, b.win_len, b.reads, b.read_off, b.read_len, b.mode)
    a, bb, go, ge = synth.SCORING
    for p in range(b.n_pairs):
        q, w = b.read_codes(p), b.window_codes(p)
        i, j, s = 0, int(b.planted_start[p]), 0
        ops = list(b.planted_ops[p])
        while ops and ops[0][0] == "D":  # leading / trailing deletions are free in semi-global
            j += ops.pop(0)[1]
        while ops and ops[-1][0] == "D":
            ops.pop()
        for op, L in ops:
            if op == "M":
                s += sum(a if q[i + t] == w[j + t] else bb for t in range(L))
                i += L
                j += L
            elif op == "I":
                s -= go + L * ge
                i += L
            else:
                s -= go + L * ge
                j += L
        assert o["score"][p] >= s


def test_error_rates_match_the_recipe():
    b = synth.config1(n_pairs=4000, ref_len=500_000, record=True)
    n_m = n_i = n_d = 0
    ins_len = []
    for ops in b.planted_ops:
        for op, L in ops:
            if op == "M":
                n_m += L
            elif op == "I":
                n_i += 1
                ins_len.append(L)
            else:
                n_d += 1
    events = (n_i + n_d) / (4000 * 150)
    assert 0.002 < events < 0.004  # 0.3% indels per step
    subs = 0
    for p in range(500):
        q, w = b.read_codes(p), b.window_codes(p)
        if all(op == "M" for op, _ in b.planted_ops[p]):
            s = int(b.planted_start[p])
            subs += int((q != w[s:s + 150]).sum())
    assert 0.005 < subs / (500 * 150) < 0.02


def test_determinism_and_config_shapes():
    assert synth.config0().digest() == synth.config0().digest()
    c3 = synth.config3(n_pairs=5000, ref_len=300_000)
    assert c3.read_len.min() >= 50 and c3.read_len.max() <= 250
    assert np.array_equal(c3.win_len, (3 * c3.read_len) // 2 + 64)
    assert 0.45 < c3.mode.mean() < 0.55
    c2 = synth.config2(n_pairs=5000, ref_len=300_000)
    assert (c2.win_len == 1000).all() and (c2.mode == 1).all()
    assert 0.08 < c2.random_partner.mean() < 0.12
    s = synth.serving_like(500)
    assert set(np.unique(s.read_len)) <= {100, 150, 250}


def test_long_reference_batch_offsets_and_rebase():
    """Windows past 2^31 and 2^32 of a > 4 Gbp packed reference, each inside a
    random stretch; unaligned read offsets; the rebased copy holds the same
    window bases and reads."""
    b, starts = synth.long_reference_batch(600)
    assert len(b.ref) * 16 == synth.LONG_REF_LEN > (1 << 32)
    end = b.win_off + b.win_len
    assert ((b.win_off < (1 << 31)) & (end > (1 << 31))).sum() >= 50
    assert ((b.win_off < (1 << 32)) & (end > (1 << 32))).sum() >= 50
    assert (end == synth.LONG_REF_LEN).sum() >= 50 and (end <= synth.LONG_REF_LEN).all()
    inside = np.zeros(b.n_pairs, bool)
    for s0 in starts:
        inside |= (b.win_off >= s0) & (end <= s0 + (1 << 16))
    assert inside.all()
    assert len(np.unique(b.read_off % 16)) == 16
    small = synth.rebase_windows(b)
    assert small.ref_packed is False and len(small.ref) == int(b.win_len.sum()) + 16
    for p in range(0, b.n_pairs, 7):
        assert np.array_equal(small.window_codes(p), b.window_codes(p))
        assert np.array_equal(small.read_codes(p), b.read_codes(p))
