"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer outputs must be identical element by element: score, start and end
coordinates, CIGAR runs and per-pair status (the GPU-only saturation note
excluded).  Sizes span many work items, several tiles of 16 / 64 lanes and
ragged tails; the full-size config-1 batch is checked on a sample of pairs
in the launch configuration the benchmark times.
"""
import os

import numpy as np
import pytest

import gpu_util as U
import synth

pytestmark = pytest.mark.gpu

SC = (1, -4, 6, 1)
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ctx():
    import torch

    import paper_1402_4876_amd as mica
    torch.cuda.set_device(0)
    c = mica.Context(0)
    yield c
    c.close()


def _pairs_batch(pairs, modes):
    """Batch from explicit (read codes, window codes) lists."""
    rl = np.array([len(q) for q, _ in pairs], np.int32)
    wl = np.array([len(r) for _, r in pairs], np.int32)
    ref = np.concatenate([np.asarray(r, np.uint8) for _, r in pairs] + [np.zeros(16, np.uint8)])
    win_off = np.concatenate([[0], np.cumsum(wl.astype(np.int64))[:-1]])
    codes = np.zeros((len(pairs), max(int(rl.max()), 1)), np.uint8)
    for k, (q, _) in enumerate(pairs):
        codes[k, :len(q)] = q
    return synth._finish("explicit", ref, win_off, wl, codes, rl, np.asarray(modes, np.uint8))


def test_hand_examples(ctx):
    import test_oracle_pins as P
    pairs = [(q, r) for _, q, r, *_ in P.HAND]
    modes = [m for m, *_ in P.HAND]
    b = _pairs_batch(pairs, modes)
    g = U.run_gpu(ctx, b, SC)
    U.assert_same(g, U.run_oracle(b, SC), what="hand")
    # and the stated values themselves
    for k, (_, _, _, score, coords, cig) in enumerate(P.HAND):
        assert g["score"][k] == score
        assert (g["read_start"][k], g["read_end"][k], g["ref_start"][k], g["ref_end"][k]) == coords


def test_tie_cases(ctx):
    import test_oracle_pins as P
    for mode, sc, q, r in P.TIES:
        b = _pairs_batch([(q, r)] * 5, [mode] * 5)
        U.assert_same(U.run_gpu(ctx, b, sc), U.run_oracle(b, sc), what="tie %s" % (sc,))


@pytest.mark.parametrize("seed,sc", [(1, (1, -4, 6, 1)), (2, (3, 0, 2, 1)), (3, (2, -3, 5, 2)),
                                     (4, (1, -1, 1, 1)), (5, (5, -4, 0, 1))])
def test_tiny_random_mixed(ctx, seed, sc):
    b = synth.tiny_random(1500, 70, 120, seed)
    o = U.run_oracle(b, sc)
    U.assert_same(U.run_gpu(ctx, b, sc), o, what="persistent")
    U.assert_same(U.run_gpu(ctx, b, sc, plain=True), o, what="plain")
    U.assert_same(U.run_gpu(ctx, b, sc, force_int32=True), o, what="int32")


def test_score_only_paths(ctx):
    b = synth.tiny_random(1500, 256, 300, 9)
    o = U.run_oracle(b, SC, trace=False)
    U.assert_same(U.run_gpu(ctx, b, SC, trace=False), o, trace=False, what="k16")
    U.assert_same(U.run_gpu(ctx, b, SC, trace=False, force_int32=True), o, trace=False, what="k32")


def test_config0(ctx):
    b = synth.config0()
    o = U.run_oracle(b, SC, trace=False)
    U.assert_same(U.run_gpu(ctx, b, SC, trace=False, force_int32=True), o, trace=False, what="c0 int32")
    U.assert_same(U.run_gpu(ctx, b, SC, trace=False), o, trace=False, what="c0 int16")
    ot = U.run_oracle(b, SC)
    U.assert_same(U.run_gpu(ctx, b, SC), ot, what="c0 full")


def test_config1_mini(ctx):
    b = synth.config1(n_pairs=20000, ref_len=2_000_000)
    U.assert_same(U.run_gpu(ctx, b, SC), U.run_oracle(b, SC), what="c1 mini")


def test_config2_mini(ctx):
    b = synth.config2(n_pairs=6000, ref_len=2_000_000)
    U.assert_same(U.run_gpu(ctx, b, SC), U.run_oracle(b, SC), what="c2 mini")


def test_config3_mini_persistent_equals_plain(ctx):
    b = synth.config3(n_pairs=20000, ref_len=2_000_000)
    o = U.run_oracle(b, SC)
    gp = U.run_gpu(ctx, b, SC)
    U.assert_same(gp, o, what="c3 persistent")
    gq = U.run_gpu(ctx, b, SC, plain=True)
    U.assert_equal_outputs(gp, gq, "plain vs persistent")


def test_forced_saturation_rerun(ctx):
    """Scaling every score by 150 saturates int16 on 250 bp reads only; those pairs
    are recomputed in int32, and results equal the oracle's (score x 150)."""
    b = synth.serving_like(3000, seed=1)
    k = 150
    sck = tuple(k * x for x in SC)
    g = U.run_gpu(ctx, b, sck)
    o = U.run_oracle(b, SC)
    U.assert_same(g, o, score_scale=k, what="scaled")
    sat = (g["status"] & 1) != 0
    assert sat.any(), "no pair saturated"
    assert not sat[b.read_len == 100].any()
    assert sat[b.read_len == 250].mean() > 0.5


def test_edge_cases(ctx):
    rng = np.random.default_rng(3)
    R = lambda n: rng.integers(0, 4, n, dtype=np.uint8)  # noqa: E731
    pairs, modes = [], []
    for mode in (0, 1):
        for q, r in [(R(0), R(10)), (R(10), R(0)), (R(0), R(0)), (R(1), R(1)), (R(1), R(7)),
                     (R(16), R(16)), (R(17), R(33)), (R(256), R(300)), (R(255), R(8)), (R(3), R(900)),
                     (R(40), R(40))]:
            pairs.append((q, r))
            modes.append(mode)
    b = _pairs_batch(pairs, modes)
    U.assert_same(U.run_gpu(ctx, b, SC), U.run_oracle(b, SC), what="edges")
    U.assert_same(U.run_gpu(ctx, b, SC, cap=1), U.run_oracle(b, SC, cap=1), cap=1, what="cap1")
    U.assert_same(U.run_gpu(ctx, b, SC, cap=0), U.run_oracle(b, SC, cap=0), cap=0, what="cap0")


def test_long_reads_wave_per_pair(ctx):
    """Reads of 257..1024 bases use the 64-lane class; windows up to 1,300."""
    rng = np.random.default_rng(4)
    pairs, modes = [], []
    for k in range(24):
        m = int(rng.integers(257, 1025))
        n = int(rng.integers(m // 2, 1300))
        r = rng.integers(0, 4, n, dtype=np.uint8)
        q = rng.integers(0, 4, m, dtype=np.uint8)
        if n >= m and k % 2 == 0:
            s = int(rng.integers(0, n - m + 1))
            q = r[s:s + m].copy()
            q[rng.integers(0, m, 5)] = rng.integers(0, 4, 5)
        pairs.append((q, r))
        modes.append(k % 3 == 0)
    b = _pairs_batch(pairs, modes)
    U.assert_same(U.run_gpu(ctx, b, SC), U.run_oracle(b, SC), what="long")
    U.assert_same(U.run_gpu(ctx, b, SC, force_int32=True), U.run_oracle(b, SC), what="long int32")


def test_long_window(ctx):
    rng = np.random.default_rng(5)
    pairs = [(rng.integers(0, 4, m, dtype=np.uint8), rng.integers(0, 4, 8192, dtype=np.uint8)) for m in (5, 150, 600)]
    pairs[1] = (pairs[1][1][4000:4150].copy(), pairs[1][1])
    b = _pairs_batch(pairs + pairs, [0, 0, 0, 1, 1, 1])
    U.assert_same(U.run_gpu(ctx, b, SC), U.run_oracle(b, SC), what="n=8192")


def test_pair_status_codes(ctx):
    import torch

    import paper_1402_4876_amd as mica
    b = synth.tiny_random(64, 30, 40, 11)
    dev = mica.to_device(b)
    win_off = dev["win_off"].clone()
    read_off = dev["read_off"].clone()
    read_len = dev["read_len"].clone()
    mode = dev["mode"].clone()
    win_off[3] = dev["ref_len"] - 2           # window past the end of the reference
    read_off[5] = dev["reads_len"] + 100      # read outside the read buffer
    read_len[7] = 31                          # above max_read_len (30)
    mode[9] = 3                               # not a mode
    out = mica.align(ctx, dev["ref2b"], win_off, dev["win_len"], dev["reads2b"], read_off, read_len,
                     mode=mode, out_cigar=True, ref_len=dev["ref_len"], reads_len=dev["reads_len"],
                     max_read_len=30, max_win_len=40)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    if b.win_len[3] > 2:
        assert st[3] == mica.ST_WIN_OOB
    assert st[5] == mica.ST_READ_OOB
    assert st[7] == mica.ST_LEN_LIMIT
    assert st[9] == mica.ST_LEN_LIMIT
    for p in (5, 7, 9):
        assert out["score"][p].item() == 0 and out["n_cigar"][p].item() == 0
    keep = np.setdiff1d(np.arange(64), [3, 5, 7, 9])
    o = U.run_oracle(b, SC, idx=keep)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    U.assert_same(g, o, idx=keep, what="others")


def test_batch_order_and_repeats(ctx):
    b = synth.config3(n_pairs=6000, ref_len=1_000_000)
    g1 = U.run_gpu(ctx, b, SC)
    g2 = U.run_gpu(ctx, b, SC)
    U.assert_equal_outputs(g1, g2, "repeat")
    perm = np.random.default_rng(6).permutation(b.n_pairs)
    gp = U.run_gpu(ctx, b.subset(perm), SC)
    U.assert_equal_outputs(gp, {k: v[perm] for k, v in g1.items()}, "permuted")


def test_default_mode_without_mode_array(ctx):
    b = synth.tiny_random(500, 40, 60, 12, mode=1)
    U.assert_same(U.run_gpu(ctx, b, SC, mode=None), U.run_oracle(b, SC), what="default local")


def test_pack_2bit_on_gpu(ctx):
    import torch

    import paper_1402_4876_amd as mica
    codes = np.random.default_rng(7).integers(0, 4, 100003, dtype=np.uint8)
    w = mica.pack_2bit(torch.from_numpy(codes).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(w.cpu().numpy().view(np.uint32), mica.pack_codes(codes))


def _spans_consistent(g):
    """Every pair's CIGAR consumes exactly its reported read and window spans."""
    cig = g["cigar"].astype(np.uint32)
    nc = g["n_cigar"]
    assert (nc >= 0).all()
    col = np.arange(cig.shape[1])[None, :] < nc[:, None]
    L = np.where(col, cig >> 4, 0)
    op = cig & 15
    read_span = (L * ((op == 0) | (op == 1))).sum(axis=1)
    ref_span = (L * ((op == 0) | (op == 2))).sum(axis=1)
    assert np.array_equal(read_span, g["read_end"] - g["read_start"])
    assert np.array_equal(ref_span, g["ref_end"] - g["ref_start"])


@pytest.mark.parametrize("launch", ["one_class", "persistent", "plain"])
def test_config1_full_size_sampled(ctx, launch):
    """The benchmark's batch (10^6 pairs, far more work items than resident waves):
    in the launch the benchmark times (one read length: its class kernel, as with
    min_read_len = max_read_len = 150) and through both general launch styles;
    sampled pairs against the oracle, every pair against properties that hold
    at any size."""
    b = synth.config1()
    g = U.run_gpu(ctx, b, SC, max_read_len=150, max_win_len=400, plain=launch == "plain",
                  min_read_len=150 if launch == "one_class" else 0)
    idx = np.sort(np.random.default_rng(8).choice(b.n_pairs, 3000, replace=False))
    U.assert_same(g, U.run_oracle(b, SC, idx=idx), idx=idx, what="c1 sample")
    assert not g["status"].any()
    assert (g["read_start"] == 0).all() and (g["read_end"] == 150).all()
    assert (g["score"] <= 150).all()
    assert (g["ref_start"] <= g["ref_end"]).all() and (g["ref_end"] <= 400).all()
    _spans_consistent(g)


def test_config2_full_size_sampled(ctx):
    """The 5 x 10^5-pair local workload as the benchmark runs it (one class):
    sampled pairs against the oracle, every pair against local-mode properties."""
    b = synth.config2()
    g = U.run_gpu(ctx, b, SC, max_read_len=150, max_win_len=int(b.win_len.max()), min_read_len=150)
    idx = np.sort(np.random.default_rng(9).choice(b.n_pairs, 2000, replace=False))
    U.assert_same(g, U.run_oracle(b, SC, idx=idx), idx=idx, what="c2 sample")
    assert not (g["status"] & ~1).any()
    assert (g["score"] >= 0).all() and (g["score"] <= 150).all()
    assert (g["read_start"] <= g["read_end"]).all() and (g["read_end"] <= 150).all()
    _spans_consistent(g)


def test_config3_full_size_sampled(ctx):
    """The 2 x 10^6-pair mixed workload in its persistent launch: sampled pairs
    against the oracle (both modes, every read length), every pair against
    properties that hold at any size."""
    b = synth.config3()
    g = U.run_gpu(ctx, b, SC, max_read_len=int(b.read_len.max()), max_win_len=int(b.win_len.max()))
    idx = np.sort(np.random.default_rng(10).choice(b.n_pairs, 2000, replace=False))
    U.assert_same(g, U.run_oracle(b, SC, idx=idx), idx=idx, what="c3 sample")
    assert not (g["status"] & ~1).any()
    assert (g["read_end"] <= b.read_len).all() and (g["ref_end"] <= b.win_len).all()
    sg = b.mode == 0
    assert (g["read_start"][sg] == 0).all() and (g["read_end"][sg] == b.read_len[sg]).all()
    _spans_consistent(g)


def test_min_read_len_hint(ctx):
    """A batch of one length class (bounded by min_read_len) runs its class
    kernel instead of the persistent ones, with the same results; a pair
    below the bound is rejected per pair."""
    import paper_1402_4876_amd as mica
    b = synth.config1(n_pairs=5000, ref_len=1_000_000)
    o = U.run_oracle(b, SC)
    g = U.run_gpu(ctx, b, SC, min_read_len=150)
    U.assert_same(g, o, what="one class")
    U.assert_equal_outputs(g, U.run_gpu(ctx, b, SC), "hinted vs not")
    g2 = U.run_gpu(ctx, b, SC, min_read_len=150, max_read_len=150)
    U.assert_same(g2, o, what="tight bounds")
    mixed = synth.tiny_random(800, 60, 90, 21)
    gm = U.run_gpu(ctx, mixed, SC, min_read_len=20)
    low = mixed.read_len < 20
    assert (gm["status"][low] == mica.ST_LEN_LIMIT).all()
    keep = np.nonzero(~low)[0]
    U.assert_same(gm, U.run_oracle(mixed, SC, idx=keep), idx=keep, what="above the bound")
