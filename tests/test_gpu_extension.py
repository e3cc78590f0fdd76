"""GPU parity of the extension mode (mode 2: DP from a seed anchor with
clipped read ends) against the CPU oracle, through the C ABI.

Integer outputs must be identical element by element.  Cases cover random
pairs under several scorings, anchor scores and clipping penalties, batches
that mix all three modes, per-pair and default anchor scores, empty reads
and windows, anchors large enough to saturate 16-bit scores (re-run in
32 bits), forced 32-bit kernels, plain per-bucket launches, the mode mask,
maximum sizes and a seed-extension workload at full size (sampled).
"""
import numpy as np
import pytest

import gpu_util as U
import synth

pytestmark = pytest.mark.gpu

SC = (1, -4, 6, 1)


@pytest.fixture(scope="module")
def ctx():
    import torch

    import paper_1402_4876_amd as mica
    torch.cuda.set_device(0)
    c = mica.Context(0)
    yield c
    c.close()


def _with_h0(b, lo, hi, seed):
    b.h0 = np.random.default_rng(seed).integers(lo, hi + 1, b.n_pairs).astype(np.int32)
    return b


@pytest.mark.parametrize("seed,sc,clip", [(1, (1, -4, 6, 1), 5), (2, (3, 0, 2, 1), 0), (3, (2, -3, 5, 2), 12),
                                          (4, (1, -1, 1, 1), 1 << 20), (5, (5, -4, 0, 1), 3),
                                          (6, (1, -4, 6, 1), 0)])
def test_tiny_random_extension(ctx, seed, sc, clip):
    b = _with_h0(synth.tiny_random(1500, 70, 120, seed, mode=2), 0, 60, seed)
    o = U.run_oracle(b, sc, clip=clip)
    U.assert_same(U.run_gpu(ctx, b, sc, clip=clip), o, what="graph")
    U.assert_same(U.run_gpu(ctx, b, sc, clip=clip, plain=True), o, what="plain")
    U.assert_same(U.run_gpu(ctx, b, sc, clip=clip, force_int32=True), o, what="int32")
    ot = U.run_oracle(b, sc, clip=clip, trace=False)
    U.assert_same(U.run_gpu(ctx, b, sc, clip=clip, trace=False), ot, trace=False, what="score only")


@pytest.mark.parametrize("seed", [7, 8])
def test_mixed_three_modes(ctx, seed):
    b = synth.tiny_random(3000, 300, 420, seed)
    b.mode = np.random.default_rng(seed).integers(0, 3, b.n_pairs).astype(np.uint8)
    _with_h0(b, 0, 40, seed + 1)
    o = U.run_oracle(b, SC, clip=6)
    U.assert_same(U.run_gpu(ctx, b, SC, clip=6), o, what="persistent + plain")
    U.assert_same(U.run_gpu(ctx, b, SC, clip=6, plain=True), o, what="plain")


def test_default_anchor_score(ctx):
    b = synth.tiny_random(800, 60, 100, 9, mode=2)
    o = U.run_oracle(b, SC, h0=None, default_h0=25, clip=4)
    U.assert_same(U.run_gpu(ctx, b, SC, h0=None, default_h0=25, clip=4), o, what="per-pair modes")
    U.assert_same(U.run_gpu(ctx, b, SC, h0=None, default_h0=25, clip=4, mode="default"), o, what="default mode")


def test_empty_reads_and_windows(ctx):
    """m = 0 gives the anchor; n = 0 gives the anchor, or all insertions when
    o + m e is within the clipping penalty."""
    rng = np.random.default_rng(10)
    R = lambda n: rng.integers(0, 4, n, dtype=np.uint8)  # noqa: E731
    pairs = [(R(0), R(10)), (R(10), R(0)), (R(0), R(0)), (R(3), R(0)), (R(1), R(1)), (R(1), R(9)), (R(9), R(1)),
             (R(16), R(16)), (R(17), R(49)), (R(256), R(300)), (R(255), R(8)), (R(3), R(900))]
    import test_gpu_parity as TP
    b = TP._pairs_batch(pairs, [2] * len(pairs))
    for clip in (0, 8, 9, 10, 100):
        for h0 in (0, 7, 50):
            b.h0 = np.full(b.n_pairs, h0, np.int32)
            o = U.run_oracle(b, SC, clip=clip)
            U.assert_same(U.run_gpu(ctx, b, SC, clip=clip), o, what="clip %d h0 %d" % (clip, h0))
            U.assert_same(U.run_gpu(ctx, b, SC, clip=clip, cap=1), U.run_oracle(b, SC, clip=clip, cap=1), cap=1,
                          what="cap1 clip %d h0 %d" % (clip, h0))


def test_large_anchor_scores_saturate_and_rerun(ctx):
    """Anchors near and above the 16-bit range go through the saturating
    kernels; saturated pairs are recomputed in 32 bits.  Anchors outside
    0..2^20 are rejected per pair."""
    b = synth.tiny_random(2000, 120, 200, 12, mode=2)
    rng = np.random.default_rng(12)
    b.h0 = rng.choice(np.array([0, 50, 32000, 32700, 32760, 40000, 1 << 20, -1, (1 << 20) + 1], np.int64),
                      b.n_pairs).astype(np.int32)
    o = U.run_oracle(b, SC, clip=5)
    g = U.run_gpu(ctx, b, SC, clip=5)
    U.assert_same(g, o, what="large h0")
    bad = (b.h0 < 0) | (b.h0 > (1 << 20))
    assert (o["status"][bad] == 4).all()
    assert ((g["status"] & 1) != 0)[(b.h0 >= 32700) & ~bad & (b.read_len > 0) & (b.win_len > 0)].any()
    U.assert_same(U.run_gpu(ctx, b, SC, clip=5, plain=True), o, what="large h0 plain")


def test_anchor_bound_skips_saturating_kernels(ctx):
    """With a host bound on the anchor scores that keeps every extension in
    16-bit scores, the batch launches no saturation-checking kernels and no
    re-run, with the same results; pairs above the bound are rejected per
    pair.  A bound too large for that keeps the saturating path."""
    b = synth.tiny_random(3000, 150, 190, 14, mode=2)
    rng = np.random.default_rng(14)
    b.h0 = rng.integers(19, 61, b.n_pairs).astype(np.int32)
    o = U.run_oracle(b, SC, clip=5)
    g = U.run_gpu(ctx, b, SC, clip=5, max_ext_h0=60)
    U.assert_same(g, o, what="bounded anchors")
    U.assert_equal_outputs(g, U.run_gpu(ctx, b, SC, clip=5), "bound vs none")
    b.h0[::7] = 61
    g = U.run_gpu(ctx, b, SC, clip=5, max_ext_h0=60)
    assert (g["status"][::7] == 4).all()
    keep = np.nonzero(b.h0 <= 60)[0]
    U.assert_same(g, U.run_oracle(b, SC, clip=5, idx=keep), idx=keep, what="below the bound")
    b.h0[::7] = 32700
    g = U.run_gpu(ctx, b, SC, clip=5, max_ext_h0=32700)
    U.assert_same(g, U.run_oracle(b, SC, clip=5), what="large bound")
    assert ((g["status"] & 1) != 0).any()


def test_scaled_scoring_saturates(ctx):
    """Scores x 60 on reads up to 700 bases leave int16 for long reads only."""
    b = _with_h0(synth.tiny_random(400, 700, 760, 13, mode=2), 0, 30, 13)
    k = 60
    g = U.run_gpu(ctx, b, tuple(k * x for x in SC), h0=b.h0 * k, clip=5 * k)
    o = U.run_oracle(b, SC, clip=5)
    U.assert_same(g, o, score_scale=k, what="scaled")
    assert ((g["status"] & 1) != 0).any()


def test_mode_mask(ctx):
    """Pairs whose mode is outside the announced mask are rejected; the
    others are computed as without a mask."""
    import paper_1402_4876_amd as mica
    b = synth.tiny_random(600, 50, 80, 14)
    b.mode = np.random.default_rng(14).integers(0, 3, b.n_pairs).astype(np.uint8)
    _with_h0(b, 0, 30, 14)
    for mask in (0b001, 0b010, 0b100, 0b011, 0b101, 0b110, 0b111):
        g = _run_masked(ctx, b, mask, clip=3)
        inside = ((mask >> b.mode) & 1) != 0
        idx = np.nonzero(inside)[0]
        U.assert_same(g, U.run_oracle(b, SC, clip=3, idx=idx), idx=idx, what="mask %d" % mask)
        assert (g["status"][~inside] == mica.ST_LEN_LIMIT).all()


def _run_masked(ctx, b, mask, clip):
    import torch

    import paper_1402_4876_amd as mica
    dev = mica.to_device(b)
    n = b.n_pairs
    out = {k: torch.full((n,), -7, dtype=torch.int32, device="cuda")
           for k in ("score", "read_end", "ref_end", "status", "read_start", "ref_start", "n_cigar")}
    out["cigar"] = torch.full((n, 64), -7, dtype=torch.int32, device="cuda")
    mica.align(ctx, dev["ref2b"], dev["win_off"], dev["win_len"], dev["reads2b"], dev["read_off"], dev["read_len"],
               mode=dev["mode"], out_cigar=True, ref_len=dev["ref_len"], reads_len=dev["reads_len"], out=out,
               ext_h0=torch.as_tensor(b.h0).cuda(), ext_clip=clip, mode_mask=mask)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def test_maximum_sizes(ctx):
    rng = np.random.default_rng(15)
    pairs = []
    for m, n in ((1024, 8192), (1024, 1100), (1000, 8192), (300, 8192), (64, 8192)):
        r = rng.integers(0, 4, n, dtype=np.uint8)
        q = r[:m].copy() if m <= n else rng.integers(0, 4, m, dtype=np.uint8)
        q[rng.integers(0, m, 8)] = rng.integers(0, 4, 8)
        q[m * 3 // 4:] = rng.integers(0, 4, m - m * 3 // 4)
        pairs.append((q, r))
    import test_gpu_parity as TP
    b = TP._pairs_batch(pairs, [2] * len(pairs))
    b.h0 = np.array([30, 0, 1000, 20, 5], np.int32)
    for clip in (0, 20, 1 << 20):
        o = U.run_oracle(b, SC, clip=clip, cap=4096)
        U.assert_same(U.run_gpu(ctx, b, SC, clip=clip, cap=4096), o, cap=4096, what="max clip %d" % clip)
        U.assert_same(U.run_gpu(ctx, b, SC, clip=clip, cap=4096, force_int32=True), o, cap=4096,
                      what="max int32 clip %d" % clip)


@pytest.mark.parametrize("clip", [0, 5, 1 << 20])
def test_extension_workload_mini(ctx, clip):
    b = synth.extension_like(20000, seed=1, ref_len=2_000_000)
    o = U.run_oracle(b, SC, clip=clip)
    U.assert_same(U.run_gpu(ctx, b, SC, clip=clip), o, what="ext mini clip %d" % clip)
    clipped = o["read_end"] < b.read_len
    if clip == 1 << 20:
        assert not clipped.any()
    elif clip == 0:
        assert clipped[b.junk].mean() > 0.5


def test_extension_workload_full_size_sampled(ctx):
    """The 1,000,000-pair seed-extension batch in the benchmark's launch
    configuration; 6,000 pairs spread over the batch are checked."""
    b = synth.extension_like(1_000_000, ref_len=100_000_000)
    g = U.run_gpu(ctx, b, SC, clip=5)
    idx = np.unique(np.random.default_rng(16).integers(0, b.n_pairs, 6000))
    U.assert_same(g, U.run_oracle(b, SC, clip=5, idx=idx), idx=idx, what="ext full")
