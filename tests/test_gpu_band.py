"""Routing of the banded traceback (DP section; the band bound of the
traceback): after the score-only fill each pair's band follows from its
score and end cell; bands of up to 16 diagonals are refilled at once, those
of 17-64 by the side-list launch, wider ones (or, in packed 16 bits, pairs
whose refill values could reach the upper clamp) by the full traceback.

The expected routing is computed here, on the host, from the oracle's score
and end cell with the bound written out (deletions Ld <= (a min(i*, j*) -
gain - o) / e, insertions Li <= (a i* - gain - o) / (a + e), gain = the score
over the start: S, or S - h0 for an extension), and compared with the
library's per-batch counts; every output is compared with the oracle.  The
batches put pairs on both sides of every width boundary (16/17, 32/33,
64/65)."""
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


def _class_d0(m):
    """Dummy rows above a read of m bases in the default class table (16
    lanes x ceil(m / 16) rows for reads up to 256 bases)."""
    return 16 * np.maximum(1, (m + 15) // 16) - m


def _routing(b, o, sc, mode, packed16):
    a, _, op, e = sc
    S = o["score"].astype(np.int64)
    ie = o["read_end"].astype(np.int64)
    je = o["ref_end"].astype(np.int64)
    h0 = b.h0.astype(np.int64) if mode == 2 else np.zeros(b.n_pairs, np.int64)
    gain = S - h0
    ad = a * np.minimum(ie, je) - gain - op
    ai = a * ie - gain - op
    ld = np.where(ad >= 0, ad // e, 0)
    li = np.where(ai >= 0, ai // (a + e), 0)
    ds = je - ie
    lo = np.maximum(ds - ld, -ie)
    hi = np.minimum(ds + li, je)
    has = (ie >= 1) & (je >= 1)
    W = np.where(has, hi - lo + 1, 0)
    m = b.read_len.astype(np.int64)
    n = b.win_len.astype(np.int64)
    hib = h0 + a * np.minimum(m, n) if mode == 2 else a * np.minimum(m, n) - _class_d0(m)
    clamp = packed16 & ((hib + 16 * e + op > 32767) | (16 * e + op > 32767))
    full = has & ((W > 64) | clamp)
    deferred = has & ~full & (W > 16)
    return W, full, deferred


def _check(ctx, b, sc, mode, int32, clip=0):
    o = U.run_oracle(b, sc, clip=clip)
    g = U.run_gpu(ctx, b, sc, force_int32=int32, clip=clip, max_ext_h0=60 if mode == 2 else 0)
    st = ctx.last_stats()
    U.assert_same(g, o, what="band mix mode %d int32 %s" % (mode, int32))
    W, full, deferred = _routing(b, o, sc, mode, not int32)
    assert st["n_saturated"] == 0
    assert st["n_fallback"] == int(full.sum()), (st, int(full.sum()))
    assert st["n_deferred"] == int(deferred.sum()), (st, int(deferred.sum()))
    return W, full, deferred


@pytest.mark.parametrize("int32", [False, True])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_band_width_routing(ctx, mode, int32):
    b = synth.band_mix(3000, mode, seed=0)
    W, full, deferred = _check(ctx, b, SC, mode, int32, clip=5 if mode == 2 else 0)
    # both sides of every width boundary are present
    for w in (1, 16, 17, 32, 33, 64, 65):
        assert (W == w).sum() >= 3, (w, int((W == w).sum()))


def test_packed_refill_clamp_goes_to_full_traceback(ctx):
    """Scores large enough that a packed 16-bit refill of a long read could
    reach the clamp (a min(m, n) - d0 + 16 e + o > 32767) while the fill
    itself stays exact: those pairs take the full traceback even when their
    band is narrow; shorter reads of the same batch keep the band."""
    sc = (218, -30, 100, 100)
    b = synth.band_mix(1500, 0, seed=2)
    W, full, _ = _check(ctx, b, sc, 0, False)
    m = b.read_len.astype(np.int64)
    hib = sc[0] * np.minimum(m, b.win_len.astype(np.int64)) - _class_d0(m)
    clamp = hib + 16 * sc[3] + sc[2] > 32767
    assert full[clamp].all()
    assert (clamp & (W >= 1) & (W <= 64)).sum() >= 20
    assert (~full & (W >= 1)).sum() >= 100
    # the same pairs in 32 bits keep every band of up to 64 diagonals
    _check(ctx, b, sc, 0, True)
