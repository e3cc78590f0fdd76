"""GPU parity at the offsets a resident multi-gigabase reference reaches.

The reference here is longer than 2^32 bases (4.36 Gbp, 1.09 GB packed, on
the device); windows start below 2^31, straddle 2^31 and 2^32, lie past 2^32
and end at the reference's last base.  Reads sit at offsets that are not
multiples of 16 (a word boundary anywhere inside a read).  The oracle aligns
the same pairs against the windows copied out of the packed reference into a
small code array (offsets rebased), so it needs no multi-gigabyte code array.
Every output is compared element by element: through mica_dp_align_batch
(persistent, plain and 32-bit launches, all three modes) and through the
serving loop.
"""
import time

import numpy as np
import pytest

import gpu_util as U
import synth

pytestmark = pytest.mark.gpu

SC = (1, -4, 6, 1)
CLIP = 5


@pytest.fixture(scope="module")
def longref():
    import torch

    import paper_1402_4876_amd as mica
    torch.cuda.set_device(0)
    b, _ = synth.long_reference_batch(4000)
    small = synth.rebase_windows(b)
    o = U.run_oracle(small, SC, h0=b.h0, clip=CLIP)
    ctx = mica.Context(0)
    yield b, o, ctx
    ctx.close()


def test_windows_reach_past_2g_and_4g(longref):
    b, _, _ = longref
    end = b.win_off + b.win_len
    assert len(b.ref) * 16 > (1 << 32)
    assert ((b.win_off < (1 << 31)) & (end > (1 << 31))).sum() >= 100
    assert ((b.win_off < (1 << 32)) & (end > (1 << 32))).sum() >= 100
    assert (b.win_off >= (1 << 32)).sum() >= 100
    assert (end == len(b.ref) * 16).sum() >= 100
    assert (b.read_off % 16 != 0).mean() > 0.8


@pytest.mark.parametrize("launch", ["persistent", "plain", "int32"])
def test_batch_api_long_reference(longref, launch):
    b, o, ctx = longref
    print("long reference, %s launch, %d pairs" % (launch, b.n_pairs), flush=True)
    g = U.run_gpu(ctx, b, SC, clip=CLIP, plain=launch == "plain", force_int32=launch == "int32")
    U.assert_same(g, o, what="long reference " + launch)


def test_served_long_reference(longref):
    """Semi-global and local requests served from the resident 4.36 Gbp
    reference (reads at unaligned offsets) equal the oracle."""
    import paper_1402_4876_amd as mica
    from paper_1402_4876_amd.pack import pack_codes
    b, o, _ = longref
    keep = np.nonzero(b.mode != 2)[0]
    reads_words = pack_codes(b.reads)
    sizes = np.random.default_rng(9).integers(1, 400, 64)
    reqs, k = [], 0
    for s in sizes:
        if k >= len(keep):
            break
        reqs.append(keep[k:k + int(s)])
        k += int(s)
    print("serving %d requests from a %d-base reference" % (len(reqs), len(b.ref) * 16), flush=True)
    srv = mica.Server(b.ref, len(b.ref) * 16, slots=3, hbm_budget_bytes=8 << 30)
    try:
        for rid, idx in enumerate(reqs):
            srv.submit(rid, reads_words, b.read_off[idx].astype(np.uint64), b.read_len[idx],
                       b.win_off[idx].astype(np.uint64), b.win_len[idx], mode=b.mode[idx].astype(np.uint8))
        got, left, t0 = {}, set(range(len(reqs))), time.time()
        while left:
            for i in srv.poll():
                got[i] = srv.fetch(i)
                left.discard(i)
            assert time.time() - t0 < 120, "requests not finished"
            time.sleep(0.002)
    finally:
        srv.close()
    idx = np.concatenate(reqs)
    g = {key: np.concatenate([got[r][key] for r in range(len(reqs))]) for key in got[0]}
    sub = {key: (v[idx] if key != "cigar" else v[idx]) for key, v in o.items()}
    U.assert_same(g, sub, what="served long reference")
