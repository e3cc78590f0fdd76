"""The allocation-free call (mica_dp_align_batch_noalloc) against the batch
entry point it mirrors (mica_dp_align_batch), through the C ABI: identical
outputs, element by element, on two calls in a row (the second smaller, so
the fixed array still holds the first call's contents), in every launch
style and output set."""
import numpy as np
import pytest

import gpu_util as U
import synth

pytestmark = pytest.mark.gpu

SC = (1, -4, 6, 1)


def run_noalloc(batch, scoring=SC, trace=True, cap=64, force_int32=False, plain=False, clip=0):
    import torch

    import paper_1402_4876_amd as mica
    dev = mica.to_device(batch)
    n = batch.n_pairs
    keys = ["score", "read_end", "ref_end", "status"] + (["read_start", "ref_start", "n_cigar"] if trace else [])
    out = {k: torch.full((n,), -7, dtype=torch.int32, device="cuda") for k in keys}
    if trace:
        out["cigar"] = torch.full((n, cap), -7, dtype=torch.int32, device="cuda")
    h0 = None if batch.h0 is None else torch.as_tensor(np.asarray(batch.h0, np.int32)).cuda()
    torch.cuda.synchronize()
    mica.align_noalloc(dev["ref2b"], dev["win_off"], dev["win_len"], dev["reads2b"], dev["read_off"],
                       dev["read_len"], mode=dev["mode"], scoring=scoring, out_cigar=trace, cigar_cap=cap,
                       force_int32=force_int32, plain=plain, ref_len=dev["ref_len"], reads_len=dev["reads_len"],
                       out=out, ext_h0=h0, ext_clip=clip)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.fixture(scope="module")
def ctx():
    import torch

    import paper_1402_4876_amd as mica
    torch.cuda.set_device(0)
    c = mica.Context(0)
    yield c
    c.close()


def _mixed(n, seed):
    """Semi-global, local and extension pairs of U{0..260}-base reads."""
    b = synth.tiny_random(n, 260, 460, seed)
    b.mode = (np.arange(n) % 3).astype(np.uint8)
    b.h0 = np.random.default_rng(seed).integers(0, 80, n).astype(np.int32)
    return b


@pytest.mark.parametrize("variant", ["persistent", "plain", "int32", "score_only"])
def test_noalloc_equals_batch_entry_two_calls(ctx, variant):
    kw = dict(plain=variant == "plain", force_int32=variant == "int32", trace=variant != "score_only", clip=5)
    big, small = _mixed(30000, 1), _mixed(2500, 2)
    for what, b in (("first call", big), ("second, smaller call", small)):
        print("no-alloc %s: %s, %d pairs" % (variant, what, b.n_pairs), flush=True)
        g_na = run_noalloc(b, **kw)
        g_ctx = U.run_gpu(ctx, b, SC, **kw)
        U.assert_equal_outputs(g_na, g_ctx, "%s %s" % (variant, what))
    o = U.run_oracle(small, SC, trace=kw["trace"], clip=5)
    U.assert_same(g_na, o, trace=kw["trace"], what="no-alloc vs oracle " + variant)


def test_noalloc_config1_shape(ctx):
    """Reads of one length class (150 bp vs 400 bp windows), 200,000 pairs: more
    work items than the fixed array's traceback slots."""
    b = synth.config1(n_pairs=200_000, ref_len=2_000_000)
    g_na = run_noalloc(b)
    U.assert_equal_outputs(g_na, U.run_gpu(ctx, b, SC), "c1 shape")
    idx = np.arange(0, b.n_pairs, 97)
    U.assert_same(g_na, U.run_oracle(b, SC, idx=idx), idx=idx, what="c1 shape sample")
