"""Helpers for GPU parity tests: run the library and the oracle on one batch."""
import numpy as np

KEYS_TRACE = ("score", "read_start", "read_end", "ref_start", "ref_end", "n_cigar")
KEYS_END = ("score", "read_end", "ref_end")


def run_gpu(ctx, batch, scoring=(1, -4, 6, 1), trace=True, cap=64, force_int32=False, plain=False,
            max_read_len=None, max_win_len=None, mode="batch", h0="batch", default_h0=0, clip=0,
            min_read_len=0, max_ext_h0=0):
    import torch
    import paper_1402_4876_amd as mica
    dev = mica.to_device(batch)
    if isinstance(h0, str):
        h0 = batch.h0
    h0_dev = None if h0 is None else torch.as_tensor(np.asarray(h0, np.int32)).cuda()
    md = dev["mode"] if mode == "batch" else None
    # every output starts as a sentinel, so a pair the kernels skip cannot
    # pass on values left in reused device memory
    n = batch.n_pairs
    keys = ["score", "read_end", "ref_end", "status"] + (["read_start", "ref_start", "n_cigar"] if trace else [])
    sentinel = {k: torch.full((n,), -7, dtype=torch.int32, device="cuda") for k in keys}
    if trace:
        sentinel["cigar"] = torch.full((n, cap), -7, dtype=torch.int32, device="cuda")
    out = mica.align(ctx, dev["ref2b"], dev["win_off"], dev["win_len"], dev["reads2b"], dev["read_off"],
                     dev["read_len"], mode=md, scoring=scoring, out_cigar=trace, cigar_cap=cap,
                     force_int32=force_int32, plain=plain, ref_len=dev["ref_len"], reads_len=dev["reads_len"],
                     max_read_len=max_read_len, max_win_len=max_win_len,
                     default_mode=int(batch.mode[0]) if mode != "batch" and batch.n_pairs else 0, out=sentinel,
                     ext_h0=h0_dev, ext_default_h0=default_h0, ext_clip=clip, min_read_len=min_read_len,
                     max_ext_h0=max_ext_h0)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def run_oracle(batch, scoring=(1, -4, 6, 1), trace=True, cap=64, idx=None, h0="batch", default_h0=0, clip=0):
    import oracle
    b = batch if idx is None else batch.subset(idx)
    if isinstance(h0, str):
        h0 = b.h0
    elif h0 is not None and idx is not None:
        h0 = np.asarray(h0)[idx]
    return oracle.align_batch(b.ref, b.win_off, b.win_len, b.reads, b.read_off, b.read_len, b.mode, scoring,
                              trace=trace, cigar_cap=cap, h0=h0, default_h0=default_h0, clip=clip)


def assert_same(g, o, trace=True, cap=64, idx=None, score_scale=1, what=""):
    """Element-wise equality (integer outputs: exact) of GPU and oracle results."""
    sel = slice(None) if idx is None else idx
    for k in (KEYS_TRACE if trace else KEYS_END):
        gk = g[k][sel]
        ok = o[k] * (score_scale if k == "score" else 1)
        bad = np.nonzero(gk != ok)[0]
        assert len(bad) == 0, "%s %s: %d mismatches, first pairs %s gpu %s oracle %s" % (
            what, k, len(bad), bad[:5], gk[bad[:5]], ok[bad[:5]])
    st = g["status"][sel].astype(np.uint32) & ~np.uint32(1)  # saturation is a GPU-only note
    bad = np.nonzero(st != o["status"])[0]
    assert len(bad) == 0, "%s status: %s gpu %s oracle %s" % (what, bad[:5], st[bad[:5]], o["status"][bad[:5]])
    if trace:
        ncig = np.minimum(np.abs(o["n_cigar"]), cap)
        col = np.arange(cap)[None, :] < ncig[:, None]
        diff = ((g["cigar"][sel].astype(np.uint32) != o["cigar"]) & col).any(axis=1)
        bad = np.nonzero(diff)[0]
        assert len(bad) == 0, "%s cigar differs for %d pairs, first %s" % (what, len(bad), bad[:5])


def assert_equal_outputs(g1, g2, what=""):
    """Two GPU results are identical (CIGAR words compared up to n_cigar)."""
    for k in g1:
        if k == "cigar":
            continue
        assert np.array_equal(g1[k], g2[k]), "%s %s" % (what, k)
    if "cigar" in g1:
        cap = g1["cigar"].shape[1]
        ncig = np.minimum(np.abs(g1["n_cigar"]), cap)
        col = np.arange(cap)[None, :] < ncig[:, None]
        assert not ((g1["cigar"] != g2["cigar"]) & col).any(), "%s cigar" % what
