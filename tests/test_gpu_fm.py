"""GPU parity of the few-mismatch search (FM index on the device) against the
CPU oracle's definition, through the C ABI.

Every output (best mismatch count, hit counts, leftmost best position,
status) must be identical per read.  Cases: planted reads with 0-3
substitutions and indels, random reads, reads at the reference's ends,
reads longer than the reference, reads too short for k + 1 parts, reads in
a tandem repeat (repetitive at small max_occ, searched at large), reads at
unaligned offsets, out-of-range reads, k = 0, 1, 2, and the 10^6-read
workload on the 100 Mbp reference, sampled.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1402_4876_amd import pack_codes

pytestmark = pytest.mark.gpu

KEYS = ("best_mm", "n_best", "n_hits", "pos", "status")


def _reference(seed=1, n=1_000_000):
    rng = np.random.default_rng(seed)
    ref = rng.integers(0, 4, n, dtype=np.uint8)
    unit = rng.integers(0, 4, 9, dtype=np.uint8)
    ref[500_000:500_900] = np.tile(unit, 100)          # a tandem repeat
    ref[700_000:700_300] = ref[100_000:100_300]        # a duplicated stretch
    ref[800_000:800_300] = ref[100_000:100_300]
    ref[800_150] = (ref[800_150] + 1) % 4             # ... with one difference
    return ref


def _reads(ref, seed=2, n=3000):
    rng = np.random.default_rng(seed)
    L = len(ref)
    reads = []
    for t in range(n):
        kind = t % 12
        m = int(rng.integers(20, 251))
        if kind == 11:
            reads.append(rng.integers(0, 4, m, dtype=np.uint8))
            continue
        if kind == 10:
            p = int(rng.integers(500_000, 500_900 - m)) if m < 880 else 500_000
            reads.append(ref[p:p + m].copy())
            continue
        if kind == 9:
            p = 100_000 + int(rng.integers(0, 300 - min(m, 300)))
            m = min(m, 300)
        elif kind == 8:
            p = L - m if t % 24 == 8 else 0
        else:
            p = int(rng.integers(0, L - m))
        q = ref[p:p + m].copy()
        nsub = kind % 4
        for w in rng.choice(m, nsub, replace=False):
            q[w] = (q[w] + rng.integers(1, 4)) % 4
        if kind == 7:  # an indel
            w = int(rng.integers(5, m - 5))
            q = np.concatenate([q[:w], q[w + 2:], ref[p + m:p + m + 2]]) if t % 2 else \
                np.concatenate([q[:w], rng.integers(0, 4, 1, dtype=np.uint8), q[w:-1]])
        reads.append(q)
    reads += [ref[:2].copy(), ref[10:12].copy(), ref[:1].copy(), rng.integers(0, 4, 1024, dtype=np.uint8)]
    return reads


def _upload(reads, aligned=True):
    """Flat reads at 16-base-aligned offsets (or back to back)."""
    if aligned:
        m = np.array([len(q) for q in reads], np.int32)
        codes = np.zeros((len(reads), max(int(m.max()), 1)), np.uint8)
        for i, q in enumerate(reads):
            codes[i, :len(q)] = q
        flat, off = synth.pack_reads_layout(codes, m)
    else:
        flat = np.concatenate(reads + [np.zeros(1, np.uint8)])
        off = np.concatenate([[0], np.cumsum([len(q) for q in reads])[:-1]]).astype(np.int64)
    m = np.array([len(q) for q in reads], np.int32)
    dev = (torch.from_numpy(pack_codes(flat).view(np.int32)).cuda(), torch.from_numpy(off).cuda(),
           torch.from_numpy(m).cuda())
    return flat, off, m, dev


@pytest.fixture(scope="module")
def small():
    import paper_1402_4876_amd as mica
    torch.cuda.set_device(0)
    ref = _reference()
    ix = mica.FmIndex(pack_codes(ref), len(ref))
    yield ref, ix
    ix.close()


def _gpu(ix, dev, n_bases, k, max_occ):
    out = ix.search(dev[0], dev[1], dev[2], k=k, max_occ=max_occ, reads_len=n_bases)
    torch.cuda.synchronize()
    return {key: v.cpu().numpy() for key, v in out.items()}


def _same(g, o, what):
    for key in KEYS:
        gk = g[key].astype(np.int64) if key != "status" else g[key].astype(np.uint32)
        ok = o[key].astype(np.int64) if key != "status" else o[key]
        bad = np.nonzero(gk != ok)[0]
        assert len(bad) == 0, "%s %s: %d differ, first %s gpu %s oracle %s" % (
            what, key, len(bad), bad[:5], gk[bad[:5]], ok[bad[:5]])


@pytest.mark.parametrize("k", [0, 1, 2])
@pytest.mark.parametrize("max_occ", [1, 8, 64])
def test_small_reference(small, k, max_occ):
    ref, ix = small
    reads = _reads(ref)
    flat, off, m, dev = _upload(reads)
    o = oracle.kmm_search(ref, flat, off, m, k=k, max_occ=max_occ)
    g = _gpu(ix, dev, len(flat), k, max_occ)
    _same(g, o, "k=%d max_occ=%d" % (k, max_occ))
    if max_occ == 64:
        assert (o["status"] == oracle.ST_REPETITIVE).any() and (o["best_mm"] == k).any()


def test_unaligned_read_offsets(small):
    ref, ix = small
    reads = _reads(ref, seed=3, n=1200)
    flat, off, m, dev = _upload(reads, aligned=False)
    o = oracle.kmm_search(ref, flat, off, m, k=2, max_occ=32)
    _same(_gpu(ix, dev, len(flat), 2, 32), o, "unaligned")


def test_out_of_range_reads(small):
    ref, ix = small
    reads = _reads(ref, seed=4, n=60)
    flat, off, m, dev = _upload(reads)
    off_bad = off.copy()
    off_bad[5] = len(flat) + 10
    dev = (dev[0], torch.from_numpy(off_bad).cuda(), dev[2])
    o = oracle.kmm_search(ref, flat, off_bad, m, k=2, max_occ=64)
    assert o["status"][5] == oracle.ST_READ_OOB
    _same(_gpu(ix, dev, len(flat), 2, 64), o, "oob")


def test_tiny_references():
    """References shorter than one occurrence block, and of a block's length."""
    import paper_1402_4876_amd as mica
    rng = np.random.default_rng(5)
    for n in (1, 5, 191, 192, 193, 383, 384, 1000):
        ref = rng.integers(0, 4, n, dtype=np.uint8)
        ix = mica.FmIndex(pack_codes(ref), n)
        reads = [ref[max(0, s):max(0, s) + L].copy() for s, L in ((0, 3), (n - 3, 3), (n // 2, 10), (0, n))
                 if L <= n and s >= 0] + [rng.integers(0, 4, 6, dtype=np.uint8)]
        flat, off, m, dev = _upload(reads)
        for k in (0, 1, 2):
            o = oracle.kmm_search(ref, flat, off, m, k=k, max_occ=1000)
            _same(_gpu(ix, dev, len(flat), k, 1000), o, "n=%d k=%d" % (n, k))
        ix.close()


def test_full_size_workload_sampled():
    """10^6 reads of 150 bp (1% substitutions, 0.3% indels) against the
    100 Mbp reference, as the benchmark searches them; 240 reads spread
    over the batch are checked against the oracle."""
    import paper_1402_4876_amd as mica
    b = synth.config1()
    ix = mica.FmIndex(pack_codes(b.ref), len(b.ref))
    dev = (torch.from_numpy(pack_codes(b.reads).view(np.int32)).cuda(), torch.from_numpy(b.read_off).cuda(),
           torch.from_numpy(b.read_len).cuda())
    g = _gpu(ix, dev, len(b.reads), 2, 64)
    idx = np.unique(np.random.default_rng(6).integers(0, b.n_pairs, 240))
    o = oracle.kmm_search(b.ref, b.reads, b.read_off[idx], b.read_len[idx], k=2, max_occ=64)
    _same({key: v[idx] for key, v in g.items()}, o, "full")
    hit = g["best_mm"] >= 0
    assert 0.3 < hit.mean() < 0.8  # reads with indels or > 2 substitutions go on to DP
    ix.close()


def test_search_argument_errors(small):
    """Bad k, max_occ or arrays are refused before any launch; an empty batch is a no-op."""
    import paper_1402_4876_amd as mica
    ref, ix = small
    reads = _reads(ref, seed=8, n=10)
    flat, off, m, dev = _upload(reads)
    for k, mo in ((3, 64), (-1, 64), (2, 0), (2, 70000)):
        with pytest.raises(mica.MicaError):
            ix.search(dev[0], dev[1], dev[2], k=k, max_occ=mo, reads_len=len(flat))
    with pytest.raises(ValueError):
        ix.search(dev[0], dev[1], dev[2][:5], k=2)
    e = ix.search(dev[0], dev[1][:0], dev[2][:0], k=2, reads_len=len(flat))
    torch.cuda.synchronize()
    assert e["best_mm"].numel() == 0


def test_concurrent_streams(small):
    """Two batches searched at once on two streams equal their one-by-one results."""
    ref, ix = small
    a = _upload(_reads(ref, seed=9, n=800))
    b = _upload(_reads(ref, seed=10, n=900))
    ga = _gpu(ix, a[3], len(a[0]), 2, 64)
    gb = _gpu(ix, b[3], len(b[0]), 2, 64)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s1):
        oa = ix.search(a[3][0], a[3][1], a[3][2], k=2, max_occ=64, reads_len=len(a[0]), stream=s1)
    with torch.cuda.stream(s2):
        ob = ix.search(b[3][0], b[3][1], b[3][2], k=2, max_occ=64, reads_len=len(b[0]), stream=s2)
    torch.cuda.synchronize()
    for key in KEYS:
        assert np.array_equal(oa[key].cpu().numpy(), ga[key]) and np.array_equal(ob[key].cpu().numpy(), gb[key])
