"""End-to-end parity of the host pipeline (FASTQ in, SAM out) against records
composed from the CPU oracles.

The expected record of every read is built here from oracle.kmm_search (the
few-mismatch search), the seed placements of the read's exact parts (found
with bytes.find), oracle.align_batch (semi-global DP of each window) and the
pipeline's stated rules (include/mica_pipe.h); every SAM field must match.
Batches are small so that a file spans several batches on both slots.
"""
import os
import threading

import numpy as np
import pytest

import oracle
from paper_1402_4876_amd import pack_codes

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SC = (1, -4, 6, 1)
CAP = 32
BASES = "ACGT"


def _reference(n=400_000, seed=11):
    rng = np.random.default_rng(seed)
    ref = rng.integers(0, 4, n, dtype=np.uint8)
    ref[200_000:200_900] = np.tile(rng.integers(0, 4, 9, dtype=np.uint8), 100)  # tandem repeat
    ref[300_000:300_400] = ref[50_000:50_400]                                   # a duplicate
    return ref


def _records(ref, n=2500, seed=12):
    rng = np.random.default_rng(seed)
    L = len(ref)
    recs = []
    for i in range(n):
        kind = i % 10
        m = int(rng.integers(25, 251))
        p = int(rng.integers(0, L - m - 5))
        q = ref[p:p + m].copy()
        if kind in (1, 2):  # substitutions
            for w in rng.choice(m, kind + 1 if kind == 2 else 1, replace=False):
                q[w] = (q[w] + rng.integers(1, 4)) % 4
        elif kind in (3, 4):  # a deletion or an insertion of 1-3 bases
            L_ = int(rng.integers(1, 4))
            w = int(rng.integers(10, m - 10))
            if kind == 3:
                q = np.concatenate([q[:w], ref[p + w + L_:p + m + L_]])
            else:
                q = np.concatenate([q[:w], rng.integers(0, 4, L_, dtype=np.uint8), q[w:m - L_]])
        elif kind == 5:  # indel plus substitutions
            w = int(rng.integers(10, m - 10))
            q = np.concatenate([q[:w], ref[p + w + 2:p + m + 2]])
            for x in rng.choice(m, 3, replace=False):
                q[x] = (q[x] + 1) % 4
        elif kind == 6:
            q = rng.integers(0, 4, m, dtype=np.uint8)
        elif kind == 7:
            p = 200_000 + int(rng.integers(0, 900 - min(m, 880)))
            q = ref[p:p + min(m, 880)].copy()
        seq = "".join(BASES[c] for c in q)
        if kind == 8 and i % 20 == 8:
            seq = seq[:5] + "N" + seq[6:]
        qual = "".join(chr(33 + int(x)) for x in rng.integers(0, 41, len(seq)))
        recs.append(("read%d" % i, seq, qual))
    recs.append(("empty", "", ""))
    recs.append(("short", "AC", "II"))
    return recs


def _write_fastq(path, recs):
    with open(path, "w") as f:
        for name, seq, qual in recs:
            f.write("@%s extra words\n%s\n+\n%s\n" % (name, seq, qual))


def _find_all(hay, needle):
    out, s = [], hay.find(needle)
    while s >= 0:
        out.append(s)
        s = hay.find(needle, s + 1)
    return out


def _expected(ref, recs, k, max_occ, band, min_score, ref_name="chrT"):
    a, b = SC[0], SC[1]
    L = len(ref)
    hay = bytes(ref.tolist())
    codes = []
    ok = []
    for _, seq, _ in recs:
        good = all(c in BASES for c in seq)
        ok.append(good)
        codes.append(np.array([BASES.index(c) for c in seq], np.uint8) if good else np.zeros(0, np.uint8))
    off = np.concatenate([[0], np.cumsum([len(c) for c in codes])[:-1]]).astype(np.int64)
    flat = np.concatenate(codes + [np.zeros(1, np.uint8)])
    lens = np.array([len(c) for c in codes], np.int32)
    o1 = oracle.kmm_search(ref, flat, off, lens, k=k, max_occ=max_occ)
    # DP windows of the reads without a hit
    wins = []  # (read, win_start, win_len)
    for r, c in enumerate(codes):
        m = len(c)
        if not ok[r] or o1["status"][r] != 0 or o1["best_mm"][r] >= 0 or m == 0:
            continue
        seeds = []
        for j in range(k + 1):
            s0, e0 = j * m // (k + 1), (j + 1) * m // (k + 1)
            occ = _find_all(hay, bytes(c[s0:e0].tolist()))
            seeds.append(min(occ) - s0 if occ else None)
        for j, cj in enumerate(seeds):
            if cj is None or any(seeds[jj] is not None and abs(cj - seeds[jj]) <= band for jj in range(j)):
                continue
            ws, we = max(0, cj - band), min(L, cj + m + band)
            if we > ws:
                wins.append((r, ws, we - ws))
    dp = {}
    if wins:
        wr = np.array([w[0] for w in wins])
        o2 = oracle.align_batch(ref, np.array([w[1] for w in wins], np.int64), np.array([w[2] for w in wins], np.int32),
                                flat, off[wr], lens[wr], np.zeros(len(wins), np.uint8), SC, trace=True, cigar_cap=CAP)
        for t, (r, ws, wl) in enumerate(wins):
            dp.setdefault(r, []).append((t, ws))
    lines = []
    for r, (name, seq, qual) in enumerate(recs):
        m = len(seq)
        unmapped = "%s\t4\t*\t0\t0\t*\t*\t0\t0\t%s\t%s" % (name, seq or "*", qual or "*")
        if not ok[r] or o1["status"][r] != 0:
            lines.append(unmapped)
            continue
        if o1["best_mm"][r] >= 0:
            mm = int(o1["best_mm"][r])
            lines.append("%s\t0\t%s\t%d\t%d\t%dM\t*\t0\t0\t%s\t%s\tNM:i:%d\tAS:i:%d" % (
                name, ref_name, o1["pos"][r] + 1, 60 if o1["n_best"][r] == 1 else 0, m, seq, qual, mm,
                (m - mm) * a + mm * b))
            continue
        cands = [(int(o2["score"][t]), ws + int(o2["ref_start"][t]), t) for t, ws in dp.get(r, [])
                 if o2["status"][t] == 0]
        if not cands:
            lines.append(unmapped)
            continue
        bs = max(c[0] for c in cands)
        tied = [c for c in cands if c[0] == bs]
        _, pos, t = min(tied, key=lambda c: c[1])
        if bs < min_score:
            lines.append(unmapped)
            continue
        ops = [(int(w) >> 4, "MID"[int(w) & 15]) for w in o2["cigar"][t][:o2["n_cigar"][t]]]
        nm, qp, rp = 0, 0, pos
        for Lop, op in ops:
            if op == "M":
                nm += int((codes[r][qp:qp + Lop] != ref[rp:rp + Lop]).sum())
                qp += Lop
                rp += Lop
            elif op == "I":
                nm += Lop
                qp += Lop
            else:
                nm += Lop
                rp += Lop
        cig = "".join("%d%s" % (Lop, op) for Lop, op in ops)
        lines.append("%s\t0\t%s\t%d\t%d\t%s\t*\t0\t0\t%s\t%s\tNM:i:%d\tAS:i:%d" % (
            name, ref_name, pos + 1, 60 if len(tied) == 1 else 0, cig, seq, qual, nm, bs))
    return lines


@pytest.mark.parametrize("k,band,min_score,batch", [(2, 32, 0, 700), (1, 48, 20, 1000), (2, 16, -50, 3000)])
def test_pipeline_matches_oracle_records(tmp_path, k, band, min_score, batch):
    import paper_1402_4876_amd as mica
    ref = _reference()
    recs = _records(ref)
    fq = tmp_path / "reads.fq"
    sam = tmp_path / "out.sam"
    _write_fastq(fq, recs)
    pipe = mica.Pipeline(pack_codes(ref), len(ref), "chrT", k=k, max_occ=64, band=band, min_score=min_score,
                         batch_reads=batch, format_threads=3)
    st = pipe.run(fq, sam)
    pipe.close()
    got = [l for l in open(sam).read().split("\n") if l and not l.startswith("@")]
    head = [l for l in open(sam).read().split("\n") if l.startswith("@")]
    assert head[1] == "@SQ\tSN:chrT\tLN:%d" % len(ref)
    want = _expected(ref, recs, k, 64, band, min_score)
    assert len(got) == len(want) == len(recs)
    bad = [i for i, (g, w) in enumerate(zip(got, want)) if g != w]
    assert not bad, "%d records differ; first:\n%s\n%s" % (len(bad), got[bad[0]], want[bad[0]])
    assert st["reads"] == len(recs) and st["batches"] == -(-len(recs) // batch)
    assert st["mapped_search"] > 0 and st["mapped_dp"] > 0 and st["unmapped"] > 0
    assert st["non_acgt"] > 0 and st["repetitive"] > 0
    assert st["mapped_search"] + st["mapped_dp"] + st["unmapped"] == st["reads"]


def test_pipeline_rejects_malformed_fastq(tmp_path):
    import paper_1402_4876_amd as mica
    ref = np.random.default_rng(13).integers(0, 4, 5000, dtype=np.uint8)
    fq = tmp_path / "bad.fq"
    fq.write_text("@r1\nACGT\n+\nIII\n")
    pipe = mica.Pipeline(pack_codes(ref), len(ref), "chrT", batch_reads=100, format_threads=1)
    with pytest.raises(mica.MicaError):
        pipe.run(fq, tmp_path / "out.sam")
    with pytest.raises(mica.MicaError):
        pipe.run(tmp_path / "missing.fq", tmp_path / "out.sam")
    # the pipeline stays usable
    fq.write_text("@r1\n%s\n+\n%s\n" % ("".join("ACGT"[c] for c in ref[100:160]), "I" * 60))
    st = pipe.run(fq, tmp_path / "out.sam")
    assert st["reads"] == 1 and st["mapped_search"] == 1
    line = [l for l in open(tmp_path / "out.sam").read().split("\n") if l.startswith("r1")][0]
    assert line.split("\t")[3] == "101" and line.split("\t")[5] == "60M"
    pipe.close()


def test_pipeline_input_forms(tmp_path):
    """CRLF line ends, blank lines between records, a missing final newline
    and lower-case bases give the same alignments as the plain file."""
    import paper_1402_4876_amd as mica
    ref = _reference()
    recs = _records(ref, n=600, seed=14)[:-2]
    plain = tmp_path / "plain.fq"
    _write_fastq(plain, recs)
    odd = tmp_path / "odd.fq"
    body = "\r\n\r\n".join("@%s\r\n%s\r\n+\r\n%s" % r for r in recs)  # blank lines between records
    odd.write_bytes(body.encode())                                             # and no final newline
    low = tmp_path / "low.fq"
    with open(low, "w") as f:
        for name, seq, qual in recs:
            f.write("@%s\n%s\n+%s\n%s\n" % (name, seq.lower(), name, qual))
    pipe = mica.Pipeline(pack_codes(ref), len(ref), "chrT", batch_reads=250, format_threads=2)
    outs = {}
    for tag, fq in (("plain", plain), ("odd", odd), ("low", low)):
        pipe.run(fq, tmp_path / (tag + ".sam"))
        outs[tag] = [l.split("\t") for l in open(tmp_path / (tag + ".sam")).read().split("\n")
                     if l and not l.startswith("@")]
    pipe.close()
    assert outs["plain"] == outs["odd"]
    assert len(outs["low"]) == len(outs["plain"])
    for a, b in zip(outs["plain"], outs["low"]):
        assert a[:9] == b[:9] and a[10:] == b[10:] and a[9].lower() == b[9]


def test_pipeline_reads_from_a_pipe(tmp_path):
    """A FIFO (read through the buffered reader, not mapped) gives the same
    SAM records as the regular file (mapped in place)."""
    import paper_1402_4876_amd as mica
    ref = _reference()
    recs = _records(ref, n=900, seed=15)
    plain = tmp_path / "plain.fq"
    _write_fastq(plain, recs)
    fifo = tmp_path / "reads.fifo"
    os.mkfifo(fifo)
    data = plain.read_bytes()

    def feed():
        with open(fifo, "wb") as f:
            f.write(data)

    pipe = mica.Pipeline(pack_codes(ref), len(ref), "chrT", batch_reads=300, format_threads=2)
    pipe.run(plain, tmp_path / "plain.sam")
    t = threading.Thread(target=feed, daemon=True)
    t.start()
    st = pipe.run(fifo, tmp_path / "fifo.sam")
    t.join(timeout=30)
    pipe.close()
    assert not t.is_alive()
    a = open(tmp_path / "plain.sam").read()
    b = open(tmp_path / "fifo.sam").read()
    assert st["reads"] == len(recs) and a == b


def test_pipeline_writes_to_a_pipe(tmp_path):
    """SAM written into a FIFO (in order through the stream, not by
    positional writes) equals the SAM written into a regular file."""
    import paper_1402_4876_amd as mica
    ref = _reference()
    recs = _records(ref, n=900, seed=16)
    fq = tmp_path / "reads.fq"
    _write_fastq(fq, recs)
    fifo = tmp_path / "out.fifo"
    os.mkfifo(fifo)
    got = []

    def drain():
        with open(fifo, "rb") as f:
            got.append(f.read())

    pipe = mica.Pipeline(pack_codes(ref), len(ref), "chrT", batch_reads=300, format_threads=3)
    pipe.run(fq, tmp_path / "plain.sam")
    t = threading.Thread(target=drain, daemon=True)
    t.start()
    st = pipe.run(fq, fifo)
    t.join(timeout=30)
    pipe.close()
    assert not t.is_alive() and st["reads"] == len(recs)
    assert got[0] == (tmp_path / "plain.sam").read_bytes()
