#!/usr/bin/env python3
"""Benchmark of the DP phase on one MI355X: GCUPS and % of the integer roofline.

Default workload (one "step" = one call of mica_dp_align_batch over the whole
batch, inputs already resident in HBM): 1,000,000 reads of 150 bp against
400 bp windows of a seeded random 100 Mbp reference, semi-global affine DP,
packed int16 scores with int32 re-run of saturated pairs, outputs score,
start/end coordinates and CIGAR.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--config c1|c0|c2|c3] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GCUPS (150bp semi-global affine DP) + % int roofline; p50/p99 served latency"

# Integer VALU peak of MI355X: 256 CUs x 64 lanes x 2.4 GHz = 3.93e13 32-bit
# ops/s; packed 16-bit ops (v_pk_*) do two per lane: 7.86e13 ops/s.
PEAK_I16_TOPS = 256 * 64 * 2 * 2.4e9 / 1e12
PEAK_I32_TOPS = 256 * 64 * 2.4e9 / 1e12
# Algorithmic integer ops per cell (binary ops, a 3-way max counts 2):
# semi-global score+end 9, +4 direction compares = 13; local score+best 11, +5 = 16.
OPS_PER_CELL = {("sg", True): 13, ("sg", False): 9, ("local", True): 16, ("local", False): 11,
                ("ext", True): 16, ("ext", False): 11}
EXT_CLIP = 5  # clipping penalty of the seed-extension workload

# HBM bytes moved by the DP launches of one step, from two rocprofv3 passes
# (FETCH_SIZE, WRITE_SIZE) of this script, scaled by what the counters read
# for a 1 GiB device copy (2048 bytes per FETCH_SIZE unit, 1024 per
# WRITE_SIZE unit); the summaries are under profiles/.  They hold only for
# the build they were taken on: the DP kernels' sources and the build script
# (compiler flags; resident-wave targets live in the sources), identified by
# one SHA-256; for any other build the bench line reports traffic as null.
MEASURED_TRAFFIC = {
    # config: (build sha256, fetch bytes, write bytes)
    "c1": ("bab58b60f45863bf65ef5a187a5b215fe18b78cfb97aa35d468bd8a7b3c23846", 3229168128, 2685101696),
    "c2": ("bab58b60f45863bf65ef5a187a5b215fe18b78cfb97aa35d468bd8a7b3c23846", 3101558400, 7240992096),
    "c3": ("bab58b60f45863bf65ef5a187a5b215fe18b78cfb97aa35d468bd8a7b3c23846", 11805670912, 9037802912),
    "ext": ("bab58b60f45863bf65ef5a187a5b215fe18b78cfb97aa35d468bd8a7b3c23846", 3151174912, 1461079552),
    # the search kernel: its own sources (fm_source_sha)
    "bwt": ("7bd545de6e0822eccd77eca98f46c872f8b688666e356e26c45b01fc1e9a9b7b", 12810119168, 26541056),
}


def _sha_of(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + fh.read())
    return h.hexdigest()


def kernel_source_sha():
    """SHA-256 of every source the DP fill kernels are built from, plus the build script."""
    csrc = os.path.join(ROOT, "paper_1402_4876_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc)
                   if f in ("dp_common.h", "dp_fill.h", "band.h", "plan.h", "dp_misc.hip") or
                   f.startswith(("fill_", "persistent_", "side_")))
    return _sha_of(files + [os.path.join(ROOT, "paper_1402_4876_amd", "build.py")])


def fm_source_sha():
    csrc = os.path.join(ROOT, "paper_1402_4876_amd", "csrc")
    return _sha_of([os.path.join(csrc, f) for f in ("fm_search.hip", "fm_common.h", "fm_match.h")] +
                   [os.path.join(ROOT, "paper_1402_4876_amd", "build.py")])


def usable_cores():
    """Host cores this process may run on: its CPU affinity, capped by a cgroup CPU quota."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    for path in ("/sys/fs/cgroup/cpu.max", "/sys/fs/cgroup/cpu/cpu.cfs_quota_us"):
        try:
            with open(path) as fh:
                parts = fh.read().split()
        except OSError:
            continue
        if path.endswith("cpu.max") and parts and parts[0] != "max":
            n = min(n, max(1, int(int(parts[0]) / int(parts[1]))))
        elif path.endswith("quota_us") and parts and int(parts[0]) > 0:
            with open("/sys/fs/cgroup/cpu/cpu.cfs_period_us") as fh:
                n = min(n, max(1, int(int(parts[0]) / int(fh.read().split()[0]))))
        break
    return n


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_batch(cfg, pairs):
    import synth
    if cfg == "c0":
        return synth.config0(**({"n_pairs": pairs} if pairs else {}))
    if cfg == "c1":
        return synth.config1(**({"n_pairs": pairs} if pairs else {}))
    if cfg == "c2":
        return synth.config2(**({"n_pairs": pairs} if pairs else {}))
    if cfg == "c3":
        return synth.config3(**({"n_pairs": pairs} if pairs else {}))
    if cfg == "ext":
        return synth.extension_like(pairs or 1_000_000, ref_len=100_000_000)
    raise SystemExit("unknown config " + cfg)


WORKLOADS = {
    "c0": ("1,000 reads of 150 bp vs their own 200 bp windows, semi-global, int32, score + end", "sg", False, True),
    "c1": ("1,000,000 reads of 150 bp vs 400 bp windows of a 100 Mbp reference, semi-global, "
           "int16 + int32 re-run, score + start/end + CIGAR", "sg", True, False),
    "c2": ("500,000 mate-rescue reads of 150 bp vs 1,000 bp windows, local, int16 + int32 re-run, "
           "score + start/end + CIGAR", "local", True, False),
    "c3": ("2,000,000 pairs, reads U{50..250} bp vs 1.5m+64 bp windows, half local, one persistent "
           "launch, score + start/end + CIGAR", "mixed", True, False),
    "ext": ("1,000,000 seed extensions: read tails U{0..150} bp vs tail+32 bp windows, anchor score "
            "U{19..60}, clipping penalty 5, int16 + int32 re-run, score + start/end + CIGAR", "ext", True, False),
    "bwt": ("few-mismatch search (k = 2, max_occ 64) of the 1,000,000 c1 reads of 150 bp against the whole "
            "100 Mbp reference through its FM index", "bwt", False, False),
    "pipe": ("host pipeline: the 1,000,000 c1 reads of 150 bp as a FASTQ file through the few-mismatch search "
             "(k = 2) and semi-global DP of seed windows (band 32) into a SAM file, 100 Mbp reference",
             "pipe", True, False),
}
BWT_K, BWT_MAX_OCC = 2, 64
PIPE_BAND = 32
# algorithmic bytes of one read's search: per backward-search step (one per
# read base over the k + 1 parts) two 64-byte occurrence blocks, plus the
# read's 2-bit words, its descriptor (12 B) and outputs (24 B)
BWT_BYTES_PER_STEP = 128


def small_batch_latency(ctx, reps=50):
    """Per-call latency of the 1,000-pair, 150 x 200 int32 batch (too small to
    fill the GPU): host time from the call to its completion, median and min."""
    import torch

    import paper_1402_4876_amd as mica
    import synth
    b = synth.config0()
    dev = mica.to_device(b)
    n = b.n_pairs
    out = {k: torch.empty(n, dtype=torch.int32, device="cuda") for k in ("score", "read_end", "ref_end", "status")}
    mm, nn = int(b.read_len.max()), int(b.win_len.max())

    def call():
        mica.align(ctx, dev["ref2b"], dev["win_off"], dev["win_len"], dev["reads2b"], dev["read_off"],
                   dev["read_len"], force_int32=True, max_read_len=mm, max_win_len=nn, ref_len=dev["ref_len"],
                   reads_len=dev["reads_len"], out=out)
        torch.cuda.synchronize()

    for _ in range(5):
        call()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        call()
        ts.append((time.perf_counter() - t0) * 1e3)
    ts.sort()
    return {"workload": "1,000 pairs, 150 x 200, int32, score + end (one graph launch, synchronised)",
            "median_ms": round(ts[len(ts) // 2], 3), "min_ms": round(ts[0], 3)}


def cpu_baseline(batch, gpu_out, want_trace, target_s=12.0):
    """Time the CPU oracle on a bounded sample of the same pairs, on every host core
    this process may use."""
    import oracle
    threads = usable_cores()
    sc = (1, -4, 6, 1)
    h0 = batch.h0 if batch.h0 is not None else np.zeros(batch.n_pairs, np.int32)
    ext = dict(clip=EXT_CLIP)
    oracle.align_batch(batch.ref, batch.win_off[:64], batch.win_len[:64], batch.reads, batch.read_off[:64],
                       batch.read_len[:64], batch.mode[:64], sc, trace=want_trace, threads=threads,
                       h0=h0[:64], **ext)
    n = min(batch.n_pairs, 20000)
    idx = np.arange(n)
    t0 = time.time()
    o = oracle.align_batch(batch.ref, batch.win_off[idx], batch.win_len[idx], batch.reads, batch.read_off[idx],
                           batch.read_len[idx], batch.mode[idx], sc, trace=want_trace, threads=threads,
                           h0=h0[idx], **ext)
    dt = time.time() - t0
    if dt < target_s / 3 and n < batch.n_pairs:
        n = int(min(batch.n_pairs, n * target_s / max(dt, 1e-3)))
        idx = np.arange(n)
        t0 = time.time()
        o = oracle.align_batch(batch.ref, batch.win_off[idx], batch.win_len[idx], batch.reads,
                               batch.read_off[idx], batch.read_len[idx], batch.mode[idx], sc,
                               trace=want_trace, threads=threads, h0=h0[idx], **ext)
        dt = time.time() - t0
    cells = float(np.dot(batch.read_len[idx].astype(np.int64), batch.win_len[idx].astype(np.int64)))
    # parity of the GPU result on the same sample
    keys = ["score", "read_end", "ref_end"] + (["read_start", "ref_start", "n_cigar"] if want_trace else [])
    mism = {k: int((gpu_out[k][idx] != o[k]).sum()) for k in keys}
    st = (gpu_out["status"][idx].astype(np.uint32) & ~np.uint32(1)) != o["status"]
    mism["status"] = int(st.sum())
    if want_trace:
        cap = o["cigar"].shape[1]
        ncig = np.minimum(np.abs(o["n_cigar"]), cap)
        col = np.arange(cap)[None, :] < ncig[:, None]
        mism["cigar"] = int((((gpu_out["cigar"][idx].astype(np.uint32) != o["cigar"]) & col).any(axis=1)).sum())
    # one core on the first 10,000 pairs
    i1 = np.arange(min(batch.n_pairs, 10000))
    t1c = time.time()
    oracle.align_batch(batch.ref, batch.win_off[i1], batch.win_len[i1], batch.reads, batch.read_off[i1],
                       batch.read_len[i1], batch.mode[i1], sc, trace=want_trace, threads=1, h0=h0[i1], **ext)
    dt1 = time.time() - t1c
    cells1 = float(np.dot(batch.read_len[i1].astype(np.int64), batch.win_len[i1].astype(np.int64)))
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            cpu_model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    base = {"value": round(cells / dt / 1e9, 4), "unit": "GCUPS", "cores": threads, "kind": "oracle",
            "sample": "first %d pairs of the same batch (%.3g cells), %s, %.1f s" % (
                n, cells, "with traceback" if want_trace else "score + end", dt),
            "single_core_gcups": round(cells1 / dt1 / 1e9, 4), "cpu_model": cpu_model}
    parity = {"pairs": n, "mismatches": mism, "exact": all(v == 0 for v in mism.values())}
    return base, parity


def serving_bench(n_per_rate=2000, warmup=200, pool_reads=200_000, slots=4, fracs=(0.3, 0.6, 0.9),
                  fifo_baseline=True, parity_requests=4):
    """Open-loop serving of config-4 requests: a 3 Gbp reference resident on the
    GPU; each request is a distinct range (1..10,000 reads) of a pool of planted
    {100, 150, 250} bp reads (windows 1.5 m + 64, semi-global, full outputs);
    arrivals are a Poisson stream replayed by the library's own submitter
    thread.  Latency = finish - scheduled arrival, on the server.

    Measured: the closed-loop capacity (lambda_max) of the continuous-batching
    server and of the FIFO baseline (one request per batch, one slot); each
    server at 0.3 / 0.6 / 0.9 of its own lambda_max; the batching server also
    at the FIFO baseline's rates.  A rate at or above a server's lambda_max is
    marked overloaded.  A few requests' outputs are kept for the parity check
    of the CPU-baseline leg."""
    import synth
    import paper_1402_4876_amd as mica
    from paper_1402_4876_amd.pack import pack_codes
    ref_len = 3_000_000_000
    t0 = time.time()
    ref = synth.serving_reference(ref_len)
    pool = synth.serving_pool(ref, ref_len, pool_reads)
    words = pack_codes(pool.reads)
    ro = pool.read_off.astype(np.uint64)
    rl = pool.read_len.astype(np.int32)
    wo = pool.win_off.astype(np.uint64)
    wl = pool.win_len.astype(np.int32)
    cells = rl.astype(np.int64) * wl.astype(np.int64)
    csum = np.concatenate([[0], np.cumsum(cells)])
    log("serving: reference and a %d-read pool in %.1fs" % (pool_reads, time.time() - t0))
    keep = {}

    def run(srv, first, count, arrival, id0, keep_ids=()):
        """Replay one schedule, forget every finished request except keep_ids
        (fetched for the parity check); returns the wall span on the server."""
        srv.replay(words, ro, rl, wo, wl, first, count, arrival, first_id=id0)
        want = set(range(id0, id0 + len(first)))
        t_first = float(np.min(arrival)) if len(arrival) else srv.now()
        while want:
            got = srv.poll()
            for i in got:
                if i in keep_ids:
                    keep[i] = srv.fetch(i)
                else:
                    srv.forget(i)
                want.discard(i)
            if not got:
                time.sleep(0.0005)
        lag = srv.replay_wait()
        return srv.now() - t_first, lag

    def closed_loop(srv, n, key, id0):
        first, count = synth.request_schedule(len(rl), n, key)
        now = srv.now()
        arrival = np.full(n, now, np.float64)
        span, _ = run(srv, first, count, arrival, id0)
        return n / span, float((csum[first + count] - csum[first]).sum()) / span / 1e9

    def open_loop(srv, rate, key, id0, keep_ids=()):
        n = warmup + n_per_rate
        first, count = synth.request_schedule(len(rl), n, key)
        arr = synth.poisson_arrivals(rate, n, seed_key=key)
        start = srv.now() + 0.01
        # warm-up requests first, then the measured ones on the same clock
        run(srv, first[:warmup], count[:warmup], start + arr[:warmup], id0)
        srv.reset_stats()
        span, lag = run(srv, first[warmup:], count[warmup:], start + arr[warmup:], id0 + warmup, keep_ids)
        st = srv.stats()
        return {"rate_rps": round(rate, 1), "p50_ms": round(st["p50_s"] * 1e3, 3),
                "p99_ms": round(st["p99_s"] * 1e3, 3), "gcups": round(st["gcups"], 1),
                "replay_lag_ms": round(lag * 1e3, 3)}

    out = {"reference_bases": ref_len, "requests_per_rate": n_per_rate, "warmup_requests": warmup,
           "request_pool_reads": pool_reads, "distinct_requests": True,
           "mean_cells_per_request": round(float(cells.mean() * 5000.5), 1), "submitter": "library replay thread"}
    # the same reads as one batch through the batch API (the served mix's
    # own batch rate: three read-length classes, semi-global, full outputs)
    import torch
    dev_ref = torch.as_tensor(np.ascontiguousarray(ref).view(np.int32)).cuda()
    dev_reads = torch.as_tensor(np.ascontiguousarray(words).view(np.int32)).cuda()
    dwo, dwl = torch.as_tensor(wo.view(np.int64)).cuda(), torch.as_tensor(wl).cuda()
    dro, drl = torch.as_tensor(ro.view(np.int64)).cuda(), torch.as_tensor(rl).cuda()
    bctx = mica.Context()
    try:
        def step():
            return mica.align(bctx, dev_ref, dwo, dwl, dev_reads, dro, drl, out_cigar=True, cigar_cap=64,
                              max_read_len=int(rl.max()), max_win_len=int(wl.max()), ref_len=ref_len,
                              reads_len=len(pool.reads), min_read_len=int(rl.min()))
        for _ in range(2):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(5):
            step()
        torch.cuda.synchronize()
        bms = (time.perf_counter() - t1) * 1e3 / 5
    finally:
        bctx.close()
    del dev_ref, dev_reads, dwo, dwl, dro, drl
    torch.cuda.empty_cache()
    # (the server runs the default plan too: a plan autotuned on these reads
    # made the one batch faster, 2,963 -> 3,244 GCUPS, but not the served
    # stream, whose batches are about 17,000 reads)
    out["batch_same_reads"] = {"reads": int(len(rl)), "ms": round(bms, 3),
                               "gcups": round(float(cells.sum()) / (bms * 1e-3) / 1e9, 1), "plan": "default"}
    log("serving: the pool as one batch: %s" % out["batch_same_reads"])
    srv = mica.Server(ref, ref_len, slots=slots)
    sample_ids = []
    try:
        closed_loop(srv, 100, 90, 10_000_000)
        lam, lam_gcups = closed_loop(srv, 2000, 91, 20_000_000)
        out["lambda_max_rps"] = round(lam, 1)
        out["gcups_at_lambda_max"] = round(lam_gcups, 1)
        out["served_over_batch_same_reads"] = round(lam_gcups / out["batch_same_reads"]["gcups"], 3)
        out["batching"] = {"slots": slots, "rates": []}
        for i, f in enumerate(fracs):
            id0 = 30_000_000 + i * 1_000_000
            kid = set(range(id0 + warmup, id0 + warmup + parity_requests)) if i == 1 else ()
            r = open_loop(srv, f * lam, 100 + i, id0, kid)
            sample_ids += sorted(kid)
            r["frac_of_own_max"] = f
            r["overloaded"] = f >= 1.0
            out["batching"]["rates"].append(r)
            log("serving batching %.1f x max: %s" % (f, r))
    except Exception:
        srv.close()
        raise
    if fifo_baseline:
        fifo = mica.Server(ref, ref_len, slots=1, fifo=True)
        try:
            fl, _ = closed_loop(fifo, 300, 92, 40_000_000)
            out["fifo_baseline"] = {"slots": 1, "lambda_max_rps": round(fl, 1), "rates": []}
            for i, f in enumerate(fracs):
                r = open_loop(fifo, f * fl, 200 + i, 50_000_000 + i * 1_000_000)
                r["frac_of_own_max"] = f
                r["overloaded"] = f >= 1.0
                out["fifo_baseline"]["rates"].append(r)
                log("serving fifo %.1f x its max: %s" % (f, r))
        finally:
            fifo.close()
        # the batching server at the FIFO baseline's own rates (loads both sustain)
        out["batching_at_fifo_rates"] = []
        try:
            for i, f in enumerate(fracs):
                rate = f * fl
                r = open_loop(srv, rate, 300 + i, 60_000_000 + i * 1_000_000)
                r["frac_of_own_max"] = round(rate / lam, 4)
                r["overloaded"] = rate >= lam
                out["batching_at_fifo_rates"].append(r)
                log("serving batching at fifo %.1f x max: %s" % (f, r))
        finally:
            srv.close()
    else:
        srv.close()
    # outputs of a few served requests, with their pairs, for the CPU-baseline leg
    sample = []
    for rid in sample_ids:
        i = rid - 30_000_000 - 1_000_000 - warmup
        first, count = synth.request_schedule(len(rl), warmup + n_per_rate, 101)
        f, c = int(first[warmup + i]), int(count[warmup + i])
        sample.append((np.arange(f, f + c), keep.get(rid)))
    out["_parity"] = (pool, sample)
    return out


def serving_parity(pool, sample):
    """The served outputs of a few requests against the oracle (CPU-baseline leg)."""
    import oracle
    import synth
    mism = {}
    pairs = 0
    for idx, got in sample:
        if got is None:
            mism["missing"] = mism.get("missing", 0) + 1
            continue
        b = synth.rebase_windows(pool.subset(idx))
        o = oracle.align_batch(b.ref, b.win_off, b.win_len, b.reads, b.read_off, b.read_len, b.mode, trace=True,
                               cigar_cap=64, threads=usable_cores())
        pairs += len(idx)
        for k in ("score", "read_start", "read_end", "ref_start", "ref_end", "n_cigar"):
            mism[k] = mism.get(k, 0) + int((got[k] != o[k]).sum())
        mism["status"] = mism.get("status", 0) + int(((got["status"] & ~np.uint32(1)) != o["status"]).sum())
        ncig = np.minimum(np.abs(o["n_cigar"]), 64)
        col = np.arange(64)[None, :] < ncig[:, None]
        mism["cigar"] = mism.get("cigar", 0) + int((((got["cigar"] != o["cigar"]) & col).any(axis=1)).sum())
    return {"requests": len(sample), "pairs": pairs, "mismatches": mism, "exact": all(v == 0 for v in mism.values())}


def bwt_bench(args):
    """The few-mismatch search phase on the c1 reads and reference: reads/s,
    HBM roofline of the search kernel, oracle baseline and parity sample."""
    import torch

    import paper_1402_4876_amd as mica
    import synth
    from paper_1402_4876_amd import pack_codes
    t0 = time.time()
    b = synth.config1(**({"n_pairs": args.pairs} if args.pairs else {}))
    log("generated reads and reference in %.1fs" % (time.time() - t0))
    ix = mica.FmIndex(pack_codes(b.ref), len(b.ref))
    info = ix.info()
    log("FM index: %.1f s build, %.2f GB on the device" % (info["build_seconds"], info["device_bytes"] / 1e9))
    reads2b = torch.from_numpy(pack_codes(b.reads).view(np.int32)).cuda()
    read_off = torch.from_numpy(b.read_off).cuda()
    read_len = torch.from_numpy(b.read_len).cuda()
    n = b.n_pairs
    out = {key: torch.empty(n, dtype=torch.int32, device="cuda") for key in ("best_mm", "n_best", "n_hits", "status")}
    out["pos"] = torch.empty(n, dtype=torch.int64, device="cuda")

    def step():
        ix.search(reads2b, read_off, read_len, k=BWT_K, max_occ=BWT_MAX_OCC, reads_len=len(b.reads), out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the search is one kernel launch on the current stream: events there time it
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for _ in range(args.steps):
        step()
    ev[1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    kernel_ms = ev[0].elapsed_time(ev[1]) / args.steps
    m = b.read_len.astype(np.int64)
    alg = float((m * BWT_BYTES_PER_STEP + (m + 15) // 16 * 4 + 36).sum())
    # The bound is HBM, priced on the bytes that really cross it (FETCH_SIZE
    # + WRITE_SIZE counters of this build).  The algorithmic model counts
    # every occurrence block a backward-search step reads; the first steps of
    # every search share a few blocks that stay in L2, so that model exceeds
    # what HBM moves and is reported beside it only.
    roof = {"bound": "hbm", "achieved": None, "peak": 8000.0, "unit": "GB/s", "frac": None, "traffic": None,
            "kernel": "k_fm_search", "kernel_ms": round(kernel_ms, 4), "bytes_per_read": round(alg / n, 1),
            "algorithmic_gbps": round(alg / (kernel_ms * 1e-3) / 1e9, 1)}
    meas = MEASURED_TRAFFIC.get("bwt")
    if meas and meas[0] == fm_source_sha():
        roof["traffic"] = meas[1] + meas[2]
        roof["traffic_split"] = {"fetch": meas[1], "write": meas[2]}
        achieved = roof["traffic"] / (kernel_ms * 1e-3) / 1e9
        roof["achieved"] = round(achieved, 1)
        roof["frac"] = round(achieved / 8000.0, 4)
    else:
        roof["traffic_note"] = "no FETCH_SIZE/WRITE_SIZE counters taken for this build: achieved not priced"
    g = {key: v.cpu().numpy() for key, v in out.items()}
    res = {
        "metric": "reads/s (few-mismatch BWT search, k = 2)", "value": round(n / (ms * 1e-3), 1), "unit": "reads/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": WORKLOADS["bwt"][0], "name": "bwt", "reads": n, "ref_bases": len(b.ref),
                   "index_build_s": round(info["build_seconds"], 1), "index_gb": round(info["device_bytes"] / 1e9, 3)},
        "roofline": roof,
        "found_frac": round(float((g["best_mm"] >= 0).mean()), 4),
        "repetitive": int((g["status"] == mica.ST_REPETITIVE).sum()),
    }
    if not args.no_cpu_baseline:
        import oracle
        threads = usable_cores()
        idx = np.arange(min(n, 64))
        t0 = time.time()
        o = oracle.kmm_search(b.ref, b.reads, b.read_off[idx], b.read_len[idx], k=BWT_K, max_occ=BWT_MAX_OCC,
                              threads=threads)
        dt = time.time() - t0
        if dt < 4 and len(idx) < n:
            idx = np.arange(min(n, int(len(idx) * 12 / max(dt, 1e-3))))
            t0 = time.time()
            o = oracle.kmm_search(b.ref, b.reads, b.read_off[idx], b.read_len[idx], k=BWT_K,
                                  max_occ=BWT_MAX_OCC, threads=threads)
            dt = time.time() - t0
        mism = {key: int((g[key][idx].astype(np.int64) != o[key].astype(np.int64)).sum())
                for key in ("best_mm", "n_best", "n_hits", "pos", "status")}
        res["cpu_baseline"] = {"value": round(len(idx) / dt, 2), "unit": "reads/s", "cores": threads,
                               "kind": "oracle", "sample": "first %d reads, every placement against the "
                               "100 Mbp reference, %.1f s" % (len(idx), dt)}
        res["parity_sample"] = {"reads": int(len(idx)), "mismatches": mism, "exact": all(v == 0 for v in mism.values())}
    ix.close()
    print(json.dumps(res), flush=True)
    return 0


def pipe_bench(args):
    """End-to-end host pipeline: FASTQ file in, SAM file out (files in TMPDIR)."""
    import shutil
    import tempfile

    import paper_1402_4876_amd as mica
    import synth
    from paper_1402_4876_amd import pack_codes
    t0 = time.time()
    b = synth.config1(**({"n_pairs": args.pairs} if args.pairs else {}))
    tmp = tempfile.mkdtemp(prefix="mica_pipe_", dir=os.environ.get("TMPDIR", "/tmp"))
    try:
        fq = os.path.join(tmp, "reads.fq")
        sam = os.path.join(tmp, "out.sam")
        letters = np.frombuffer(b"ACGT", np.uint8)
        with open(fq, "wb") as f:
            qual = b"I" * 150
            seqs = letters[b.reads]
            for r in range(b.n_pairs):
                o = int(b.read_off[r])
                m = int(b.read_len[r])
                f.write(b"@r%d\n%s\n+\n%s\n" % (r, seqs[o:o + m].tobytes(), qual[:m]))
        fq_bytes = os.path.getsize(fq)
        log("wrote %d reads as FASTQ (%.0f MB) in %.1fs" % (b.n_pairs, fq_bytes / 1e6, time.time() - t0))
        pipe = mica.Pipeline(pack_codes(b.ref), len(b.ref), "chrS", k=BWT_K, max_occ=BWT_MAX_OCC, band=PIPE_BAND,
                             min_score=0, batch_reads=args.pipe_batch, format_threads=args.pipe_threads)
        for _ in range(args.warmup):
            pipe.run(fq, sam)
        runs = []
        for _ in range(max(1, args.steps)):
            runs.append(pipe.run(fq, sam))
        pipe.close()
        sam_bytes = os.path.getsize(sam)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    st = runs[-1]
    sec = float(np.mean([r["seconds"] for r in runs]))
    res = {
        "metric": "reads/s (FASTQ to SAM, both phases)", "value": round(b.n_pairs / sec, 1), "unit": "reads/s",
        "n_gpus": 1, "steps": len(runs), "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i16", "data": "synthetic",
        "config": {"workload": WORKLOADS["pipe"][0], "name": "pipe", "reads": b.n_pairs, "batch_reads": args.pipe_batch,
                   "format_threads": args.pipe_threads,
                   "fastq_mb": round(fq_bytes / 1e6, 1), "sam_mb": round(sam_bytes / 1e6, 1)},
        "stages_s": {"parse": round(st["parse_seconds"], 3), "gpu": round(st["gpu_seconds"], 3),
                     "format_write": round(st["format_seconds"], 3), "wall": round(st["seconds"], 3)},
        "reads_by_outcome": {"search": st["mapped_search"], "dp": st["mapped_dp"], "unmapped": st["unmapped"]},
    }
    print(json.dumps(res), flush=True)
    return 0


def copy_calibration(nbytes=1 << 30, reps=3):
    """A device-to-device copy of known size: what FETCH_SIZE / WRITE_SIZE read for it
    gives the counter-to-bytes factor used for the DP kernel's HBM traffic."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": nbytes, "launches": reps}), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c1", choices=sorted(WORKLOADS))
    ap.add_argument("--pairs", type=int, default=0, help="override the pair count (testing only)")
    ap.add_argument("--plain", action="store_true", help="per-bucket launches instead of the persistent one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving (request stream) measurement")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per arrival rate")
    ap.add_argument("--serve-slots", type=int, default=4, help="in-flight slots of the serving measurement")
    ap.add_argument("--serve-only", action="store_true", help="only the serving measurement (no batch step)")
    ap.add_argument("--no-fifo", action="store_true", help="skip the FIFO serving baseline")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="c1 only: skip the short runs of c2, c3 and the extensions appended to its line")
    ap.add_argument("--pipe-batch", type=int, default=1 << 18, help="reads per batch of the host pipeline")
    ap.add_argument("--pipe-threads", type=int, default=8, help="SAM formatting threads of the host pipeline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (scale for the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
    if args.serve_only:
        res = serving_bench(n_per_rate=args.serve_requests, warmup=max(args.serve_requests // 10, 20),
                            slots=args.serve_slots, fifo_baseline=not args.no_fifo)
        served = res.pop("_parity")
        if not args.no_cpu_baseline:
            res["parity_sample"] = serving_parity(*served)
        print(json.dumps({"serving": res}), flush=True)
        return 0
    if args.gpus == 1 and args.config == "bwt":
        return bwt_bench(args)
    if args.gpus == 1 and args.config == "pipe":
        return pipe_bench(args)
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(pairs are independent; see the sharding notes). Run with --gpus 1.", file=sys.stderr)
        return 2

    import torch

    import paper_1402_4876_amd as mica

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    desc, mode_kind, want_trace, force_i32 = WORKLOADS[args.config]
    t0 = time.time()
    batch = make_batch(args.config, args.pairs)
    log("generated %s: %d pairs, %.3g cells in %.1fs" % (args.config, batch.n_pairs, batch.cells(), time.time() - t0))
    dev = mica.to_device(batch)
    n = batch.n_pairs
    cells = float(batch.cells())
    max_m = int(batch.read_len.max())
    min_m = int(batch.read_len.min())
    # reads of one 16-base length class (default plan, up to 256 bases) run
    # that class's own kernel rather than the persistent ones
    one_class = n > 0 and min_m >= 1 and (min_m - 1) // 16 == (max_m - 1) // 16 and max_m <= 256
    max_n = int(batch.win_len.max())
    cap = 64

    def new_out():
        o = {k: torch.empty(n, dtype=torch.int32, device="cuda") for k in
             ("score", "read_end", "ref_end", "status", "read_start", "ref_start", "n_cigar")}
        o["cigar"] = torch.empty((n, cap), dtype=torch.int32, device="cuda")
        return o

    out = new_out()
    ctx = mica.Context()
    # a batch of one mode passes no per-pair mode array
    uniform = bool((batch.mode == batch.mode[0]).all()) if n else True
    mode_arg = None if uniform else dev["mode"]
    default_mode = int(batch.mode[0]) if (uniform and n) else 0
    mode_mask = int(np.bitwise_or.reduce(1 << np.unique(batch.mode).astype(np.int64))) if n else 0
    ext_h0 = torch.as_tensor(batch.h0).cuda() if batch.h0 is not None else None
    # the anchor scores' bound, known where the batch was made (lets a batch
    # whose extensions fit 16-bit scores skip the saturation-checking kernels)
    max_h0 = int(batch.h0.max()) if batch.h0 is not None and n else 0
    if mode_kind == "mixed":
        loc = batch.mode == 1
        ops = float(np.dot(batch.read_len.astype(np.int64), batch.win_len.astype(np.int64) *
                           np.where(loc, OPS_PER_CELL[("local", want_trace)], OPS_PER_CELL[("sg", want_trace)])))
    else:
        ops = cells * OPS_PER_CELL[(mode_kind, want_trace)]
    peak = PEAK_I32_TOPS if force_i32 else PEAK_I16_TOPS
    # measured VALU roof of this GPU (the spec figure assumes 2.4 GHz under load)
    valu_i16, valu_i32 = mica.measure_valu_peak(torch.cuda.current_device())
    peak_meas = valu_i32 if force_i32 else valu_i16

    autotune = None
    if args.config == "c3" and not args.plain:
        # the plan is tuned on a sample of the batch (every 16-base read-length
        # range, bit-exact gate against the default plan), then both launch
        # styles run with the tuned plan
        k = min(n, 200_000)
        t0 = time.time()
        entries = ctx.autotune(dev["ref2b"], dev["win_off"][:k], dev["win_len"][:k], dev["reads2b"],
                               dev["read_off"][:k], dev["read_len"][:k], mode=dev["mode"][:k],
                               out_cigar=want_trace, cigar_cap=cap, max_read_len=max_m, max_win_len=max_n,
                               ref_len=dev["ref_len"], reads_len=dev["reads_len"], reps=3)
        autotune = {"sample_pairs": k, "seconds": round(time.time() - t0, 1),
                    "ranges": [{"m": [e["m_lo"], e["m_hi"]], "lanes": e["lanes"], "rows": e["rows"],
                                "ms": round(e["ms"], 4), "default_ms": round(e["default_ms"], 4),
                                "candidates": e["n_candidates"], "rejected": e["n_rejected"]} for e in entries]}
        log("autotune: %d ranges in %.1fs; %d changed from the default plan" % (
            len(entries), time.time() - t0,
            sum(1 for e in entries if abs(e["ms"] - e["default_ms"]) > 1e-12)))

    def run_leg(plain, out):
        """Warm-up, then args.steps timed steps of one launch style: host time per
        step, the fill kernels' summed event time and per-step device times."""
        def step():
            mica.align(ctx, dev["ref2b"], dev["win_off"], dev["win_len"], dev["reads2b"], dev["read_off"],
                       dev["read_len"], mode=mode_arg, default_mode=default_mode, out_cigar=want_trace,
                       cigar_cap=cap, force_int32=force_i32, plain=plain, max_read_len=max_m, max_win_len=max_n,
                       ref_len=dev["ref_len"], reads_len=dev["reads_len"], out=out, mode_mask=mode_mask,
                       ext_h0=ext_h0, ext_clip=EXT_CLIP, min_read_len=min_m, max_ext_h0=max_h0)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ctx.set_timing(True)
        ctx.read_timing()
        # events on the launch stream around every step (the align call enqueues
        # the whole graph there): per-step device times for the median and minimum
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs[0].record()
        for i in range(args.steps):
            step()
            evs[i + 1].record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step_ms = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps))
        fill_ms, nb = ctx.read_timing()
        ctx.set_timing(False)
        ms = (t1 - t0) * 1e3 / args.steps
        fill_avg_ms = fill_ms / max(nb, 1)
        achieved = ops / (fill_avg_ms * 1e-3) / 1e12
        return {"ms": ms, "fill_ms": fill_avg_ms, "step_ms": step_ms, "gcups": cells / (ms * 1e-3) / 1e9,
                "achieved": achieved}

    leg = run_leg(args.plain, out)
    stats = ctx.last_stats()
    ms, fill_avg_ms, step_ms, gcups, achieved = leg["ms"], leg["fill_ms"], leg["step_ms"], leg["gcups"], leg["achieved"]
    # transfers of the same batch, timed apart from the steps: inputs from
    # pinned host memory to the device, outputs back
    host_in = {k: v.cpu().pin_memory() for k, v in dev.items() if isinstance(v, torch.Tensor)}
    host_out = {k: torch.empty(v.shape, dtype=v.dtype, pin_memory=True) for k, v in out.items()}
    te = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    te[0].record()
    for k, v in host_in.items():
        dev[k].copy_(v, non_blocking=True)
    te[1].record()
    for k, v in out.items():
        host_out[k].copy_(v, non_blocking=True)
    te[2].record()
    torch.cuda.synchronize()
    h2d_ms, d2h_ms = te[0].elapsed_time(te[1]), te[1].elapsed_time(te[2])
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": "TOP/s",
            "frac": round(achieved / peak, 4), "traffic": None,
            "kernel": ("k_fill_bucket" if args.plain or one_class else "k_fill_persistent") +
            " (all fill launches of one step)", "kernel_ms": round(fill_avg_ms, 4),
            "ops_per_cell": round(ops / cells, 3),
            "peak_measured": round(peak_meas, 3), "frac_of_measured": round(achieved / peak_meas, 4),
            "valu_measured": {"i16x2": round(valu_i16, 3), "i32": round(valu_i32, 3)}}
    meas = MEASURED_TRAFFIC.get(args.config + ("_plain" if args.plain else ""))
    if meas and meas[0] == kernel_source_sha():
        roof["traffic"] = meas[1] + meas[2]
        roof["traffic_split"] = {"fetch": meas[1], "write": meas[2]}
    else:
        roof["traffic_note"] = "no FETCH_SIZE/WRITE_SIZE counters taken for this build"
    host = {k: v.cpu().numpy() for k, v in out.items()}
    res = {
        "metric": METRIC, "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "i32" if force_i32 else "i16", "data": "synthetic",
        "config": {"workload": desc, "name": args.config, "pairs": n, "cells": cells,
                   "launch": "plain per-bucket" if args.plain else (
                       "one class: its own kernel" if one_class else "persistent"),
                   "plan": "autotuned" if autotune else "default"},
        "roofline": roof,
        "step_ms": {"median": round(step_ms[len(step_ms) // 2], 4), "min": round(step_ms[0], 4),
                    "max": round(step_ms[-1], 4)},
        "transfers": {"h2d_ms": round(h2d_ms, 3), "d2h_ms": round(d2h_ms, 3),
                      "h2d_mb": round(sum(v.numel() * v.element_size() for v in host_in.values()) / 1e6, 1),
                      "d2h_mb": round(sum(v.numel() * v.element_size() for v in out.values()) / 1e6, 1),
                      "gcups_with_transfers": round(cells / ((ms + h2d_ms + d2h_ms) * 1e-3) / 1e9, 2)},
        "saturated_pairs": int(stats["n_saturated"]),
        "wide_band_pairs": int(stats["n_fallback"]),
        "deferred_band_pairs": int(stats["n_deferred"]),
        "resident_waves": int(stats["n_waves"]),
    }
    if autotune is not None:
        res["autotune"] = autotune
        # the plain one-launch-per-length-bucket kernels on the same batch and
        # plan, and a bit-exact comparison of every output of the two styles
        out_plain = new_out()
        lp = run_leg(True, out_plain)
        host_plain = {k: v.cpu().numpy() for k, v in out_plain.items()}
        ncig = np.minimum(np.abs(host["n_cigar"]), cap)
        col = np.arange(cap)[None, :] < ncig[:, None]
        diff = {k: int((host[k] != host_plain[k]).sum()) for k in host if k != "cigar"}
        diff["cigar"] = int((((host["cigar"] != host_plain["cigar"]) & col).any(axis=1)).sum())
        res["plain_per_bucket"] = {
            "value": round(lp["gcups"], 2), "ms_per_step": round(lp["ms"], 4), "kernel_ms": round(lp["fill_ms"], 4),
            "achieved": round(lp["achieved"], 3), "frac": round(lp["achieved"] / peak, 4),
            "frac_of_measured": round(lp["achieved"] / peak_meas, 4),
            "step_ms_median": round(lp["step_ms"][len(lp["step_ms"]) // 2], 4),
            "outputs_differing_from_persistent": diff, "bit_exact_vs_persistent": all(v == 0 for v in diff.values())}
        res["persistent_over_plain"] = round(gcups / lp["gcups"], 4)
        log("c3 persistent %.1f GCUPS, plain %.1f GCUPS, bit-exact %s" % (
            gcups, lp["gcups"], res["plain_per_bucket"]["bit_exact_vs_persistent"]))
    if args.config == "c1":
        res["small_batch_latency"] = small_batch_latency(ctx)
    served = None
    if not args.no_serving:
        res["serving"] = serving_bench(n_per_rate=args.serve_requests, warmup=max(args.serve_requests // 10, 20),
                                       slots=args.serve_slots)
        served = res["serving"].pop("_parity")
    if not args.no_cpu_baseline:
        base, parity = cpu_baseline(batch, host, want_trace)
        res["cpu_baseline"] = base
        res["parity_sample"] = parity
        if served is not None:
            res["serving"]["parity_sample"] = serving_parity(*served)
    if args.config == "c1" and not args.no_other_workloads and not args.pairs:
        res["other_workloads"] = other_workloads()
    print(json.dumps(res), flush=True)
    return 0


def other_workloads(steps=5, warmup=2, timeout_s=420):
    """Short runs of the other DP workloads (c2, c3 with its plain-launch
    comparison, the seed extensions), each in a child process after the c1
    measurement, so that one bench invocation reports every DP workload.
    A failed or timed-out run is reported as such; it never fails the c1 line."""
    import subprocess
    out = {}
    for cfg in ("c2", "c3", "ext"):
        cmd = [sys.executable, os.path.abspath(__file__), "--config", cfg, "--no-cpu-baseline", "--no-serving",
               "--steps", str(steps), "--warmup", str(warmup)]
        log("other workloads: %s" % cfg)
        try:
            r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=timeout_s)
            line = r.stdout.strip().splitlines()[-1] if r.stdout.strip() else ""
            if r.returncode != 0 or not line:
                out[cfg] = {"error": "exit status %d" % r.returncode}
                continue
            d = json.loads(line)
        except subprocess.TimeoutExpired:
            out[cfg] = {"error": "timed out after %d s" % timeout_s}
            continue
        except (ValueError, OSError) as e:
            out[cfg] = {"error": str(e)}
            continue
        roof = d["roofline"]
        e = {"value": d["value"], "unit": d["unit"], "ms_per_step": d["ms_per_step"], "steps": d["steps"],
             "frac": roof["frac"], "frac_of_measured": roof["frac_of_measured"], "kernel_ms": roof["kernel_ms"],
             "ops_per_cell": roof["ops_per_cell"], "traffic": roof.get("traffic"), "launch": d["config"]["launch"],
             "plan": d["config"]["plan"], "workload": d["config"]["workload"],
             "wide_band_pairs": d["wide_band_pairs"], "deferred_band_pairs": d["deferred_band_pairs"]}
        if "plain_per_bucket" in d:
            pl = d["plain_per_bucket"]
            e["plain_per_bucket"] = {"value": pl["value"], "frac": pl["frac"],
                                     "bit_exact_vs_persistent": pl["bit_exact_vs_persistent"]}
            e["persistent_over_plain"] = d["persistent_over_plain"]
        out[cfg] = e
    return out


if __name__ == "__main__":
    sys.exit(main())
