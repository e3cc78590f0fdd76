"""GPU tests of the serving loop (mica_server_*): results of requests served
through continuous batching equal the oracle, a request's results do not
depend on what shares its batch, and the FIFO baseline, statistics and error
paths behave."""
import time

import numpy as np
import pytest

import synth
import gpu_util as U
from paper_1402_4876_amd.pack import pack_codes

pytestmark = pytest.mark.gpu

SC = (1, -4, 6, 1)


def _requests(batch, sizes):
    """Split a batch into requests (index arrays) of the given sizes."""
    out, k = [], 0
    for s in sizes:
        out.append(np.arange(k, min(k + s, batch.n_pairs)))
        k += s
    return [r for r in out if len(r)]


def _submit(srv, batch, reads_words, rid, idx):
    mode = batch.mode[idx].astype(np.uint8)
    srv.submit(rid, reads_words, batch.read_off[idx].astype(np.uint64), batch.read_len[idx],
               batch.win_off[idx].astype(np.uint64), batch.win_len[idx], mode=mode)


def _wait(srv, ids, timeout=120.0):
    left, got = set(ids), {}
    t0 = time.time()
    while left:
        for i in srv.poll():
            if i in left:
                got[i] = srv.fetch(i)
                left.discard(i)
        if left and time.time() - t0 > timeout:
            raise AssertionError("requests not finished: %s" % sorted(left)[:5])
        time.sleep(0.002)
    return got


def _concat(results, order):
    keys = results[order[0]].keys()
    return {k: np.concatenate([results[i][k] for i in order]) for k in keys}


@pytest.fixture(scope="module")
def served():
    import torch

    import paper_1402_4876_amd as mica
    torch.cuda.set_device(0)
    b = synth.serving_like(6000, ref_len=2_000_000, seed=3)
    b.mode[::2] = 1  # half local
    ref_words = pack_codes(b.ref)
    reads_words = pack_codes(b.reads)
    sizes = list(np.random.default_rng(5).integers(1, 700, 40))
    reqs = _requests(b, sizes)
    srv = mica.Server(ref_words, len(b.ref), slots=3, hbm_budget_bytes=4 << 30)
    try:
        for rid, idx in enumerate(reqs):
            _submit(srv, b, reads_words, 100 + rid, idx)
        res = _wait(srv, [100 + r for r in range(len(reqs))])
        st = srv.stats()
    finally:
        srv.close()
    return b, ref_words, reads_words, reqs, res, st


def test_served_results_equal_oracle(served):
    b, _, _, reqs, res, st = served
    order = [100 + r for r in range(len(reqs))]
    g = _concat(res, order)
    idx = np.concatenate(reqs)
    o = U.run_oracle(b, SC, idx=idx)
    U.assert_same(g, o, what="served")
    assert st["p50_s"] > 0 and st["p99_s"] >= st["p50_s"] and st["gcups"] > 0


def test_request_alone_equals_in_mix(served):
    """Served alone (its own batch) a request gives exactly its in-mix results."""
    import paper_1402_4876_amd as mica
    b, ref_words, reads_words, reqs, res, _ = served
    srv = mica.Server(ref_words, len(b.ref), slots=1, hbm_budget_bytes=2 << 30, fifo=True)
    try:
        for r in (0, 7, len(reqs) - 1):
            _submit(srv, b, reads_words, 5000 + r, reqs[r])
            alone = _wait(srv, [5000 + r])[5000 + r]
            U.assert_equal_outputs(alone, res[100 + r], "request %d alone vs in mix" % r)
    finally:
        srv.close()


def test_fifo_baseline_and_errors(served):
    import paper_1402_4876_amd as mica
    b, ref_words, reads_words, reqs, res, _ = served
    srv = mica.Server(ref_words, len(b.ref), slots=1, hbm_budget_bytes=2 << 30, fifo=True)
    try:
        for r in range(5):
            _submit(srv, b, reads_words, r, reqs[r])
        with pytest.raises(mica.MicaError):
            _submit(srv, b, reads_words, 0, reqs[0])  # id still in use
        got = _wait(srv, list(range(5)))
        for r in range(5):
            U.assert_equal_outputs(got[r], res[100 + r], "fifo request %d" % r)
        st = srv.stats()
        assert st["p99_s"] >= st["p50_s"] > 0
        with pytest.raises(mica.MicaError):
            srv.fetch(0)  # already fetched
        big = np.arange(70000) % b.n_pairs
        with pytest.raises(mica.MicaError):
            _submit(srv, b, reads_words, 99, big)  # over one serving batch
        # an empty request finishes too
        srv.submit(77, reads_words, np.zeros(0, np.uint64), np.zeros(0, np.int32), np.zeros(0, np.uint64),
                   np.zeros(0, np.int32))
        assert _wait(srv, [77])[77]["score"].shape == (0,)
    finally:
        srv.close()


def test_replayed_schedule_equals_oracle(served):
    """Requests submitted by the library's replay thread at scheduled times
    (ranges of one read pool) are served exactly; the replay keeps up."""
    import paper_1402_4876_amd as mica
    b, ref_words, reads_words, _, _, _ = served
    first, count = synth.request_schedule(b.n_pairs, 30, 7, max_reads=300)
    srv = mica.Server(ref_words, len(b.ref), slots=3, hbm_budget_bytes=4 << 30)
    try:
        t0 = srv.now() + 0.01
        arrival = t0 + np.arange(30) * 0.002
        srv.replay(reads_words, b.read_off.astype(np.uint64), b.read_len, b.win_off.astype(np.uint64), b.win_len,
                   first, count, arrival, first_id=900, mode=b.mode.astype(np.uint8))
        got = _wait(srv, list(range(900, 930)))
        lag = srv.replay_wait()
        assert 0 <= lag < 0.5
        st = srv.stats()
        assert st["p99_s"] >= st["p50_s"] > 0
    finally:
        srv.close()
    for r in range(30):
        idx = np.arange(first[r], first[r] + count[r])
        U.assert_same(got[900 + r], U.run_oracle(b, SC, idx=idx), what="replayed request %d" % r)


def test_tight_hbm_budget_serves_long_windows():
    """With a budget that leaves the slots little room beyond their staging,
    batches of long windows still run (with fewer resident waves) and are
    exact; a budget below the fixed needs is refused."""
    import paper_1402_4876_amd as mica
    b = synth.tiny_random(600, 200, 3000, 17)
    ref_words = pack_codes(b.ref)
    reads_words = pack_codes(b.reads)
    fixed = 3 * (26 << 20) + len(ref_words) * 4  # the slots' staging (25.3 MiB each) and the reference
    with pytest.raises(mica.MicaError):  # less than 64 MiB of workspace per slot
        mica.Server(ref_words, len(b.ref), slots=3, hbm_budget_bytes=fixed + (100 << 20))
    srv = mica.Server(ref_words, len(b.ref), slots=3, hbm_budget_bytes=fixed + 3 * (80 << 20))
    try:
        reqs = _requests(b, [100] * 6)
        for rid, idx in enumerate(reqs):
            _submit(srv, b, reads_words, rid, idx)
        got = _wait(srv, list(range(len(reqs))))
    finally:
        srv.close()
    g = _concat(got, list(range(len(reqs))))
    U.assert_same(g, U.run_oracle(b, SC, idx=np.concatenate(reqs)), what="tight budget")


def test_plan_loaded_into_the_slots(served, tmp_path):
    """A kernel plan given to the server (loaded while requests are queued and
    running, which it waits for) changes which kernels run but not the
    results; a file the contexts refuse is an error."""
    import paper_1402_4876_amd as mica
    b, ref_words, reads_words, reqs, res, _ = served
    ctx = mica.Context()
    try:
        ctx.set_plan(1, 256, 64, 4)  # every read of the mix in the 64-lane, 4-row class
        plan = tmp_path / "plan.json"
        ctx.save_plan(str(plan))
    finally:
        ctx.close()
    bad = tmp_path / "bad.json"
    bad.write_text("{not a plan")
    srv = mica.Server(ref_words, len(b.ref), slots=3, hbm_budget_bytes=4 << 30)
    try:
        for r in range(10):
            _submit(srv, b, reads_words, 700 + r, reqs[r])
        srv.load_plan(str(plan))
        for r in range(10, 20):
            _submit(srv, b, reads_words, 700 + r, reqs[r])
        got = _wait(srv, [700 + r for r in range(20)])
        with pytest.raises(mica.MicaError):
            srv.load_plan(str(bad))
        with pytest.raises(mica.MicaError):
            srv.load_plan(str(tmp_path / "missing.json"))
    finally:
        srv.close()
    for r in range(20):
        U.assert_equal_outputs(got[700 + r], res[100 + r], "request %d under the loaded plan" % r)
