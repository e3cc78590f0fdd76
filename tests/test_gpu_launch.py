"""GPU tests of the launch layer: HIP-graph launches, every kernel plan (lanes x
rows per lane), and the autotuner with its bit-exactness gate and plan file.

Plans and launch styles change only how the DP runs, so every variant must
reproduce the oracle exactly (integer outputs, element by element).
"""
import json

import numpy as np
import pytest

import synth
import gpu_util as U

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


def _run(ctx, dev, batch, graph=True, plain=False, out=None):
    import torch

    import paper_1402_4876_amd as mica
    o = mica.align(ctx, dev["ref2b"], dev["win_off"], dev["win_len"], dev["reads2b"], dev["read_off"],
                   dev["read_len"], mode=dev["mode"], scoring=SC, out_cigar=True, cigar_cap=64, graph=graph,
                   plain=plain, ref_len=dev["ref_len"], reads_len=dev["reads_len"],
                   max_read_len=int(batch.read_len.max()), max_win_len=int(batch.win_len.max()), out=out)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def test_graph_replays_match_eager(ctx):
    """One instantiated graph launched again and again (with the program's own GPU
    work and synchronisations in between) gives the eager result every time."""
    import torch

    import paper_1402_4876_amd as mica
    b = synth.config3(n_pairs=3000, ref_len=1_000_000)
    dev = mica.to_device(b)
    eager = _run(ctx, dev, b, graph=False)
    U.assert_same(eager, U.run_oracle(b, SC), what="eager")
    x = torch.randn(512, 512, device="cuda")
    n = b.n_pairs
    for rep in range(4):
        # outputs start from garbage so a replay that writes nothing cannot pass
        out = {k: torch.full((n,), -7, dtype=torch.int32, device="cuda")
               for k in ("score", "read_end", "ref_end", "status", "read_start", "ref_start", "n_cigar")}
        out["cigar"] = torch.full((n, 64), -7, dtype=torch.int32, device="cuda")
        g = _run(ctx, dev, b, graph=True, out=out)
        U.assert_equal_outputs(eager, g, "graph replay %d" % rep)
        y = (x @ x).sum().item()  # eager work of the program between replays
        assert np.isfinite(y)
    # timing events inside the graph, and the plain launch sequence as a graph
    ctx.set_timing(True)
    g = _run(ctx, dev, b, graph=True)
    ms, nb = ctx.read_timing()
    ctx.set_timing(False)
    assert nb == 1 and ms > 0
    U.assert_equal_outputs(eager, g, "graph with timing")
    U.assert_equal_outputs(eager, _run(ctx, dev, b, graph=True, plain=True), "plain graph")


def test_graph_grid_update_between_sizes(ctx):
    """The same launch sequence with a different number of pairs (grid sizes are
    updated on the instantiated graph): each size equals the oracle."""
    import paper_1402_4876_amd as mica
    for n in (2000, 37, 900):
        b = synth.config1(n_pairs=n, ref_len=500_000)
        g = _run(ctx, mica.to_device(b), b, graph=True)
        U.assert_same(g, U.run_oracle(b, SC), what="n=%d" % n)


def _length_batch(m_lo, m_hi, n_pairs, seed):
    """Pairs with read lengths in [m_lo, m_hi], windows 1.5m+64, half local."""
    rng = np.random.default_rng(seed)
    pairs, modes = [], []
    for k in range(n_pairs):
        m = int(rng.integers(m_lo, m_hi + 1))
        n = int(1.5 * m) + 64
        r = rng.integers(0, 4, n, dtype=np.uint8)
        s = int(rng.integers(0, n - m + 1))
        q = r[s:s + m].copy()
        nmut = max(1, m // 40)
        q[rng.integers(0, m, nmut)] = rng.integers(0, 4, nmut)
        if k % 5 == 0:
            q = rng.integers(0, 4, m, dtype=np.uint8)
        pairs.append((q, r))
        modes.append(k % 2)
    rl = np.array([len(q) for q, _ in pairs], np.int32)
    wl = np.array([len(r) for _, r in pairs], np.int32)
    ref = np.concatenate([r for _, r in pairs] + [np.zeros(16, np.uint8)])
    win_off = np.concatenate([[0], np.cumsum(wl.astype(np.int64))[:-1]])
    codes = np.zeros((n_pairs, int(rl.max())), np.uint8)
    for k, (q, _) in enumerate(pairs):
        codes[k, :len(q)] = q
    return synth._finish("lengths", ref, win_off, wl, codes, rl, np.asarray(modes, np.uint8))


@pytest.mark.parametrize("m_lo,m_hi,plans", [
    (1, 16, [(16, 1), (16, 2), (64, 4), (64, 8), (64, 16)]),
    (97, 112, [(16, 7), (16, 8), (16, 16), (64, 4), (64, 8), (64, 16)]),
    (145, 160, [(16, 10), (16, 11), (64, 4), (64, 8)]),
    (241, 256, [(16, 16), (64, 4), (64, 8), (64, 16)]),
    (300, 380, [(64, 8), (64, 16)]),
])
def test_every_plan_matches_oracle(m_lo, m_hi, plans):
    """Each (lanes, rows) plan of a length range reproduces the oracle, through the
    persistent and the plain launch."""
    import paper_1402_4876_amd as mica
    b = _length_batch(m_lo, m_hi, 200, seed=m_lo)
    o = U.run_oracle(b, SC)
    dev = mica.to_device(b)
    for lanes, rows in plans:
        c = mica.Context(0)
        try:
            c.set_plan(m_lo, m_hi, lanes, rows)
            for plain in (False, True):
                U.assert_same(_run(c, dev, b, plain=plain), o, what="plan %dx%d plain=%s" % (lanes, rows, plain))
        finally:
            c.close()


def test_set_plan_rejects_bad_plans(ctx):
    import paper_1402_4876_amd as mica
    with pytest.raises(mica.MicaError):
        ctx.set_plan(1, 100, 16, 6)  # 96 rows cannot cover 100 bases
    with pytest.raises(mica.MicaError):
        ctx.set_plan(1, 10, 64, 5)   # no such plan
    with pytest.raises(mica.MicaError):
        ctx.set_plan(0, 10, 16, 1)


def test_autotune_gate_plan_file(tmp_path):
    """The autotuner picks, per 16-base range, a plan whose outputs equal the default
    plan's; results after tuning equal the oracle; the plan file round-trips and is
    refused on another device kind."""
    import paper_1402_4876_amd as mica
    b = synth.config3(n_pairs=6000, ref_len=1_000_000)
    dev = mica.to_device(b)
    c = mica.Context(0)
    try:
        ent = c.autotune(dev["ref2b"], dev["win_off"], dev["win_len"], dev["reads2b"], dev["read_off"],
                         dev["read_len"], mode=dev["mode"], out_cigar=True, ref_len=dev["ref_len"],
                         reads_len=dev["reads_len"], reps=2)
        assert len(ent) >= 10
        for e in ent:
            assert e["lanes"] * e["rows"] >= e["m_hi"]
            assert e["n_rejected"] == 0, e  # every candidate plan reproduces the default's outputs
            assert e["ms"] <= e["default_ms"] + 1e-9
            assert e["n_pairs"] >= 256 and e["n_candidates"] >= 2
        o = U.run_oracle(b, SC)
        U.assert_same(_run(c, dev, b), o, what="tuned")
        path = tmp_path / "plan.json"
        c.save_plan(path)
        plan = json.loads(path.read_text())
        assert plan["arch"].startswith("gfx") and plan["n_cu"] > 0
        c2 = mica.Context(0)
        try:
            c2.load_plan(path)
            c2.save_plan(tmp_path / "plan2.json")
            assert json.loads((tmp_path / "plan2.json").read_text()) == plan
            U.assert_same(_run(c2, dev, b), o, what="loaded plan")
            bad_plan = dict(plan, arch="gfx000")
            bad = tmp_path / "bad.json"
            bad.write_text(json.dumps(bad_plan))
            with pytest.raises(mica.MicaError):
                c2.load_plan(bad)
            c2.save_plan(tmp_path / "plan3.json")  # a refused file leaves the plan as it was
            assert json.loads((tmp_path / "plan3.json").read_text()) == plan
        finally:
            c2.close()
    finally:
        c.close()
