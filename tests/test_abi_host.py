"""Host-side checks of the C ABI library (no GPU compute calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(mica_\w+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    from paper_1402_4876_amd import _lib
    lib = _lib.load()
    names = declared_functions()
    assert "mica_dp_align_batch" in names and len(names) >= 8
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTS)


def test_struct_layout_matches_header(tmp_path):
    """ctypes mirrors of the C structs: same size and field offsets as gcc gives."""
    import subprocess
    from paper_1402_4876_amd import _lib
    structs = {"mica_batch_t": _lib.Batch, "mica_scoring_t": _lib.Scoring, "mica_batch_stats_t": _lib.BatchStats,
               "mica_tune_entry_t": _lib.TuneEntry, "mica_fm_batch_t": _lib.FmBatch,
               "mica_pipe_params_t": _lib.PipeParams, "mica_pipe_stats_t": _lib.PipeStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mica_dp.h"', '#include "mica_fm.h"',
             '#include "mica_pipe.h"',
             'int main(void) {']
    for cname, cls in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got["%s.%s" % (cname, f)]) == getattr(cls, f).offset, (cname, f)


def test_invalid_arguments_fail_before_any_device_call():
    from paper_1402_4876_amd import _lib
    lib = _lib.load()
    b = _lib.Batch()
    s = _lib.Scoring(1, -4, 6, 1)
    assert lib.mica_dp_align_batch(None, ctypes.byref(b), ctypes.byref(s), 0, None) == -1
    assert b"NULL" in lib.mica_last_error()
    assert lib.mica_pack_2bit(None, -1, None, None) == -1
    assert lib.mica_pack_2bit(None, 10, None, None) == -1
    assert lib.mica_ctx_set_plan(None, 1, 10, 16, 1) == -1
    n_out = ctypes.c_int32(7)
    assert lib.mica_ctx_autotune(None, ctypes.byref(b), ctypes.byref(s), 0, None, 1, None, 0,
                                 ctypes.byref(n_out)) == -1
    assert lib.mica_ctx_save_plan(None, b"/nonexistent/plan.json") == -1
    hs = ctypes.c_void_p()
    assert lib.mica_server_create(0, None, 0, 0, 0, ctypes.byref(s), 0, ctypes.byref(hs)) == -1  # 0 slots
    assert lib.mica_server_create(0, None, 0, 0, 1, ctypes.byref(s), 1 << 20, ctypes.byref(hs)) == -1  # flag
    assert not hs.value
    k = ctypes.c_int64()
    assert lib.mica_server_submit(None, 1, None, None, None, None, None, None, 0, 0.0) == -1
    assert lib.mica_server_poll(None, None, 0, ctypes.byref(k)) == -1
    assert lib.mica_server_fetch(None, 1, None, None, None, None, None, None, 0, None, None) == -1
    assert lib.mica_server_stats(None, None, None, None) == -1
    assert lib.mica_server_destroy(None) == 0
    assert lib.mica_ctx_load_plan(None, b"/nonexistent/plan.json") == -1
    assert lib.mica_ctx_destroy(None) == 0
    h = ctypes.c_void_p()
    rc = lib.mica_ctx_create(-1, 0, ctypes.byref(h))
    assert rc in (-1, -4) and not h.value


def test_pack_layout():
    from paper_1402_4876_amd.pack import pack_codes, unpack_words
    codes = np.random.default_rng(0).integers(0, 4, 1000, dtype=np.uint8)
    w = pack_codes(codes)
    assert w.dtype == np.uint32 and len(w) == 63
    # base k sits at bits 2*(k % 16) of word k // 16
    for k in (0, 1, 15, 16, 17, 999):
        assert (int(w[k // 16]) >> (2 * (k % 16))) & 3 == codes[k]
    assert (int(w[-1]) >> (2 * (1000 % 16))) == 0  # unused high bits are zero
    assert np.array_equal(unpack_words(w, 1000), codes)


def test_binding_refuses_missing_library(tmp_path, monkeypatch):
    from paper_1402_4876_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _lib.load()


def test_suffix_array_matches_sorting():
    """The library's SA-IS against plain sorting of all suffixes (host only)."""
    import paper_1402_4876_amd as mica
    rng = np.random.default_rng(7)
    cases = [np.zeros(0, np.uint8), np.zeros(1, np.uint8), np.zeros(50, np.uint8), np.full(33, 3, np.uint8),
             np.tile(np.array([0, 1], np.uint8), 40), np.tile(np.array([2, 2, 1], np.uint8), 30),
             np.tile(rng.integers(0, 4, 7, dtype=np.uint8), 20)]
    cases += [rng.integers(0, 4, int(n), dtype=np.uint8) for n in rng.integers(2, 600, 40)]
    cases += [rng.integers(0, 2, 300, dtype=np.uint8), rng.integers(0, 4, 5000, dtype=np.uint8)]
    for t in cases:
        s = bytes((t + 1).tolist()) + b"\x00"
        want = sorted(range(len(s)), key=lambda i: s[i:])
        assert mica.suffix_array(t).tolist() == want, len(t)


def test_fm_entry_points_reject_bad_arguments():
    from paper_1402_4876_amd import _lib
    lib = _lib.load()
    sa = np.zeros(4, np.uint32)
    bad = np.array([0, 4, 1], np.uint8)
    assert lib.mica_fm_suffix_array(bad.ctypes.data, 3, sa.ctypes.data) == -1
    assert lib.mica_fm_suffix_array(None, 3, sa.ctypes.data) == -1
    h = ctypes.c_void_p()
    assert lib.mica_fm_create(0, None, 10, ctypes.byref(h)) == -1 and not h.value
    b = _lib.FmBatch()
    assert lib.mica_fm_search(None, ctypes.byref(b), None) == -1
    assert lib.mica_fm_info(None, None, None) == -1
    assert lib.mica_fm_destroy(None) == 0
    prm = _lib.PipeParams()
    assert lib.mica_pipe_create(0, None, 10, b"ref", ctypes.byref(prm), ctypes.byref(h)) == -1 and not h.value
    words = np.zeros(4, np.uint32)
    assert lib.mica_pipe_create(0, words.ctypes.data, 10, b"ref", ctypes.byref(prm), ctypes.byref(h)) == -1
    assert b"out of range" in lib.mica_last_error()
    assert lib.mica_pipe_run(None, b"a.fq", b"b.sam", None) == -1
    assert lib.mica_pipe_destroy(None) == 0


def test_noalloc_rejects_too_many_pairs_before_any_device_call():
    """The allocation-free call refuses batches beyond its fixed workspace on
    the host (MICA_ERR_LIMIT), and validates like the batch call."""
    from paper_1402_4876_amd import _lib
    lib = _lib.load()
    s = _lib.Scoring(1, -4, 6, 1)
    b = _lib.Batch()
    assert lib.mica_dp_align_batch_noalloc(ctypes.byref(b), None, 0, None) == -1
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the call fails first
    for f in ("ref2b", "win_off", "win_len", "reads2b", "read_off", "read_len", "score", "read_end", "ref_end",
              "status"):
        setattr(b, f, fake)
    b.n_pairs = _lib.NOALLOC_MAX_PAIRS + 1
    b.max_read_len, b.max_win_len = 150, 400
    assert lib.mica_dp_align_batch_noalloc(ctypes.byref(b), ctypes.byref(s), 0, None) == -2
    assert b"4,194,304" in lib.mica_last_error()
    assert lib.mica_dp_align_batch_noalloc(ctypes.byref(b), ctypes.byref(s), 1 << 20, None) == -1  # flag
    b.n_pairs = 10
    for bad in (-1, (1 << 20) + 1):
        b.max_ext_h0 = bad
        assert lib.mica_dp_align_batch_noalloc(ctypes.byref(b), ctypes.byref(s), 0, None) == -1
        assert b"max_ext_h0" in lib.mica_last_error()
