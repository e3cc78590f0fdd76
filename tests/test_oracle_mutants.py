"""The oracle's pins must catch plausible mistakes.

Each case copies gotoh.c, plants one mistake (a dropped term, a wrong sign,
a transposed operand, a flipped comparison or tie-break), compiles the copy
with gcc and checks that the brute-force / hand-example pins reject it.
Mistakes are planted on the CPU only, in a temporary copy of the oracle.
"""
import ctypes
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

import brute
import oracle
import test_oracle_pins as P

SRC = os.path.join(os.path.dirname(oracle.__file__), "gotoh.c")
HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

MUTANTS = {
    "dropped_extend_on_D": ("AT(D, i, j - 1) - e,", "AT(D, i, j - 1),"),
    "dropped_open_on_I": ("AT(H, i - 1, j) - o - e);", "AT(H, i - 1, j) - e);"),
    "I_uses_left_not_up": ("AT(I, i - 1, j) - e", "AT(I, i, j - 1) - e"),
    "diag_uses_up": ("AT(H, i - 1, j - 1) + s, imax", "AT(H, i - 1, j) + s, imax"),
    "sg_column0_positive": ("AT(H, i, 0) = local ? 0 : -(o + i * e);", "AT(H, i, 0) = local ? 0 : (o + i * e);"),
    "no_local_floor": ("if (local) h = imax(h, 0);", ""),
    "sg_end_tie_largest_j": ("if (AT(H, m, j) > best) {", "if (AT(H, m, j) >= best) {"),
    "local_tie_largest_i": ("        if (AT(H, i, j) > best) {", "        if (AT(H, i, j) >= best) {"),
    "trace_D_before_diag": (
        "if (AT(H, i, j) == AT(H, i - 1, j - 1) + s) {",
        "if (AT(H, i, j) == AT(D, i, j)) { st = ST_D; } else if (AT(H, i, j) == AT(H, i - 1, j - 1) + s) {"),
    "trace_extend_before_open": (
        "if (AT(D, i, j) == AT(H, i, j - 1) - o - e) st = ST_H;",
        "if (AT(D, i, j) != AT(D, i, j - 1) - e) st = ST_H;"),
    "trace_I_extend_before_open": (
        "if (AT(I, i, j) == AT(H, i - 1, j) - o - e) st = ST_H;",
        "if (AT(I, i, j) != AT(I, i - 1, j) - e) st = ST_H;"),
    "trace_no_local_zero_stop": ("if (local && AT(H, i, j) == 0) break;", "if (local && i == 0) break;"),
    "cigar_I_D_swapped": ("enum { OP_M = 0, OP_I = 1, OP_D = 2 };", "enum { OP_M = 0, OP_I = 2, OP_D = 1 };"),
    "ext_clip_strict": ("if ((int64_t)gbest >= (int64_t)best - J->clip) {",
                        "if ((int64_t)gbest > (int64_t)best - J->clip) {"),
    "ext_row0_gap_without_open": ("AT(H, 0, j) = ext ? (j == 0 ? h0 : h0 - (o + j * e)) : 0;",
                                  "AT(H, 0, j) = ext ? (j == 0 ? h0 : h0 - j * e) : 0;"),
    "ext_early_end_ignores_anchor": ("best = ext ? h0 : 0;", "best = 0;"),
    "ext_col0_without_start_score": ("AT(H, i, 0) = local ? 0 : (ext ? h0 : 0) - (o + i * e);",
                                     "AT(H, i, 0) = local ? 0 : -(o + i * e);"),
    "ext_trace_row0_no_deletions": ("for (; j > 0; j--) ops[nops++] = OP_D;", "j = 0;"),
}


def build_mutant(name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, name
    # built inside the repository's (git-ignored) build folder, removed again
    # once loaded
    base = os.path.join(ROOT, "_build")
    os.makedirs(base, exist_ok=True)
    with tempfile.TemporaryDirectory(prefix="oracle_mut_", dir=base) as d:
        c = os.path.join(d, "m.c")
        so = os.path.join(d, "m.so")
        open(c, "w").write(text.replace(old, new))
        subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-pthread", c, "-o", so])
        return ctypes.CDLL(so)


def _bind(lib):
    return oracle.bind(lib)


def _brute_small():
    rng = np.random.default_rng(5)
    for sc in ((1, -4, 6, 1), (3, 0, 2, 1)):
        for mode in (0, 1):
            pairs = [(rng.integers(0, 4, int(rng.integers(0, 6)), dtype=np.uint8),
                      rng.integers(0, 4, int(rng.integers(0, 6)), dtype=np.uint8)) for _ in range(150)]
            got = oracle.align_pairs(pairs, mode=mode, scoring=sc, threads=1)
            for p, (q, r) in enumerate(pairs):
                score, (ei, ej), (si, sj), cig = brute.canonical(q, r, mode, sc)
                assert (got["score"][p], got["read_end"][p], got["ref_end"][p], got["read_start"][p],
                        got["ref_start"][p]) == (score, ei, ej, si, sj)
                assert oracle.decode_cigar(got["cigar"][p], got["n_cigar"][p]) == "".join(cig)


def _brute_ext_small():
    import test_oracle_extension as X
    rng = np.random.default_rng(7)
    for sc in ((1, -4, 6, 1), (3, 0, 2, 1)):
        pairs = [(tuple(rng.integers(0, 4, int(rng.integers(0, 5)))), tuple(rng.integers(0, 4, int(rng.integers(0, 5)))))
                 for _ in range(120)]
        for h0, clip in ((0, 0), (6, 2), (9, 50)):
            X._check(pairs, sc, h0, clip)
    X.test_extension_closed_forms()


PINS = [lambda: [P.test_hand_example(row) for row in P.HAND],
        lambda: [P.test_gap_open_extend_tie_case(row) for row in P.TIES],
        P.test_closed_forms,
        P.test_cigar_rescores_to_score_and_spans_coordinates,
        _brute_small,
        _brute_ext_small]


def pins_pass(lib):
    """Run the committed pins with ``lib`` in place of the oracle library."""
    saved = oracle._lib
    oracle._lib = _bind(lib)
    try:
        for pin in PINS:
            try:
                pin()
            except AssertionError:
                return False
        return True
    finally:
        oracle._lib = saved


def test_unmutated_oracle_passes_compact_pins():
    assert pins_pass(oracle._load())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    # A planted mistake may also make the traceback walk out of its matrices and
    # crash; each mutant therefore runs in a child process, and a crash counts
    # as caught.  Exit code 0 means every pin passed (mutant missed).
    code = ("import sys; sys.path[:0] = %r; import test_oracle_mutants as T; "
            "sys.exit(0 if T.pins_pass(T.build_mutant(%r)) else 3)" % ([HERE, ROOT], name))
    rc = subprocess.run([sys.executable, "-c", code], timeout=300,
                        stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL).returncode
    assert rc != 0, name
