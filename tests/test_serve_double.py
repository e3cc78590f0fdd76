"""CPU checks of the serving logic and the host C/C++ code under sanitizers.

- The serving core (queue, continuous batching, slot threads, hand-back,
  replay, statistics: paper_1402_4876_amd/csrc/serve_core.h) driven by the
  host test double tests/serve_double.cpp, whose slots compute with the CPU
  oracle after injected delays; built with AddressSanitizer +
  UndefinedBehaviorSanitizer, and again with ThreadSanitizer.
- The CPU oracle itself (oracle/gotoh.c, oracle/kmm.c) built with
  AddressSanitizer + UndefinedBehaviorSanitizer and run on hand examples,
  edge cases and random batches by a small driver.
- The few-mismatch search's base comparisons
  (paper_1402_4876_amd/csrc/fm_match.h, the device helpers of the search
  kernel) built as host code with AddressSanitizer +
  UndefinedBehaviorSanitizer and compared with base-by-base counts.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "_build", "sanitized")
CSRC = os.path.join(ROOT, "paper_1402_4876_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
ORACLE = os.path.join(ROOT, "oracle")

ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
TSAN = ["-fsanitize=" + "thread"]


def _build(name, cxx_srcs, c_srcs, flags):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in c_srcs:
        obj = os.path.join(BUILD, "%s_%s.o" % (name, os.path.basename(src)))
        subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-pthread", "-c", src, "-o", obj] + flags)
        objs.append(obj)
    exe = os.path.join(BUILD, name)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-pthread", "-I", INCLUDE, "-I", CSRC] + cxx_srcs +
                          objs + flags + ["-o", exe])
    return exe


def _run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, "%s failed (%d):\n%s\n%s" % (os.path.basename(exe), r.returncode, r.stdout[-3000:],
                                                           r.stderr[-6000:])
    return r.stdout


def test_serving_core_test_double_asan_ubsan():
    exe = _build("serve_double_asan", [os.path.join(ROOT, "tests", "serve_double.cpp")],
                 [os.path.join(ORACLE, "gotoh.c")], ASAN)
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1", "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert "all checks passed" in out


def test_serving_core_test_double_tsan():
    exe = _build("serve_double_tsan", [os.path.join(ROOT, "tests", "serve_double.cpp")],
                 [os.path.join(ORACLE, "gotoh.c")], TSAN)
    out = _run(exe, {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"})
    assert "all checks passed" in out


def test_oracle_under_asan_ubsan():
    exe = _build("oracle_asan", [os.path.join(ROOT, "tests", "oracle_sanitize.cpp")],
                 [os.path.join(ORACLE, "gotoh.c"), os.path.join(ORACLE, "kmm.c")], ASAN)
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1"})
    assert "oracle under sanitizers: ok" in out


def test_search_base_comparisons_under_asan_ubsan():
    exe = _build("fm_match_asan", [os.path.join(ROOT, "tests", "fm_match_check.cpp")], [], ASAN)
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1", "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert "stretches ok" in out
