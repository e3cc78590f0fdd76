"""Build libmica_dp.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1402_4876_amd.build   (or call build()).
Every source under csrc/ is compiled to an object in parallel, then linked.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.environ.get("MICA_LIB_OUT", os.path.join(HERE, "libmica_dp.so"))
BUILD = os.environ.get("MICA_BUILD_DIR", BUILD)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("MICA_ARCH", "gfx950")
FLAGS = [
    "-O3", "--offload-arch=" + ARCH, "-fPIC", "-std=c++17",
    # no packed fp32 instructions (this code has no fp32 math anyway)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE, "-I" + CSRC,
] + os.environ.get("MICA_EXTRA_FLAGS", "").split()
SOURCES = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, err))
    return obj


def build(verbose: bool = True) -> str:
    """Compile every HIP source for gfx950 and link the shared library."""
    os.makedirs(BUILD, exist_ok=True)
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))) as ex:
        # longest first: the persistent kernels and the traceback fills
        order = sorted(SOURCES, key=lambda f: (not f.startswith("persistent"), not f.endswith("_1.hip")))
        objs = list(ex.map(_compile, order))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built %s in %.1fs" % (LIB, time.time() - t0), file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()


def resource_report(sources=None):
    """Per-kernel VGPRs, spills and occupancy from the compiler (gfx950).

    Returns a list of (kernel, vgprs, vgpr_spills, scratch_bytes_per_lane,
    waves_per_simd).  Kernels compiled for one wave more than their
    spill-free budget (see fill_waves and persist_waves) spill in their
    set-up and walk; the step loops of the plain fill kernels do not spill,
    those of a few of the persistent kernels' longest classes reload a value
    or three per step.
    """
    import re
    rows = []
    for src in sources or [f for f in SOURCES if f.startswith(("fill_", "persistent_", "side_"))]:
        cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", os.devnull,
                                 "-Rpass-analysis=kernel-resource-usage"]
        out = subprocess.run(cmd, capture_output=True, text=True).stderr
        for blk in out.split("Function Name: ")[1:]:
            name = blk.split()[0]
            get = lambda k: int((re.search(k + r": (\d+)", blk) or [0, -1])[1])  # noqa: E731
            rows.append((name, get("VGPRs"), get("VGPRs Spill"), get(r"ScratchSize \[bytes/lane\]"),
                         get(r"Occupancy \[waves/SIMD\]")))
    return rows
