"""Builds libsnp.so (the HIP library behind include/snp.h) for gfx950.

    python -m paper_2510_08491_amd.build [--jobs N]

Each .hip source is compiled to an object with hipcc, in parallel, then linked
into paper_2510_08491_amd/libsnp.so.  The microbenchmark executable is built
beside it.  Compilation is always redone (the caller asked for a build).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsnp.so")
MICROBENCH = os.path.join(HERE, "snp_microbench")

SOURCES = ["api.hip", "preprocess.hip", "binning.hip", "raster.hip", "loss.hip", "sh.hip", "train.hip", "relight.hip"]
ARCH = "gfx950"
# packed FP32 instructions are disabled on purpose (the compiler would form
# them from ordinary float code)
COMMON = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-munsafe-fp-atomics",
          # atomics here are issued on already reduced values; the compiler's
          # atomic optimizer would wrap each one in a loop over the lanes
          "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
          # an occupancy request that the LDS of a large batch already rules out
          "-Wno-pass-failed", "-Wshadow"]
PER_FILE = {
    # float64 key path: one fixed operation order, no contraction
    "preprocess.hip": ["-ffp-contract=off"],
}


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # the host pass does not know the packed-fp32 target feature; drop that note
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    return r.returncode, out


def build(jobs: int = 8, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([cc, *COMMON, *PER_FILE.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        results = list(ex.map(_run, cmds))
    for (rc, out), cmd in zip(results, cmds):
        if verbose and out:
            print(out)
        if rc != 0:
            raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + out)
    tmp = LIB + ".tmp"
    rc, out = _run([cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp])
    if rc != 0:
        raise RuntimeError("link failed:\n" + out)
    os.replace(tmp, LIB)
    rc, out = _run([cc, *COMMON, os.path.join(CSRC, "microbench.hip"), "-o", MICROBENCH])
    if rc != 0:
        raise RuntimeError("microbench build failed:\n" + out)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.verbose))


if __name__ == "__main__":
    sys.exit(main())
