"""Build libpifcm.so (HIP kernels + host runtime + C ABI) for gfx950, in-tree.

    python paper_2002_01981_amd/build.py

Each translation unit is compiled in parallel into _build/, then linked into
paper_2002_01981_amd/libpifcm.so.  Every build compiles from scratch.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libpifcm.so")
ARCH = os.environ.get("PIFCM_ARCH", "gfx950")

# Packed fp32 instructions are disabled for all device code.
HIPFLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]

SOURCES = ["gather_c4.hip", "gather_c2_6.hip", "gather_c7_10.hip", "gather_c11_13.hip",
           "gather_c14_16.hip", "pointwise.hip", "ring.hip", "ring2.hip", "adjoint.hip", "scratch.hip", "pifcm_host.cpp"]


def _hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _compile(src: str, verbose: bool, build_dir: str, defines):
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [_hipcc(), *HIPFLAGS, *[f"-D{d}" for d in defines], *lang, "-c",
           os.path.join(CSRC, src), "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{msgs}")
    if verbose:
        print(f"  {src}: {time.time() - t0:.1f}s", flush=True)
        if msgs.strip():
            print(msgs, flush=True)
    return obj


def build(verbose: bool = False, jobs: int | None = None, out: str = LIB,
          build_dir: str = BUILD, defines=()) -> str:
    """Compile every source and link `out`.  `defines` are extra -D macros
    (kernel variants for experiments); `out`/`build_dir` place the result."""
    os.makedirs(build_dir, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1), 8)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, build_dir, defines), SOURCES))
    tmp = out + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=LIB)
    ap.add_argument("--build-dir", default=BUILD)
    ap.add_argument("-D", dest="defines", action="append", default=[])
    args = ap.parse_args()
    t = time.time()
    path = build(verbose=True, out=args.out, build_dir=args.build_dir, defines=args.defines)
    print(f"built {path} in {time.time() - t:.1f}s")
    sys.exit(0)
