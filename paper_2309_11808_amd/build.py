"""Build libspod.so for gfx950 with hipcc, in place (next to this file).

    python -m paper_2309_11808_amd.build [--jobs N] [--verbose]

Every library source under csrc/ is compiled to an object under _build/ at
the repository root and linked into paper_2309_11808_amd/libspod.so; the
plain C caller csrc/spod_bench.cpp becomes paper_2309_11808_amd/spod_bench.
The build always recompiles (it is the "does it build" check as well as the
build).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libspod.so")
ARCH = "gfx950"

SOURCES = ["api.cpp", "batch.cpp", "ooc.cpp", "fft.hip", "gram.hip", "eig.hip", "modes.hip",
           "backward.hip", "coeffs.hip", "fft_general.hip"]

# Packed FP32 instructions are kept out of all device code (the compiler would
# otherwise form v_pk_* FP32 ops from ordinary float code).
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Wall", "-Wno-unused-function", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libspod)")


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, src + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [_hipcc()] + lang + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (r.stderr or "").splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{err}")
    if err.strip() and verbose:
        print(err, file=sys.stderr)
    return obj


def build(jobs: int = 0, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libspod.so failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    # spod_bench: a plain C-ABI caller of the library (hardware-counter runs)
    drv = os.path.join(PKG, "spod_bench")
    cmd = [_hipcc(), "-x", "hip"] + [c for c in COMMON if c != "-fPIC"] + [
        os.path.join(CSRC, "spod_bench.cpp"), "-L", PKG, "-lspod", "-Wl,-rpath,$ORIGIN",
        "-o", drv + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"building spod_bench failed:\n{r.stderr}")
    os.replace(drv + ".tmp", drv)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=0)
    ap.add_argument("--verbose", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.verbose))


if __name__ == "__main__":
    main()
