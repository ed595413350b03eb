"""Build the HIP libraries libspfc.so (SAV-BDF2 stepper) and libspfc_fno.so (FNO
surrogate) for gfx950, in-tree next to this file.

Usage: python -m paper_2012_15133_amd.build [--jobs N]
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libspfc.so")
FNO_SRC = os.path.join(HERE, "fno")
FNO_LIB = os.path.join(HERE, "libspfc_fno.so")
FNO_SOURCES = ["fno_kernels.hip", "fno.cpp"]
# roctx (ranges around the ABI calls) from the ROCm install
LINK = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
SOURCES = [f"kern_{p}_{k}.hip" for p in ("f64", "f32") for k in ("inv", "real", "fwd", "aux")] + [
    "finalize.hip", "solver.cpp"]

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("SPFC_OFFLOAD_ARCH", "gfx950")

# packed FP32 instructions are kept out of every kernel
FLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # hipcc's host pass does not know the packed-fp32 target feature; that warning is noise
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    return out


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile both libraries (all objects in one pool); returns the stepper's path."""
    os.makedirs(BUILD, exist_ok=True)
    objs, fobjs, cmds = [], [], []
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmds.append([HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
    for src in FNO_SOURCES:
        obj = os.path.join(BUILD, "fno_" + os.path.splitext(src)[0] + ".o")
        fobjs.append(obj)
        cmds.append([HIPCC, *FLAGS, "-I", FNO_SRC, "-c", os.path.join(FNO_SRC, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=jobs or min(len(cmds), os.cpu_count() or 1)) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out:
                print(out)
    for lib, ob in ((LIB, objs), (FNO_LIB, fobjs)):
        tmp = lib + ".tmp"
        _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *ob, *LINK])
        os.replace(tmp, lib)
    return LIB


def build_emulator() -> str:
    """Host-only run of the line-FFT schedule, used by the CPU tests."""
    src = os.path.join(ROOT, "tests", "native", "fft_emul.cpp")
    out = os.path.join(BUILD, "libfft_emul.so")
    os.makedirs(BUILD, exist_ok=True)
    _run([HIPCC, "-x", "hip", f"--offload-arch={ARCH}", "-O1", "-std=c++17", "-fPIC", "-shared",
          "-o", out, src])
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.verbose))
    print(FNO_LIB)
    sys.exit(0)
