"""Build liblddmm.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1605_02060_amd.build   (or build() from Python)
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblddmm.so")

SOURCES = ["flow.hip", "fft.hip", "control.hip", "grad.hip", "runtime.hip", "cnn.hip", "hist.hip",
           "align.hip", "masks.hip"]
ARCH = "gfx950"


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def common_flags():
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-I", CSRC, "-I", INCLUDE,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument"]


# Sources whose kernels compute the same step in two implementations (the sweeps:
# grid-stride and LDS-staged; the FFT passes: single and batched launches of one
# line transform): multiply-add fusion only within one source expression, so
# both give the same bits.
CONTRACT_ON = {"flow.hip", "fft.hip"}
# Sources whose FP64 arithmetic restates a definition operation by operation
# (histogram quantiles and the intensity map; affine sampling positions, where
# a whole-number position must stay whole; the guard's energies E = R + D, whose
# rounding otherwise followed the compiler's fusion choice for the surrounding
# code): no multiply-add fusion at all.
CONTRACT_OFF = {"hist.hip", "align.hip", "control.hip"}


def flags_for(src):
    """Compiler flags of one source (include paths included)."""
    extra = (["-ffp-contract=on"] if src in CONTRACT_ON else
             ["-ffp-contract=off"] if src in CONTRACT_OFF else [])
    return [*common_flags(), *extra]


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *flags_for(src), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def build_host_asan(out_dir, driver, verbose=False) -> str:
    """Build an executable from `driver` (C++) and every source, with
    AddressSanitizer on the host code only (the device code is built as usual,
    so that the objects carry their kernels), to check the host runtime
    (argument validation, geometry, workspace layout) on the CPU.  The driver may
    only call paths that return before any device work.  Returns the
    executable's path."""
    os.makedirs(out_dir, exist_ok=True)
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer", "-I", CSRC, "-I",
             INCLUDE, "-Wno-unused-command-line-argument", "-Wno-unused-result",
             "-Xarch_host", "-fsanitize=address"]

    def host_obj(src):
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".asan.o")
        cmd = [hipcc(), f"--offload-arch={ARCH}", *flags, "-Xclang", "-target-feature",
               "-Xclang", "-packed-fp32-ops", "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed for {src}:\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(host_obj, SOURCES))
    exe = os.path.join(out_dir, "host_abi_checks")
    cmd = [hipcc(), f"--offload-arch={ARCH}", *flags, "-x", "c++", driver, "-x", "none", *objs,
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"host link failed:\n{r.stderr}")
    if verbose:
        print(f"built {exe}")
    return exe


if __name__ == "__main__":
    try:
        build()
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
