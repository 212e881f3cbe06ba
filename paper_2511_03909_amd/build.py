"""Build libwect.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc.

    python -m paper_2511_03909_amd.build [--asm DIR]

The library is written next to this file; the Python binding loads it from
there.  Every call recompiles.
"""
from __future__ import annotations

import argparse
import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libwect.so")
ARCH = "gfx950"

# kernel translation units are compiled in parallel, then linked with the host runtime
SOURCES = ["k_simp_fwd.hip", "k_cub_fwd.hip", "k_reduce.hip", "k_simp_bwd.hip", "k_smooth_bwd.hip",
           "k_lower_star.hip", "k_image.hip", "wect_static.hip", "k_calib.hip", "wect_api.cpp"]

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    # float32 heights: no contraction into fused multiply-add, denormals kept
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    # hardware float atomics for the adjoint's accumulation
    "-munsafe-fp-atomics",
    # never form packed float32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build(asm_dir: str | None = None, verbose: bool = False) -> str:
    cc = hipcc()
    tmp = os.path.join(PKG, "_build")
    os.makedirs(tmp, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(tmp, src + ".o")
        cmds.append([cc, f"--offload-arch={ARCH}", *COMMON, "-I", INCLUDE, "-I", CSRC, "-c",
                     os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(run, c) for c in cmds]:
            f.result()
    out_tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out_tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out_tmp, LIB)
    if asm_dir:
        os.makedirs(asm_dir, exist_ok=True)
        # device assembly of the kernels, for inspection
        for src in SOURCES:
            if not src.endswith(".hip"):
                continue
            cmd = [cc, f"--offload-arch={ARCH}", *COMMON, "-I", INCLUDE, "-I", CSRC, "--cuda-device-only", "-S",
                   os.path.join(CSRC, src), "-o", os.path.join(asm_dir, src[:-4] + ".s")]
            subprocess.run(cmd, check=True)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--asm", default=None, help="also write the device assembly into this folder")
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.asm, a.v))


if __name__ == "__main__":
    sys.exit(main())
