"""Build libqtask.so in-tree: HIP kernels with hipcc for gfx950, host C++
with ROCm's clang, linked by hipcc.  ``python -m paper_2210_01076_amd.build``
or ``__graft_entry__.build()``."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libqtask.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")
ARCH = "gfx950"

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
             # packed FP32 instructions are kept out of the generated code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             # the op switch of the pass kernel branches on wave-uniform
             # values only: keeping it a plain switch (instead of a chain of
             # structured flow blocks) lets every case update the amplitude
             # registers in place
             "-mllvm", "-structurizecfg-skip-uniform-regions",
             # FP64 multiply-adds as three-address v_fma_f64: the two-address
             # v_fmac form ties the result to the addend's register, which
             # forces copies wherever an op updates an amplitude in place
             "-Xclang", "-target-feature", "-Xclang", "-fmacf64-inst",
             # the same for FP32: v_fmac_f32 comes with the dl-insts feature
             # (whose dot-product instructions the kernels do not use)
             "-Xclang", "-target-feature", "-Xclang", "-dl-insts",
             "-Wall", "-Wno-unused-function"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__=1",
             "-I" + os.path.join(ROCM, "include"), "-Wall", "-Wextra", "-Wno-unused-parameter"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), out))
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.join(OUT_DIR, "obj"), exist_ok=True)
    jobs = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        obj = os.path.join(OUT_DIR, "obj", os.path.basename(src) + ".o")
        jobs.append([HIPCC] + HIP_FLAGS + ["-c", src, "-o", obj])
    for src in sorted(glob.glob(os.path.join(CSRC, "*.cpp"))):
        obj = os.path.join(OUT_DIR, "obj", os.path.basename(src) + ".o")
        jobs.append([CLANG] + CXX_FLAGS + ["-c", src, "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for out in ex.map(_run, jobs):
            if verbose and out.strip():
                print(out)
    objs = [j[-1] for j in jobs]
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
