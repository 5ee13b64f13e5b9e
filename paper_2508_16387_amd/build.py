"""Build the gfx950 HIP library ``libm2c.so`` in-tree.

Every ``csrc/*.hip`` file is compiled to an object with hipcc for gfx950 and
the objects are linked into one shared library next to this file.  Packed
FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libm2c.so")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", CSRC, "-I", INCLUDE,
]


# Per-source additions.  The stiffened-gas and option stage kernels are
# scheduled for instruction-level parallelism: at their two (FP64) or three
# (mixed) waves per SIMD the extra registers cost no occupancy, and the
# 384^3 stage launch measured 2.68 -> 2.64 ms.  The general-EOS kernels keep
# the default scheduler: with it some dropped to one wave per SIMD, and held
# to two waves they measured slower (128^3 charge 230 -> 241 us).
EXTRA_FLAGS = {
    "k_stage.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
    "k_stage_opts.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
}


def flags_for(src: str):
    """Compiler flags of one source file."""
    return [*FLAGS, *EXTRA_FLAGS.get(os.path.basename(src), [])]


def hipcc() -> str:
    return os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str, build_dir: str = BUILD, defines=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src)[:-4] + ".o")
    cmd = [hipcc(), *flags_for(src), *[f"-D{d}" for d in defines], "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    if r.stderr.strip():
        # keep compiler warnings visible, minus the host-pass note about the
        # device-only target feature
        lines = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l]
        if any(l.strip() for l in lines):
            sys.stderr.write("\n".join(lines) + "\n")
    return obj


def build(jobs: int = 8, out: str = LIB, defines=()) -> str:
    """Compile and link; ``out`` and ``defines`` give variant builds
    (compile-time tuning knobs such as M2C_STAGE_WAVES)."""
    build_dir = BUILD if out == LIB else out + ".objs"
    os.makedirs(build_dir, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir, defines), srcs))
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
