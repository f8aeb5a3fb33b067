"""Build libmfhex.so (HIP, gfx950) in-tree.

``python -m paper_2109_05072_amd.build`` compiles every ``csrc/*.hip`` and
``csrc/*.cpp`` with hipcc into ``paper_2109_05072_amd/libmfhex.so``.
Object files go to ``paper_2109_05072_amd/_build/`` (not committed).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmfhex.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-munsafe-fp-atomics",                                     # hardware FP64/FP32 atomic add
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",  # no packed FP32 VALU ops
    "-Wall", "-Wno-unused-result", f"-I{INCLUDE}",
]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = jobs or min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)), 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    build_probe(verbose)
    return LIB


PROBE_SRCS = [os.path.join(HERE, "probe", "hbm_stream.hip"), os.path.join(HERE, "probe", "fp64_rate.hip")]
PROBE_LIB = os.path.join(HERE, "libhbmprobe.so")


def build_probe(verbose: bool = False) -> str:
    """The measuring kernels the benchmark times next to the operator: HBM streaming (read / copy /
    fill) and FP64 pipe throughput (matrix-core and vector FMA chains)."""
    tmp = PROBE_LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-shared"] + PROBE_SRCS + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {PROBE_SRCS}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
