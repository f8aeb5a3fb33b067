"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the CPU code (no GPU).

Two drivers under tests/sanitize/ are compiled with -fsanitize=address,undefined
(-fno-sanitize-recover: any report fails the run) and executed:
  oracle_main.c -- every entry point of the FP64 oracle on tiny perturbed
                   meshes, p = 1..4, both rules, mass and diffusion, with and
                   without Dirichlet rows, plus the 1D rules at every size;
  host_main.cpp -- the library's host set-up code: the 1D Gauss / Gauss-Lobatto
                   rules and B, D tables (basis.cpp) for p = 1..8, and the
                   tetrahedral rule and basis tables (tet.cpp) for p = 1..6.
Each driver also checks facts the mathematics fixes (volume, affine nullity,
symmetry, exactness, partition of unity), so a run that skipped work fails."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, OMP_NUM_THREADS="1", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, tmp_path, exe):
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=tmp_path)
    assert r.returncode == 0, f"build failed:\n{r.stderr[-4000:]}"
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, cwd=tmp_path, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, f"sanitized run failed ({r.returncode}):\n{r.stdout[-2000:]}\n{r.stderr[-6000:]}"
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fopenmp"] + SAN + [
        "-o", exe, os.path.join(HERE, "sanitize", "oracle_main.c"), "-lm"]
    assert "sanitize oracle: OK" in _run(cmd, tmp_path, exe)


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="g++ or the HIP headers not found")
def test_host_setup_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "host_san")
    csrc = os.path.join(ROOT, "paper_2109_05072_amd", "csrc")
    cmd = ["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", f"-I{ROOT}/include"] + SAN + [
        "-o", exe, os.path.join(HERE, "sanitize", "host_main.cpp"), os.path.join(csrc, "basis.cpp"),
        os.path.join(csrc, "tet.cpp")]
    assert "sanitize host: OK" in _run(cmd, tmp_path, exe)
