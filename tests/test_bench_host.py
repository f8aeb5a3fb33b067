"""Host-side checks of the benchmark's bookkeeping (no GPU)."""
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_late_factor_slots_match_the_launch_tables():
    # the benchmark names the dominant kernel as the profile summaries do, which needs the late-factor
    # batch of each launch variant; it must agree with the table the kernels are instantiated from
    import bench
    src = open(os.path.join(ROOT, "paper_2109_05072_amd", "csrc", "mfhex_internal.h")).read()
    for name, mirror in (("kVarLate", bench.LATE_FACTOR_SLOTS), ("kVarPre", bench.PREFETCH_SLOTS)):
        body = re.search(name + r"\[9\]\[5\]\s*=\s*\{(.*?)\};", src, re.S).group(1)
        rows = [[int(v) for v in r.split(",")] for r in re.findall(r"\{([^{}]*)\}", body)]
        assert len(rows) == 9 and all(len(r) == 5 for r in rows)
        table = {(i + 2, v): n for i, r in enumerate(rows) for v, n in enumerate(r) if n}
        assert table == mirror, name


def test_measuring_library_exports():
    # the benchmark's measuring kernels (HBM streaming, FP64 pipe rates) load and export their entry points
    import ctypes
    from paper_2109_05072_amd import build as libbuild
    if not os.path.exists(libbuild.PROBE_LIB):
        import pytest
        pytest.skip("libhbmprobe.so not built")
    lib = ctypes.CDLL(libbuild.PROBE_LIB)
    for name in ("hbm_stream", "fp64_rate", "fp64_rate_flops_per_wave_iter"):
        assert hasattr(lib, name), name
    f = lib.fp64_rate_flops_per_wave_iter
    f.argtypes, f.restype = [ctypes.c_int], ctypes.c_double
    assert [f(k) for k in range(3)] == [4 * 2 * 16 * 16 * 4, 4 * 2 * 4 * 4 * 4 * 4, 8 * 2 * 64]
