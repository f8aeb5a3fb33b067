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
