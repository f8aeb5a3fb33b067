"""Summaries of rocprofv3 output for the fused apply kernels.

``python -m paper_2109_05072_amd.prof_summary trace <dir> <command...>``
    kernel-trace statistics (``*_kernel_stats.csv``) -> text table
    (``trace-tet``, ``trace-probe``: the same, hashed over the tetrahedral kernel sources or the
    measuring kernels).
``python -m paper_2109_05072_amd.prof_summary traffic <fetch_dir> <write_dir> <command...>``
    FETCH_SIZE / WRITE_SIZE per dispatch of each apply kernel, scaled by what
    the same counters read for the 1 GiB device-to-device copy that
    ``bench.py --calib-copy`` runs (the copy reads and writes exactly 2^30
    bytes), -> HBM bytes per launch.  The kernel source hash is recorded so
    that a later reader can tell whether the numbers still describe the
    current kernels.

The benchmark reads the traffic summary back (``read_traffic``) and reports
it only while the source hash matches.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/apply_kernels.hpp", "csrc/mfhex_internal.h", "csrc/geom.hpp", "csrc/diag_kernels.hpp")
TET_SOURCES = ("csrc/tet_kernels.hip", "csrc/tet.h")
PROBE_SOURCES = ("probe/hbm_stream.hip", "probe/fp64_rate.hip")
COPY_BYTES = 1 << 30


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    m = re.match(r"void mfhex::k_apply<(\d+), (\d+), (\w+), (\d), (\w+), (\w+), (\d+), (\d+)(?:, (\d+))?"
                 r"(?:, (true|false))?(?:, (true|false))?(?:, (true|false))?(?:, (\d+))?(?:, (true|false))?"
                 r"(?:, (\d+))?>", name)
    if m:
        P, Q, colloc, mode, vark, T, G, NT, VC, otf, det, stage, late, mx, pre = m.groups()
        kind = {"0": "mass", "1": "diffusion", "2": "rhs"}[mode]
        vc = f" VC={VC}" if VC and VC != "1" else ""
        geo = " otf" if otf == "true" else ""
        dt = " det" if det == "true" else ""
        st = " staged" if stage == "true" else ""
        lt = f" late{late}" if late and late != "0" else ""
        lt += f" pre{pre}" if pre and pre != "0" else ""
        mc = " mfma" if mx == "true" else ""
        return (f"k_apply p={int(P) - 1} q={Q} {kind}{' kappa' if vark == 'true' else ''}{geo} {T} G={G} NT={NT}"
                f"{vc}{dt}{st}{lt}{mc}")
    m = re.match(r"void mfhex::k_apply_gf<(\d+), (\d+), (\w+), (\w+), (\d+), (\d+), (\w+)(?:, (true|false))?>", name)
    if m:
        P, Q, vark, T, G, NT, pf, det = m.groups()
        late = "" if pf == "true" else " late-factors"
        dt = " det" if det == "true" else ""
        return (f"k_apply_gf p={int(P) - 1} q={Q} diffusion{' kappa' if vark == 'true' else ''} {T} G={G} NT={NT}"
                f"{late}{dt}")
    m = re.match(r"void mfhex::k_mass<(\d+), (\d+), (\w+), (\w+), (\d+), (\d+), (\d+)(?:, (true|false))?>", name)
    if m:
        P, Q, colloc, T, G, NT, VC, det = m.groups()
        vc = f" VC={VC}" if VC != "1" else ""
        return f"k_mass p={int(P) - 1} q={Q} {T} G={G} NT={NT}{vc}{' det' if det == 'true' else ''}"
    m = re.match(r"void mfhex::tet::\(anonymous namespace\)::k_tet_apply<(\d+), (\d+)>", name)
    if m:
        return f"k_tet_apply p={m.group(1)} q={m.group(2)}"
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0].split("<")[0].split("::")[-1][:60]


def _find(d: str, suffix: str) -> str:
    fs = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not fs:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return fs[0]


def trace_summary(d: str, command: str, sources=KERNEL_SOURCES) -> str:
    rows = list(csv.DictReader(open(_find(d, "kernel_stats.csv"))))
    out = [f"# rocprofv3 kernel trace summary", f"# command: {command}",
           f"# kernel source hash: {kernel_source_hash(sources)}",
           f"{'kernel':<60} {'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'pct':>6}"]
    for r in rows:
        out.append(f"{_short(r['Name']):<60} {int(r['Calls']):>6} {float(r['AverageNs']) / 1e3:>10.2f} "
                   f"{float(r['MinNs']) / 1e3:>10.2f} {float(r['MaxNs']) / 1e3:>10.2f} "
                   f"{float(r['Percentage']):>6.2f}")
    return "\n".join(out) + "\n"


def _counter(d: str, counter: str):
    per = defaultdict(list)
    dur = defaultdict(list)
    for r in csv.DictReader(open(_find(d, "counter_collection.csv"))):
        if r["Counter_Name"] != counter:
            continue
        per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        dur[r["Kernel_Name"]].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return per, dur


def traffic_summary(fetch_dir: str, write_dir: str, command: str) -> str:
    fe, fdur = _counter(fetch_dir, "FETCH_SIZE")
    wr, _ = _counter(write_dir, "WRITE_SIZE")
    copy = [k for k in fe if "copyBuffer" in k or "copy" in k.lower()]
    # the calibration copy is the dispatch with by far the largest fetch among the copy kernels
    cf = max(v for k in copy for v in fe[k])
    cw = max(v for k in copy if k in wr for v in wr[k])
    f_scale = COPY_BYTES / (cf * 1024.0)
    w_scale = COPY_BYTES / (cw * 1024.0)
    out = [f"# HBM traffic per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB per dispatch)",
           f"# command: {command}",
           f"# kernel source hash: {kernel_source_hash()}",
           f"# calibration: 1 GiB device copy reads FETCH_SIZE={cf:.1f} KiB, WRITE_SIZE={cw:.1f} KiB -> "
           f"scale fetch x{f_scale:.4f}, write x{w_scale:.4f}",
           f"{'kernel':<60} {'fetch_KiB':>12} {'write_KiB':>12} {'traffic_bytes':>15} {'avg_us':>9}"]
    for k in fe:
        if ("k_apply" not in k and "k_mass" not in k) or k not in wr:
            continue
        f = sum(fe[k]) / len(fe[k])
        w = sum(wr[k]) / len(wr[k])
        t = f * 1024 * f_scale + w * 1024 * w_scale
        out.append(f"{_short(k):<60} {f:>12.1f} {w:>12.1f} {t:>15.0f} {sum(fdur[k]) / len(fdur[k]) / 1e3:>9.2f}")
    return "\n".join(out) + "\n"


_TABLE_COLS = (
    ("waves/SIMD", "waves_per_simd", "{:.2f}"), ("valu_busy", "valu_busy", "{:.3f}"),
    ("wait_any", "wait_any/wave", "{:.3f}"), ("wait_inst", "wait_inst_any/wave", "{:.3f}"),
    ("wait_lds", "wait_inst_lds/wave", "{:.3f}"), ("lds_confl", "lds_conflict", "{:.3f}"),
    ("VALU_insts", "SQ_INSTS_VALU", "{:.3e}"), ("LDS_insts", "SQ_INSTS_LDS", "{:.3e}"),
    ("SALU_insts", "SQ_INSTS_SALU", "{:.3e}"), ("EA_RDREQ", "TCC_EA0_RDREQ_sum", "{:.3e}"),
    ("EA_WRREQ", "TCC_EA0_WRREQ_sum", "{:.3e}"), ("L2_hit", "l2_hit", "{:.3f}"),
)


def _derived(m: dict) -> dict:
    """Derived ratios from one kernel's mean counter values (see `counter_summary`)."""
    der = {}
    if "SQ_WAVE_CYCLES" in m and m.get("GRBM_GUI_ACTIVE", 0) > 0:
        simd_cycles = m["GRBM_GUI_ACTIVE"] / 8 * 1024
        der["waves_per_simd"] = 4 * m["SQ_WAVE_CYCLES"] / simd_cycles
        if "SQ_ACTIVE_INST_VALU" in m:
            der["valu_busy"] = 4 * m["SQ_ACTIVE_INST_VALU"] / simd_cycles
    if m.get("SQ_WAVE_CYCLES", 0) > 0:
        for c in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS"):
            if c in m:
                der[c.lower().replace("sq_", "") + "/wave"] = m[c] / m["SQ_WAVE_CYCLES"]
    if "SQ_LDS_BANK_CONFLICT" in m and m.get("SQ_LDS_IDX_ACTIVE", 0) > 0:
        der["lds_conflict"] = m["SQ_LDS_BANK_CONFLICT"] / m["SQ_LDS_IDX_ACTIVE"]
    if m.get("TCC_HIT_sum", 0) + m.get("TCC_MISS_sum", 0) > 0:
        der["l2_hit"] = m["TCC_HIT_sum"] / (m["TCC_HIT_sum"] + m["TCC_MISS_sum"])
    return der


def _counter_table(header, per_kernel: dict) -> str:
    """One row per kernel: derived ratios and the instruction / memory-request counts behind them."""
    w = max([len(k) for k in per_kernel] + [6])
    out = list(header)
    out.append(f"{'kernel':<{w}} " + " ".join(f"{c:>10}" for c, _, _ in _TABLE_COLS))
    for k, m in per_kernel.items():
        v = dict(m)
        v.update(_derived(m))
        out.append(f"{k:<{w}} " + " ".join(f"{(fmt.format(v[key]) if key in v else '-'):>10}"
                                          for _, key, fmt in _TABLE_COLS))
    return "\n".join(out) + "\n"


_TABLE_NOTE = ("# derived (SQ wave-cycle counters count quad-cycles): waves/SIMD = 4*SQ_WAVE_CYCLES/(GRBM_GUI_ACTIVE/8)/1024; "
               "valu_busy = 4*SQ_ACTIVE_INST_VALU/(GRBM_GUI_ACTIVE/8)/1024; wait_any, wait_inst, wait_lds = "
               "SQ_WAIT_ANY, SQ_WAIT_INST_ANY, SQ_WAIT_INST_LDS per SQ_WAVE_CYCLES; lds_confl = "
               "SQ_LDS_BANK_CONFLICT/SQ_LDS_IDX_ACTIVE; L2_hit = TCC_HIT/(TCC_HIT+TCC_MISS); instruction and "
               "request counts are per dispatch, summed over the GPU")


def counter_summary(dirs, command: str, sources=KERNEL_SOURCES) -> str:
    """Per-kernel averages of the counters found in the ``--pmc`` runs under `dirs` (one directory per
    pass), as a table of derived ratios where their inputs were collected:
      waves/SIMD  = 4 SQ_WAVE_CYCLES / (GRBM_GUI_ACTIVE / 8 XCDs) / 1024 SIMDs  (mean resident waves; the SQ
                    wave-cycle counters count quad-cycles, GRBM_GUI_ACTIVE single cycles summed over the 8 XCDs)
      valu_busy   = 4 SQ_ACTIVE_INST_VALU / (GRBM_GUI_ACTIVE / 8) / 1024  (share of SIMD cycles issuing VALU)
      wait_*      = SQ_WAIT_ANY, SQ_WAIT_INST_ANY, SQ_WAIT_INST_LDS over SQ_WAVE_CYCLES (same unit both sides)
      lds_confl   = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE, L2_hit = TCC_HIT / (TCC_HIT + TCC_MISS)
    Counter values are per dispatch, summed over the GPU by rocprofv3."""
    vals = defaultdict(lambda: defaultdict(list))
    for d in dirs:
        for r in csv.DictReader(open(_find(d, "counter_collection.csv"))):
            vals[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    per = {}
    for k in vals:
        sk = _short(k)
        if sk.startswith("k_apply") or sk.startswith("k_mass") or sk.startswith("k_tet"):
            per[sk] = {c: sum(v) / len(v) for c, v in vals[k].items()}
    header = [f"# rocprofv3 counters per dispatch (mean over dispatches)", f"# command: {command}",
              f"# kernel source hash: {kernel_source_hash(sources)}", _TABLE_NOTE]
    return _counter_table(header, per)


def condense(path: str) -> str:
    """Rewrite a per-counter listing (one block per kernel, one ``COUNTER value`` line each) as the table
    `counter_summary` prints, keeping the listing's header lines."""
    header, per, cur = [], {}, None
    for line in open(path).read().splitlines():
        if line.startswith("#"):
            if not line.startswith("# derived"):
                header.append(line)
        elif line.startswith("    = "):
            continue
        elif line.startswith("    "):
            c, v = line.split()
            per[cur][c] = float(v)
        elif line.strip():
            cur = line.strip()
            per[cur] = {}
    return _counter_table(header + [_TABLE_NOTE], per)


def read_traffic(path: str):
    """{short kernel name: traffic bytes} if the summary matches the current kernel sources, else {}."""
    if not os.path.exists(path):
        return {}
    txt = open(path).read()
    m = re.search(r"kernel source hash: (\w+)", txt)
    if not m or m.group(1) != kernel_source_hash():
        return {}
    res = {}
    for line in txt.splitlines():
        if line.startswith("k_apply") or line.startswith("k_mass"):
            parts = line.split()
            name = " ".join(parts[:-4])
            res[name] = float(parts[-2])
    return res


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "trace":
        sys.stdout.write(trace_summary(sys.argv[2], " ".join(sys.argv[3:])))
    elif mode == "trace-tet":
        sys.stdout.write(trace_summary(sys.argv[2], " ".join(sys.argv[3:]), TET_SOURCES))
    elif mode == "trace-probe":
        sys.stdout.write(trace_summary(sys.argv[2], " ".join(sys.argv[3:]), PROBE_SOURCES))
    elif mode == "counters":
        # counters <dir1,dir2,...> <cmd...>
        sys.stdout.write(counter_summary(sys.argv[2].split(","), " ".join(sys.argv[3:])))
    elif mode == "condense":
        sys.stdout.write(condense(sys.argv[2]))
    elif mode == "traffic":
        sys.stdout.write(traffic_summary(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:])))
    else:
        raise SystemExit("usage: prof_summary trace <dir> <cmd...> | traffic <fetch_dir> <write_dir> <cmd...>")
