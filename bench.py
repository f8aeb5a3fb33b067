#!/usr/bin/env python3
"""Benchmark of the matrix-free BP3 apply on one MI355X.

Workload (default): the diffusion (stiffness, BP3) operator in FP64 with
Gauss quadrature q = p+2, orders p = 3..8, each on a cubic hexahedral mesh of
the unit cube with about 1e7 nodes (elements per direction
round((1e7^(1/3) - 1)/p)), interior vertices perturbed by U(+-0.1 h),
homogeneous Dirichlet, input U[-1,1].  Synthetic inputs stand in for the CEED
bake-off meshes.  One step = one apply at every order; value = nodes
processed per second over the step (GDOF/s).

Before timing, each operator is autotuned on this GPU (mfhex_tune: every
launch variant whose result agrees with the default, median of three rounds;
--no-tune times the built-in defaults).  The timed region runs the K steps order by order (K back-to-back applies of
each operator, as an operator is applied inside CG; --interleaved runs them
step by step).  Per order each apply is bracketed by HIP events on the launch
stream; the
roofline fraction uses the algorithmic bytes of one apply,
  8 N (x) + 8 N (y) + 4 E (p+1)^3 (restriction) + 48 E q^3 (geometric factors),
over the measured duration, against 8 TB/s.  The CPU baseline times the FP64
oracle (dense, no sum factorization) on a bounded sample on the host cores.

The same run times a 1 GiB device copy and reports each order's fraction of
that measured rate next to the datasheet fraction.

Prints ONE JSON line.  Untimed extras of the default run (skipped with
--no-extras): the HBM ceiling from streaming kernels written for it
(read-only sweep, copy, fill); the same BP3 sweep at about 1e8 nodes per
order; and the second half of the metric, FP64 vs mixed-precision CG to a
1e-10 relative residual at about 3e7 nodes, p = 3, 5, 7.  Further extras:
--cg adds Jacobi / p-multigrid preconditioned CG; --tet adds the tetrahedral
P_p apply (matrix-core basis products, p = 2..6) with its FP64 MFMA and HBM
fractions.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDOF/s of BP3 apply per order p; mixed-vs-FP64 CG time to 1e-10 resid"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # MI355X dense FP64 (vector and matrix)
PAPER_V100_CUDA_GEN = {1: 0.510, 2: 1.420, 3: 1.872, 4: 2.300, 5: 2.344, 6: 2.683, 7: 2.639, 8: 2.609}


def alg_bytes(N: int, E: int, p: int, q: int, g: int = 6, s: int = 8, nvec: int = 1) -> int:
    return s * N * nvec * 2 + 4 * E * (p + 1) ** 3 + s * g * E * q ** 3


def alg_flops(E: int, p: int, q: int, kind: str = "diffusion", colloc: bool = False, otf: bool = False) -> int:
    P, Q = p + 1, q
    interp = 0 if colloc else 4 * (Q * P ** 3 + Q * Q * P * P + Q ** 3 * P)
    if kind == "mass":
        return E * (interp + Q ** 3)
    # in-kernel factors: 3 adjugate rows (27), detJ (5), 6 products (30), scaling (8) per point,
    # and 3 Q^2 Jacobian columns (36 each) per element
    geo = (70 * Q ** 3 + 108 * Q ** 2) if otf else 0
    return E * (interp + 12 * Q ** 4 + 15 * Q ** 3 + geo)


def alg_bytes_otf(N: int, E: int, ne: int, p: int) -> int:
    """In-kernel factors: x, y, offsets and the vertex coordinates (each vertex read once)."""
    return 8 * N * 2 + 4 * E * (p + 1) ** 3 + 24 * (ne + 1) ** 3


def cpu_baseline(p: int, budget_s: float = 12.0) -> dict:
    import oracle
    import synth
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))

    def run(ne):
        vert = synth.mesh_vertices(ne, ne, ne)
        pr = oracle.Problem(ne, ne, ne, p, p + 2, oracle.GAUSS, oracle.DIFFUSION, 1, vert)
        x = synth.uniform_vector(pr.n_nodes)
        t0 = time.perf_counter()
        oracle.apply(pr, x, nthreads=cores)
        return pr.n_nodes, time.perf_counter() - t0

    ne = 2
    n, t = run(ne)
    # grow the mesh until one apply takes about a quarter of the budget, then time three applies
    while t < budget_s / 5 and ne < 96:
        ne = max(ne + 1, int(ne * min(2.0, (budget_s / 4 / max(t, 1e-3)) ** (1 / 3))))
        n, t = run(ne)
    ts = sorted([t] + [run(ne)[1] for _ in range(2)])
    t = ts[1]
    return {"value": n / t / 1e9, "unit": "GDOF/s", "cores": cores, "kind": "oracle",
            "sample": f"BP3 FP64 apply, p={p}, q={p + 2}, {ne}^3 elements ({n} DOFs), median of 3 applies "
                      f"({t:.2f} s each), dense-tabulation oracle, OpenMP {cores} threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--orders", type=str, default="3,4,5,6,7,8")
    ap.add_argument("--dofs", type=float, default=1e7)
    ap.add_argument("--kind", choices=["diffusion", "mass"], default="diffusion",
                    help="diffusion = BP3 (default), mass = BP1")
    ap.add_argument("--batched", action="store_true",
                    help="also time the batched collocated apply (BP5 / BP6, 4/8/32 right-hand sides)")
    ap.add_argument("--batched-config", type=str, default="",
                    help="only time one batched collocated configuration p,ncomp,nrhs[,variant] at about 3e7 "
                         "nodes per field (for profiling runs)")
    ap.add_argument("--adjoint", action="store_true",
                    help="also time the variable-coefficient forward / backward (p=4, 1e7 DOFs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the untimed extras of the default run (HBM ceiling probe, the 1e8-node sweep and "
                         "the FP64 vs mixed CG comparison)")
    ap.add_argument("--cg", action="store_true",
                    help="also time Jacobi- and p-multigrid-preconditioned CG next to FP64 vs mixed CG")
    ap.add_argument("--tet", action="store_true",
                    help="also time the tetrahedral P_p diffusion apply (matrix-core basis products), p=2..6")
    ap.add_argument("--no-tune", action="store_true",
                    help="time the built-in launch defaults instead of autotuning each operator before timing")
    ap.add_argument("--otf", action="store_true",
                    help="diffusion with the geometric factors evaluated in the kernel (no stored factors)")
    ap.add_argument("--sweep", action="store_true", help="report the time of every launch variant (stderr)")
    ap.add_argument("--interleaved", action="store_true",
                    help="time the steps one by one (one apply of every order per step) instead of order by order")
    ap.add_argument("--fp64-rate", action="store_true",
                    help="only measure the FP64 pipes: 16x16x4 and 4x4x4 matrix-core and vector FMA chains")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after timing, copy 1 GiB device-to-device twice (a kernel of known traffic, "
                         "used to scale the HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the multi-GPU path is a design "
                          "(element-partition sharding with a face exchange), not built"}), flush=True)
        sys.exit(2)

    import torch
    import synth
    import paper_2109_05072_amd as mf

    torch.cuda.set_device(0)
    if args.fp64_rate:
        print(json.dumps({"fp64_rate": fp64_rates(), "peak_tflops": FP64_PEAK_TFLOPS}), flush=True)
        return
    if args.batched_config:
        print(json.dumps(batched_one([int(v) for v in args.batched_config.split(",")], args.steps, args.warmup)),
              flush=True)
        if args.calib_copy:
            calib_copy()
        return
    orders = [int(s) for s in args.orders.split(",") if s]
    ops, xs, ys, meta = {}, {}, {}, {}
    for p in orders:
        ne = synth.elems_for_dofs(args.dofs, p)
        vert = synth.mesh_vertices(ne, ne, ne)
        op = mf.Operator(ne, ne, ne, p, vert, kind=args.kind, quad="gauss", dirichlet=(args.kind == "diffusion"),
                         otf=args.otf)
        x = torch.from_numpy(synth.uniform_vector(op.n_nodes)).cuda()
        ops[p], xs[p], ys[p] = op, x, torch.empty_like(x)
        if args.sweep:
            sweep_variants(op, x, p)
        if not args.no_tune:
            op.tune()  # the launch variant for this operator on this GPU (untimed set-up)
        meta[p] = dict(ne=ne, N=op.n_nodes, E=op.n_elem, q=p + 2, epb=op.get_config())
        print(f"# setup p={p}: {ne}^3 elements, {op.n_nodes} DOFs, launch (variant, elems, threads, depth) "
              f"{meta[p]['epb']}",
              file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        for p in orders:
            ops[p].apply(xs[p], ys[p])
    torch.cuda.synchronize()

    evs = {p: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)] for p in orders}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.interleaved:
        # step by step: one apply of every order per step
        for s in range(args.steps):
            for p in orders:
                e0, e1 = evs[p][s]
                e0.record()
                ops[p].apply(xs[p], ys[p])
                e1.record()
    else:
        # the same K steps order by order: K back-to-back applies of each operator (t_apply of the
        # measurement plan; an operator inside CG is applied back to back the same way)
        for p in orders:
            for s in range(args.steps):
                e0, e1 = evs[p][s]
                e0.record()
                ops[p].apply(xs[p], ys[p])
                e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    ms_per_step = wall / args.steps * 1e3
    dofs_per_step = sum(meta[p]["N"] for p in orders)
    value = dofs_per_step / (ms_per_step / 1e3) / 1e9
    per_p = []
    for p in orders:
        t_ms = float(np.mean([a.elapsed_time(b) for a, b in evs[p]]))
        m = meta[p]
        byts = (alg_bytes_otf(m["N"], m["E"], m["ne"], p) if args.otf else
                alg_bytes(m["N"], m["E"], p, m["q"], g=6 if args.kind == "diffusion" else 1))
        fl = alg_flops(m["E"], p, m["q"], args.kind, otf=args.otf)
        gbs = byts / (t_ms / 1e3) / 1e9
        per_p.append({"p": p, "elements_per_dim": m["ne"], "dofs": m["N"], "ms": round(t_ms, 4),
                      "gdofs": round(m["N"] / (t_ms / 1e3) / 1e9, 3), "alg_bytes": byts,
                      "alg_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                      "alg_tflops": round(fl / (t_ms / 1e3) / 1e12, 2),
                      "fp64_alu_frac": round(fl / (t_ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS, 4),
                      "launch": {"variant": m["epb"][0], "elements_per_group": m["epb"][1],
                                 "threads_per_group": m["epb"][2], "groups_per_block": m["epb"][3]},
                      "paper_v100_cuda_gen_gdofs": PAPER_V100_CUDA_GEN.get(p)})
    # measured device-copy rate on this GPU (1 GiB read + 1 GiB written per copy, median of 5): the
    # practical HBM ceiling next to the datasheet peak
    copy_gbs = measure_copy_gbs()
    for r in per_p:
        r["copy_frac"] = round(r["alg_gbs"] / copy_gbs, 4)
    dom = max(per_p, key=lambda r: r["ms"])
    from paper_2109_05072_amd.prof_summary import read_traffic
    lg = dom["launch"]
    if args.kind == "diffusion":
        tag = "otf " if args.otf else ""
        traffic = read_traffic(os.path.join(ROOT, "profiles", f"bp3{'_otf' if args.otf else ''}_apply_traffic.txt"))
        gf = 9 <= lg["variant"] <= 14
        kname = "k_apply_gf" if gf else "k_apply"
        late = LATE_FACTOR_SLOTS.get((dom["p"] + 2, lg["variant"]))
        pre = PREFETCH_SLOTS.get((dom["p"] + 2, lg["variant"]))
        suffix = (" late-factors" if lg["variant"] == 14 else
                  f" late{late}{f' pre{pre}' if pre else ''}" if late and not args.otf else "")
        dom_name = (f"{kname} p={dom['p']} q={dom['p'] + 2} diffusion {tag}double G={lg['elements_per_group']} "
                    f"NT={lg['threads_per_group']}{suffix}")
    else:
        traffic = read_traffic(os.path.join(ROOT, "profiles", "bp1_apply_traffic.txt"))
        dom_name = (f"k_mass p={dom['p']} q={dom['p'] + 2} double G={lg['elements_per_group']} "
                    f"NT={lg['threads_per_group']}")
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GDOF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded perturbed unit-cube hex meshes, U[-1,1] inputs)",
        "config": {"workload": (f"BP3 diffusion apply FP64{' (geometric factors in-kernel)' if args.otf else ''}, "
                                f"Gauss q=p+2, p={','.join(map(str, orders))}, "
                                f"~{args.dofs:.0e} DOFs per order, perturbed hex mesh, Dirichlet")
                   if args.kind == "diffusion" else
                               (f"BP1 mass apply FP64, Gauss q=p+2, p={','.join(map(str, orders))}, "
                                f"~{args.dofs:.0e} DOFs per order, perturbed hex mesh"),
                   "orders": orders, "dofs_per_step": dofs_per_step,
                   "timing": "interleaved steps" if args.interleaved else "steps order by order (back-to-back applies)"},
        "roofline": ({"bound": "hbm", "kernel": dom_name,
                      "achieved": dom["alg_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": dom["hbm_frac"], "traffic": traffic.get(dom_name),
                      "alg_bytes_per_launch": dom["alg_bytes"], "measured_copy_gbs": round(copy_gbs, 1),
                      "frac_of_copy": dom["copy_frac"]}
                     if not args.otf or dom["hbm_frac"] >= dom["fp64_alu_frac"] else
                     {"bound": "alu", "kernel": dom_name, "achieved": dom["alg_tflops"],
                      "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": dom["fp64_alu_frac"],
                      "traffic": traffic.get(dom_name), "alg_bytes_per_launch": dom["alg_bytes"],
                      "hbm_frac": dom["hbm_frac"]}),
        "per_order": per_p,
    }
    if args.calib_copy:
        calib_copy()
    for p in orders:
        ops[p].close()
    del ops, xs, ys
    torch.cuda.empty_cache()
    default_extras = args.kind == "diffusion" and not args.otf and not args.no_extras
    if default_extras:
        # the practical HBM ceiling, measured by streaming kernels written for it (read-only sweep,
        # copy, fill), next to the datasheet peak
        out["hbm_ceiling"] = hbm_ceiling()
        out["roofline"]["frac_of_read_ceiling"] = round(dom["alg_gbs"] / out["hbm_ceiling"]["read_gbs"], 4)
        for r in per_p:
            r["read_ceiling_frac"] = round(r["alg_gbs"] / out["hbm_ceiling"]["read_gbs"], 4)
        # the second gate size of the sweep: about 1e8 nodes per order
        out["per_order_1e8"] = per_order_sweep(orders, 1e8, steps=5, tune=not args.no_tune)
    if args.cg or default_extras:
        # the second half of the metric: FP64 vs mixed-precision CG to a 1e-10 relative residual at
        # about 3e7 nodes, p = 3, 5, 7 (preconditioned variants only with --cg)
        out["cg"] = cg_compare(precond=args.cg)
    if args.batched:
        out["batched"] = batched_sweep()
    if args.tet:
        out["tet"] = tet_bench()
    if args.adjoint:
        out["adjoint"] = adjoint_bench()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(dom["p"])
    print(json.dumps(out), flush=True)


# (q, variant) -> points per factor-load batch of the launch variants that load the geometric
# factors in the pointwise stage (kVarLate in csrc/mfhex_internal.h), so that the dominant kernel
# is named as the profile summaries name it
LATE_FACTOR_SLOTS = {(5, 2): 2, (6, 1): 2, (7, 2): 3, (7, 3): 3, (8, 1): 2, (8, 4): 2, (9, 2): 2, (9, 4): 2, (10, 2): 4, (10, 3): 2}
# of those, (q, variant) -> points per lane still prefetched at the group start (kVarPre)
PREFETCH_SLOTS = {(7, 2): 3, (7, 3): 3, (8, 4): 2}


def measure_copy_gbs(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """GB/s of a device-to-device copy of nbytes (read + write counted), median of reps."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / float(np.median(ts)) / 1e9


def fp64_rates(nblocks: int = 2048, iters: int = 4096, reps: int = 3) -> list:
    """FP64 throughput of the matrix-core and vector pipes (libhbmprobe.so: chains of 16x16x4 and
    4x4x4 FP64 MFMA and of v_fma_f64 with independent accumulators, registers only), median of reps
    event-timed launches of nblocks x 256 threads."""
    import ctypes as C
    import torch
    from paper_2109_05072_amd import build as libbuild
    if not os.path.exists(libbuild.PROBE_LIB):
        raise RuntimeError(f"{libbuild.PROBE_LIB} is not built (run __graft_entry__.build())")
    lib = C.CDLL(libbuild.PROBE_LIB)
    lib.fp64_rate.argtypes = [C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_void_p]
    lib.fp64_rate.restype = C.c_int
    lib.fp64_rate_flops_per_wave_iter.argtypes = [C.c_int]
    lib.fp64_rate_flops_per_wave_iter.restype = C.c_double
    out = torch.empty(nblocks * 256, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    res = []
    for kind, name in ((0, "mfma_f64_16x16x4"), (1, "mfma_f64_4x4x4_4blocks"), (2, "v_fma_f64")):
        def run():
            rc = lib.fp64_rate(kind, out.data_ptr(), nblocks, iters, stream)
            if rc != 0:
                raise RuntimeError(f"fp64_rate({kind}) failed: {rc}")
        run()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            run()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        t = float(np.median(ts))
        flops = nblocks * 256 / 64 * iters * lib.fp64_rate_flops_per_wave_iter(kind)
        res.append({"kind": name, "ms": round(t * 1e3, 4), "tflops": round(flops / t / 1e12, 2),
                    "frac_of_peak": round(flops / t / 1e12 / FP64_PEAK_TFLOPS, 4)})
    if not bool(torch.isfinite(out).all()):
        raise RuntimeError("fp64 rate probe produced non-finite results")
    del out
    torch.cuda.empty_cache()
    return res


def hbm_ceiling(nbytes: int = 4 << 30, reps: int = 5) -> dict:
    """Bandwidth of streaming kernels written for this measurement (libhbmprobe.so): a read-only
    sweep, a copy and a fill of nbytes, 16-byte accesses, plain and non-temporal, over a few grid
    sizes; the best median of each kind.  Copy counts read + write bytes."""
    import ctypes as C
    import torch
    from paper_2109_05072_amd import build as libbuild
    if not os.path.exists(libbuild.PROBE_LIB):
        raise RuntimeError(f"{libbuild.PROBE_LIB} is not built (run __graft_entry__.build())")
    lib = C.CDLL(libbuild.PROBE_LIB)
    lib.hbm_stream.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p]
    lib.hbm_stream.restype = C.c_int
    n = nbytes // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    grids = (1024, 2048, 4096, 8192, 16384)
    part = torch.empty(max(grids), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    best = {}
    for kind, name, mult in ((0, "read", 1), (1, "copy", 2), (2, "fill", 1)):
        for nt in (0, 1):
            for g in grids:
                def run():
                    rc = lib.hbm_stream(kind, nt, a.data_ptr(), b.data_ptr(), n, part.data_ptr(), g, stream)
                    if rc != 0:
                        raise RuntimeError(f"hbm_stream({kind}, {nt}, grid {g}) failed: {rc}")
                run()
                ts = []
                for _ in range(reps):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    run()
                    e1.record()
                    torch.cuda.synchronize()
                    ts.append(e0.elapsed_time(e1) / 1e3)
                gbs = mult * nbytes / float(np.median(ts)) / 1e9
                if gbs > best.get(name, (0.0,))[0]:
                    best[name] = (gbs, {"grid": g, "nontemporal": bool(nt)})
    # the read kernel's result checks that it really read the data
    lib.hbm_stream(0, 0, a.data_ptr(), b.data_ptr(), n, part.data_ptr(), 1024, stream)
    total = float(part[:1024].sum())
    if total != float(n):
        raise RuntimeError(f"read probe summed {total}, expected {n}")
    del a, b, part
    torch.cuda.empty_cache()
    out = {f"{k}_gbs": round(v[0], 1) for k, v in best.items()}
    out.update({f"{k}_launch": v[1] for k, v in best.items()})
    out["bytes"] = nbytes
    out["frac_of_peak"] = {k: round(v[0] / HBM_PEAK_GBS, 4) for k, v in best.items()}
    return out


def per_order_sweep(orders, dofs: float, steps: int = 5, tune: bool = True) -> list:
    """BP3 FP64 apply at about `dofs` nodes per order (one operator at a time, autotuned unless
    tune=False): median of `steps` event-timed back-to-back applies after two warm-ups, with the
    roofline fraction against 8 TB/s."""
    import torch
    import synth
    import paper_2109_05072_amd as mf
    res = []
    for p in orders:
        ne = synth.elems_for_dofs(dofs, p)
        vert = synth.mesh_vertices(ne, ne, ne)
        op = mf.Operator(ne, ne, ne, p, vert, kind="diffusion", quad="gauss", dirichlet=True)
        x = torch.from_numpy(synth.uniform_vector(op.n_nodes)).cuda()
        y = torch.empty_like(x)
        if tune:
            op.tune()
        for _ in range(2):
            op.apply(x, y)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for e0, e1 in ev:
            e0.record()
            op.apply(x, y)
            e1.record()
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
        byts = alg_bytes(op.n_nodes, op.n_elem, p, p + 2)
        gbs = byts / (ms / 1e3) / 1e9
        cfg = op.get_config()
        r = {"p": p, "elements_per_dim": ne, "dofs": op.n_nodes, "ms": round(ms, 4),
             "gdofs": round(op.n_nodes / (ms / 1e3) / 1e9, 3), "alg_bytes": byts, "alg_gbs": round(gbs, 1),
             "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
             "launch": {"variant": cfg[0], "elements_per_group": cfg[1], "threads_per_group": cfg[2]}}
        res.append(r)
        print(f"# 1e8 {r}", file=sys.stderr, flush=True)
        op.close()
        del op, x, y, vert
        torch.cuda.empty_cache()
    return res


def sweep_variants(op, x, p, reps=10, rounds=3, nrhs=1):
    """Median over interleaved rounds of the apply time of every launch configuration (stderr)."""
    import torch
    import paper_2109_05072_amd as mf
    y = torch.empty_like(x)
    default = op.get_config(nrhs=nrhs)
    depths = (1, 2, 4) if op.kind == "mass" else (1,)
    cfgs = []
    for v in range(17):
        for d in depths:
            try:
                op.set_config(v, nrhs=nrhs, groups_per_block=d)
            except mf.MFHexError:
                continue
            cfgs.append((v, d, op.get_config(nrhs=nrhs)[1:]))
            for _ in range(3):
                op.apply(x, y)
    times = {c[:2]: [] for c in cfgs}
    for _ in range(rounds):
        for v, d, _g in cfgs:
            op.set_config(v, nrhs=nrhs, groups_per_block=d)
            op.apply(x, y)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                op.apply(x, y)
            e1.record()
            torch.cuda.synchronize()
            times[(v, d)].append(e0.elapsed_time(e1) / reps)
    op.set_config(default[0], nrhs=nrhs, groups_per_block=default[3])
    res = sorted(((float(np.median(times[(v, d)])), v, g) for v, d, g in cfgs))
    print(f"# sweep p={p} nrhs={nrhs} (median of {rounds}): " + "  ".join(f"v{v} {g}: {ms:.4f} ms" for ms, v, g in res),
          file=sys.stderr, flush=True)


def _time(fn, reps=5):
    import torch
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def batched_sweep(orders=(3, 4, 5, 6, 7, 8), dofs=3e7, ncomps=(1, 3), nrhss=(4, 8, 32)):
    """Collocated (Gauss-Lobatto q=p+1) diffusion, BP5 (ncomp=1) and BP6 (ncomp=3), several
    right-hand sides per launch, autotuned launch variant; throughput in field-DOF/s."""
    import torch
    import synth
    import paper_2109_05072_amd as mf
    res = []
    for p in orders:
        ne = synth.elems_for_dofs(dofs, p)
        vert = synth.mesh_vertices(ne, ne, ne)
        for nc in ncomps:
            op = mf.Operator(ne, ne, ne, p, vert, kind="diffusion", quad="gll", ncomp=nc, dirichlet=True)
            for nr in nrhss:
                nvec = nc * nr
                x = torch.rand(op.n_nodes, nvec, dtype=torch.float64, device="cuda") * 2 - 1
                y = torch.empty_like(x)
                if os.environ.get("MFHEX_BENCH_SWEEP"):
                    sweep_variants(op, x, p, reps=3, nrhs=nr)
                variant = op.tune(nrhs=nr)
                ms = _time(lambda: op.apply(x, y), reps=3)
                byts = alg_bytes(op.n_nodes, op.n_elem, p, p + 1, nvec=nvec)
                fl = alg_flops(op.n_elem, p, p + 1, colloc=True) * nvec
                res.append({"p": p, "ncomp": nc, "nrhs": nr, "dofs_per_field": op.n_nodes, "ms": round(ms, 3),
                            "gdofs_fields": round(op.n_nodes * nvec / (ms / 1e3) / 1e9, 2),
                            "alg_gbs": round(byts / (ms / 1e3) / 1e9, 1),
                            "hbm_frac": round(byts / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                            "alg_tflops": round(fl / (ms / 1e3) / 1e12, 2), "variant": list(variant)})
                print(f"# batched {res[-1]}", file=sys.stderr, flush=True)
                del x, y
                torch.cuda.empty_cache()
            op.close()
            del op
            torch.cuda.empty_cache()
    return res


def calib_copy():
    """Two 1 GiB device-to-device copies: a kernel of known traffic for scaling the byte counters."""
    import torch
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def batched_one(cfg, steps: int, warmup: int, dofs: float = 3e7) -> dict:
    """One batched collocated configuration (p, ncomp, nrhs[, variant]): the default (or given) launch,
    `steps` back-to-back applies after `warmup`, event-timed."""
    import torch
    import synth
    import paper_2109_05072_amd as mf
    p, nc, nr = cfg[:3]
    ne = synth.elems_for_dofs(dofs, p)
    op = mf.Operator(ne, ne, ne, p, synth.mesh_vertices(ne, ne, ne), kind="diffusion", quad="gll", ncomp=nc,
                     dirichlet=True)
    if len(cfg) > 3:
        op.set_config(cfg[3], nrhs=nr)
    x = torch.rand(op.n_nodes, nc * nr, dtype=torch.float64, device="cuda") * 2 - 1
    y = torch.empty_like(x)
    for _ in range(warmup):
        op.apply(x, y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        op.apply(x, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / max(steps, 1)
    return {"p": p, "ncomp": nc, "nrhs": nr, "launch": list(op.get_config(nrhs=nr)), "ms": round(ms, 4),
            "gdofs_fields": round(op.n_nodes * nc * nr / (ms / 1e3) / 1e9, 2)}


def adjoint_bench(p=4, dofs=1e7):
    """Variable-coefficient diffusion y = A(kappa) u and the backward of 0.5||y - f||^2 (grad wrt
    u and kappa), p=4, q=6, about 1e7 DOFs; checked by central differences (exact: the loss is
    quadratic in kappa and in u)."""
    import numpy as np
    import torch
    import synth
    import paper_2109_05072_amd as mf
    from paper_2109_05072_amd.autograd import diffusion
    ne = synth.elems_for_dofs(dofs, p)
    vert = synth.mesh_vertices(ne, ne, ne)
    op = mf.Operator(ne, ne, ne, p, vert, kind="diffusion", quad="gauss", dirichlet=True, variable_kappa=True)
    kap = torch.from_numpy(synth.kappa_field(op.qpoint_coords().cpu().numpy())).cuda()
    n = op.n_nodes
    nn = p * ne + 1
    ijk = np.arange(n)
    ix, iy, iz = ijk % nn, (ijk // nn) % nn, ijk // (nn * nn)
    interior = ((ix > 0) & (ix < nn - 1) & (iy > 0) & (iy < nn - 1) & (iz > 0) & (iz < nn - 1)).astype(float)
    u = torch.from_numpy(synth.uniform_vector(n, seed=1)).cuda()
    f = torch.from_numpy(synth.uniform_vector(n, seed=2) * interior).cuda()
    uu = u.clone().requires_grad_(True)
    kk = kap.clone().requires_grad_(True)

    def loss(a, b):
        r = diffusion(a, b, op) - f
        return 0.5 * (r * r).sum()

    fwd_ms = _time(lambda: op.set_kappa(kap) or op.apply(u), reps=5)
    r = op.apply(u) - f
    bwd_ms = _time(lambda: (op.apply_adjoint(r), op.kappa_grad(u, r)), reps=5)
    kg_ms = _time(lambda: op.kappa_grad(u, r), reps=5)
    Lv = loss(uu, kk)
    gu, gk = torch.autograd.grad(Lv, [uu, kk])
    rng = np.random.default_rng(synth.SEED_DIR)
    fd = []
    with torch.no_grad():
        for _ in range(2):
            d = torch.from_numpy(rng.standard_normal(tuple(kap.shape))).cuda()
            eps = 1e-2 * float(kap.norm() / d.norm())
            num = float((loss(u, kap + eps * d) - loss(u, kap - eps * d)) / (2 * eps))
            an = float((gk * d).sum())
            fd.append({"wrt": "kappa", "rel_err": abs(num - an) / abs(an)})
            du = torch.from_numpy(rng.standard_normal(n)).cuda()
            eps = 1e-2 * float(u.norm() / du.norm())
            num = float((loss(u + eps * du, kap) - loss(u - eps * du, kap)) / (2 * eps))
            an = float((gu * du).sum())
            fd.append({"wrt": "u", "rel_err": abs(num - an) / abs(an)})
    out = {"p": p, "q": p + 2, "dofs": n, "qpts": op.n_elem * (p + 2) ** 3, "forward_ms": round(fwd_ms, 3),
           "backward_ms": round(bwd_ms, 3), "kappa_grad_ms": round(kg_ms, 3), "fd_checks": fd}
    op.close()
    return out


def tet_dims(p: int, q: int):
    P, Q = (p + 1) * (p + 2) * (p + 3) // 6, q ** 3
    r = lambda n, m: (n + m - 1) // m * m
    return P, Q, r(Q, 16), r(P, 4), r(P, 16)


def tet_bench(orders=(2, 3, 4, 5, 6), dofs=1e7, reps=20):
    """Tetrahedral P_p apply at about `dofs` nodes per order (Kuhn split of the perturbed box)."""
    import torch
    import synth
    import paper_2109_05072_amd as mf
    res = []
    for p in orders:
        ne = synth.elems_for_dofs(dofs, p)
        op = mf.TetOperator(ne, ne, ne, p, synth.mesh_vertices(ne, ne, ne))
        x = torch.from_numpy(synth.uniform_vector(op.n_nodes)).cuda()
        y = torch.empty_like(x)
        for _ in range(3):
            op.apply(x, y)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in ev:
            e0.record()
            op.apply(x, y)
            e1.record()
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
        P, Q, Qp, Pk, Pn = tet_dims(p, op.q)
        E, N = op.n_elem, op.n_nodes
        useful = E * (12.0 * Q * P + 15.0 * Q)          # two products of 3Q x P per element + the 3x3 per point
        # p <= 3: the library groups the 12 tetrahedra of two hexahedra per wavefront and computes their
        # restriction from the block coordinates (no offset array); otherwise 16 elements per
        # wavefront with a stored int32 restriction
        pairs = p <= 3
        groups = ((ne + 1) // 2) * ne * ne if pairs else -(-E // 16)
        issued = groups * 2048.0 * (3 * (Qp // 16) * (Pk // 4) + 12 * (Qp // 16) * (Pn // 16))
        byts = 8 * N + 8 * N + (0 if pairs else 4 * E * P) + 48 * E * Q
        t = ms / 1e3
        r = {"p": p, "q": op.q, "elements": E, "dofs": N, "basis_per_elem": P, "points_per_elem": Q, "ms": round(ms, 4),
             "gdofs": round(N / t / 1e9, 3), "useful_tflops": round(useful / t / 1e12, 2),
             "mfma_frac_useful": round(useful / t / 1e12 / FP64_PEAK_TFLOPS, 4),
             "issued_mfma_tflops": round(issued / t / 1e12, 2),
             "mfma_frac_issued": round(issued / t / 1e12 / FP64_PEAK_TFLOPS, 4),
             "alg_bytes": byts, "alg_gbs": round(byts / t / 1e9, 1), "hbm_frac": round(byts / t / 1e9 / HBM_PEAK_GBS, 4),
             "flop_per_byte": round(useful / byts, 2)}
        res.append(r)
        print(f"# tet {r}", file=sys.stderr, flush=True)
        op.close()
        del op, x, y
        torch.cuda.empty_cache()
    return res


def cg_compare(orders=(3, 5, 7), dofs=3e7, precond=True):
    """FP64 CG vs mixed-precision (reliable-update) CG to a true relative residual of 1e-10 on BP3,
    Gauss q = p+2, sin forcing; with precond also Jacobi and p-multigrid preconditioned CG."""
    import torch
    import synth
    import paper_2109_05072_amd as mf
    res = []
    for p in orders:
        ne = synth.elems_for_dofs(dofs, p)
        vert = synth.mesh_vertices(ne, ne, ne)
        op = mf.Operator(ne, ne, ne, p, vert, kind="diffusion", quad="gauss", dirichlet=True, f32=True, rhs=True)
        f = synth.sin_forcing(op.qpoint_coords().cpu().numpy())
        b = op.rhs(torch.from_numpy(f).cuda())
        r64 = op.cg(b, maxit=20000, rtol=1e-10, mode="f64")
        rmx = op.cg(b, maxit=20000, rtol=1e-10, mode="mixed")
        d = float((rmx.x - r64.x).norm() / r64.x.norm())
        ue = torch.from_numpy(synth.sin_solution(op.node_coords().cpu().numpy())).cuda()
        row = {"p": p, "q": p + 2, "elements_per_dim": ne, "dofs": op.n_nodes,
               "f64_s": round(r64.seconds, 4), "f64_iters": r64.iters, "f64_status": r64.status,
               "mixed_s": round(rmx.seconds, 4), "mixed_iters": rmx.iters, "mixed_status": rmx.status,
               "replacements": rmx.replacements, "fell_back_to_f64": rmx.fell_back_to_f64,
               "speedup": round(r64.seconds / rmx.seconds, 3), "rel_diff_x_mixed_vs_f64": d,
               "f64_rel_resid": r64.rel_resid_true, "mixed_rel_resid": rmx.rel_resid_true,
               "max_err_vs_exact_f64": float((r64.x - ue).abs().max()),
               "max_err_vs_exact_mixed": float((rmx.x - ue).abs().max())}
        if not precond:
            res.append(row)
            print(f"# cg {row}", file=sys.stderr, flush=True)
            op.close()
            del op, b, r64, rmx, ue
            torch.cuda.empty_cache()
            continue
        j64 = op.cg(b, maxit=20000, rtol=1e-10, mode="f64", precond="jacobi")
        jmx = op.cg(b, maxit=20000, rtol=1e-10, mode="mixed", precond="jacobi")
        t0 = time.perf_counter()
        nlev = op.mg_setup()
        torch.cuda.synchronize()
        mg_setup_s = time.perf_counter() - t0
        rmg = op.cg(b, maxit=2000, rtol=1e-10, mode="f64", precond="mg")
        mg_lv = [lv[0] for lv in op.mg_levels()]
        t0 = time.perf_counter()
        op.mg_setup(dtype=torch.float32)
        torch.cuda.synchronize()
        mg32_setup_s = time.perf_counter() - t0
        rmg32 = op.cg(b, maxit=2000, rtol=1e-10, mode="f64", precond="mg")
        d = float((rmx.x - r64.x).norm() / r64.x.norm())
        ue = torch.from_numpy(synth.sin_solution(op.node_coords().cpu().numpy())).cuda()
        res.append({"p": p, "dofs": op.n_nodes, "f64_s": round(r64.seconds, 4), "f64_iters": r64.iters,
                    "mixed_s": round(rmx.seconds, 4), "mixed_iters": rmx.iters, "replacements": rmx.replacements,
                    "fell_back_to_f64": rmx.fell_back_to_f64, "speedup": round(r64.seconds / rmx.seconds, 3),
                    "rel_diff_x_mixed_vs_f64": d, "f64_rel_resid": r64.rel_resid_true,
                    "mixed_rel_resid": rmx.rel_resid_true,
                    "max_err_vs_exact_f64": float((r64.x - ue).abs().max()),
                    "max_err_vs_exact_mixed": float((rmx.x - ue).abs().max()),
                    "jacobi_f64_s": round(j64.seconds, 4), "jacobi_f64_iters": j64.iters,
                    "jacobi_mixed_s": round(jmx.seconds, 4), "jacobi_mixed_iters": jmx.iters,
                    "jacobi_mixed_replacements": jmx.replacements, "jacobi_f64_rel_resid": j64.rel_resid_true,
                    "jacobi_mixed_rel_resid": jmx.rel_resid_true,
                    "jacobi_rel_diff_x_vs_f64": float((j64.x - r64.x).norm() / r64.x.norm()),
                    "speedup_jacobi_mixed_vs_f64": round(r64.seconds / jmx.seconds, 3),
                    "mg_levels": mg_lv, "mg_setup_s": round(mg_setup_s, 4),
                    "mg_s": round(rmg.seconds, 4), "mg_iters": rmg.iters, "mg_rel_resid": rmg.rel_resid_true,
                    "mg_rel_diff_x_vs_f64": float((rmg.x - r64.x).norm() / r64.x.norm()),
                    "speedup_mg_vs_f64": round(r64.seconds / rmg.seconds, 3),
                    "max_err_vs_exact_mg": float((rmg.x - ue).abs().max()),
                    "mg32_setup_s": round(mg32_setup_s, 4), "mg32_s": round(rmg32.seconds, 4),
                    "mg32_iters": rmg32.iters, "mg32_rel_resid": rmg32.rel_resid_true,
                    "mg32_rel_diff_x_vs_f64": float((rmg32.x - r64.x).norm() / r64.x.norm()),
                    "speedup_mg32_vs_f64": round(r64.seconds / rmg32.seconds, 3)})
        print(f"# cg {res[-1]}", file=sys.stderr, flush=True)
        op.close()
        del op
        torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    main()
