#!/usr/bin/env python3
"""Throughput of the NUFFT hot path on one MI355X, in nonuniform points per second.

One step = the whole path over one batch of points: set the points (bin-sort),
a type 1 transform (spread, FFT, deconvolve) and a type 2 transform
(precorrect, FFT, interpolate) on the same sorted points; the type 2 is the
adjoint of the type 1 plan (opposite sign), i.e. the paper's type 2 with sign
+1.  Each step therefore moves 2 M points through the method; value =
2 M K / (time of K steps), inputs resident in HBM, plan creation excluded.

The default workload is 2D with 1024 x 1024 modes, M = 1e7 points iid uniform
in [-pi, pi)^2, complex64 strengths with N(0,1) parts, eps = 1e-5 (w = 6),
single precision.  Other workloads (--workload) are for exploration.

Prints one JSON line.  The per-stage HIP-event timers of the library give the
dominant kernel's average launch time, from which the roofline fraction is
computed against algorithmic bytes; the oracle is timed on a bounded sample
of the same workload on the host's cores.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "NU points/sec at eps=1e-5 (2D/3D, type 1/2); batched vs plain speedup"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (dim, modes, M, point kind, eps, precision)
    "2d": (2, (1024, 1024), 10_000_000, "uniform", 1e-5, "f32"),
    "2d-cluster": (2, (1024, 1024), 10_000_000, "cluster", 1e-5, "f32"),
    "2d-small": (2, (64, 64), 100_000, "uniform", 1e-5, "f32"),
    "3d": (3, (128, 128, 128), 1 << 24, "uniform", 1e-5, "f32"),
    # 1D (beyond the paper, Sec. I-B): 2^20 modes, 1e7 points
    "1d": (1, (1 << 20,), 10_000_000, "uniform", 1e-5, "f32"),
    "3d-gauss": (3, (128, 128, 128), 1 << 24, "gaussian", 1e-5, "f32"),
    # one GPU's share of the 2D workload split over 8 GPUs (points sharded, full grid)
    "2d-shard": (2, (1024, 1024), 1_250_000, "uniform", 1e-5, "f32"),
    # shapes of the application's slicing (3D type 2) and merging (3D type 1) steps,
    # Sec. V: random Ewald-sphere caps of 32^2 / 128^2 points, eps 1e-12 in fp64
    "mtip-slice": (3, (41, 41, 41), 1000 * 32 * 32, "ewald32", 1e-12, "f64"),
    "mtip-merge": (3, (81, 81, 81), 1000 * 128 * 128, "ewald128", 1e-12, "f64"),
}

# Type 3 workloads (points and frequencies both nonuniform; beyond the paper,
# Sec. I-B / Sec. VI): dim, M points uniform on [-xw, xw)^d, K frequencies
# uniform on [-sw, sw)^d, eps, precision.  sw = N/2 makes the spreading grid
# about that of a type 1 with N modes per dimension.
T3_WORKLOADS = {
    "2d-type3": (2, 10_000_000, 10_000_000, math.pi, 512.0, 1e-5, "f32"),
    "3d-type3": (3, 1 << 24, 1 << 24, math.pi, 64.0, 1e-5, "f32"),
}

# Kernel sources whose change invalidates committed hardware-counter figures.
KERNEL_SOURCES = ["paper_2102_08463_amd/csrc/spread_kernels.h"]


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(stage, dim, M, ncells, rsz):
    """Bytes one spread / interp launch must move at least: per point the
    sorted coordinates (dim reals), the permutation entry (4 B) and the
    strength or result (one complex); plus the fine grid once (one complex
    per cell, written by spreading and read by interpolation)."""
    per_pt = dim * rsz + 4 + 2 * rsz
    return M * per_pt + ncells * 2 * rsz


def load_traffic(kernel, workload):
    """Counter-measured HBM bytes per launch from profiles/, if taken on the
    current kernel source; None otherwise."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    e = d.get(f"{workload}:{kernel}")
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def load_counters(kernel, workload):
    """Counter-derived utilisation (VALU busy, LDS busy, LDS bank-conflict
    stall, occupancy) of one kernel from profiles/counters.json, if taken on
    the current kernel source; None otherwise."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    e = d.get(f"{workload}:{kernel}")
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return {k: e[k] for k in ("valu_busy", "lds_util", "lds_bank_conflict", "occupancy",
                              "valu_insts_per_cu_cycle") if k in e}


def cpu_model():
    """The host CPU's model string (first 'model name' of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(data, sample, sample_1core):
    """Time the oracle (plain FP64 three-step NUFFT: C/OpenMP spreading and
    interpolation, scipy FFT) on the first `sample` points with all host
    threads, and on the first `sample_1core` points with one thread: one
    type 1 and one type 2 each, like one GPU step."""
    from oracle import direct, nufft as onufft
    pts64, c64, f64 = data["pts64"], data["c64"], data["f64"]
    modes, eps = data["modes"], data["eps"]
    nall = direct.num_threads()

    def run(n, threads):
        direct.set_threads(threads)
        sub = tuple(a[:n] for a in pts64)
        t0 = time.perf_counter()
        onufft.type1(sub, c64[:n], modes, eps, iflag=-1, workers=threads)
        onufft.type2(sub, f64, eps, iflag=+1, workers=threads)
        return time.perf_counter() - t0

    M = len(c64)
    n = min(sample, M)
    print(f"[bench] timing the oracle on {n} points, {nall} threads", file=sys.stderr, flush=True)
    dt = run(n, nall)
    n1 = min(sample_1core, M)
    print(f"[bench] timing the oracle on {n1} points, 1 thread", file=sys.stderr, flush=True)
    dt1 = run(n1, 1)
    direct.set_threads(nall)
    model = cpu_model()
    return {"value": 2 * n / dt, "unit": "NU points/s", "cores": nall, "kind": "oracle",
            "cpu": model,
            "sample": f"first {n} of the same points ({data['workload']} workload), one type 1 + "
                      f"one type 2 (same modes and eps), FP64, {nall} threads (C loops and FFT), "
                      f"{dt:.2f} s wall",
            "one_core": {"value": 2 * n1 / dt1, "unit": "NU points/s", "cores": 1,
                         "sample": f"first {n1} of the same points, one type 1 + one type 2, "
                                   f"one thread, {dt1:.2f} s wall"}}


SELECTOR_WEIGHTS = os.path.join(ROOT, "paper_2102_08463_amd", "data", "selector_2d_f32_1e-06.bin")


def batched_speedup(kind="uniform", ntype=1, reps=3, eps=1e-6, autotune=False):
    """Batched workload: 64 2D transforms, modes uniform in {64..512}^2, M
    lognormal (median 2e5, 1e4..4e6), fp32, eps 1e-6.
      plain            one plan per transform with the library defaults,
                       setpts + execute each, in sequence
      batched_default  one Batch with the library's default bins and msub
      batched_selected one Batch with the learned selector's bins and msub
                       (mnufft_batch_select: batched density features, one
                       network pass and the argmin on the device), the
                       selection time included in its speedup
      batched_autotuned (autotune=True) one Batch with the autotuner's picks
                       per transform, its speedup given with and without the
                       search time
    Plan creation is excluded throughout."""
    import numpy as np
    import torch

    import workloads
    from paper_2102_08463_amd import Batch, Plan, lib as L

    n_modes, n_points = workloads.batch_descriptors(64)
    pts = [[torch.from_numpy(np.asarray(a, np.float32)).cuda()
            for a in workloads.points(kind, M, 2, 100 + t)] for t, M in enumerate(n_points)]
    data = [torch.from_numpy(workloads.strengths(M if ntype == 1 else nm[::-1], 200 + t)
                             .astype(np.complex64)).cuda().reshape(-1)
            for t, (M, nm) in enumerate(zip(n_points, n_modes))]
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(n):
            out = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n, out

    plans = [Plan(ntype, nm, 1, eps, None, dtype=torch.complex64) for nm in n_modes]

    def plain():
        for p, x, d in zip(plans, pts, data):
            p.setpts(*x)
            p.execute(d)
    t_plain, _ = timed(plain, reps)
    for p in plans:
        p.destroy()

    cat = [torch.cat([x[d] for x in pts]) for d in range(2)]
    dcat = torch.cat(data)

    def run_batch(binsize, msub):
        b = Batch(ntype, n_modes, n_points, eps=eps, binsize=binsize, msub=msub)

        def batched():
            b.setpts(*cat)
            b.execute(dcat)
        t, _ = timed(batched, reps)
        b.destroy()
        return t

    out = {"transforms": len(n_modes), "points": int(sum(n_points)), "kind": kind, "type": ntype,
           "plain_ms": t_plain, "batched_default_ms": run_batch(None, None)}
    out["speedup_defaults"] = t_plain / out["batched_default_ms"]
    if os.path.exists(SELECTOR_WEIGHTS):
        L.selector_load(SELECTOR_WEIGHTS)
        sel_t = []
        for _ in range(reps + 1):
            t0 = time.perf_counter()
            bins, msub, src = L.batch_select(ntype, n_modes, n_points, cat[0], cat[1], eps,
                                             mode="learned")
            sel_t.append((time.perf_counter() - t0) * 1e3)
        out["selector_ms"] = float(np.median(sel_t[1:]))
        out["selector_fallbacks"] = int(sum(src))
        out["batched_selected_ms"] = run_batch(bins, msub)
        out["speedup"] = t_plain / (out["batched_selected_ms"] + out["selector_ms"])
    else:
        out["speedup"] = out["speedup_defaults"]
    if autotune:
        t0 = time.perf_counter()
        bins, msub, _ = L.batch_select(ntype, n_modes, n_points, cat[0], cat[1], eps,
                                       mode="autotune")
        out["autotune_search_ms"] = (time.perf_counter() - t0) * 1e3
        out["batched_autotuned_ms"] = run_batch(bins, msub)
        out["speedup_autotuned"] = t_plain / out["batched_autotuned_ms"]
        out["speedup_autotuned_with_search"] = t_plain / (out["batched_autotuned_ms"] +
                                                          out["autotune_search_ms"])
    return out


def sorted_order_kernels(plan, modes, pts, c, f, eps, cdt, args, dim, M, ncells, rsz, reps=10):
    """Spreading and interpolation kernel times when the strengths / results
    are kept in bin-sorted order (mnufft_execute_sorted), with the HBM
    fraction on the same algorithmic bytes: what a caller that reuses the
    points and keeps its vectors sorted gets."""
    from paper_2102_08463_amd import Plan
    perm, _ = plan.get_sort()
    cs = c[perm.long()].contiguous()
    p2 = Plan(2, modes, 1, eps, 1, dtype=cdt, method=args.method,
              binsize=tuple(int(v) for v in args.binsize.split(",")) if args.binsize else None,
              msub=args.msub, upsampfac=args.upsampfac)
    p2.setpts(*pts)
    res = {}
    for name, pl, x, stage in (("spread", plan, cs, "spread"), ("interp", p2, f, "interp")):
        pl.execute_sorted(x)
        pl.timing(reset=True)
        pl.set_timing(True)
        for _ in range(reps):
            pl.execute_sorted(x)
        st = pl.timing(reset=True)
        pl.set_timing(False)
        ms = st[stage][0] / max(st[stage][1], 1)
        algo = algorithmic_bytes(stage, dim, M, ncells, rsz)
        res[f"{name}_ms"] = ms
        res[f"{name}_frac"] = algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
    p2.destroy()
    return res


def _short_kernel(name):
    """'void mn::detail::k_x<float, 2>(args)' -> 'k_x<float, 2>'."""
    name = name.strip().strip('"')
    if name.startswith("void "):
        name = name[5:]
    for ns in ("mn::detail::", "mn::(anonymous namespace)::", "mn::"):
        name = name.replace(ns, "")
    depth, cut = 0, len(name)
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    return name[:cut]


def _base_kernel(name):
    return _short_kernel(name).split("<")[0]


def summarize_profiles(args):
    """Turn rocprofv3 CSV output (a --kernel-trace --stats run and FETCH_SIZE /
    WRITE_SIZE --pmc runs of the same bench command, plus the two counters on
    a plain copy of known size) into a markdown summary and the calibrated
    per-launch HBM traffic that the bench line reports (profiles/traffic.json)."""
    import csv
    import glob

    def csvs(d, suffix):
        return sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))

    def counters(d):
        # keyed by the kernel name with its template arguments (one row per instantiation)
        per = {}
        for f in csvs(d, "counter_collection.csv"):
            for row in csv.DictReader(open(f)):
                per.setdefault(_short_kernel(row["Kernel_Name"]), []).append(float(row["Counter_Value"]))
        return per

    stats = []
    for f in csvs(args.stats_dir, "kernel_stats.csv"):
        for row in csv.DictReader(open(f)):
            stats.append((_short_kernel(row["Name"]), int(row["Calls"]), float(row["AverageNs"]) / 1e3,
                          float(row["Percentage"])))
    stats.sort(key=lambda r: -r[3])
    if args.workload in T3_WORKLOADS:
        dim, M, K, xw, sw, eps, prec = T3_WORKLOADS[args.workload]
        desc = (f"{dim}D type 3, M = {M} points uniform on [-{xw:g}, {xw:g})^{dim}, K = {K} "
                f"frequencies uniform on [-{sw:g}, {sw:g})^{dim}, eps = {eps:g}, {prec}; one bench "
                f"step = setpts3 + execute with the library defaults.")
    else:
        dim, modes, M, kind, eps, prec = WORKLOADS[args.workload]
        desc = (f"{dim}D, modes {'x'.join(map(str, modes))}, M = {M} {kind} points, eps = "
                f"{eps:g}, {prec}; one bench step = setpts + type 1 + type 2 (adjoint) with the "
                f"library defaults.")
    lines = [f"# {args.title}", "", f"Workload `{args.workload}`: {desc}", "",
             "## Commands (repository root, on the MI355X)", "",
             "```"] + args.command + ["```", "",
             "## Kernel statistics (rocprofv3 --kernel-trace --stats)", "",
             "| kernel | calls | avg us | share % |", "|---|---|---|---|"]
    for name, calls, avg, pct in stats[:args.top]:
        lines.append(f"| `{name}` | {calls} | {avg:.1f} | {pct:.2f} |")
    if args.sq_dir:
        lines += sq_summary(args, counters_raw(args.sq_dir), stats)
    if not args.fetch_dir or args.workload in T3_WORKLOADS:
        if args.note:
            lines += ["", args.note]
        with open(args.md_out, "w") as fh:
            fh.write("\n".join(lines) + "\n")
        print(f"wrote {args.md_out}")
        return
    fetch, write = counters(args.fetch_dir), counters(args.write_dir)
    def copy_kernel(d):
        return max(v for k, vals in counters(d).items() if _base_kernel(k) == "__amd_rocclr_copyBuffer"
                   for v in vals)
    cal_f, cal_w = copy_kernel(args.cal_fetch_dir), copy_kernel(args.cal_write_dir)
    kib = args.cal_mib * 1024.0
    ff, fw = kib / cal_f, kib / cal_w
    rsz = 4 if prec == "f32" else 8
    ncells = 1
    for n in modes:
        ncells *= 2 * n  # upsampling 2 (5-smooth sizes of these powers of two are 2N)
    lines += ["", "## HBM traffic per launch (PMC, calibrated)", "",
              f"Calibration: a {args.cal_mib} MiB device copy reads FETCH_SIZE = {cal_f:.0f} KiB and "
              f"WRITE_SIZE = {cal_w:.0f} KiB per launch, so the factors are {ff:.3f} (fetch) and "
              f"{fw:.3f} (write).", "",
              "| kernel | avg us | FETCH_SIZE KiB | WRITE_SIZE KiB | traffic MB | algorithmic MB |",
              "|---|---|---|---|---|---|"]
    avg_us = {name: avg for name, calls, avg, pct in stats}
    path = args.traffic_out or os.path.join(ROOT, "profiles", "traffic.json")
    table = json.load(open(path)) if os.path.exists(path) else {}
    for k in args.kernels.split(","):
        for full in sorted(n for n in fetch if _base_kernel(n) == k and n in write):
            fk = sum(fetch[full]) / len(fetch[full])
            wk = sum(write[full]) / len(write[full])
            traffic = (fk * ff + wk * fw) * 1024.0
            stage = "spread" if "spread" in k else ("interp" if "interp" in k else None)
            algo = algorithmic_bytes(stage, dim, M, ncells, rsz) if stage else None
            lines.append(f"| `{full}` | {avg_us.get(full, float('nan')):.1f} | {fk:.0f} | {wk:.0f} | "
                         f"{traffic / 1e6:.1f} | {'%.1f' % (algo / 1e6) if algo else '-'} |")
            if not stage:
                continue
            table[f"{args.workload}:{k}"] = {"source_hash": kernel_source_hash(),
                                            "bytes_per_launch": traffic, "fetch_kib": fk,
                                            "write_kib": wk, "cal_fetch": ff, "cal_write": fw}
    if args.note:
        lines += ["", args.note]
    with open(args.md_out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    print(f"wrote {args.md_out} and {path}")


# Counter instances summed into one value per dispatch by rocprofv3: the
# graphics-block activity counter is reported once per XCD.
XCDS = 8
CUS = 256


def counters_raw(d):
    """{kernel (with template arguments): {counter: [values per dispatch]}} from a
    --pmc run's CSV."""
    import csv
    import glob
    per = {}
    for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        for row in csv.DictReader(open(f)):
            per.setdefault(_short_kernel(row["Kernel_Name"]), {}).setdefault(
                row["Counter_Name"], []).append(float(row["Counter_Value"]))
    return per


def sq_fractions(c):
    """Utilisation of one kernel from its SQ counters (averages per dispatch):
    VALU busy = SQ_ACTIVE_INST_VALU / (CUs x cycles), LDS busy =
    SQ_LDS_IDX_ACTIVE / (CUs x cycles), bank-conflict stall =
    SQ_LDS_BANK_CONFLICT / (CUs x cycles), occupancy = resident waves over
    the 32 a CU can hold (SQ_WAVE_CYCLES counted in quad-cycles), with cycles
    the kernel's GRBM_GUI_ACTIVE of one XCD (the CSV sums the XCDs)."""
    a = {k: sum(v) / len(v) for k, v in c.items()}
    cyc = a["GRBM_GUI_ACTIVE"] / XCDS
    out = {"cycles": cyc,
           "valu_busy": a["SQ_ACTIVE_INST_VALU"] / (CUS * cyc),
           "valu_insts_per_cu_cycle": a["SQ_INSTS_VALU"] / (CUS * cyc),
           "lds_util": a["SQ_LDS_IDX_ACTIVE"] / (CUS * cyc),
           "lds_bank_conflict": a["SQ_LDS_BANK_CONFLICT"] / (CUS * cyc)}
    if "SQ_WAVE_CYCLES" in a:
        out["occupancy"] = 4.0 * a["SQ_WAVE_CYCLES"] / (cyc * CUS * 32)
    return out


def sq_summary(args, raw, stats):
    """Markdown rows of the SQ fractions per kernel; records them in the
    counters table (profiles/counters.json) for the spread / interp kernels."""
    lines = ["", "## Utilisation from SQ counters (rocprofv3 --pmc)", "",
             "Fractions of the kernel's active cycles (GRBM_GUI_ACTIVE of one XCD) summed "
             "over the 256 CUs: VALU busy (SQ_ACTIVE_INST_VALU), VALU wave-instructions "
             "issued per CU and cycle (one is the issue limit), LDS busy (SQ_LDS_IDX_ACTIVE), "
             "cycles the LDS stalled on bank conflicts (SQ_LDS_BANK_CONFLICT), and occupancy "
             "(resident waves / 32 per CU, from SQ_WAVE_CYCLES).", "",
             "| kernel | VALU busy | VALU insts / CU / cycle | LDS busy | LDS bank-conflict "
             "stall | occupancy |", "|---|---|---|---|---|---|"]
    path = args.counters_out or os.path.join(ROOT, "profiles", "counters.json")
    table = json.load(open(path)) if os.path.exists(path) else {}
    extra = ["k_tile_sum", "k_tile_gather2", "k_radix_scatter", "k_binkey"]
    for k in dict.fromkeys(args.kernels.split(",") + extra):
        fulls = sorted(n for n in raw if _base_kernel(n) == k and "GRBM_GUI_ACTIVE" in raw[n])
        if not fulls:
            continue
        if k == "k_radix_scatter":  # one row over its passes
            merged = {}
            for n in fulls:
                for cn, vals in raw[n].items():
                    merged.setdefault(cn, []).extend(vals)
            rows = [(k, merged)]
        else:
            rows = [(n if len(fulls) > 1 else k, raw[n]) for n in fulls]
        for label, c in rows:
            fr = sq_fractions(c)
            lines.append(f"| `{label}` | {fr['valu_busy']:.2f} | {fr['valu_insts_per_cu_cycle']:.2f} | "
                         f"{fr['lds_util']:.2f} | {fr['lds_bank_conflict']:.2f} | "
                         f"{fr.get('occupancy', float('nan')):.2f} |")
            if ("spread" in k or "interp" in k) and len(fulls) == 1:
                table[f"{args.workload}:{k}"] = dict(fr, source_hash=kernel_source_hash())
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    return lines


def summarize_sweep(args):
    """Markdown table of bench JSON lines (one per run)."""
    rows = [json.loads(l) for l in open(args.sweep) if l.strip()]
    names = {1: "GM", 2: "GM-sort", 3: "SM"}
    lines = [f"# {args.title}", "", "```"] + args.command + ["```", "",
             "| points | dim | eps | dtype | w | method | bins | NU pts/s per step | exec type 1 | "
             "exec type 2 | setpts ms | spread ms | add-back ms | interp ms | FFT ms (both) |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for d in rows:
        c, st = d["config"], d["stage_ms_per_step"]
        lines.append(
            f"| {c['points']} | {c['dim']} | {c['eps']:g} | {d['dtype']} | {c['w']} | "
            f"{names.get(c['method'], c['method'])} | {'x'.join(map(str, c['binsize']))} | "
            f"{d['value']:.3g} | {d['exec_pts_per_s']['type1']:.3g} | {d['exec_pts_per_s']['type2']:.3g} | "
            f"{st['setpts']:.3f} | {st['spread']:.3f} | {st['addback']:.3f} | {st['interp']:.3f} | "
            f"{st['fft']:.3f} |")
    if args.note:
        lines += ["", args.note]
    with open(args.md_out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {args.md_out}")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="2d", choices=sorted(WORKLOADS) + sorted(T3_WORKLOADS))
    ap.add_argument("--method", default="auto")
    ap.add_argument("--binsize", default=None, help="comma-separated bin extents")
    ap.add_argument("--msub", type=int, default=0)
    ap.add_argument("--upsampfac", type=float, default=0.0,
                    help="fine-grid upsampling factor sigma (0 = 2)")
    ap.add_argument("--eps", type=float, default=0.0,
                    help="override the workload's tolerance (fp32 down to 1e-6, fp64 below)")
    ap.add_argument("--cpu-sample", type=int, default=10_000_000,
                    help="points the oracle is timed on (capped at M); 1e7 is about 20-30 "
                         "CPU-seconds on 16 host threads")
    ap.add_argument("--cpu-sample-1core", type=int, default=1_000_000,
                    help="points the oracle is timed on with one thread")
    ap.add_argument("--no-3d", action="store_true",
                    help="leave the 3D entry out of the default 2D line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-vs-plain speedup measurement")
    ap.add_argument("--no-sorted", action="store_true",
                    help="skip the sorted-order kernel measurement (profiling runs, so that "
                         "every spread / interp launch is of the timed kind)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (reference for HBM counters)")
    ap.add_argument("--summarize-profiles", action="store_true",
                    help="only summarize rocprofv3 CSV output (see --stats-dir etc.)")
    ap.add_argument("--stats-dir")
    ap.add_argument("--fetch-dir")
    ap.add_argument("--write-dir")
    ap.add_argument("--cal-fetch-dir")
    ap.add_argument("--cal-write-dir")
    ap.add_argument("--cal-mib", type=int, default=256)
    ap.add_argument("--sq-dir", help="rocprofv3 --pmc output with the SQ / GRBM counters")
    ap.add_argument("--counters-out", default=None,
                    help="counter table to update (default profiles/counters.json)")
    ap.add_argument("--kernels", default="k_spread_smp,k_interp_sm")
    ap.add_argument("--md-out")
    ap.add_argument("--traffic-out", default=None,
                    help="per-launch traffic table to update (default profiles/traffic.json)")
    ap.add_argument("--title", default="Kernel times and HBM traffic (MI355X)")
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--note", default="")
    ap.add_argument("--top", type=int, default=16)
    ap.add_argument("--summarize-sweep", dest="sweep", default=None, metavar="JSONL",
                    help="only tabulate bench JSON lines from JSONL into --md-out")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args)
        return
    if args.sweep:
        summarize_sweep(args)
        return
    if args.copy_calibration:
        import torch
        src = torch.ones(args.copy_calibration * (1 << 18), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library "
              f"has no multi-GPU path (sharding over GPUs is a design only).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_2102_08463_amd import Plan, lib

    if not os.path.exists(lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()

    if args.workload in T3_WORKLOADS:
        return bench_type3(args)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    res, data = measure(args, args.workload, dev)
    out = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "NU points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": res["dtype"],
        "data": "synthetic",
    }
    out.update({k: v for k, v in res.items() if k not in ("value", "ms_per_step", "dtype")})
    if args.workload == "2d" and args.eps <= 0 and not args.no_3d:
        # the metric covers 2D and 3D: the 3D workload (128^3 modes, M = 2^24
        # uniform points, eps 1e-5, fp32) as a second keyed entry
        res3, _ = measure(args, "3d", dev, sorted_order=False)
        out["3d"] = dict(res3, steps=args.steps, warmup=args.warmup)
    if not args.no_batched:
        print("[bench] batched vs plain (64 transforms)", file=sys.stderr, flush=True)
        runs = [batched_speedup(kind, ntype, autotune=(k == 0)) for k, (kind, ntype) in
                enumerate((("uniform", 1), ("cluster", 1), ("radial", 1), ("uniform", 2)))]
        out["batched_speedup"] = dict(runs[0], others=runs[1:])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(data, args.cpu_sample, args.cpu_sample_1core)
    print(json.dumps(out), flush=True)


def measure(args, workload, dev, sorted_order=True):
    """One workload: W warm-up and K timed steps of setpts + type 1 + type 2
    (adjoint) on the same points, with the library's stage timers on the
    plan's stream.  Returns (result dict, host copies of the inputs)."""
    import numpy as np
    import torch

    import workloads
    from paper_2102_08463_amd import Plan

    dim, modes, M, kind, eps, prec = WORKLOADS[workload]
    if args.eps > 0:
        eps, prec = args.eps, ("f32" if args.eps >= 1e-6 else "f64")
    rdt = np.float32 if prec == "f32" else np.float64
    cdt = torch.complex64 if prec == "f32" else torch.complex128
    print(f"[bench] workload {workload}: dim={dim} modes={modes} M={M} {kind} "
          f"eps={eps} {prec}", file=sys.stderr, flush=True)
    pts_np = [np.asarray(a, dtype=rdt) for a in workloads.points(kind, M, dim, seed=0)]
    c_np = workloads.strengths(M, seed=1).astype(np.complex64 if prec == "f32" else np.complex128)
    f_np = workloads.strengths(tuple(modes[::-1]), seed=2).astype(c_np.dtype)
    pts = [torch.from_numpy(a).to(dev) for a in pts_np]
    c = torch.from_numpy(c_np).to(dev)
    f = torch.from_numpy(f_np).to(dev)

    binsize = tuple(int(v) for v in args.binsize.split(",")) if args.binsize else None
    plan = Plan(1, modes, 1, eps, -1, dtype=cdt, method=args.method, binsize=binsize,
                msub=args.msub, device=dev, upsampfac=args.upsampfac)
    info = plan.info()

    def step():
        plan.setpts(*pts)
        plan.execute(c)
        plan.execute_adjoint(f)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.timing(reset=True)
    plan.set_timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    stages = plan.timing(reset=True)
    plan.set_timing(False)
    K = args.steps
    value = 2.0 * M * K / (total_ms * 1e-3)

    rsz = 4 if prec == "f32" else 8
    ncells = int(np.prod(info["nfine"][:dim]))
    kern_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}
    per_step = {k: v[0] / K for k, v in stages.items()}
    setpts_ms = per_step["setpts"]
    t1_ms = (per_step["zero"] + per_step["scale"] + per_step["spread"] + per_step["addback"]
             + per_step["deconv"] + per_step["fft"] / 2)
    t2_ms = per_step["precorrect"] + per_step["interp"] + per_step["fft"] / 2
    dominant = max(("spread", "interp"), key=lambda k: stages[k][0])
    algo = algorithmic_bytes(dominant, dim, M, ncells, rsz)
    achieved = algo / (kern_ms[dominant] * 1e-3) / 1e9
    sm_spread = "k_spread_smp" if prec == "f32" and dim >= 2 else "k_spread_sm"
    names = {"spread": sm_spread if info["method"] == 3 else "k_spread_gm",
             "interp": "k_interp_sm" if info["method"] == 3 else "k_interp_gm"}
    default_shape = args.eps <= 0 and args.upsampfac in (0.0, 2.0) and not args.binsize \
        and not args.msub and args.method == "auto"

    def roof(stage):
        a = algorithmic_bytes(stage, dim, M, ncells, rsz)
        ach = a / (kern_ms[stage] * 1e-3) / 1e9
        r = {"bound": "hbm", "kernel": names[stage], "achieved": ach, "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
             "traffic": load_traffic(names[stage], workload) if default_shape else None,
             "algorithmic_bytes_per_launch": a, "avg_launch_ms": kern_ms[stage]}
        cnt = load_counters(names[stage], workload) if default_shape else None
        if cnt:
            # fractions of the other two ceilings, from hardware counters of
            # the same kernel source (profiles/counters.json)
            r["fractions"] = {"hbm": ach / HBM_PEAK_GBS, "valu": cnt["valu_busy"],
                              "lds": cnt["lds_util"]}
            r["counters"] = cnt
        return r

    res = {
        "value": value,
        "ms_per_step": total_ms / K,
        "dtype": prec,
        "config": {
            "workload": f"{dim}D type 1 + type 2 per step (setpts, execute, adjoint), "
                        f"modes {'x'.join(map(str, modes))}, M={M} {kind} points, "
                        f"eps={eps:g}, {prec}",
            "dim": dim, "modes": list(modes), "M": M, "points": kind, "eps": eps,
            "w": info["w"], "fine_grid": info["nfine"][:dim], "method": info["method"],
            "binsize": info["binsize"][:dim], "msub": info["msub"],
            "upsampfac": info["upsampfac"],
        },
        "roofline": roof(dominant),
        "roofline_other": roof("interp" if dominant == "spread" else "spread"),
        "stage_ms_per_step": per_step,
        "exec_pts_per_s": {"type1": M / (t1_ms * 1e-3), "type2": M / (t2_ms * 1e-3)},
        "total_pts_per_s": {"type1": M / ((setpts_ms + t1_ms) * 1e-3),
                            "type2": M / ((setpts_ms + t2_ms) * 1e-3)},
    }
    if sorted_order and info["method"] == 3 and not args.no_sorted:
        res["sorted_order"] = sorted_order_kernels(plan, modes, pts, c, f, eps, cdt, args,
                                                   dim, M, ncells, rsz)
    plan.destroy()
    data = {"pts64": tuple(a.astype(np.float64) for a in pts_np),
            "c64": c_np.astype(np.complex128), "f64": f_np.astype(np.complex128),
            "modes": modes, "eps": eps, "workload": workload}
    return res, data


def bench_type3(args):
    """One step = setpts3 + execute of a type 3 plan; value = (M + K) / step
    time (both sets are nonuniform points).  The roofline line covers the
    longer of the spreading kernel (on the nf grid) and the interpolation
    kernel (on the inner type 2's fine grid)."""
    import numpy as np
    import torch

    import workloads
    from paper_2102_08463_amd import Plan

    dim, M, K, xw, sw, eps, prec = T3_WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rdt = np.float32 if prec == "f32" else np.float64
    cdt = torch.complex64 if prec == "f32" else torch.complex128
    print(f"[bench] workload {args.workload}: dim={dim} M={M} K={K} eps={eps} {prec}",
          file=sys.stderr, flush=True)
    x_np, s_np = workloads.type3_sets(M, K, dim, seed=0, xw=xw, sw=sw)
    x_np = [np.asarray(a, dtype=rdt) for a in x_np]
    s_np = [np.asarray(a, dtype=rdt) for a in s_np]
    c_np = workloads.strengths(M, seed=1).astype(np.complex64 if prec == "f32" else np.complex128)
    xs = [torch.from_numpy(a).to(dev) for a in x_np]
    ss = [torch.from_numpy(a).to(dev) for a in s_np]
    c = torch.from_numpy(c_np).to(dev)
    plan = Plan(3, dim, 1, eps, -1, dtype=cdt, method=args.method, msub=args.msub, device=dev,
                upsampfac=args.upsampfac)
    pad = [None] * (3 - dim)

    def step():
        plan.setpts(*xs, *pad, *ss)
        plan.execute(c)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.timing(reset=True)
    plan.set_timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    stages = plan.timing(reset=True)
    plan.set_timing(False)
    info = plan.info()
    steps = args.steps
    rsz = 4 if prec == "f32" else 8
    kern_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}
    dominant = max(("spread", "interp"), key=lambda k: stages[k][0])
    ncells = int(np.prod(info["nmodes"][:dim] if dominant == "spread" else info["nfine"][:dim]))
    algo = algorithmic_bytes(dominant, dim, M if dominant == "spread" else K, ncells, rsz)
    achieved = algo / (kern_ms[dominant] * 1e-3) / 1e9
    kernel_name = {"spread": "k_spread_smp" if prec == "f32" else "k_spread_sm",
                   "interp": "k_interp_sm"}[dominant]
    out = {
        "metric": "type 3 nonuniform points (M + K) per second",
        "value": (M + K) * steps / (total_ms * 1e-3),
        "unit": "NU points/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": total_ms / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {
            "workload": f"{dim}D type 3 per step (setpts3, execute), M={M} points uniform on "
                        f"[-{xw:g}, {xw:g})^{dim}, K={K} frequencies uniform on "
                        f"[-{sw:g}, {sw:g})^{dim}, eps={eps:g}, {prec}",
            "dim": dim, "M": M, "K": K, "eps": eps, "w": info["w"],
            "spread_grid": info["nmodes"][:dim], "inner_fine_grid": info["nfine"][:dim],
            "method": info["method"], "binsize": info["binsize"][:dim],
            "upsampfac": info["upsampfac"],
        },
        "roofline": {
            "bound": "hbm", "kernel": kernel_name, "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": None, "algorithmic_bytes_per_launch": algo,
            "avg_launch_ms": kern_ms[dominant],
        },
        "stage_ms_per_step": {k: v[0] / steps for k, v in stages.items()},
    }
    if not args.no_cpu_baseline:
        from oracle import direct, nufft as onufft
        # 3D: the oracle's FP64 fine grid alone is a few GB; 2e6 points keep the
        # sample near 20 CPU-seconds
        n = min(args.cpu_sample, M, K, 2_000_000 if dim == 3 else M)
        print(f"[bench] timing the oracle on {n} points and {n} frequencies", file=sys.stderr,
              flush=True)
        x64 = tuple(a[:n].astype(np.float64) for a in x_np)
        s64 = tuple(a[:n].astype(np.float64) for a in s_np)
        t0 = time.perf_counter()
        onufft.type3(x64, c_np[:n].astype(np.complex128), s64, eps, iflag=-1)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 2 * n / dt, "unit": "NU points/s",
                               "cores": direct.num_threads(), "kind": "oracle",
                               "sample": f"first {n} points and {n} frequencies of the same "
                                         f"sets, one type 3, FP64, {dt:.2f} s wall"}
    plan.destroy()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
