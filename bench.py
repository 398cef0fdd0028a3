"""Benchmark: BiCGStab cell-iterations/s and HBM-roofline fraction on one
MI355X, with p50/p99 solve latency of a served request stream.

Default workload (headline): one backward-Euler step of pure diffusion on a
512 x 512 x 1024 grid (268M cells) in FP32, smooth 8-mode per-cell
diffusivity in [0.5, 2], dt 1, Dirichlet 0 on every face, exactly 500
BiCGStab iterations (two-reduction organisation, shadow residual hashed from
the cell index; paper_2209_13768_amd.inputs.poisson_large).  A "step" is
that whole solve (right-hand side, initial residual, 500 iterations, FP64
true residual) restarted from the same T0, so that every step does the same
work.

Prints one JSON line:
  value      cells x iterations / seconds over all K timed steps (HIP events
             on the solve stream around the K steps; inputs resident in HBM);
  roofline   the dominant kernel's algorithmic bytes per launch over its mean
             duration, from HIP events around every 8th launch of each kernel
             inside the same timed steps; traffic = HBM bytes per launch from rocprofv3
             counters (profiles/) when taken from the current kernel
             sources, else null;
  t_eff      the paper's effective-bandwidth figure (section 3.1.3):
             A_eff = 2 D_u + D_k over the step time;
  oracle     the error against the FP64 oracle (after 10 iterations, the
             same method) and the oracle-evaluated true residual at exit;
  compare    the 256^3 FP64 convection-diffusion time integration (50 steps
             to 1e-8), the 32^3 heat workload (10 steps), the 384^3 FP32-in-
             FP64 refinement against plain FP64 (to 1e-10), CG with one
             reduction on the headline grid, each with its error against the
             oracle;
  solve_latency_ms  p50/p99 of the 2000-request serving stream (200/s, grids
             32..192 per axis, FP32 in FP64 refinement to 1e-10);
  cpu_baseline  the FP64 oracle timed on this host: 10 iterations of the
             headline solve on every core, and 1 iteration on one core.

Other workloads (--workload): convdiff (256^3 time steps, the round-one
headline), heat32, poisson_large (headline grid, other methods), mixed384,
serve, explicit, apply, ceilings (HBM copy ceilings).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILES = {
    "headline": os.path.join(ROOT, "profiles", "traffic_poisson512x512x1024_f32.json"),
    "convdiff": os.path.join(ROOT, "profiles", "traffic_convdiff256_f64.json"),
}
HEADLINE_ITERS = 500
HEADLINE_TIME_EVERY = 8   # the timed steps time one launch in 8 of each kernel


# The files that define the single-grid solver kernels and their launch
# shapes: counter figures taken from other sources are stale.
# sources of the stencil passes, and of the copy that calibrates the counters
KERNEL_SOURCES = ("device.hpp", "phases.hpp", "kernels.hip", "probes.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2209_13768_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def library_source_hash() -> str:
    """Hash of every HIP source of the library (any kernel or launch change)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2209_13768_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode())
                h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str = "convdiff"):
    """HBM bytes per launch of `kernel` from the committed counter summary of
    `workload`, if it was taken from the current kernel sources."""
    try:
        with open(TRAFFIC_FILES[workload]) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


# rocprofv3 kernel names -> the names bench.py and the library's kernel
# statistics use
KERNEL_PATTERNS = (("PhAC<", "phase_ac"), ("k_phase_act<", "phase_ac"), ("PhB2<", "phase_b2"),
                   ("PhA<", "phase_a"),
                   ("PhB<", "phase_b"), ("k_phase_c<", "phase_c"), ("PhInit<", "init"),
                   ("PhResid<", "residual"), ("PhCgA<", "cg_a"), ("k_cg_b<", "cg_b"),
                   ("PhCg1<", "cg1"),
                   ("PhExplicit<", "explicit"), ("PhApply<", "apply"), ("k_copy", "copy"))
COPY_PROBE_BYTES = 1 << 30   # --probe-copy: one copy of this many bytes (read and written)


def kernel_label(name: str):
    for pat, label in KERNEL_PATTERNS:
        if pat in name:
            return label
    return None


def counter_means(csv_path: str, counter: str):
    """Mean value of `counter` per working dispatch, by kernel label, from a
    rocprofv3 --pmc counter_collection.csv.  An iteration pass queued past
    convergence exits at its first instruction; its dispatches (under a
    fifth of the kernel's 90th-percentile value) are left out."""
    import csv
    per = {}
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] != counter:
                continue
            label = kernel_label(row["Kernel_Name"])
            if label is None:
                continue
            d = per.setdefault(label, {})
            did = row["Dispatch_Id"]
            d[did] = d.get(did, 0.0) + float(row["Counter_Value"])
    out = {}
    for k, v in per.items():
        vals = sorted(v.values())
        cut = 0.2 * vals[int(0.9 * (len(vals) - 1))]
        w = [x for x in vals if x >= cut]
        out[k] = (sum(w) / len(w), len(w))
    return out


def summarize_counters(fetch_csv: str, write_csv: str, workload: str, commands: list):
    """HBM bytes per launch of each kernel from two counter runs (FETCH_SIZE,
    WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads
    for the --probe-copy dispatch of known size.  Writes the traffic file
    the roofline line reads."""
    fetch = counter_means(fetch_csv, "FETCH_SIZE")
    write = counter_means(write_csv, "WRITE_SIZE")
    if "copy" not in fetch or "copy" not in write:
        raise SystemExit("the counter runs need the --probe-copy dispatch for calibration")
    f_fetch = COPY_PROBE_BYTES / (fetch["copy"][0] * 1024.0)
    f_write = COPY_PROBE_BYTES / (write["copy"][0] * 1024.0)
    kernels = {}
    for k in sorted(set(fetch) & set(write)):
        if k == "copy":
            continue
        fk, n = fetch[k]
        wk, _ = write[k]
        kernels[k] = {"dispatches": n, "fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
                      "hbm_bytes_per_launch": round(fk * 1024.0 * f_fetch + wk * 1024.0 * f_write)}
    out = {"source_hash": kernel_source_hash(), "workload": workload, "commands": commands,
           "copy_calibration": {"bytes_each_way": COPY_PROBE_BYTES,
                                "fetch_kib": round(fetch["copy"][0], 1),
                                "write_kib": round(write["copy"][0], 1),
                                "fetch_factor": round(f_fetch, 4), "write_factor": round(f_write, 4)},
           "kernels": kernels}
    with open(TRAFFIC_FILES[workload], "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    return out


def summarize_pmc(csvs: list, title: str, commands: list) -> str:
    """Markdown table of the mean of every counter per working dispatch, by
    kernel, from rocprofv3 --pmc counter_collection.csv files (one counter
    set per file)."""
    import csv
    names, per = [], {}
    for path in csvs:
        with open(path) as f:
            for row in csv.DictReader(f):
                c = row["Counter_Name"]
                if c not in names:
                    names.append(c)
        for c in names:
            for k, (mean, n) in counter_means(path, c).items():
                per.setdefault(k, {})[c] = (mean, n)
    lines = [f"# {title}", "", "Commands (run from the repository root on one MI355X):", "",
             "```", *commands, "```", "",
             f"Kernel sources hash (bench.kernel_source_hash): `{kernel_source_hash()}`", "",
             "Mean per working dispatch (dispatches under a fifth of the kernel's 90th "
             "percentile, passes skipped after the solve stopped, left out).", "",
             "| counter | " + " | ".join(sorted(per)) + " |",
             "|---|" + "---:|" * len(per)]
    for c in names:
        row = [f"{per[k][c][0]:.4g}" if c in per[k] else "" for k in sorted(per)]
        lines.append(f"| {c} | " + " | ".join(row) + " |")
    return "\n".join(lines) + "\n"


def summarize_trace(stats_csv: str, title: str, command: str) -> str:
    """Markdown table of a rocprofv3 --kernel-trace --stats kernel_stats.csv.
    With the run's kernel_trace.csv beside it, also the calls and average of
    the working launches: an iteration pass queued past convergence exits at
    its first instruction, and such launches (under a fifth of the kernel's
    90th-percentile duration) are left out of those two columns."""
    import csv
    import re
    trace_csv = stats_csv.replace("kernel_stats", "kernel_trace")
    durs = {}
    spans = []
    if trace_csv != stats_csv and os.path.exists(trace_csv):
        with open(trace_csv) as f:
            for r in csv.DictReader(f):
                t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
                durs.setdefault(r["Kernel_Name"], []).append((t1 - t0) / 1e3)
                spans.append((t0, t1))
    head = "| kernel | calls | total (us) | average (us) | % |"
    rule = "|---|---:|---:|---:|---:|"
    if durs:
        head += " working calls | working average (us) |"
        rule += "---:|---:|"
    lines = [f"# {title}", "", "Command (run from the repository root on one MI355X):", "",
             "```", command, "```", "",
             f"Kernel sources hash (bench.kernel_source_hash): `{kernel_source_hash()}`; "
             f"library sources hash (bench.library_source_hash): `{library_source_hash()}`", "",
             head, rule]
    with open(stats_csv) as f:
        for r in csv.DictReader(f):
            if float(r["Percentage"]) < 0.01:
                continue
            name = re.sub(r"wfa::|\(anonymous namespace\)::", "", r["Name"])
            m = re.match(r"void (\w+)<([^(]*)>\(", name)
            short = f"{m.group(1)}<{m.group(2)}>" if m else name.split("(")[0][:80]
            row = (f"| `{short}` | {int(r['Calls'])} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
            if durs:
                d = durs.get(r["Name"], []) if "wfa::" in r["Name"] else []
                if d:
                    cut = 0.2 * sorted(d)[int(0.9 * (len(d) - 1))]
                    w = [x for x in d if x >= cut]
                    row += f" {len(w)} | {sum(w) / len(w):.2f} |"
                else:
                    row += " | |"
            lines.append(row)
    if spans:
        busy, gaps = gpu_busy(spans)
        lines += ["", f"GPU busy {100 * busy:.1f}% of the span from the first kernel to the last "
                      f"(union of kernel intervals); median idle gap "
                      f"{gaps['median_us']:.1f} us; {gaps['over_20us']} gaps over 20 us, "
                      f"{gaps['over_20us_total_ms']:.1f} ms in all, of which {gaps['over_1ms']} "
                      f"over 1 ms ({gaps['over_1ms_total_ms']:.1f} ms); busy "
                      f"{100 * gaps['busy_without_over_1ms']:.1f}% of the span less those."]
    return "\n".join(lines) + "\n"


def gpu_busy(spans):
    """Fraction of [first start, last end] covered by the union of the
    (start, end) kernel intervals (ns), and the gaps between them."""
    spans = sorted(spans)
    merged = []
    for a, b in spans:
        if merged and a <= merged[-1][1]:
            merged[-1][1] = max(merged[-1][1], b)
        else:
            merged.append([a, b])
    total = merged[-1][1] - merged[0][0]
    covered = sum(b - a for a, b in merged)
    gaps = [(merged[q + 1][0] - merged[q][1]) / 1e3 for q in range(len(merged) - 1)]
    big = [g for g in gaps if g > 20.0]
    idle = [g for g in gaps if g > 1000.0]   # over 1 ms: no kernel queued at all
    rest = total - sum(idle) * 1e3
    return covered / total if total > 0 else 1.0, {
        "median_us": sorted(gaps)[len(gaps) // 2] if gaps else 0.0,
        "over_20us": len(big), "over_20us_total_ms": sum(big) / 1e3,
        "over_1ms": len(idle), "over_1ms_total_ms": sum(idle) / 1e3,
        "busy_without_over_1ms": covered / rest if rest > 0 else 1.0}


def cpu_baseline(prob, iters: int):
    """FP64 oracle (test infrastructure) on a bounded sample: `iters`
    BiCGStab iterations of the first step of the same workload."""
    import oracle
    o = oracle.Oracle(prob)
    b = o.rhs(prob.T0)
    t0 = time.perf_counter()
    _, info = o.bicgstab(b, prob.T0, 1e-300, iters)
    dt = time.perf_counter() - t0
    return {
        "value": prob.cells * info.iterations / dt,
        "unit": "cell-iters/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"first step, {info.iterations} BiCGStab iterations at "
                  f"{prob.nx}x{prob.ny}x{prob.nz} (includes the initial and final residual "
                  f"products), {dt:.1f} s",
    }


def percentile(vals, q):
    v = sorted(vals)
    if not v:
        return None
    return v[min(len(v) - 1, int(round(q / 100 * (len(v) - 1))))]


def run_convdiff(args, torch, inputs, wfa):
    """The headline workload: 256^3 convection-diffusion time steps."""
    if args.method in ("cg", "cg1"):
        raise SystemExit("CG needs a symmetric operator; the convection-diffusion workload is not")
    prob = inputs.convdiff(n=args.n)
    prec = wfa.PRECISIONS[args.precision]
    g = wfa.Grid.from_problem(prob, precision=prec)
    g.set_option(wfa.OPT_METHOD, METHODS[args.method])
    g.set_option(wfa.OPT_SHADOW, 1 if args.shadow == "hashed" else 0)
    T0 = g.field(prob.T0)
    T = g.field(prob.T0)
    stream = torch.cuda.current_stream()

    # warmup: the first steps of the time integration
    for _ in range(args.warmup):
        g.timestep(T, 1, tol=args.tol, maxit=args.maxit, check=False)
    T.copy_(T0)
    torch.cuda.synchronize()

    # the timed steps: plain launches, no per-launch events
    g.set_option(wfa.OPT_PROFILE, 0)
    infos = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    step_ms = []
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        s0 = time.perf_counter()
        infos += g.timestep(T, 1, tol=args.tol, maxit=args.maxit, check=False)
        step_ms.append((time.perf_counter() - s0) * 1e3)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    iters = sum(i.iterations for i in infos)
    value = prob.cells * iters / (total_ms * 1e-3)

    # the same steps again with HIP events around every launch (on the
    # solve stream) for the per-kernel durations of the roofline
    profile = not args.no_profile
    roofline = None
    kernels = {}
    if profile:
        T.copy_(T0)
        for _ in range(args.warmup):
            g.timestep(T, 1, tol=args.tol, maxit=args.maxit, check=False)
        T.copy_(T0)
        g.set_option(wfa.OPT_PROFILE, 1)
        for k in range(wfa.K_COUNT):
            g.kernel_stats(k, reset=True)
        # the repeat retraces the timed steps (same field, deterministic
        # kernels), so each step's iteration count is known: one chunk of
        # exactly that many iterations per step leaves no pass that exits at
        # once after convergence to dilute the per-launch averages (only the
        # converged iteration's second pass)
        pinfos = []
        for k in range(args.steps):
            # refinement reports only the total over its inner solves: there,
            # one iteration per chunk (a host check after every iteration)
            chunk = 1 if prec == wfa.F32_IR64 else infos[k].iterations + 1
            g.set_option(wfa.OPT_CHECK_EVERY, chunk)
            pinfos += g.timestep(T, 1, tol=args.tol, maxit=args.maxit, check=False)
        g.set_option(wfa.OPT_CHECK_EVERY, 0)
        torch.cuda.synchronize()
        g.set_option(wfa.OPT_PROFILE, 0)
        retraced = [i.iterations for i in pinfos] == [i.iterations for i in infos]
        for k, name in enumerate(wfa.KERNEL_NAMES):
            n, ms, by = g.kernel_stats(k)
            if n:
                kernels[name] = {"launches": n, "ms_total": round(ms, 3), "us_avg": round(ms / n * 1e3, 2),
                                 "alg_bytes_per_launch": by,
                                 "gbps": round(by / (ms / n * 1e-3) / 1e9, 1)}
        dom = max(kernels, key=lambda k: kernels[k]["ms_total"])
        kd = kernels[dom]
        achieved = kd["gbps"]
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 4),
                    "traffic": load_traffic(dom),
                    "measured": "HIP events around every launch on the solve stream, over "
                                "the timed steps repeated from the same initial field, one "
                                "chunk of the step's iteration count per step",
                    "repeat_matches_timed_iterations": retraced}
        # the measured reference: a 1 GiB device-to-device copy (one read and
        # one write stream) on the same GPU
        copy = wfa.stream_probe(COPY_PROBE_BYTES, 10)
        roofline["copy_gbps"] = round(copy, 1)
        roofline["frac_of_copy"] = round(achieved / copy, 4)
    # vector width of the counted iterations: FP32 for the refinement's inner
    # solve too (its few FP64 residual passes are left out of this figure)
    w = 8 if prec == wfa.F64 else 4
    streams = streams_of(args)
    alg_bytes_iter = (streams * w + 2 * 4) * prob.cells   # vector streams + 2 kappa reads
    whole = alg_bytes_iter * iters / (total_ms * 1e-3) / 1e9
    line = {
        "metric": "BiCGStab cell-iters/s and % HBM roofline on 1 MI355X; p50/p99 solve latency",
        "value": value,
        "unit": "cell-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f32_ir64": "f32+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"convdiff_{args.n}^3_{args.precision}", "grid": [args.n] * 3,
                   "precision": args.precision, "tol": args.tol, "method": args.method,
                   "shadow": args.shadow if args.method == "bicgstab2" else "r0",
                   "physics": "lognormal kappa, u=(1,0.5,0.25) upwind, dt=1e-2, mixed BC"},
        "iterations_per_step": iters / args.steps,
        "solve_latency_ms": {"p50": percentile(step_ms, 50), "p99": percentile(step_ms, 99)},
        "alg_bytes_per_cell_iter": streams * w + 8,
        "whole_step_gbps": round(whole, 1),
        "whole_step_frac": round(whole / HBM_PEAK_GBPS, 4),
        "roofline": roofline,
        "kernels": kernels,
        "rel_res_true_max": max(i.rel_res_true for i in infos),
        "kernel_source_hash": kernel_source_hash(),
    }
    if args.compare:
        # the other organisations on the same steps, for comparison (plain
        # launches, wall clock around the synchronised steps)
        # organisations, and the Jacobi-scaled form of the benchmark's one:
        # the same cost per iteration, far fewer iterations on this
        # diffusivity field (time to solution, not the iteration rate)
        others = [("bicgstab2", "r0", 0), ("bicgstab", "r0", 0), ("bicgstab2", "hashed", 1)]
        line["compare"] = {}
        for method, shadow, jac in others:
            if (method, shadow, jac) == (args.method, args.shadow if args.method == "bicgstab2" else "r0", 0):
                continue
            g.set_option(wfa.OPT_METHOD, METHODS[method])
            g.set_option(wfa.OPT_SHADOW, 1 if shadow == "hashed" else 0)
            g.set_option(wfa.OPT_JACOBI, jac)
            T.copy_(T0)
            for _ in range(args.warmup):
                g.timestep(T, 1, tol=args.tol, maxit=args.maxit, check=False)
            T.copy_(T0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tinfos = []
            for _ in range(args.steps):
                tinfos += g.timestep(T, 1, tol=args.tol, maxit=args.maxit, check=False)
            torch.cuda.synchronize()
            tdt = time.perf_counter() - t0
            tit = sum(i.iterations for i in tinfos)
            streams = STREAMS[method] - (2 if (method, shadow) == ("bicgstab2", "hashed") else 0)
            line["compare"][f"{method}_{shadow}" + ("_jacobi" if jac else "")] = {
                "value": prob.cells * tit / tdt, "ms_per_step": tdt / args.steps * 1e3,
                "iterations_per_step": tit / args.steps,
                "alg_bytes_per_cell_iter": streams * w + 8,
                "rel_res_true_max": max(i.rel_res_true for i in tinfos)}
        g.set_option(wfa.OPT_JACOBI, 0)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_iters)
    return line


def run_heat32(args, torch, inputs, wfa):
    """32^3 heat diffusion, FP64, 10 steps to 1e-10: a latency-bound grid."""
    prob = inputs.heat_32()
    g = wfa.Grid.from_problem(prob, precision=wfa.F64)
    g.set_option(wfa.OPT_METHOD, METHODS[args.method])
    T = g.field(prob.T0)
    g.timestep(T, 2, tol=1e-10, maxit=1000)
    T = g.field(prob.T0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = g.timestep(T, 10, tol=1e-10, maxit=1000)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = sum(i.iterations for i in infos)
    out = {"workload": "heat_32^3_f64_10steps", "method": args.method, "seconds": dt,
           "ms_per_step": dt / 10 * 1e3, "us_per_iteration": dt / iters * 1e6,
           "iterations": iters, "cell_iters_per_s": prob.cells * iters / dt,
           "rel_res_true_max": max(i.rel_res_true for i in infos)}
    # the same steps on the tile shape the autotuner picks for this grid
    # (tuning is not timed; the tuned grid's results are checked below too)
    Tt = g.field(prob.T0)
    gt = wfa.Grid.from_problem(prob, precision=wfa.F64)
    gt.set_option(wfa.OPT_METHOD, METHODS[args.method])
    tune = gt.autotune(args.method, iters=20)
    gt.timestep(Tt, 2, tol=1e-10, maxit=1000)
    Tt = gt.field(prob.T0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tinfos = gt.timestep(Tt, 10, tol=1e-10, maxit=1000)
    torch.cuda.synchronize()
    tdt = time.perf_counter() - t0
    titers = sum(i.iterations for i in tinfos)
    out["tuned"] = {"ry": tune["ry"], "zc": tune["zc"], "seconds": tdt,
                    "ms_per_step": tdt / 10 * 1e3, "us_per_iteration": tdt / titers * 1e6,
                    "iterations": titers,
                    "rel_res_true_max": max(i.rel_res_true for i in tinfos)}
    wfa.tune_clear()
    if not args.no_cpu:
        import oracle
        o = oracle.Oracle(prob)
        c0 = time.perf_counter()
        To, io = o.timestep(prob.T0, 10, 1e-10, 1000)
        cdt = time.perf_counter() - c0
        out["cpu_baseline"] = {"seconds": cdt, "iterations": sum(i.iterations for i in io),
                               "cores": oracle.num_threads(), "kind": "oracle"}
        for key, field in (("rel_err_vs_oracle", T), ("rel_err_vs_oracle_tuned", Tt)):
            Tg = field.cpu().numpy()
            out[key] = float(((Tg - To) ** 2).sum() ** 0.5 / (To ** 2).sum() ** 0.5)
    return out


def run_poisson_large(args, torch, inputs, wfa):
    """512x512x1024 FP32 pure diffusion, exactly 500 BiCGStab iterations."""
    prob = inputs.poisson_large()
    g = wfa.Grid.from_problem(prob, precision=wfa.F32)
    g.set_option(wfa.OPT_METHOD, METHODS[args.method])
    g.set_option(wfa.OPT_SHADOW, 1 if args.shadow == "hashed" else 0)
    T = g.field(prob.T0)
    b = g.rhs(T)
    x = g.field()
    g.solve(b, x, tol=1e-300, maxit=20, method=args.method)
    # a fixed iteration count: one host check at the end
    g.set_option(wfa.OPT_CHECK_EVERY, 500)
    times = []
    for _ in range(args.repeats):
        x.copy_(T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = g.solve(b, x, tol=1e-300, maxit=500, method=args.method)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    best = min(times)
    # one more repeat with HIP events around every launch: per-kernel times
    g.set_option(wfa.OPT_PROFILE, 1)
    for k in range(wfa.K_COUNT):
        g.kernel_stats(k, reset=True)
    x.copy_(T)
    g.solve(b, x, tol=1e-300, maxit=500, method=args.method)
    torch.cuda.synchronize()
    kernels = {}
    for k, name in enumerate(wfa.KERNEL_NAMES):
        n, ms, by = g.kernel_stats(k)
        if n:
            kernels[name] = {"us_avg": round(ms / n * 1e3, 1), "gbps": round(by / (ms / n * 1e-3) / 1e9, 1)}
    streams = streams_of(args)
    kappa_reads = 1 if args.method in ("cg", "cg1") else 2   # one per operator product
    bytes_iter = (streams * 4 + 4 * kappa_reads) * prob.cells
    return {"workload": "poisson_512x512x1024_f32_500it", "method": args.method,
            "shadow": args.shadow if args.method == "bicgstab2" else "r0",
            "seconds_best": best, "seconds": times, "iterations": info.iterations,
            "cell_iters_per_s": prob.cells * info.iterations / best,
            "gbps": bytes_iter * info.iterations / best / 1e9,
            "frac_8tbs": bytes_iter * info.iterations / best / 8e12,
            "kernels": kernels, "rel_res_recursive": info.rel_res_recursive}


def run_mixed384(args, torch, inputs, wfa):
    """384^3 convection-diffusion (u x4): FP32 inside FP64 refinement vs
    plain FP64 BiCGStab (with and without Jacobi scaling), to 1e-12 and to
    1e-10, all with the two-reduction BiCGStab and r^ = r0 (the refinement's
    inner FP32 solve is Jacobi-scaled).  On this strongly convective problem
    the hashed shadow residual needs 30-40% more iterations than r0."""
    prob = inputs.convdiff_384(n=args.n if args.n != 256 else 384)
    out = {"workload": f"mixed_{prob.nx}^3", "method": "bicgstab2", "shadow": "r0",
           "results": []}
    Tref = None
    for tol in (1e-10, 1e-12):
        # refinement with the default inner tolerance (1e-4) and with 1e-3,
        # which needs one more refinement but cheaper inner solves here
        for name, prec, jac, itol in (("f64", wfa.F64, 0, None), ("f64_jacobi", wfa.F64, 1, None),
                                      ("f32_ir64", wfa.F32_IR64, 0, None),
                                      ("f32_ir64_inner1e-3", wfa.F32_IR64, 0, 1e-3)):
            g = wfa.Grid.from_problem(prob, precision=prec)
            g.set_option(wfa.OPT_METHOD, METHODS["bicgstab2"])
            g.set_option(wfa.OPT_JACOBI, jac)
            if itol is not None:
                g.set_option(wfa.OPT_IR_INNER_TOL, int(round(itol * 1e12)))
            T = g.field(prob.T0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = g.timestep(T, 1, tol=tol, maxit=100000, check=False)[0]
            if info.status != wfa.OK:
                print(f"{name} tol {tol}: status {info.status}: {wfa.last_error()}", file=sys.stderr)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rec = {"precision": name, "tol": tol, "seconds": dt, "iterations": info.iterations,
                   "refinements": info.refinements, "rel_res_true": info.rel_res_true,
                   "status": info.status}
            if name == "f64":
                Tref = T.double().clone()
            else:
                rec["rel_diff_vs_f64"] = float((T - Tref).norm() / Tref.norm())
            out["results"].append(rec)
            del g
    return out


def run_serve(args, torch, inputs, wfa, keep_fields=False):
    """Poisson request stream (200/s) of heat-step solves on grids with dims
    in {32,...,192}, FP32 inside FP64 refinement to 1e-10.  keep_fields: the
    result also carries the solved device fields (key "_fields")."""
    reqs = inputs.request_stream(count=args.requests)
    prec = wfa.PRECISIONS[args.serve_precision]
    fields = []
    for rq in reqs:       # inputs resident in HBM before the clock starts
        fields.append(torch.from_numpy(rq.problem().T0).to("cuda"))
    torch.cuda.synchronize()
    sv = wfa.Server(args.budget_gb << 30, max_slots=args.slots)
    sv.set_option(wfa.OPT_PERSISTENT, args.serve_persistent)
    sv.set_option(wfa.OPT_CHECK_EVERY, args.serve_round)
    sv.set_option(wfa.OPT_METHOD, METHODS[args.serve_method])
    sv.set_option(wfa.OPT_CG1_MAX_CELLS, args.serve_cg1_max_cells)
    sv.set_option(wfa.OPT_IR_INNER_TOL, int(round(args.serve_inner_tol * 1e12)))
    classes = None
    if args.serve_classes is not None:
        classes = [int(v) for v in args.serve_classes.split(",") if v.strip()][:3]
        bounds = classes + [0] * (3 - len(classes))
        for opt in (wfa.OPT_SIZE_CLASS_3, wfa.OPT_SIZE_CLASS_2, wfa.OPT_SIZE_CLASS_1):
            sv.set_option(opt, 0)
        for opt, v in zip((wfa.OPT_SIZE_CLASS_1, wfa.OPT_SIZE_CLASS_2, wfa.OPT_SIZE_CLASS_3),
                          bounds):
            if v:
                sv.set_option(opt, v)
    tickets = {}
    t_start = time.perf_counter()
    for q, rq in enumerate(reqs):
        now = time.perf_counter() - t_start
        if rq.arrival > now:
            time.sleep(rq.arrival - now)
        h = 1.0 / (max(rq.nx, rq.ny, rq.nz) + 1)
        tickets[q] = (sv.submit(fields[q], h=h, dt=1e-3, alpha=1.0, precision=prec,
                                tol=1e-10, maxit=20000), time.perf_counter() - t_start)
    sv.drain()
    t_end = time.perf_counter() - t_start
    lat, cell_it, fails, its, passes = [], 0, 0, 0, 0
    limit = args.serve_cg1_max_cells
    for q, rq in enumerate(reqs):
        code, info = sv.poll(tickets[q][0])
        if code != wfa.OK:
            fails += 1
        lat.append((tickets[q][1] - rq.arrival) + info.seconds)
        cells = rq.nx * rq.ny * rq.nz
        cell_it += cells * info.iterations
        its += info.iterations
        # a CG iteration is one operator pass, a BiCGStab iteration two (the
        # stream's heat requests are all symmetric)
        cg = args.serve_method == "cg1" and (limit == 0 or cells <= limit)
        passes += info.iterations * (1 if cg else 2)
    sv.close()
    extra = {"_fields": fields} if keep_fields else {}
    return {**extra, "workload": f"serve_{args.requests}req_200rps", "precision": args.serve_precision,
            "method": args.serve_method, "inner_tol": args.serve_inner_tol,
            "cg1_max_cells": args.serve_cg1_max_cells if args.serve_method == "cg1" else None,
            "round": {"iterations": args.serve_round,
                      "launch": "persistent" if args.serve_persistent else "per pass"},
            "size_classes": ("library default (up to 96^3, 152^3, larger)" if classes is None
                             else {"upper_bounds_cells": classes}),
            "requests": len(reqs), "failed": fails, "makespan_s": t_end,
            "latency_ms": {"p50": percentile(lat, 50) * 1e3, "p99": percentile(lat, 99) * 1e3,
                           "mean": sum(lat) / len(lat) * 1e3},
            "iterations_mean": its / len(reqs), "passes_mean": passes / len(reqs),
            "cell_iters_per_s": cell_it / t_end, "slots": args.slots,
            "budget_gb": args.budget_gb}


def run_apply(args, torch, inputs, wfa):
    """y = A x alone (wfa_stencil_apply): the 256^3 convection-diffusion
    operator in FP64 and the 512x512x1024 diffusion operator in FP32, both
    with a per-cell diffusivity; 2w + 4 bytes per cell."""
    out = {"workload": "stencil_apply", "results": []}
    for label, prob, prec, w in (("convdiff_256^3_f64", inputs.convdiff(n=256), wfa.F64, 8),
                                 ("poisson_512x512x1024_f32", inputs.poisson_large(), wfa.F32, 4)):
        g = wfa.Grid.from_problem(prob, precision=prec)
        x = g.field(prob.T0)
        y = g.field()
        reps = 50
        for _ in range(3):
            g.apply(x, y)
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            g.apply(x, y)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        by = (2 * w + 4) * prob.cells
        out["results"].append({"grid": label, "us_per_apply": round(us, 2),
                               "alg_gbps": round(by / (us * 1e-6) / 1e9, 1),
                               "frac_8tbs": round(by / (us * 1e-6) / 8e12, 4)})
        del g, x, y
    return out


def run_explicit(args, torch, inputs, wfa):
    """Explicit forward-time heat steps (Eq. 2, omega = 1/10, constant
    diffusivity, Dirichlet 0) on 512x512x1024 in FP32: the paper's explicit
    benchmark kernel.  One step per pass is bounded by 2w bytes per
    cell-step; the fused form (temporal blocking, up to 4 steps per pass)
    moves 2w bytes per pass."""
    nx, ny, nz = 512, 512, 1024
    h = inputs.grid_spacing(nx, ny, nz)
    cells = nx * ny * nz
    steps = 96
    out = {"workload": "explicit_heat_512x512x1024_f32", "steps": steps,
           "bound_cell_steps_per_s_one_pass_per_step_8tbs": 8e12 / 8}
    for label, fuse in (("one_step_per_pass", 1), ("fused", 0)):
        g = wfa.Grid(nx, ny, nz, h=h, dt=0.1 * h * h, alpha=1.0, precision=wfa.F32)
        g.set_option(wfa.OPT_EXPLICIT_FUSE, fuse)
        T = g.field(inputs.random_field(6, (nz, ny, nx), dtype="float32"))
        g.explicit(T, 8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.explicit(T, steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        g.set_option(wfa.OPT_PROFILE, 1)
        for k in range(wfa.K_COUNT):
            g.kernel_stats(k, reset=True)
        g.explicit(T, steps)
        torch.cuda.synchronize()
        kid = wfa.K_EXPLICIT if fuse == 1 else wfa.K_EXPLICIT_FUSED
        n, ms, by = g.kernel_stats(kid)
        per_pass = steps / n
        out[label] = {"seconds": dt, "cell_steps_per_s": cells * steps / dt,
                      "steps_per_pass": per_pass,
                      "kernel_us_avg": ms / n * 1e3,
                      "kernel_alg_gbps": by / (ms / n * 1e-3) / 1e9,
                      "equivalent_gbps_one_pass_per_step": 8 * cells * steps / dt / 1e9}
        del g
    out["speedup_fused"] = out["fused"]["cell_steps_per_s"] / out["one_step_per_pass"]["cell_steps_per_s"]
    return out


# ---------------------------------------------------------------------------
# headline: 512 x 512 x 1024 FP32, 500 fixed iterations per step
# ---------------------------------------------------------------------------
_T_START = time.perf_counter()


def progress(msg: str) -> None:
    """One line per finished phase on stderr (the JSON line goes to stdout)."""
    print(f"[bench {time.perf_counter() - _T_START:7.1f} s] {msg}", file=sys.stderr, flush=True)


def cpu_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable}


def rel_l2(a, b) -> float:
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def kernel_table(g, wfa) -> dict:
    kernels = {}
    for k, name in enumerate(wfa.KERNEL_NAMES):
        n, ms, by = g.kernel_stats(k)
        if n:
            kernels[name] = {"launches": n, "ms_total": round(ms, 3),
                             "us_avg": round(ms / n * 1e3, 2), "alg_bytes_per_launch": by,
                             "gbps": round(by / (ms / n * 1e-3) / 1e9, 1)}
    return kernels


def copy_ceiling(torch, wfa, nbytes: int = COPY_PROBE_BYTES) -> dict:
    """The measured copy ceilings on this GPU: the library's nontemporal copy
    kernel and hipMemcpyAsync device-to-device (torch's copy_), GB/s read +
    written."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    kern = wfa.bandwidth_probe(wfa.PROBE_COPY, src, dst, reps=10)
    dst.copy_(src)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    memcpy = 2.0 * nbytes * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    out = {"copy_kernel_gbps": round(kern, 1), "memcpy_d2d_gbps": round(memcpy, 1)}
    out.update(mix_ceilings(torch, wfa, nbytes))
    return out


# the stream mix of each pass of the two-reduction BiCGStab: pass 1 reads
# x, r, p, v, t and the diffusivity and writes x, r, p, v; pass 2 reads r, v
# and the diffusivity and writes t
KERNEL_MIX = {"phase_ac": "mix_6r4w_gbps", "phase_b2": "mix_3r1w_gbps"}


def mix_ceilings(torch, wfa, stream_bytes: int) -> dict:
    """GB/s of the library's stream-mix probes (the two passes' read/write
    mixes, nontemporal, 16 B per lane) with streams of `stream_bytes`."""
    out = {}
    for kind, key in ((wfa.PROBE_MIX_6R4W, "mix_6r4w_gbps"), (wfa.PROBE_MIX_3R1W, "mix_3r1w_gbps")):
        nr, nw = wfa.PROBE_STREAMS[kind]
        src = torch.ones(nr * stream_bytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty(nw * stream_bytes, dtype=torch.uint8, device="cuda")
        out[key] = round(wfa.bandwidth_probe(kind, src, dst, reps=10), 1)
        del src, dst
    torch.cuda.empty_cache()
    return out


def oracle_sample(prob, T0_32, iters: int):
    """The FP64 oracle (test infrastructure) on the headline solve: `iters`
    iterations of the same method (two-reduction BiCGStab, hashed shadow)
    from the same FP32-rounded T0, on every core, then one iteration on one
    core.  Returns (cpu_baseline, x_iters)."""
    import numpy as np
    import oracle
    o = oracle.Oracle(prob)
    T0 = T0_32.astype(np.float64)
    b = o.rhs(T0)
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    x, info = o.bicgstab2(b, T0, 1e-300, iters, hashed_shadow=True)
    dt = time.perf_counter() - t0
    # one core: one iteration on the first 128 z-planes of the same fields
    # (the oracle streams every vector through memory, so its rate per cell
    # does not depend on the grid's depth)
    nzs = min(128, prob.nz)
    slab = prob.with_(nz=nzs, kappa=prob.kappa[:nzs].copy(), T0=T0[:nzs].copy())
    os_ = oracle.Oracle(slab)
    bs = os_.rhs(slab.T0)
    oracle.set_num_threads(1)
    t1 = time.perf_counter()
    _, info1 = os_.bicgstab2(bs, slab.T0, 1e-300, 1, hashed_shadow=True)
    dt1 = time.perf_counter() - t1
    oracle.set_num_threads(threads)
    del os_, bs
    base = {
        "value": prob.cells * info.iterations / dt,
        "unit": "cell-iters/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{info.iterations} iterations of the headline solve (two-reduction BiCGStab, "
                  f"hashed shadow, FP64) on the full {prob.nx}x{prob.ny}x{prob.nz} grid, "
                  f"including the initial residual and the final true residual, {dt:.1f} s",
        "one_core": {"value": slab.cells * info1.iterations / dt1, "cores": 1,
                     "sample": f"1 iteration of the same solve on the first {nzs} z-planes "
                               f"({slab.nx}x{slab.ny}x{nzs}), including the initial and "
                               f"final residual products, {dt1:.1f} s"},
        **cpu_info(),
    }
    return base, x, o, b


def leg_c2(args, torch, inputs, wfa, oracle_mod):
    """256^3 convection-diffusion, FP64, the 50-step time integration to 1e-8
    (two-reduction BiCGStab, hashed shadow), with the oracle-evaluated true
    residual of every step's result and the first iterates against the
    oracle's."""
    import numpy as np
    prob = inputs.convdiff(n=256)
    g = wfa.Grid.from_problem(prob, precision=wfa.F64)
    g.set_option(wfa.OPT_METHOD, METHODS["bicgstab2"])
    g.set_option(wfa.OPT_SHADOW, 1)
    o = oracle_mod.Oracle(prob)
    T = g.field(prob.T0)
    g.timestep(T, 1, tol=1e-8, maxit=20000, check=False)      # warm-up
    T = g.field(prob.T0)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    infos, worst, Tprev = [], 0.0, prob.T0
    total_ms = 0.0
    for k in range(args.c2_steps):
        torch.cuda.synchronize()
        e0.record(stream)
        infos += g.timestep(T, 1, tol=1e-8, maxit=20000, check=False)
        e1.record(stream)
        torch.cuda.synchronize()
        total_ms += e0.elapsed_time(e1)
        Tn = T.cpu().numpy()
        if k < 3 or k == args.c2_steps - 1:   # the oracle's operator on this step's system
            worst = max(worst, o.true_relres(o.rhs(Tprev), Tn))
        Tprev = Tn
        if (k + 1) % 10 == 0:
            progress(f"c2: {k + 1} steps")
    iters = sum(i.iterations for i in infos)
    b = o.rhs(prob.T0)
    first = {}
    for k in (1, 2):
        xo, _ = o.bicgstab2(b, prob.T0, 1e-300, k, hashed_shadow=True)
        x, _ = g.solve(g.field(b), g.field(prob.T0), tol=1e-300, maxit=k, method="bicgstab2",
                       check=False)
        first[f"k{k}"] = rel_l2(x.cpu().numpy(), xo)
    return {"workload": "convdiff_256^3_f64", "steps": args.c2_steps, "tol": 1e-8,
            "method": "bicgstab2", "shadow": "hashed",
            "value": prob.cells * iters / (total_ms * 1e-3),
            "ms_per_step": total_ms / args.c2_steps, "iterations_per_step": iters / args.c2_steps,
            "status_ok_steps": sum(1 for i in infos if i.status == wfa.OK),
            "rel_res_true_max": max(i.rel_res_true for i in infos),
            "oracle": {"rel_res_true_oracle_operator_max": worst,
                       "checked_steps": sorted({1, 2, 3, args.c2_steps}),
                       "first_iterates_rel_l2": first,
                       "note": "cond ~1e5: a converged x is fixed only to ~cond*tol, so the "
                               "gate is the oracle-evaluated true residual <= tol"}}


def leg_c1(args, torch, inputs, wfa, oracle_mod):
    """32^3 heat, FP64, 10 steps to 1e-10, against the oracle's 10 steps."""
    prob = inputs.heat_32()
    g = wfa.Grid.from_problem(prob, precision=wfa.F64)
    g.set_option(wfa.OPT_METHOD, METHODS["bicgstab2"])
    T = g.field(prob.T0)
    g.timestep(T, 2, tol=1e-10, maxit=1000)
    T = g.field(prob.T0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = g.timestep(T, 10, tol=1e-10, maxit=1000)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = sum(i.iterations for i in infos)
    o = oracle_mod.Oracle(prob)
    To, _ = o.timestep(prob.T0, 10, 1e-10, 1000)
    return {"workload": "heat_32^3_f64_10steps", "ms_per_step": dt / 10 * 1e3,
            "us_per_iteration": dt / iters * 1e6, "iterations": iters,
            "oracle": {"rel_l2_vs_oracle": rel_l2(T.cpu().numpy(), To),
                       "bound_cond_2tol": 13.6 * 2 * 1e-10}}


def leg_c4(args, torch, inputs, wfa, oracle_mod):
    """384^3 convection-diffusion (u x4): FP32 inside FP64 refinement (inner
    tolerance 1e-3) against plain FP64, both two-reduction BiCGStab with
    r^ = r0.  One step to 1e-10 (the comparison tolerance), then a time
    integration of args.c4_steps steps to 1e-12 (the workload's tolerance),
    each from the previous step's result; oracle-evaluated true residuals of
    the first and last steps."""
    prob = inputs.convdiff_384()
    o = oracle_mod.Oracle(prob)
    out = {"workload": "mixed_384^3_u4"}
    variants = (("f64", wfa.F64, None), ("f32_ir64", wfa.F32_IR64, 1e-3))

    def grid(prec, itol):
        g = wfa.Grid.from_problem(prob, precision=prec)
        g.set_option(wfa.OPT_METHOD, METHODS["bicgstab2"])
        if itol is not None:
            g.set_option(wfa.OPT_IR_INNER_TOL, int(round(itol * 1e12)))
        return g

    # one step to 1e-10
    b = o.rhs(prob.T0)
    step1, ref = {}, None
    for name, prec, itol in variants:
        g = grid(prec, itol)
        T = g.field(prob.T0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = g.timestep(T, 1, tol=1e-10, maxit=100000, check=False)[0]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        Tn = T.cpu().numpy()
        rec = {"seconds": dt, "iterations": info.iterations, "refinements": info.refinements,
               "status": info.status, "rel_res_true": info.rel_res_true,
               "rel_res_true_oracle_operator": o.true_relres(b, Tn)}
        if ref is None:
            ref = Tn
        else:
            rec["rel_l2_vs_f64"] = rel_l2(Tn, ref)
        step1[name] = rec
        del g, T
    step1["speedup_f32_ir64"] = step1["f64"]["seconds"] / step1["f32_ir64"]["seconds"]
    out["step1_tol1e-10"] = step1

    # time integration to 1e-12
    steps = args.c4_steps
    integ, finals = {"steps": steps, "tol": 1e-12}, {}
    for name, prec, itol in variants:
        g = grid(prec, itol)
        T = g.field(prob.T0)
        prev = prob.T0
        its, refs, worst, oracle_checks, ok = 0, 0, 0.0, {}, 0
        t_total = 0.0
        for k in range(1, steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = g.timestep(T, 1, tol=1e-12, maxit=100000, check=False)[0]
            torch.cuda.synchronize()
            t_total += time.perf_counter() - t0
            its += info.iterations
            refs += info.refinements
            ok += info.status == wfa.OK
            worst = max(worst, info.rel_res_true)
            if k in (1, steps):   # the oracle's operator on this step's system
                Tn = T.cpu().numpy()
                oracle_checks[str(k)] = o.true_relres(o.rhs(prev), Tn)
            if k == 1 or k == steps - 1:
                prev = T.cpu().numpy()
        finals[name] = T.cpu().numpy()
        integ[name] = {"seconds": t_total, "ms_per_step": t_total / steps * 1e3,
                       "iterations_per_step": its / steps, "refinements_per_step": refs / steps,
                       "status_ok_steps": ok, "rel_res_true_max": worst,
                       "rel_res_true_oracle_operator": oracle_checks}
        del g, T
    integ["f32_ir64"]["rel_l2_vs_f64_final"] = rel_l2(finals["f32_ir64"], finals["f64"])
    integ["speedup_f32_ir64"] = integ["f64"]["seconds"] / integ["f32_ir64"]["seconds"]
    out[f"{steps}_steps_tol1e-12"] = integ
    return out


def leg_cg1(args, torch, prob, wfa):
    """CG with one reduction (the paper's solver, one pass per iteration) on
    the headline grid: 500 iterations, HIP-event timed."""
    g = wfa.Grid.from_problem(prob, precision=wfa.F32)
    g.set_option(wfa.OPT_METHOD, METHODS["cg1"])
    g.set_option(wfa.OPT_CHECK_EVERY, HEADLINE_ITERS + 1)
    T0 = g.field(prob.T0)
    T = g.field(prob.T0)
    g.timestep(T, 1, tol=1e-300, maxit=50, check=False)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps, its = 3, 0
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        T.copy_(T0)
        its += g.timestep(T, 1, tol=1e-300, maxit=HEADLINE_ITERS, check=False)[0].iterations
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del g
    return {"workload": "poisson_512x512x1024_f32_500it", "method": "cg1",
            "value": prob.cells * its / (ms * 1e-3), "ms_per_step": ms / reps,
            "alg_bytes_per_cell_iter": 10 * 4 + 4}


def leg_serve(args, torch, inputs, wfa, oracle_mod):
    """The 2000-request stream: p50/p99 latency (arrival to completion),
    throughput, and for a sample of 50 requests the oracle-evaluated true
    residual and, for those up to 64^3 cells, the distance to the oracle's
    own solve."""
    import numpy as np
    args.requests = getattr(args, "requests", 2000)
    out = run_serve(args, torch, inputs, wfa, keep_fields=True)
    fields = out.pop("_fields")
    reqs = inputs.request_stream(count=args.requests)
    rng = np.random.default_rng(7)
    sample = sorted(rng.choice(len(reqs), size=min(50, len(reqs)), replace=False).tolist())
    worst_res, worst_err, n_err = 0.0, 0.0, 0
    for q in sample:
        prob = reqs[q].problem()
        o = oracle_mod.Oracle(prob)
        b = o.rhs(prob.T0)
        x = fields[q].cpu().numpy()
        worst_res = max(worst_res, o.true_relres(b, x))
        if prob.cells <= 64 ** 3:
            xo, _ = o.bicgstab(b, prob.T0, 1e-12, 2000)
            worst_err = max(worst_err, rel_l2(x, xo))
            n_err += 1
    out["oracle"] = {"sampled_requests": len(sample),
                     "rel_res_true_oracle_operator_max": worst_res,
                     "rel_l2_vs_oracle_max": worst_err, "compared_requests": n_err,
                     "note": "tol 1e-10; the heat operators have cond <= ~450, so the bound "
                             "cond * 2 * tol is <= ~1e-7"}
    return out


def run_headline(args, torch, inputs, wfa):
    import numpy as np
    prob = inputs.poisson_large()
    g = wfa.Grid.from_problem(prob, precision=wfa.F32)
    g.set_option(wfa.OPT_METHOD, METHODS["bicgstab2"])
    g.set_option(wfa.OPT_SHADOW, 1)
    g.set_option(wfa.OPT_RECOMPUTE_T, args.recompute_t)
    g.set_option(wfa.OPT_CHECK_EVERY, HEADLINE_ITERS + 1)   # one host check per solve
    T0 = g.field(prob.T0)
    T = g.field(prob.T0)
    stream = torch.cuda.current_stream()

    def step():
        T.copy_(T0)
        return g.timestep(T, 1, tol=1e-300, maxit=HEADLINE_ITERS, check=False)[0]

    progress("headline inputs resident")
    for _ in range(args.warmup):
        step()
    progress(f"{args.warmup} warm-up steps done")
    # the timed steps, with HIP events around every HEADLINE_TIME_EVERY-th
    # launch of each kernel on the solve stream (the host never waits on
    # them inside the steps; sampling keeps their cost off the steps' time)
    profile = not args.no_profile
    g.set_option(wfa.OPT_PROFILE, HEADLINE_TIME_EVERY if profile else 0)
    for k in range(wfa.K_COUNT):
        g.kernel_stats(k, reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    infos = []
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        infos.append(step())
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    iters = sum(i.iterations for i in infos)
    value = prob.cells * iters / (total_ms * 1e-3)
    progress(f"{args.steps} timed steps done: {value:.4g} cell-iters/s")
    kernels = kernel_table(g, wfa) if profile else {}
    g.set_option(wfa.OPT_PROFILE, 0)
    # what the per-launch events cost: two more steps without them
    plain = None
    if profile:
        torch.cuda.synchronize()
        e0.record(stream)
        pit = sum(step().iterations for _ in range(2))
        e1.record(stream)
        torch.cuda.synchronize()
        plain = prob.cells * pit / (e0.elapsed_time(e1) * 1e-3)
    x500 = T.cpu().numpy()
    roofline = None
    ceiling = copy_ceiling(torch, wfa)
    if profile:
        dom = max(kernels, key=lambda k: kernels[k]["ms_total"])
        achieved = kernels[dom]["gbps"]
        best = max(ceiling["copy_kernel_gbps"], ceiling["memcpy_d2d_gbps"])
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 4),
                    "traffic": load_traffic(dom, "headline"),
                    "measured": f"HIP events around every {HEADLINE_TIME_EVERY}th launch of "
                                "each kernel on the solve stream inside the timed steps",
                    "copy_ceiling_gbps": ceiling, "frac_of_best_copy": round(achieved / best, 4)}
        if dom in KERNEL_MIX:
            roofline["frac_of_own_mix"] = round(achieved / ceiling[KERNEL_MIX[dom]], 4)
        for k, key in KERNEL_MIX.items():
            if k in kernels:
                kernels[k]["of_own_mix"] = round(kernels[k]["gbps"] / ceiling[key], 4)
    # two-reduction, hashed shadow: 9 + 3 vector streams, or 8 + 2 when pass 1
    # forms t again instead of pass 2 storing it
    streams = 10 if args.recompute_t else 12
    alg_cell_iter = streams * 4 + 2 * 4
    whole = alg_cell_iter * prob.cells * iters / (total_ms * 1e-3) / 1e9
    # the paper's effective bandwidth (section 3.1.3): A_eff = 2 D_u + D_k
    # with the updated fields D_u = {x, r, p, v, t} and the read-only ones
    # D_k = {r^, kappa}: (2 * 5 + 2) * w bytes per cell and iteration
    a_eff = (2 * 5 + 2) * 4
    t_eff = a_eff * prob.cells * iters / (total_ms * 1e-3) / 1e9
    line = {
        "metric": "BiCGStab cell-iters/s and % HBM roofline on 1 MI355X; p50/p99 solve latency",
        "value": value,
        "unit": "cell-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "poisson_512x512x1024_f32_500it", "grid": [512, 512, 1024],
                   "cells": prob.cells, "precision": "f32",
                   "iterations_per_step": HEADLINE_ITERS, "method": "bicgstab2",
                   "shadow": "hashed", "recompute_t": bool(args.recompute_t),
                   "physics": "pure diffusion, 8-mode smooth kappa in [0.5,2], dt=1, "
                              "Dirichlet 0, T0~U[0,1)",
                   "step": "one backward-Euler step restarted from T0: rhs + initial residual "
                           "+ 500 iterations + FP64 true residual"},
        "iterations": [i.iterations for i in infos],
        "value_without_launch_events": plain,
        "alg_bytes_per_cell_iter": alg_cell_iter,
        "whole_step_gbps": round(whole, 1),
        "whole_step_frac": round(whole / HBM_PEAK_GBPS, 4),
        "t_eff": {"a_eff_bytes_per_cell_iter": a_eff, "gbps": round(t_eff, 1),
                  "frac": round(t_eff / HBM_PEAK_GBPS, 4)},
        "roofline": roofline,
        "kernels": kernels,
        "kernel_source_hash": kernel_source_hash(),
    }
    legs = [] if args.legs == "none" else args.legs.split(",")
    oracle_mod = None
    if not args.no_cpu or legs:
        import oracle as oracle_mod
    # error against the FP64 oracle: the GPU's 10th iterate against the
    # oracle's (same method, same x0 and b); the oracle's operator on the
    # 500-iteration result
    ora = {"rel_res_true_500": max(i.rel_res_true for i in infos),
           "rel_res_recursive_500": infos[-1].rel_res_recursive}
    if not args.no_cpu:
        T0_32 = T0.cpu().numpy()
        base, x10o, o, b = oracle_sample(prob, T0_32, 10)
        progress("oracle sample done")
        line["cpu_baseline"] = base
        x10, _ = g.solve(g.field(b), g.field(T0_32), tol=1e-300, maxit=10, method="bicgstab2",
                         check=False)
        ora["rel_l2_x10_vs_oracle"] = rel_l2(x10.cpu().numpy(), x10o)
        ora["rel_res_true_500_oracle_operator"] = o.true_relres(b, x500)
        ora["note"] = ("FP32 against the FP64 oracle: cond ~1e6 here, so cond * 6e-8 >> 1e-5 and "
                       "no 1e-5 gate applies (the tests gate the first iterates); the 500-"
                       "iteration FP32 iterate does not reduce the residual at this condition "
                       "number, the workload measures bandwidth")
        del o, b, x10o
    line["oracle"] = ora
    del g, T, T0
    torch.cuda.empty_cache()
    compare = {}
    if "cg1" in legs:
        compare["cg1"] = leg_cg1(args, torch, prob, wfa)
        progress("leg cg1 done")
    if "c2" in legs:
        compare["c2"] = leg_c2(args, torch, inputs, wfa, oracle_mod)
        progress("leg c2 done")
    if "c1" in legs:
        compare["c1"] = leg_c1(args, torch, inputs, wfa, oracle_mod)
        progress("leg c1 done")
    if "c4" in legs:
        compare["c4"] = leg_c4(args, torch, inputs, wfa, oracle_mod)
        progress("leg c4 done")
    if "serve" in legs:
        sv = leg_serve(args, torch, inputs, wfa, oracle_mod)
        progress("leg serve done")
        compare["serve"] = sv
        line["solve_latency_ms"] = {"p50": sv["latency_ms"]["p50"], "p99": sv["latency_ms"]["p99"],
                                    "source": f"serving stream, {sv['requests']} requests at "
                                              "200/s, arrival to completion"}
    line["compare"] = compare
    return line


def run_ceilings(args, torch, inputs, wfa):
    """HBM bandwidth ceilings: the library's probe kernels (copy, 16 and 32
    bytes per lane, nontemporal and plain; read only; write only) over 1 and
    4 GiB with 2048 to 16384 workgroups, hipMemcpyAsync device to device, and
    the two passes' stream mixes (six reads and four writes; three reads and
    one write) with streams of 128 MiB and 1 GiB."""
    out = {"workload": "hbm_ceilings", "results": []}
    for gib in (1, 4):
        nbytes = gib << 30
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        dst.fill_(0)
        for kind, name in enumerate(wfa.PROBE_NAMES[:wfa.PROBE_MIX_6R4W]):
            for blocks in (2048, 4096, 8192, 16384):
                gbps = wfa.bandwidth_probe(kind, src, dst, reps=10, blocks=blocks)
                out["results"].append({"bytes": nbytes, "kind": name, "blocks": blocks,
                                       "gbps": round(gbps, 1)})
        stream = torch.cuda.current_stream()
        dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(10):
            dst.copy_(src)
        e1.record(stream)
        torch.cuda.synchronize()
        out["results"].append({"bytes": nbytes, "kind": "hipMemcpyAsync_d2d", "blocks": None,
                               "gbps": round(2.0 * nbytes * 10 / (e0.elapsed_time(e1) * 1e-3)
                                             / 1e9, 1)})
        del src, dst
        torch.cuda.empty_cache()
    # the passes' stream mixes, with streams of a 256^3 FP64 and a
    # 512x512x1024 FP32 vector
    for sb in (128 << 20, 1 << 30):
        for kind in (wfa.PROBE_MIX_6R4W, wfa.PROBE_MIX_3R1W):
            nr, nw = wfa.PROBE_STREAMS[kind]
            src = torch.ones(nr * sb, dtype=torch.uint8, device="cuda")
            dst = torch.empty(nw * sb, dtype=torch.uint8, device="cuda")
            for blocks in (2048, 4096, 8192, 16384):
                gbps = wfa.bandwidth_probe(kind, src, dst, reps=10, blocks=blocks)
                out["results"].append({"bytes": sb, "kind": wfa.PROBE_NAMES[kind],
                                       "blocks": blocks, "gbps": round(gbps, 1)})
            del src, dst
            torch.cuda.empty_cache()
    best = {}
    for r in out["results"]:
        key = (f"{r['kind']}_{r['bytes'] >> 30}GiB" if r["bytes"] >= 1 << 30
               else f"{r['kind']}_{r['bytes'] >> 20}MiB")
        best[key] = max(best.get(key, 0.0), r["gbps"])
    out["best"] = best
    return out


METHODS = {"bicgstab": 0, "cg": 1, "bicgstab2": 2, "cg1": 3}
STREAMS = {"bicgstab": 17, "cg": 10, "bicgstab2": 14, "cg1": 10}


def streams_of(args) -> int:
    """Vector streams per iteration; the hashed shadow residual of the
    two-reduction BiCGStab is computed, not read, in both passes."""
    s = STREAMS[args.method]
    return s - 2 if args.method == "bicgstab2" and args.shadow == "hashed" else s


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "convdiff", "heat32", "poisson_large", "mixed384", "serve",
                             "explicit", "apply", "ceilings"])
    ap.add_argument("--method", default="bicgstab2",
                    choices=["bicgstab", "bicgstab2", "cg", "cg1"],
                    help="cg, cg1 (one reduction per iteration): the symmetric workloads only "
                         "(poisson_large, heat32)")
    ap.add_argument("--shadow", default="hashed", choices=["r0", "hashed"],
                    help="shadow residual of the two-reduction BiCGStab: r0 (stored) or a "
                         "field hashed from the cell index (computed, one stream less per pass)")
    ap.add_argument("--compare", type=int, default=1,
                    help="also time the textbook three-pass BiCGStab on the same steps")
    ap.add_argument("--n", type=int, default=256, help="grid cells per axis")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32", "f32_ir64"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=20000)
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--budget-gb", type=int, default=64)
    ap.add_argument("--cpu-iters", type=int, default=120)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-precision", default="f32_ir64", choices=["f32_ir64", "f64"],
                    help="serve: precision of every request")
    ap.add_argument("--serve-round", type=int, default=4,
                    help="serve: iterations per round between host reads of the scalars")
    ap.add_argument("--serve-method", default="bicgstab2", choices=["bicgstab2", "cg1"],
                    help="serve: cg1 = the (symmetric) heat requests iterate with CG with one "
                         "reduction")
    ap.add_argument("--serve-cg1-max-cells", type=int, default=0,
                    help="serve with --serve-method cg1: larger requests keep BiCGStab (0: none)")
    ap.add_argument("--serve-inner-tol", type=float, default=1e-3,
                    help="serving: relative tolerance of the FP32 inner solves (the "
                         "library's default is 1e-4; 1e-3 measured faster on the stream)")
    ap.add_argument("--serve-classes", default=None,
                    help="serve: comma-separated upper cell-count bounds of the server's size "
                         "classes (each class has its own worker thread and stream); '' = one "
                         "class; default: the library's")
    ap.add_argument("--serve-persistent", type=int, default=0, choices=[0, 1],
                    help="serve: 1 = each round is one cooperative launch per precision")
    ap.add_argument("--legs", default="c2,c1,c4,cg1,serve",
                    help="headline: comma-separated comparison legs to run (c2 = 256^3 FP64 "
                         "time integration, c1 = 32^3 heat, c4 = 384^3 refinement vs FP64, cg1 = "
                         "CG with one reduction on the headline grid, serve = request stream); "
                         "'none' for the headline alone")
    ap.add_argument("--recompute-t", type=int, default=0, choices=[0, 1],
                    help="two-reduction BiCGStab: 1 = pass 1 forms t = A s again instead of "
                         "pass 2 storing it (bitwise the same iterates, two streams fewer)")
    ap.add_argument("--c4-steps", type=int, default=20,
                    help="headline: steps of the 384^3 refinement-vs-FP64 time integration leg "
                         "to 1e-12 (50: the workload's full length, about 145 s)")
    ap.add_argument("--c2-steps", type=int, default=50,
                    help="headline: steps of the 256^3 FP64 time integration leg")
    ap.add_argument("--no-profile", action="store_true",
                    help="time without per-launch events (no roofline)")
    ap.add_argument("--probe-copy", action="store_true",
                    help="start with one 1 GiB device copy (a dispatch of known traffic that "
                         "calibrates hardware byte counters)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU work: turn two rocprofv3 --pmc counter_collection.csv files "
                         "(FETCH_SIZE, WRITE_SIZE; both runs with --probe-copy) into the traffic "
                         "file the roofline line reads")
    ap.add_argument("--counter-commands", nargs="*", default=[],
                    help="with --summarize-counters: the commands that made the two files")
    ap.add_argument("--summarize-pmc", nargs="+", metavar="CSV",
                    help="no GPU work: print a markdown table of the per-dispatch means of the "
                         "counters in rocprofv3 --pmc counter_collection.csv files (title and "
                         "commands from --pmc-title and --counter-commands)")
    ap.add_argument("--pmc-title", default="rocprofv3 counters")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("STATS_CSV", "TITLE", "COMMAND"),
                    help="no GPU work: print a markdown summary of a rocprofv3 --kernel-trace "
                         "--stats kernel_stats.csv")
    args = ap.parse_args()

    if args.summarize_pmc:
        print(summarize_pmc(args.summarize_pmc, args.pmc_title, args.counter_commands), end="")
        return
    if args.summarize_trace:
        print(summarize_trace(*args.summarize_trace), end="")
        return
    if args.summarize_counters:
        out = summarize_counters(*args.summarize_counters, workload=f"{args.workload}",
                                 commands=args.counter_commands)
        print(json.dumps(out))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the solver has no "
                          "multi-GPU path",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2209_13768_amd import inputs, wfa

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.probe_copy:
        print(json.dumps({"copy_probe_gbps": wfa.stream_probe(COPY_PROBE_BYTES, 1)}), file=sys.stderr)
    run = {"headline": run_headline, "convdiff": run_convdiff, "heat32": run_heat32,
           "poisson_large": run_poisson_large, "apply": run_apply, "ceilings": run_ceilings,
           "mixed384": run_mixed384, "serve": run_serve, "explicit": run_explicit}[args.workload]
    print(json.dumps(run(args, torch, inputs, wfa)))


if __name__ == "__main__":
    main()
