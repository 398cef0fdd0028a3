"""Benchmark: BiCGStab cell-iterations/s and HBM-roofline fraction on one MI355X.

Default workload (a "step" = one backward-Euler time step = one BiCGStab
solve of the whole grid): 256^3 convection-diffusion, FP64, log-normal
per-cell diffusivity (mu 0, sigma 1), velocity (1, 0.5, 0.25) with
first-order upwind, dt 1e-2, x- Dirichlet 1 / x+ Dirichlet 0 / y, z
zero-flux, BiCGStab to a relative residual of 1e-8, solved with the
two-reduction organisation of BiCGStab and a shadow residual hashed from
the cell index (--shadow r0 stores r^ = r0 instead); the r^ = r0 form and
the textbook three-pass BiCGStab are timed on the same steps for
comparison.  Inputs are synthetic and seeded
(paper_2209_13768_amd.inputs.convdiff).

Prints one JSON line.  `value` = cells x BiCGStab iterations / seconds over
the K timed steps (inputs resident in HBM, HIP-event timing on the solve
stream, plain launches).  `roofline` is for the kernel with the largest
share of GPU time; its average duration comes from HIP events around every
launch of that kernel while the same K steps run again from the same
initial field; `traffic` is the HBM bytes per launch measured
with rocprofv3 counters (profiles/) when they were taken from the current
kernel sources, else null.  `cpu_baseline` times the FP64 CPU oracle on a
bounded sample of the same workload on this host.

Other workloads (--workload): heat32 (32^3, 10 steps), poisson_large
(512x512x1024 FP32, 500 iterations), mixed384 (FP32 inside FP64 refinement
vs FP64), serve (Poisson request stream through the batching server),
explicit (forward-time steps, one and several per pass), apply (the
operator alone).  --method cg and cg1 apply to the symmetric workloads.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_convdiff256_f64.json")


# The files that define the single-grid solver kernels and their launch
# shapes: counter figures taken from other sources are stale.
KERNEL_SOURCES = ("device.hpp", "phases.hpp", "kernels.hip")


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


def load_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    if it was taken from the current kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


# rocprofv3 kernel names -> the names bench.py and the library's kernel
# statistics use
KERNEL_PATTERNS = (("PhAC<", "phase_ac"), ("PhB2<", "phase_b2"), ("PhA<", "phase_a"),
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
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    return out


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
    if trace_csv != stats_csv and os.path.exists(trace_csv):
        with open(trace_csv) as f:
            for r in csv.DictReader(f):
                durs.setdefault(r["Kernel_Name"], []).append(
                    (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
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
    return "\n".join(lines) + "\n"


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


def run_serve(args, torch, inputs, wfa):
    """Poisson request stream (200/s) of heat-step solves on grids with dims
    in {32,...,192}, FP32 inside FP64 refinement to 1e-10."""
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
    return {"workload": f"serve_{args.requests}req_200rps", "precision": args.serve_precision,
            "method": args.serve_method,
            "cg1_max_cells": args.serve_cg1_max_cells if args.serve_method == "cg1" else None,
            "round": {"iterations": args.serve_round,
                      "launch": "persistent" if args.serve_persistent else "per pass"},
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
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="convdiff",
                    choices=["convdiff", "heat32", "poisson_large", "mixed384", "serve", "explicit",
                             "apply"])
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
    ap.add_argument("--serve-persistent", type=int, default=0, choices=[0, 1],
                    help="serve: 1 = each round is one cooperative launch per precision")
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
    ap.add_argument("--summarize-trace", nargs=3, metavar=("STATS_CSV", "TITLE", "COMMAND"),
                    help="no GPU work: print a markdown summary of a rocprofv3 --kernel-trace "
                         "--stats kernel_stats.csv")
    args = ap.parse_args()

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
    run = {"convdiff": run_convdiff, "heat32": run_heat32, "poisson_large": run_poisson_large,
           "apply": run_apply,
           "mixed384": run_mixed384, "serve": run_serve, "explicit": run_explicit}[args.workload]
    print(json.dumps(run(args, torch, inputs, wfa)))


if __name__ == "__main__":
    main()
