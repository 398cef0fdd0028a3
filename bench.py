"""Benchmark: BiCGStab cell-iterations/s and HBM-roofline fraction on one MI355X.

Workload (a "step" = one backward-Euler time step = one BiCGStab solve of the
whole grid): 256^3 convection-diffusion, FP64, log-normal per-cell
diffusivity (mu 0, sigma 1), velocity (1, 0.5, 0.25) with first-order
upwind, dt 1e-2, x- Dirichlet 1 / x+ Dirichlet 0 / y, z zero-flux, BiCGStab
to a relative residual of 1e-8.  Inputs are synthetic and seeded
(paper_2209_13768_amd.inputs.convdiff).

Prints one JSON line.  `value` = cells x BiCGStab iterations / seconds over
the K timed steps (inputs resident in HBM, HIP-event timing on the solve
stream).  `roofline` is for the kernel with the largest share of GPU time;
its average duration comes from HIP events around every launch of that
kernel in the timed region; `traffic` is the HBM bytes per launch measured
with rocprofv3 counters (profiles/) when they were taken from the current
kernel sources, else null.  `cpu_baseline` times the FP64 CPU oracle on a
bounded sample of the same workload on this host.
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


def kernel_source_hash() -> str:
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="grid cells per axis")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32", "f32_ir64"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=20000)
    ap.add_argument("--cpu-iters", type=int, default=120)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="time without per-launch events (no roofline)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the solver has no "
                          "multi-GPU path (see DESIGN.md for how it would shard)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2209_13768_amd import inputs, wfa

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    prob = inputs.convdiff(n=args.n)
    prec = wfa.PRECISIONS[args.precision]
    g = wfa.Grid.from_problem(prob, precision=prec)
    T0 = g.field(prob.T0)
    T = g.field(prob.T0)
    stream = torch.cuda.current_stream()

    # warmup: the first steps of the time integration
    for _ in range(args.warmup):
        g.timestep(T, 1, tol=args.tol, maxit=args.maxit)
    T.copy_(T0)
    torch.cuda.synchronize()

    profile = not args.no_profile
    g.set_option(wfa.OPT_PROFILE, 1 if profile else 0)
    for k in range(wfa.K_COUNT):
        g.kernel_stats(k, reset=True)
    infos = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    step_ms = []
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        s0 = time.perf_counter()
        infos += g.timestep(T, 1, tol=args.tol, maxit=args.maxit)
        step_ms.append((time.perf_counter() - s0) * 1e3)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    iters = sum(i.iterations for i in infos)
    value = prob.cells * iters / (total_ms * 1e-3)

    roofline = None
    kernels = {}
    if profile:
        for k, name in enumerate(wfa.KERNEL_NAMES):
            n, ms, by = g.kernel_stats(k)
            if n:
                kernels[name] = {"launches": n, "ms_total": ms, "ms_avg": ms / n,
                                 "alg_bytes_per_launch": by,
                                 "gbps": by / (ms / n * 1e-3) / 1e9}
        dom = max(kernels, key=lambda k: kernels[k]["ms_total"])
        kd = kernels[dom]
        achieved = kd["gbps"]
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 4),
                    "traffic": load_traffic(dom)}
    w = 4 if prec == wfa.F32 else 8
    alg_bytes_iter = (17 * w + 2 * 4) * prob.cells   # 17 vector streams + 2 kappa reads
    whole = alg_bytes_iter * iters / (total_ms * 1e-3) / 1e9

    step_ms_sorted = sorted(step_ms)

    def pct(p):
        return step_ms_sorted[min(len(step_ms_sorted) - 1, int(round(p / 100 * (len(step_ms_sorted) - 1))))]

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
                   "precision": args.precision, "tol": args.tol,
                   "physics": "lognormal kappa, u=(1,0.5,0.25) upwind, dt=1e-2, mixed BC"},
        "iterations_per_step": iters / args.steps,
        "solve_latency_ms": {"p50": pct(50), "p99": pct(99)},
        "whole_step_gbps": round(whole, 1),
        "whole_step_frac": round(whole / HBM_PEAK_GBPS, 4),
        "roofline": roofline,
        "kernels": kernels,
        "rel_res_true_max": max(i.rel_res_true for i in infos),
        "kernel_source_hash": kernel_source_hash(),
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_iters)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
