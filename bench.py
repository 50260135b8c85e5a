#!/usr/bin/env python3
"""Throughput of the TSSP step on one MI355X.

Workload (default): 3D quantum-turbulence grid, 512^3 sites on the periodic
box [0, 2 pi)^3, V = 0, g = 1, psi = exp(i theta) with theta a seeded
band-limited random phase (|m| <= 8, per-mode variance ~ |m|^-2), dt = 5e-4,
FP64 state.  One step = one real-time TSSP step (three fused axis passes).
The FP32 form of the same workload is timed in the same run.

Prints ONE JSON line.  Inputs are resident in HBM before timing starts; the
timed region is bracketed by device synchronisation and measured with HIP
events on the library's stream.  The dominant kernel's average duration comes
from per-launch HIP events inside the timed region.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_run(ctx, torch, steps, warmup, dt):
    stream = torch.cuda.current_stream()
    ctx.evolve(dt, warmup)
    torch.cuda.synchronize()
    ctx.timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    ctx.evolve(dt, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kinds = ctx.timing()
    ctx.timing(False)
    return ms, kinds


def dominant(kinds):
    name = max(kinds, key=lambda k: kinds[k]["total_ms"])
    k = kinds[name]
    avg_ms = k["total_ms"] / max(1, k["launches"])
    achieved = k["bytes"] / (avg_ms * 1e-3) / 1e9
    return name, avg_ms, achieved, k["bytes"]


def cpu_baseline(n, seed, steps=1):
    import oracle
    from paper_2301_08275_amd import inputs as I

    psi = I.phase_field(n, seed)
    lo, hi = (0.0,) * 3, (2 * 3.141592653589793,) * 3
    oracle.set_threads(0)
    t0 = time.perf_counter()
    oracle.tssp_real(psi, lo, hi, None, 1.0, 5e-4, steps)
    t = time.perf_counter() - t0
    return {"value": n ** 3 * steps / t, "unit": "site-steps/s", "cores": oracle.get_threads(),
            "kind": "oracle",
            "sample": "%d real-time step(s) of the %d^3 FP64 workload (plain radix-2 oracle, "
                      "%.1f s)" % (steps, n, t)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2301_08275_amd import gpe
    from paper_2301_08275_amd import inputs as I

    torch.cuda.set_device(0)
    # a dedicated stream (default priority): the library enqueues on it and the
    # timing events are recorded on it
    torch.cuda.set_stream(torch.cuda.Stream())
    n, seed, dt, g = args.n, 2, 5e-4, 1.0
    lo, hi = (0.0,) * 3, (2 * 3.141592653589793,) * 3
    log("generating %d^3 phase field" % n)
    psi0 = I.phase_field(n, seed)
    dev = torch.from_numpy(psi0).to("cuda")
    del psi0
    stream = torch.cuda.current_stream().cuda_stream
    sites = n ** 3

    results = {}
    for prec in (["fp64"] if args.no_fp32 else ["fp64", "fp32"]):
        log("timing %s" % prec)
        ctx = gpe.Context((n, n, n), lo, hi, g, precision=prec,
                          norm_target=(2 * 3.141592653589793) ** 3, stream=stream)
        ctx.set_state_device(dev)
        ms, kinds = time_run(ctx, torch, args.steps, args.warmup, dt)
        name, avg_ms, achieved, bytes_per = dominant(kinds)
        results[prec] = dict(ms=ms, kinds=kinds, dom=(name, avg_ms, achieved, bytes_per))
        ctx.close()
        torch.cuda.synchronize()
    del dev
    torch.cuda.empty_cache()

    r64 = results["fp64"]
    ms_step = r64["ms"] / args.steps
    value = sites * args.steps / (r64["ms"] * 1e-3)
    name, avg_ms, achieved, bytes_per = r64["dom"]
    out = {
        "metric": "TSSP site-steps/s at 512^3 FP64 vs FP32; % HBM roofline; p50/p99 solve latency",
        "value": value,
        "unit": "site-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D quantum turbulence, %d^3 periodic box [0,2pi)^3, V=0, g=1, "
                               "psi=exp(i theta) seeded random phase (|m|<=8, ~k^-2), dt=5e-4, "
                               "real-time TSSP" % n,
                   "grid": [n, n, n], "sites": sites, "dt": dt, "g": g,
                   "passes_per_step": 3},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": name, "avg_launch_ms": avg_ms, "bytes_per_launch": bytes_per},
        "kernels": {k: {"avg_ms": v["total_ms"] / max(1, v["launches"]),
                        "GBps": v["bytes"] / (v["total_ms"] / max(1, v["launches"]) * 1e-3) / 1e9}
                    for k, v in r64["kinds"].items()},
    }
    step_bytes = sum(v["bytes"] for v in r64["kinds"].values())
    out["step_hbm_frac"] = step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS
    if "fp32" in results:
        r32 = results["fp32"]
        v32 = sites * args.steps / (r32["ms"] * 1e-3)
        n32, a32, ach32, b32 = r32["dom"]
        out["fp32"] = {"value": v32, "ms_per_step": r32["ms"] / args.steps,
                       "speedup_vs_fp64": v32 / value,
                       "dominant_kernel": n32, "achieved_GBps": ach32,
                       "frac": ach32 / HBM_PEAK_GBS}
    if not args.no_cpu:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(n, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
