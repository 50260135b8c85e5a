#!/usr/bin/env python3
"""Throughput of the TSSP solver on one MI355X.

Workload (default): 3D quantum turbulence, 512^3 sites on the periodic box
[0, 2 pi)^3, V = 0, g = 1, psi = exp(i theta) with theta a seeded
band-limited random phase (integer modes 1 <= |m| <= 8, per-mode variance
~ |m|^-2, rms |grad theta| = 1), dt = 5e-4, FP64 state.  A step is one
real-time TSSP step (three fused axis passes); the particle-number,
compressible, incompressible and quantum-pressure |k|-shell spectra are
evaluated every 100 steps inside the timed region, as the workload asks.  The
FP32 form of the same workload is timed in the same run.  The serving mix
(a seeded Poisson stream of independent 2D/3D solves, FP32 or FP64) is then
run through the request server and, for comparison, one request at a time:
once arriving far faster than the GPU serves them (200/s) and once below its
capacity (8/s, about 60 % load).

Prints ONE JSON line.  Inputs are resident in HBM before timing starts; the
timed region is bracketed by device synchronisation and timed with HIP events
recorded on the stream the library launches on.  The dominant kernel's
average duration comes from per-launch HIP events inside the timed region.
HBM traffic is taken from the committed rocprofv3 counter summary when it was
made from the current kernel sources, else reported as null.

--copy-calibration times a plain device copy of 2 GiB (the reference kernel
for scaling the FETCH_SIZE / WRITE_SIZE counters) and exits.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_512.json")
KERNEL_SOURCES = ["axis_pass.h", "axis_pass.hip", "axis_pass_f64.hip", "axis_pass_f32.hip",
                  "gpe_kernels.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2301_08275_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def copy_calibration():
    import torch

    n = 1 << 27  # 2 GiB of FP64 complex
    x = torch.zeros(2 * n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 10
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = x.numel() * 8
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                      "ms": ms, "GBps_read_plus_write": 2 * nbytes / ms / 1e6}), flush=True)


def run_workload(ctx, torch, steps, warmup, dt, every, spectra):
    """Time `steps` steps with the spectra (and observables) evaluated after
    every `every`-th step.  The workload evaluates them once per `every` steps,
    so a run whose step count is not a multiple of the cadence (say 20 steps
    of a 100-step cadence) also times one more evaluation at the end of the
    timed region and counts the share of it that its steps owe: the returned
    time is the stepping with the evaluations reached, plus
    (steps / every - evaluations reached) times one evaluation."""
    stream = torch.cuda.current_stream()
    ctx.evolve(dt, warmup)
    if spectra:
        ctx.spectra()
    torch.cuda.synchronize()
    ctx.timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e_mid = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    done, nspec = 0, 0
    while done < steps:
        chunk = min(every - done % every, steps - done)
        ctx.evolve(dt, chunk)
        done += chunk
        if spectra and done % every == 0:
            ctx.spectra(with_obs=True)  # one call: observables and shell spectra
            nspec += 1
    e_mid.record(stream)
    owed = steps / every - nspec if spectra else 0.0
    if owed > 0:
        ctx.spectra(with_obs=True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_region = e0.elapsed_time(e_mid)
    ms_eval = e_mid.elapsed_time(e1) if owed > 0 else 0.0
    kinds = ctx.timing()
    ctx.timing(False)
    return dict(ms=ms_region + owed * ms_eval, ms_region=ms_region, nspec=nspec,
                owed=owed, ms_eval=ms_eval, kinds=kinds)


def kernel_table(kinds):
    out = {}
    for k, v in kinds.items():
        avg = v["total_ms"] / max(1, v["launches"])
        out[k] = {"launches": v["launches"], "avg_ms": avg, "bytes": v["bytes"],
                  "GBps": v["bytes"] / (avg * 1e-3) / 1e9}
    return out


def dominant(kinds):
    name = max(kinds, key=lambda k: kinds[k]["total_ms"])
    k = kinds[name]
    avg_ms = k["total_ms"] / max(1, k["launches"])
    return name, avg_ms, k["bytes"] / (avg_ms * 1e-3) / 1e9, k["bytes"]


def traffic_for(kernel, bytes_per_launch):
    """Measured HBM bytes per launch of `kernel` from the committed counter
    summary, or None when the summary was made from other kernel sources or
    for another workload (its algorithmic bytes per launch differ)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("kernel_hash") != kernel_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    if not k or k.get("algorithmic_bytes_per_launch") != bytes_per_launch:
        return None
    return k["hbm_bytes_per_launch"]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def fp32_accuracy_series(torch, dev, n, lo, hi, g, dt, stream, steps=1000, every=100):
    """The mixed-precision comparison: the FP64 run and both FP32 forms from
    the same state, in lockstep, compared every `every` steps (untimed):
    relative L2 distance of psi, norm drift, energy relative error, and the
    largest relative L2 error over shells of the N, compressible and
    incompressible spectra."""
    from paper_2301_08275_amd import gpe

    L3 = (hi[0] - lo[0]) ** 3
    forms = ("fp64", "fp32s", "fp32")
    ctxs = {p: gpe.Context((n,) * 3, lo, hi, g, precision=p, norm_target=L3, stream=stream)
            for p in forms}
    try:
        norm0 = {}
        for p, c in ctxs.items():
            c.set_state_device(dev)
            norm0[p] = c.observables()["norm"]
        ref = torch.empty_like(dev)
        got = torch.empty_like(dev)
        series = {p: [] for p in forms[1:]}
        for t in range(every, steps + 1, every):
            res = {}
            for p, c in ctxs.items():
                c.evolve(dt, every)
                res[p] = c.spectra(with_obs=True)
            ctxs["fp64"].get_state_device(ref)
            torch.cuda.synchronize()
            sp64, o64 = res["fp64"]
            nref = float(torch.linalg.vector_norm(ref))
            for p in forms[1:]:
                ctxs[p].get_state_device(got)
                torch.cuda.synchronize()
                sp, o = res[p]
                err = float(torch.linalg.vector_norm(got - ref)) / nref
                spec = max(float(((sp[k] - sp64[k]) ** 2).sum() ** 0.5
                                 / ((sp64[k] ** 2).sum() ** 0.5))
                           for k in ("n_k", "e_comp", "e_incomp"))
                series[p].append({"step": t, "rel_l2": err,
                                  "norm_drift": abs(o["norm"] - norm0[p]) / norm0[p],
                                  "energy_rel": abs(o["energy"] - o64["energy"])
                                  / abs(o64["energy"]),
                                  "spectra_rel": spec})
    finally:
        for c in ctxs.values():
            c.close()
    bars = {"rel_l2": 1e-4, "norm_drift": 1e-6, "energy_rel": 1e-5, "spectra_rel": 1e-4}
    out = {"workload": "%d^3 turbulence, %d steps from the same state, compared every %d"
                       % (n, steps, every), "bars": bars}
    for p, name in (("fp32s", "fp32"), ("fp32", "fp32_fft")):
        worst = {k: max(r[k] for r in series[p]) for k in bars}
        out[name] = {"end": series[p][-1], "worst": worst,
                     "meets_bars": all(worst[k] <= bars[k] for k in bars), "series": series[p]}
    return out


def cpu_baseline(n, seed, target_s=12.0, max_steps=25):
    """The oracle on the host cores: a bounded sample of the same workload,
    its step count sized by one untimed step to about target_s seconds."""
    import oracle
    from paper_2301_08275_amd import inputs as I

    psi = I.phase_field(n, seed)
    lo, hi = (0.0,) * 3, (2 * 3.141592653589793,) * 3
    oracle.set_threads(0)
    t0 = time.perf_counter()
    oracle.tssp_real(psi, lo, hi, None, 1.0, 5e-4, 1)
    t1 = time.perf_counter() - t0
    steps = max(1, min(max_steps, int(round(target_s / t1))))
    t0 = time.perf_counter()
    oracle.tssp_real(psi, lo, hi, None, 1.0, 5e-4, steps)
    t = time.perf_counter() - t0
    return {"value": n ** 3 * steps / t, "unit": "site-steps/s", "cores": oracle.get_threads(),
            "kind": "oracle", "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "sample": "%d real-time TSSP step(s) of the %d^3 FP64 turbulence workload, no "
                      "spectra (plain radix-2 C++ oracle, %.1f s)" % (steps, n, t)}


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def ground_state_bench(torch):
    """The 3D ground-state setup at 256^3: imaginary time from a Gaussian until
    |dE| < 1e-10 between checks 10 steps apart, then the trap switches to
    isotropic and the state evolves 2000 real-time steps with sigma and E
    recorded every 10 steps.  Wall time of each phase (device time, state
    resident)."""
    from paper_2301_08275_amd import gpe
    from paper_2301_08275_amd import inputs as I

    n, g = 256, 50.0
    shape, lo, hi = (n,) * 3, (-12.0,) * 3, (12.0,) * 3
    psi0 = I.gaussian(shape, lo, hi, widths=[1.0, 2.0, 4.0])
    with gpe.Context(shape, lo, hi, g, harmonic=[1.0, 2.0, 4.0]) as ctx:
        ctx.set_state(psi0)
        ctx.synchronize()
        t0 = time.perf_counter()
        steps, energy, conv = ctx.ground_state(1e-3, tol=1e-10, check_every=10, max_steps=200000)
        ctx.synchronize()
        t1 = time.perf_counter()
        o = ctx.observables()
        ctx.set_potential(harmonic=[1.0, 1.0, 1.0])
        ctx.synchronize()
        t2 = time.perf_counter()
        series = ctx.evolve_record(1e-3, 2000, 10)
        t3 = time.perf_counter()
    return {"workload": "256^3 on [-12,12)^3, trap (1, 2, 4), g = 50, dt = 1e-3",
            "ground_state": {"steps": steps, "converged": bool(conv), "seconds": t1 - t0,
                             "ms_per_step": (t1 - t0) * 1e3 / max(1, steps), "energy": energy,
                             "mu": o["mu"], "sigma": [o["sigma_x"], o["sigma_y"], o["sigma_z"]]},
            "dynamics": {"steps": 2000, "records": len(series), "seconds": t3 - t2,
                         "ms_per_step": (t3 - t2) * 1e3 / 2000,
                         "sigma_z_max": max(r["sigma_z"] for r in series),
                         "energy_drift": max(abs(r["energy"] - series[0]["energy"])
                                             for r in series) / abs(series[0]["energy"])}}


def potentials_bench(torch, dev, n, lo, hi, g, dt, steps=50):
    """The real-time step at n^3 with V = 0, with a static separable potential
    (trap, quartic, lattice on every axis: read from per-axis tables), and
    with a time-dependent one (a shaken lattice: parameters from a Python
    callback at every N-substep midpoint, tables rebuilt each step).  Device
    time of `steps` steps from HIP events on the context stream."""
    from paper_2301_08275_amd import gpe

    stream = torch.cuda.current_stream()
    L = hi[0] - lo[0]
    static = dict(w=[0.3] * 3, center=[L / 2] * 3, quartic=[1e-3] * 3, lattice=[1.0] * 3,
                  q=[2.0] * 3, phase=[0.0] * 3)

    def shaken(t):
        return dict(lattice=[1.0 + 0.5 * math.sin(10 * t)] * 3, q=[2.0] * 3,
                    phase=[0.3 * t, 0.0, 0.0])

    out = {"workload": "%d^3 turbulence state, FP64, dt = %g, %d steps per case" % (n, dt, steps)}
    with gpe.Context((n,) * 3, lo, hi, g, stream=stream.cuda_stream,
                     norm_target=L ** 3) as ctx:
        for name, setup in (("no_potential", lambda: ctx.set_potential()),
                            ("static_separable", lambda: ctx.set_separable(**static)),
                            ("time_dependent", lambda: ctx.set_potential_fn(shaken))):
            setup()
            ctx.set_state_device(dev)
            ctx.evolve(dt, 5)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            ctx.evolve(dt, steps)
            e1.record(stream)
            torch.cuda.synchronize()
            out[name + "_ms_per_step"] = e0.elapsed_time(e1) / steps
    return out


def dynamics_validation_bench(n=256, dt=1e-3, t_end=4.0, every=10):
    """The dynamics-validation run of the Results section: the 3D Gaussian
    exp(-(x^2 + 2 y^2 + 4 z^2)/(2 eps1)), eps1 = 0.25, in
    V = (x^2 + 4 y^2 + 16 z^2)/2 on [-8,8) x [-6,6) x [-4,4), n^3 points,
    sigma_x,y,z recorded every `every` steps to t_end; g = 0.1 (the figure's
    case) and g = 0 (closed form per axis: the largest deviation of sigma^2
    is reported).  Wall time per step with the records (device-resident)."""
    from paper_2301_08275_amd import gpe
    from paper_2301_08275_amd import inputs as I

    gam, eps1 = (1.0, 2.0, 4.0), 0.25
    lo, hi = (-8.0, -6.0, -4.0), (8.0, 6.0, 4.0)
    shape = (n,) * 3
    nsteps = int(round(t_end / dt))
    psi0 = I.gaussian(shape, lo, hi, widths=list(gam), eps=eps1)
    out = {"workload": "%d^3 on [-8,8)x[-6,6)x[-4,4), gamma = (1, 2, 4), eps1 = 0.25, "
                       "dt = %g, %d steps, sigma every %d" % (n, dt, nsteps, every)}
    for g in (0.1, 0.0):
        with gpe.Context(shape, lo, hi, g, harmonic=list(gam)) as ctx:
            ctx.set_state(psi0)
            ctx.synchronize()
            t0 = time.perf_counter()
            series = ctx.evolve_record(dt, nsteps, every)
            t1 = time.perf_counter()
        if g > 0:
            per = max(1, len(series) // 4)
            out["g0.1"] = {"ms_per_step": (t1 - t0) * 1e3 / nsteps,
                           "sigma_at_t": {"%.1f" % ((k + 1) * every * dt):
                                          [series[k]["sigma_x"], series[k]["sigma_y"],
                                           series[k]["sigma_z"]]
                                          for k in range(per - 1, len(series), per)}}
        else:
            worst = 0.0
            for k, o in enumerate(series):
                t = (k + 1) * every * dt
                for a, key in enumerate(("sigma_x", "sigma_y", "sigma_z")):
                    s2 = (eps1 / (2 * gam[a]) * math.cos(gam[a] * t) ** 2
                          + 1 / (2 * eps1 * gam[a]) * math.sin(gam[a] * t) ** 2)
                    worst = max(worst, abs(o[key] ** 2 - s2))
            out["g0_closed_form_max_abs_error_sigma2"] = worst
            out["g0_ms_per_step"] = (t1 - t0) * 1e3 / nsteps
    return out


def serving_bench(nreq, max_slots, chunk, rate=200.0):
    """The serving mix: requests arrive on a seeded Poisson stream (mean
    `rate` per second); continuous batching through the request server against
    the same requests solved one at a time in arrival order with the
    single-context calls.  Latency = done - arrival."""
    import numpy as np

    from paper_2301_08275_amd import gpe
    from paper_2301_08275_amd import inputs as I

    trace = I.serving_trace(nreq, rate=rate)
    psis = [I.psi0_of(r) for r in trace]
    work = sum(float(np.prod(r["shape"])) * r["nsteps"] for r in trace)

    def submit_args(r, p):
        return dict(shape=r["shape"], lo=r["lo"], hi=r["hi"], g=r["g"], psi0=p, mode=r["mode"],
                    dt=r["dt"], nsteps=r["nsteps"], precision=r["precision"], trap=r["trap"])

    srv = gpe.Server(max_slots=max_slots, chunk_steps=chunk)
    t0 = time.perf_counter()
    ids = []
    for r, p in zip(trace, psis):
        delay = t0 + r["arrival"] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        ids.append(srv.submit(**submit_args(r, p)))
    srv.wait_idle()
    res = [srv.poll(i) for i in ids]
    for i in ids:
        srv.release(i)
    srv.close()
    ok = sum(1 for x in res if x["status"] == gpe.GPE_OK)
    lat = [x["t_done"] - x["t_submit"] for x in res]
    span = max(x["t_done"] for x in res) - min(x["t_submit"] for x in res)

    # one at a time, same arrivals, single-context calls
    clock, lat1 = 0.0, []
    for r, p in zip(trace, psis):
        start = max(clock, r["arrival"])
        ts = time.perf_counter()
        with gpe.Context(r["shape"], r["lo"], r["hi"], r["g"], precision=r["precision"],
                         harmonic=r["trap"]) as ctx:
            ctx.set_state(p)
            if r["mode"] == "real":
                ctx.evolve(r["dt"], r["nsteps"])
            else:
                ctx.imag_steps(r["dt"], r["nsteps"])
            ctx.observables()
        clock = start + (time.perf_counter() - ts)
        lat1.append(clock - r["arrival"])
    span1 = clock - trace[0]["arrival"]
    return {"requests": nreq, "completed_ok": ok, "offered_rate_per_s": rate,
            "offered_site_steps": work, "max_slots": max_slots, "chunk_steps": chunk,
            "p50_latency_s": percentile(lat, 0.5), "p99_latency_s": percentile(lat, 0.99),
            "makespan_s": span, "site_steps_per_s": work / span,
            "one_at_a_time": {"p50_latency_s": percentile(lat1, 0.5),
                              "p99_latency_s": percentile(lat1, 0.99),
                              "makespan_s": span1, "site_steps_per_s": work / span1}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--spectra-every", type=int, default=100)
    ap.add_argument("--no-spectra", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the untimed FP32-against-FP64 comparison series")
    ap.add_argument("--accuracy-steps", type=int, default=1000)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="run the launch-shape tuner for the bench grid instead of loading "
                         "the shipped tuning cache")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the default launch shapes (no cache, no tuner)")
    ap.add_argument("--serving", type=int, default=256,
                    help="requests of the serving mix to run (0: skip)")
    ap.add_argument("--serving-slots", type=int, default=16)
    ap.add_argument("--no-ground-state", action="store_true",
                    help="skip the 256^3 ground state + trap-switch dynamics timing")
    ap.add_argument("--serving-chunk", type=int, default=16)
    ap.add_argument("--serving-light-rate", type=float, default=13.0,
                    help="arrival rate (1/s) of the second serving run, about 0.7 of the GPU's "
                         "capacity for the mix (0: skip)")
    ap.add_argument("--no-dynamics", action="store_true",
                    help="skip the dynamics-validation (Gaussian breathing) timing")
    ap.add_argument("--no-potentials", action="store_true",
                    help="skip the separable / time-dependent potential timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    # a dedicated stream at default priority: the library enqueues on it and
    # the timing events are recorded on it
    torch.cuda.set_stream(torch.cuda.Stream())

    from paper_2301_08275_amd import gpe
    from paper_2301_08275_amd import inputs as I

    n, seed, dt, g = args.n, 2, 5e-4, 1.0
    lo, hi = (0.0,) * 3, (2 * 3.141592653589793,) * 3
    log("generating the %d^3 phase field" % n)
    psi0 = I.phase_field(n, seed)
    dev = torch.from_numpy(psi0).to("cuda")
    del psi0
    stream = torch.cuda.current_stream().cuda_stream
    sites = n ** 3
    spectra = not args.no_spectra

    from paper_2301_08275_amd import tune_cache

    results, tuning = {}, {}
    tuning_source = "defaults"
    if not args.no_tune and not args.tune and os.path.exists(tune_cache.SHIPPED):
        gpe.gpe_tuning_load(tune_cache.SHIPPED)
        tuning_source = os.path.basename(tune_cache.SHIPPED)
    for prec in (["fp64"] if args.no_fp32 else ["fp64", "fp32", "fp32s"]):
        d = gpe.make_desc((n, n, n), lo, hi, g, prec)
        if args.tune:
            # untimed: pick the launch shapes of this shape class on this device
            log("tuning %s" % prec)
            gpe.gpe_autotune(d, steps=5)
            tuning_source = "gpe_autotune"
        tuning[prec] = dict(gpe.gpe_tuning_get(d)[0], source=tuning_source)
        log("timing %s" % prec)
        ctx = gpe.Context((n, n, n), lo, hi, g, precision=prec,
                          norm_target=(2 * 3.141592653589793) ** 3, stream=stream)
        ctx.set_state_device(dev)
        r = run_workload(ctx, torch, args.steps, args.warmup, dt, args.spectra_every, spectra)
        r["dom"] = dominant(r["kinds"])
        results[prec] = r
        ctx.close()
        torch.cuda.synchronize()
    accuracy = None
    if not args.no_fp32 and not args.no_accuracy:
        log("FP32 forms against FP64, %d steps" % args.accuracy_steps)
        accuracy = fp32_accuracy_series(torch, dev, n, lo, hi, g, dt, stream,
                                        steps=args.accuracy_steps)
    potentials = None
    if not args.no_potentials:
        log("separable and time-dependent potentials")
        potentials = potentials_bench(torch, dev, n, lo, hi, g, dt)
    del dev
    torch.cuda.empty_cache()

    def summary(r):
        step_ms = sum(v["total_ms"] for k, v in r["kinds"].items() if k.startswith("step_"))
        name, avg, ach, nbytes = r["dom"]
        return {"value": sites * args.steps / (r["ms"] * 1e-3), "ms_per_step": r["ms"] / args.steps,
                "stepping_only_ms_per_step": step_ms / args.steps,
                "dominant_kernel": name, "avg_launch_ms": avg, "achieved_GBps": ach,
                "frac": ach / HBM_PEAK_GBS, "kernels": kernel_table(r["kinds"])}

    r64 = results["fp64"]
    ms_step = r64["ms"] / args.steps
    value = sites * args.steps / (r64["ms"] * 1e-3)
    name, avg_ms, achieved, bytes_per = r64["dom"]
    step_ms = summary(r64)["stepping_only_ms_per_step"]
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
                               "psi=exp(i theta), seeded random phase |m|<=8 ~|m|^-2, dt=5e-4, "
                               "real-time TSSP, shell spectra every %d steps"
                               % (n, args.spectra_every),
                   "grid": [n, n, n], "sites": sites, "dt": dt, "g": g,
                   "spectra_every": args.spectra_every if spectra else None,
                   "spectra_evaluations_in_steps": r64["nspec"],
                   "spectra_evaluation_ms": r64["ms_eval"],
                   "spectra_evaluations_owed": r64["owed"],
                   "timing": "HIP events on the library stream around the steps and the "
                             "evaluations they reach; plus owed x one evaluation timed at the "
                             "end of the same region when the step count is not a multiple "
                             "of the cadence",
                   "passes_per_step": 3},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for(name, bytes_per),
                     "kernel": name, "avg_launch_ms": avg_ms, "bytes_per_launch": bytes_per},
        "stepping_only": {"ms_per_step": step_ms, "site_steps_per_s": sites / (step_ms * 1e-3),
                          "hbm_GBps_at_96B_per_site_step":
                              96.0 * sites / (step_ms * 1e-3) / 1e9},
        "kernels": kernel_table(r64["kinds"]),
        "tuning": tuning["fp64"],
    }
    if "fp32s" in results:
        # the reported FP32 form: FP32 state in HBM (half the bytes), FP64
        # arithmetic in every pass (one rounding per pass)
        out["fp32"] = dict(summary(results["fp32s"]), form="fp32 state, fp64 arithmetic",
                           tuning=tuning["fp32s"])
        out["fp32"]["speedup_vs_fp64"] = out["fp32"]["value"] / value
    if "fp32" in results:
        # FP32 state and FP32 FFT arithmetic: misses the norm bar on the 2D
        # trap workload and the energy bar at 1024^3 (not the reported form)
        out["fp32_fft"] = dict(summary(results["fp32"]), form="fp32 state and fp32 fft",
                               tuning=tuning["fp32"])
        out["fp32_fft"]["speedup_vs_fp64"] = out["fp32_fft"]["value"] / value
    if accuracy is not None:
        out["fp32_accuracy"] = accuracy
    if potentials is not None:
        out["potentials"] = potentials
    if not args.no_dynamics:
        log("dynamics-validation run")
        out["dynamics_validation"] = dynamics_validation_bench()
    if not args.no_ground_state:
        log("256^3 ground state and dynamics")
        out["ground_state_256"] = ground_state_bench(torch)
    if args.serving > 0:
        log("serving mix: %d requests" % args.serving)
        out["serving"] = serving_bench(args.serving, args.serving_slots, args.serving_chunk)
        if args.serving_light_rate > 0:
            log("serving mix at %.1f requests/s" % args.serving_light_rate)
            out["serving_light"] = serving_bench(args.serving, args.serving_slots,
                                                 args.serving_chunk, args.serving_light_rate)
    if not args.no_cpu:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(n, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
