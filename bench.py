#!/usr/bin/env python3
"""Benchmark of the SIPF-W step on one MI355X: particle-steps/s and the HBM roofline fraction
of the dominant kernel, float32 form (float64 masses and sums) beside the plain float64 form,
on the 128^3-grid / 2^23-particle four-blob workload (dt = 5e-4).

One "step" is the whole hot path: reaction + 3D FFT solves for m and w + spectral gradient of
v + gather / Euler-Maruyama push / mass update / deposit + diagnostics reductions (folded into
the kernels that write each value) + periodic tile binning of the particles.  Inputs are
resident in HBM before the timed region; the timed region replays the captured step graph.

Prints one JSON line.  `python bench.py --gpus N --steps K --warmup W`.
"""
import argparse
import ctypes
import hashlib
import math
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = ("particle-steps/s + HBM GB/s fraction at 128^3/2^23 (FP32 vs FP64); "
          "p50/p99 served")


def plane_path(N, s):
    """The library runs the y and x transforms of a k3 plane in one block (the plane pass)
    when the plane fits the kernel's LDS: float32 N <= 128, float64 N <= 64 (3D)."""
    return N <= (128 if s == 4 else 64)


def stage_bytes(N, P, s, lowpass=False):
    """Bytes each stage must move per step by design (reads + writes), s = 4 or 8.  On the
    plane path the "xpass" stage is the plane pass (reads the M*, W*, V half spectra, writes
    M, W, G1, G2 and, with the low-pass filter, the filtered V) and the y passes do not run."""
    G = N ** 3
    half = (N // 2 + 1) * N * N * 2 * s  # one half spectrum
    plane = plane_path(N, s)
    # float32 takes the m and w solves in change form (m* and w* stored by the forward z pass
    # and read back by the inverse one); float64 in plain form
    change = s == 4
    return {
        # reads ubar, m, v, w; writes v, and m* and w* (into ubar's array) in change form, or
        # clears ubar's array; 3 half spectra
        "zfwd": G * 4 * s + G * (3 if change else 2) * s + 3 * half,
        # M, W transformed in place; V read, its y derivative written (with the filter V in
        # place as well)
        "yfwd": 0 if plane else 6 * half,
        # M, W in place, V read and d1 V written; with the filter also the filtered V
        "xpass": (3 + 4 + (1 if lowpass else 0)) * half if plane else (8 if lowpass else 6) * half,
        # M, W in place; with the filter also d1 V in place and the filtered V -> V, d2 V
        "yinv": 0 if plane else (9 if lowpass else 4) * half,
        # reads 5 half spectra (and m*, w* in change form); writes m, w, the gather array (4
        # per node) and, in change form, the cleared ubar
        "zinv": 5 * half + (9 if change else 6) * G * s,
        # particles: read x,y,z,a; write x,y,z,a (the 4-byte particle index that keys the
        # noise is not counted) + gather array read once + deposit target written once
        "particles": P * (6 * s + 16) + G * 5 * s,
        "finalize": 0,
        # binning, per binning: count reads x,y,z and writes the rank within the tile;
        # scatter reads the ranks and one particle set and writes the other
        "binning": P * (3 * s + 4) + P * (4 + 2 * (3 * s + 8 + 4)),
    }


def resort_period(prm):
    """Re-binning period of a run: resort_every if set, else the library's default as the
    header documents it (the largest k <= 64 with sqrt(k 2 D_u dt) <= 0.45 h in 3D, 2.4 h in
    2D; 64 without noise)."""
    if prm.get("resort_every", 0) > 0:
        return int(prm["resort_every"])
    h = prm["L"] / prm["N"]
    s = math.sqrt(2.0 * prm["D_u"] * prm["dt"]) / h
    if not s > 0.0:
        return 64
    reach = 2.4 if prm.get("dim") == 2 else 0.45
    return int(min(64, max(1, math.floor((reach / s) ** 2))))

# Kernel behind each stage (the roofline names the dominant one) and the sources it is built
# from: a byte-counter summary under profiles/ only applies while these are unchanged.
STAGE_KERNEL = {"particles": ("k_particles<float, 2>", "k_particles<double, 2>"),
                "xpass": ("k_plane<float, 7>", "k_xpass<double, 7>")}
KERNEL_SOURCES = ("paper_2605_20140_amd/csrc/particles.hip",
                  "paper_2605_20140_amd/csrc/sipf_internal.h",
                  "paper_2605_20140_amd/csrc/diag_acc.h")
COPY_CAL_BYTES = 512 << 20


def _code_text(src):
    """Source text without comments and with whitespace runs collapsed: what the compiler sees
    of it, so that an edit of a comment does not invalidate a measurement of the kernel."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def sources_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "r", encoding="utf-8") as fh:
            h.update(_code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision):
    """HBM bytes per launch of the particle kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each divided by what the counter read for a device
    copy of COPY_CAL_BYTES), or None if there is none or the kernel changed since."""
    path = os.path.join(ROOT, "profiles", f"pmc_traffic_particles_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or "=" not in line:
                continue
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("sources_digest") != sources_digest():
        return None
    key = "traffic_bytes_fp32" if precision == 1 else "traffic_bytes_fp64"
    return float(kv[key]) if key in kv else None


def copy_calibration():
    """One device-to-device copy of COPY_CAL_BYTES (a blit kernel of known size: the
    reference the byte counters are scaled by)."""
    import torch
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.c_int, ctypes.c_void_p]
    src = torch.ones(COPY_CAL_BYTES // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream().cuda_stream
    rc = hip.hipMemcpyAsync(dst.data_ptr(), src.data_ptr(), COPY_CAL_BYTES, 3, st)
    torch.cuda.synchronize()
    assert rc == 0 and bool((dst == 1).all())


def run_form(ic, precision, steps, warmup, profile_steps, workload, keep_state=False, **over):
    import torch
    from paper_2605_20140_amd import sipf
    prm = dict(ic["params"], **over)
    p = sipf.make_params(precision=precision, **prm)
    torch.cuda.synchronize()
    ti = time.perf_counter()
    sim = sipf.Simulation(p, ic["X0"], ic["a0"], ic["v0"], ic["m0"], ic["w0"], device="cuda:0")
    torch.cuda.synchronize()
    init_s = time.perf_counter() - ti
    stream = torch.cuda.current_stream()
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    sim.step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)
    stage_ms = sim.step_timed(profile_steps)
    out = sim.fields(particles=keep_state)
    sim.close()
    d = out["diag"]
    s = 4 if precision == 1 else 8
    sb = stage_bytes(prm["N"], prm["P"], s, lowpass=prm.get("H0", 0) > 0)
    if prm.get("dim") == 2:
        return dict(value=prm["P"] * steps / (ms * 1e-3), ms_per_step=ms / steps,
                    init_s=init_s,
                    stages={k: round(v / profile_steps, 5) for k, v in stage_ms.items()},
                    check=dict(n_nan=d["n_nan"], step=d["step"]))
    stages = {}
    for k, tot in stage_ms.items():
        avg = tot / profile_steps  # per step (binning: amortised over its period)
        nbytes = sb[k] / resort_period(prm) if k == "binning" else sb[k]
        stages[k] = dict(ms=round(avg, 5),
                         GBs=round(nbytes / (avg * 1e-3) / 1e9, 1) if avg > 0 and nbytes else None)
    dominant = max(stages, key=lambda k: stages[k]["ms"])
    ach = sb[dominant] / (stages[dominant]["ms"] * 1e-3) / 1e9
    kname = STAGE_KERNEL.get(dominant, (dominant, dominant))[0 if precision == 1 else 1]
    traffic = (measured_traffic(workload, precision)
               if dominant == "particles" and not over else None)
    return dict(
        state=out if keep_state else None,
        value=prm["P"] * steps / (ms * 1e-3),
        ms_per_step=ms / steps,
        wall_ms_per_step=wall * 1e3 / steps,
        init_s=init_s,
        stages=stages,
        roofline=dict(bound="hbm", kernel=kname, achieved=round(ach, 1), peak=HBM_PEAK_GBS,
                      unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 4), traffic=traffic,
                      algorithmic_bytes=sb[dominant],
                      avg_launch_ms=stages[dominant]["ms"]),
        check=dict(n_nan=d["n_nan"], step=d["step"],
                   mass_rel_gap=abs(d["mass_grid"] / d["mass_particles"] - 1.0)),
    )


def host_cpu():
    """Model name and core counts of the host the CPU baseline runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = None
    return dict(model=model, nproc=os.cpu_count(), usable=usable,
                omp_num_threads=os.environ.get("OMP_NUM_THREADS"))


def _oracle_time(ic, steps):
    from oracle import step as S
    prm = ic["params"]
    op = S.Params(N=prm["N"], dt=prm["dt"], L=prm["L"], D_u=prm["D_u"], chi=prm["chi"],
                  D_m=prm["D_m"], D_w=prm["D_w"], alpha=prm["alpha"], beta=prm["beta"],
                  gamma=prm["gamma"], seed=prm["seed"])
    st = S.State(ic["X0"], ic["a0"], ic["v0"], ic["m0"], ic["w0"], 0)
    t = time.perf_counter()
    S.run(st, op, steps)
    return time.perf_counter() - t


def cpu_baseline(ic, steps=3):
    """The FP64 numpy oracle as it stands, timed on the host on bounded samples: a few steps
    of the benchmark workload (the line's figure), the whole 16^3 / 4096-particle run (100
    steps) and the first steps of the 64^3 / 2^20-particle run.  The oracle is single-threaded
    numpy (its FFTs and array operations use one thread), so `cores` is 1."""
    from paper_2605_20140_amd import workloads as W
    prm = ic["params"]
    dt = _oracle_time(ic, steps)
    small = {}
    for name, nst in (("blob16", 100), ("modes64", 3)):
        icn = W.make_initial_state(name)
        t = _oracle_time(icn, nst)
        small[name] = dict(steps=nst, seconds=round(t, 2), N=icn["params"]["N"],
                           P=icn["params"]["P"],
                           particle_steps_per_s=icn["params"]["P"] * nst / t,
                           full_run_steps=icn["params"]["steps"])
    return dict(value=prm["P"] * steps / dt, unit="particle-steps/s", cores=1, threads=1,
                kind="oracle", host=host_cpu(),
                sample=f"{steps} steps of the full workload ({prm['N']}^3 grid, {prm['P']} "
                       "particles), float64 numpy oracle, single thread", seconds=round(dt, 2),
                other_configs=small)


def precision_errors(s32, s64, L=1.0):
    """Per-field error of the float32 form against the float64 form after the same steps
    (both on the GPU, same noise): relative L2 and max norms of v, m, w; positions as the
    largest and rms minimum-image distance over L; masses as the largest relative error."""
    import numpy as np
    out = {}
    for f in ("v", "m", "w"):
        d = s32[f] - s64[f]
        out[f] = dict(l2=float(np.linalg.norm(d) / np.linalg.norm(s64[f])),
                      max=float(np.abs(d).max() / np.abs(s64[f]).max()))
    d = s32["X"] - s64["X"]
    d = np.abs(d - L * np.round(d / L)) / L
    out["X"] = dict(max=float(d.max()), rms=float(np.sqrt((d ** 2).mean())))
    out["a"] = dict(max=float(np.abs(s32["a"] / s64["a"] - 1.0).max()))
    out["total_mass"] = float(abs(s32["a"].sum() / s64["a"].sum() - 1.0))
    out["step"] = s32["diag"]["step"]
    return out


def next_rows(ic, steps=50, warmup=5, profile_steps=8):
    """The rows beyond the plain step, each timed on its own: the fourth-order deposit and
    the low-pass filter on the benchmark workload (float32), one residual resampling of its
    particles with log-normal masses, the small configurations 16^3 / 4096 and 64^3 / 2^20,
    the 256^3 / 2^25 workload (float32; per-kernel split), and the paper's 2D example at
    1024^2 / 2^22 (float32)."""
    import numpy as np
    import torch
    from paper_2605_20140_amd import sipf, workloads as W
    out = {}
    prm = ic["params"]
    for name, over in (("order4", dict(deposit_order=4)), ("lowpass", dict(H0=prm["N"] / 2.0))):
        r = run_form(ic, 1, steps, warmup, profile_steps, "", **over)
        out[name] = dict(value=r["value"], unit="particle-steps/s", ms_per_step=r["ms_per_step"],
                         particles_ms=r["stages"]["particles"]["ms"],
                         xpass_ms=r["stages"]["xpass"]["ms"], check=r["check"], **over)
    # resampling: log-normal masses (the spread a long run accumulates)
    rng = np.random.Generator(np.random.Philox(7))
    a0 = W.weighted_masses(prm["P"], 1.0, rng)
    p = sipf.make_params(precision=1, **prm)
    sim = sipf.Simulation(p, ic["X0"], a0, ic["v0"], ic["m0"], ic["w0"], device="cuda:0")
    torch.cuda.synchronize()
    t = time.perf_counter()
    info = sim.resample()
    rs_s = time.perf_counter() - t
    sim.step(2)
    d = sim.fields(particles=False)["diag"]
    sim.close()
    out["resample"] = dict(ms=rs_s * 1e3, particles_per_s=prm["P"] / rs_s, n_stoch=info["n_stoch"],
                           a0=info["a0"], note="one synchronous call incl. re-binning and "
                           "deposit, float32 form", check=dict(n_nan=d["n_nan"]))
    # the small configurations, where a step is bound by launch latency rather than HBM:
    # 16^3 / 4096 (float64) and 64^3 / 2^20 (float64 and float32), whole runs of graph replays
    for name, prec, nst in (("blob16", 0, 100), ("modes64", 0, 500), ("modes64", 1, 500)):
        icn = W.make_initial_state(name)
        r = run_form(icn, prec, nst, warmup, profile_steps, "")
        out[f"{name}_{'fp32' if prec else 'fp64'}"] = dict(
            value=r["value"], unit="particle-steps/s", ms_per_step=r["ms_per_step"],
            steps=nst, N=icn["params"]["N"], P=icn["params"]["P"],
            stages_ms={k: v["ms"] for k, v in r["stages"].items()}, check=r["check"])
    # the largest single-GPU configuration: 256^3 grid, 2^25 particles, float32
    ic5 = W.make_initial_state("blobs256")
    r = run_form(ic5, 1, steps, warmup, profile_steps, "blobs256")
    out["blobs256"] = dict(value=r["value"], unit="particle-steps/s",
                           ms_per_step=r["ms_per_step"], N=256, P=ic5["params"]["P"],
                           stages=r["stages"], roofline=r["roofline"], check=r["check"])
    del ic5
    ic2 = W.paper2d_initial_state(1024)
    r = run_form(ic2, 1, steps, warmup, profile_steps, "")
    out["paper2d"] = dict(value=r["value"], unit="particle-steps/s",
                          ms_per_step=r["ms_per_step"], N=1024, P=ic2["params"]["P"],
                          stages_ms=r["stages"], check=r["check"])
    return out


def served(nreq, budget_gib, seed=4, graphs=False):
    """Served mix: Poisson arrivals at 0.7 x the solo capacity (requests/s measured by
    running a few requests alone first), continuous batching, p50/p99 latency and the tick
    loop's host time per tick (admission hand-off, joins, launches, fence waits,
    retirement hand-off, idle)."""
    import numpy as np
    from paper_2605_20140_amd import serve, workloads as W
    from concurrent.futures import ThreadPoolExecutor
    q = W.served_mix(nreq=nreq, rate=None, steps=200, seed=seed)
    reqs = serve.make_requests(q, lazy=True)
    # every request's initial state is made on the host before the run starts (numpy
    # releases the GIL in the bulk of it), so latency never includes input generation
    with ThreadPoolExecutor(8) as ex:
        for r, ic in zip(reqs, ex.map(W.served_initial_state, q)):
            r.ic = ic
    be = serve.GpuBackend(precision=1, graphs=graphs)
    # solo capacity: the first few requests, one at a time (once untimed, so that first-use
    # costs such as module loading do not lower the rate)
    probe = reqs[:8]
    for _ in range(2):
        t = time.perf_counter()
        srv = serve.Server(be, budget_gib << 30, max_slots=1, tick_steps=50)
        srv.run([serve.Request(r.rid, 0.0, r.N, r.P, r.steps, r.params, r.ic) for r in probe])
        solo_s = (time.perf_counter() - t) / len(probe)
    rate = 0.7 / solo_s
    # one request of each size class alone, with the mix's tick length: its solo latency
    cls = lambda r: f"N{r.N}_P{'lo' if r.P < (1 << 19) else 'hi'}"
    firsts = {}
    for r in reqs:
        firsts.setdefault(cls(r), r)
    solo_by = {}
    for k, r in sorted(firsts.items()):
        srv = serve.Server(be, budget_gib << 30, max_slots=1, tick_steps=10)
        rec, _ = srv.run([serve.Request(r.rid, 0.0, r.N, r.P, r.steps, r.params, r.ic)])
        solo_by[k] = round(1e3 * rec[r.rid].latency, 1)
    rng = np.random.Generator(np.random.Philox(seed))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(reqs)))
    for r, ta in zip(reqs, arrivals):
        r.t_arrive = float(ta)
    srv = serve.Server(be, budget_gib << 30, max_slots=64, tick_steps=10)
    recs, summ = srv.run(reqs)
    be.close()
    # latency by request size: the grid and the particle count's half of the log range
    by = {}
    for r in reqs:
        key = f"N{r.N}_P{'lo' if r.P < (1 << 19) else 'hi'}"
        by.setdefault(key, []).append(recs[r.rid].latency)
    summ["latency_by_size_ms"] = {
        k: dict(n=len(v), p50=round(1e3 * float(np.percentile(v, 50)), 1),
                p99=round(1e3 * float(np.percentile(v, 99)), 1), solo=solo_by.get(k))
        for k, v in sorted(by.items())}
    summ.update(rate_per_s=rate, solo_service_s=solo_s, hbm_budget_gib=budget_gib,
                max_slots=64, tick_steps=10, form="fp32",
                step_path="captured graph per batch" if graphs else "allocation-free batched step",
                mix="N in {32,64,128}, P = 2^U(16,22), chi = 10^U(-3,-2), 200 steps, dt 1e-3")
    summ["p99_over_p50"] = summ["latency_p99_s"] / summ["latency_p50_s"]
    return summ


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="blobs128")
    ap.add_argument("--profile-steps", type=int, default=24)
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-next-rows", action="store_true",
                    help="skip the order-4 / low-pass / resampling / 2D measurements")
    ap.add_argument("--served-requests", type=int, default=256,
                    help="requests in the served-mix run (0: skip it)")
    ap.add_argument("--served-graphs", action="store_true",
                    help="served mix through sipf_step_batch's captured graphs instead of "
                         "the allocation-free batched step")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device-to-device copy of 512 MiB (the reference "
                         "the byte counters are scaled by)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the library has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    from paper_2605_20140_amd import workloads as W
    ic = W.make_initial_state(args.workload)
    prm = ic["params"]
    keep = not args.no_fp64
    r32 = run_form(ic, 1, args.steps, args.warmup, args.profile_steps, args.workload,
                   keep_state=keep)
    r64 = (None if args.no_fp64 else
           run_form(ic, 0, args.steps, args.warmup, args.profile_steps, args.workload,
                    keep_state=keep))
    errs = precision_errors(r32.pop("state"), r64.pop("state"), prm["L"]) if keep else None
    r32.pop("state", None)
    if args.copy_calibration:
        copy_calibration()
    nxt = None if args.no_next_rows else next_rows(ic)
    srv = (served(args.served_requests, 32, graphs=args.served_graphs)
           if args.served_requests > 0 else None)
    cpu = None if args.no_cpu_baseline else cpu_baseline(ic)
    line = {
        "metric": METRIC,
        "value": r32["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": prm["N"], "P": prm["P"], "dt": prm["dt"],
                   "form": "fp32 positions/fields/FFT, fp64 masses and sums",
                   "parallelism": "single GPU"},
        "roofline": r32["roofline"],
        "cpu_baseline": cpu,
        "init_s": r32["init_s"],
        "stages": r32["stages"],
        "check": r32["check"],
        "served": srv,
        "next_rows": nxt,
        "fp32_vs_fp64": errs,
        "fp64": None if r64 is None else {
            "value": r64["value"], "ms_per_step": r64["ms_per_step"], "dtype": "f64",
            "init_s": r64["init_s"],
            "roofline": r64["roofline"], "stages": r64["stages"], "check": r64["check"]},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
