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
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = ("particle-steps/s + HBM GB/s fraction at 128^3/2^23 (FP32 vs FP64); "
          "p50/p99 served")


def stage_bytes(N, P, s):
    """Bytes each stage must move per step by design (reads + writes), s = 4 or 8."""
    G = N ** 3
    half = (N // 2 + 1) * N * N * 2 * s  # one half spectrum
    return {
        "zfwd": G * 4 * s + G * 2 * s + 3 * half,
        "yfwd": 6 * half,
        "xpass": 6 * half,
        "yinv": 9 * half,
        "zinv": 5 * half + G * s + G * 6 * s,
        # particles: read x,y,z,a; write x,y,z,a (SURVEY per-particle figure; the 4-byte
        # noise key is not counted) + gather array read once + deposit target written once
        "particles": P * (6 * s + 16) + G * 5 * s,
        "finalize": 0,
        # binning, per binning: count reads x,y,z and writes (tile, rank); scatter reads the
        # keys and one particle set and writes the other
        "binning": P * (3 * s + 8) + P * (8 + 2 * (3 * s + 8 + 4)),
    }


RESORT_EVERY = 8  # library default binning period


def run_form(ic, precision, steps, warmup, profile_steps):
    import torch
    from paper_2605_20140_amd import sipf
    prm = ic["params"]
    p = sipf.make_params(precision=precision, **prm)
    sim = sipf.Simulation(p, ic["X0"], ic["a0"], ic["v0"], ic["m0"], ic["w0"], device="cuda:0")
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
    out = sim.fields(particles=False)
    sim.close()
    d = out["diag"]
    s = 4 if precision == 1 else 8
    sb = stage_bytes(prm["N"], prm["P"], s)
    stages = {}
    for k, tot in stage_ms.items():
        avg = tot / profile_steps  # per step (binning: amortised over its period)
        nbytes = sb[k] / RESORT_EVERY if k == "binning" else sb[k]
        stages[k] = dict(ms=round(avg, 5),
                         GBs=round(nbytes / (avg * 1e-3) / 1e9, 1) if avg > 0 and nbytes else None)
    dominant = max(stages, key=lambda k: stages[k]["ms"])
    ach = sb[dominant] / (stages[dominant]["ms"] * 1e-3) / 1e9
    return dict(
        value=prm["P"] * steps / (ms * 1e-3),
        ms_per_step=ms / steps,
        wall_ms_per_step=wall * 1e3 / steps,
        stages=stages,
        roofline=dict(bound="hbm", kernel=dominant, achieved=round(ach, 1), peak=HBM_PEAK_GBS,
                      unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 4), traffic=None,
                      algorithmic_bytes=sb[dominant]),
        check=dict(n_nan=d["n_nan"], step=d["step"],
                   mass_rel_gap=abs(d["mass_grid"] / d["mass_particles"] - 1.0)),
    )


def cpu_baseline(ic):
    """FP64 numpy oracle, one step of the same workload on the host (bounded sample)."""
    from oracle import step as S
    prm = ic["params"]
    op = S.Params(N=prm["N"], dt=prm["dt"], L=prm["L"], D_u=prm["D_u"], chi=prm["chi"],
                  D_m=prm["D_m"], D_w=prm["D_w"], alpha=prm["alpha"], beta=prm["beta"],
                  gamma=prm["gamma"], seed=prm["seed"])
    st = S.State(ic["X0"], ic["a0"], ic["v0"], ic["m0"], ic["w0"], 0)
    t = time.perf_counter()
    S.step(st, op)
    dt = time.perf_counter() - t
    return dict(value=prm["P"] / dt, unit="particle-steps/s", cores=1, kind="oracle",
                sample=f"1 step of the full workload ({prm['N']}^3 grid, {prm['P']} particles), "
                       "float64 numpy oracle, single thread", seconds=round(dt, 2))


def served(nreq, budget_gib, seed=4):
    """Served mix: Poisson arrivals at 0.7 x the solo capacity (requests/s measured by
    running a few requests alone first), continuous batching, p50/p99 latency."""
    import numpy as np
    from paper_2605_20140_amd import serve, workloads as W
    q = W.served_mix(nreq=nreq, rate=None, steps=200, seed=seed)
    reqs = serve.make_requests(q)
    be = serve.GpuBackend(precision=1)
    # solo capacity: the first few requests, one at a time
    probe = reqs[:4]
    t = time.perf_counter()
    srv = serve.Server(be, budget_gib << 30, max_slots=1, tick_steps=50)
    srv.run([serve.Request(r.rid, 0.0, r.N, r.P, r.steps, r.params, r.ic) for r in probe])
    solo_s = (time.perf_counter() - t) / len(probe)
    rate = 0.7 / solo_s
    rng = np.random.Generator(np.random.Philox(seed))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(reqs)))
    for r, ta in zip(reqs, arrivals):
        r.t_arrive = float(ta)
    srv = serve.Server(be, budget_gib << 30, max_slots=64, tick_steps=10)
    _, summ = srv.run(reqs)
    summ.update(rate_per_s=rate, solo_service_s=solo_s, hbm_budget_gib=budget_gib,
                max_slots=64, tick_steps=10, form="fp32",
                mix="N in {32,64,128}, P = 2^U(16,22), chi = 10^U(-3,-2), 200 steps, dt 1e-3")
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
    ap.add_argument("--served-requests", type=int, default=48,
                    help="requests in the served-mix run (0: skip it)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device copy of 512 MiB (reference for byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): this build has no "
              "multi-GPU path; the sharding design is described in DESIGN.md.", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    from paper_2605_20140_amd import workloads as W
    ic = W.make_initial_state(args.workload)
    prm = ic["params"]
    r32 = run_form(ic, 1, args.steps, args.warmup, args.profile_steps)
    r64 = None if args.no_fp64 else run_form(ic, 0, args.steps, args.warmup, args.profile_steps)
    if args.copy_calibration:
        src = torch.empty(512 << 20, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    srv = served(args.served_requests, 32) if args.served_requests > 0 else None
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
        "stages": r32["stages"],
        "check": r32["check"],
        "served": srv,
        "fp64": None if r64 is None else {
            "value": r64["value"], "ms_per_step": r64["ms_per_step"], "dtype": "f64",
            "roofline": r64["roofline"], "stages": r64["stages"], "check": r64["check"]},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
