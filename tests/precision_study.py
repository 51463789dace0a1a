"""Per-field error of the float32 form against the FP64 oracle over whole runs (test
infrastructure: it imports the oracle; not collected by pytest).

Two stages, so that the slow oracle can run on any host:

  python tests/precision_study.py gpu CASE OUT.npz      (needs the GPU and libsipf.so)
      runs CASE in the float32 form (and the float64 form) through the C ABI and saves the
      final states;
  python tests/precision_study.py oracle CASE OUT.npz [REF.npz]   (CPU only)
      runs the oracle on the same seeded inputs for the same steps and prints the relative
      L2 and max errors of v, m, w, the largest minimum-image position error and the largest
      relative mass error of each saved GPU state (REF.npz: where the oracle's final state
      is cached; OUT.npz "-" runs and caches the oracle only).

CASE is "modes64" (64^3 grid, random-mode ECM field, dt 1e-3, 500 steps) or "blobs128"
(128^3 grid, four blobs, dt 5e-4, 1000 steps), each with 2^16 particles so that the oracle
finishes in minutes; the field errors, which dominate, do not depend on the particle count.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

CASES = {"modes64": dict(P=1 << 16), "blobs128": dict(P=1 << 16)}


def initial(case):
    from paper_2605_20140_amd import workloads as W
    return W.make_initial_state(case, **CASES[case])


def run_gpu(case, out):
    from _parity import gpu_sim
    ic = initial(case)
    steps = ic["params"]["steps"]
    res = {}
    # the float32 form's state is stored exactly in float32; the float64 form's full state
    # only where it stays small (64^3)
    for prec in ((1, 0) if ic["params"]["N"] <= 64 else (1,)):
        sim = gpu_sim(ic, precision=prec)
        sim.step(steps)
        o = sim.fields()
        sim.close()
        tag = "fp32" if prec else "fp64"
        for k in ("v", "m", "w", "X"):
            res[f"{tag}_{k}"] = o[k].astype(np.float32) if prec else o[k]
        res[f"{tag}_a"] = o["a"]
        res[f"{tag}_step"] = o["diag"]["step"]
    np.savez_compressed(out, **res)
    print(f"{case}: {steps} steps saved to {out}", flush=True)


def errors(got, ref, L):
    from _parity import rel_errors, min_image
    e = {}
    for f in ("v", "m", "w"):
        l2, mx = rel_errors(got[f], getattr(ref, f))
        e[f] = dict(l2=l2, max=mx)
    d = np.abs(min_image(got["X"] - ref.X, L)) / L
    e["X"] = dict(max=float(d.max()), rms=float(np.sqrt((d ** 2).mean())))
    e["a"] = dict(max=float(np.abs(got["a"] / ref.a - 1.0).max()))
    return e


def oracle_final(case, cache=None):
    """The oracle's state after the case's steps (read from / written to cache if given)."""
    from oracle import step as S
    from _parity import oracle_params, oracle_state
    ic = initial(case)
    if cache and os.path.exists(cache):
        z = np.load(cache)
        return S.State(z["X"], z["a"], z["v"], z["m"], z["w"], int(z["n"])), 0.0
    t = time.time()
    ref = S.run(oracle_state(ic), oracle_params(ic["params"]), ic["params"]["steps"])
    dt = time.time() - t
    if cache:
        np.savez(cache, X=ref.X, a=ref.a, v=ref.v, m=ref.m, w=ref.w, n=ref.n)
    return ref, dt


def run_oracle(case, saved, cache=None):
    ic = initial(case)
    steps = ic["params"]["steps"]
    z = np.load(saved) if saved != "-" else {}
    ref, t = oracle_final(case, cache)
    assert ref.n == steps
    L = ic["params"]["L"]
    out = dict(case=case, steps=steps, P=ic["params"]["P"], N=ic["params"]["N"],
               oracle_s=round(t, 1))
    for tag in ("fp32", "fp64"):
        if f"{tag}_v" not in z:
            continue
        got = {k: z[f"{tag}_{k}"].astype(np.float64) for k in ("v", "m", "w", "X", "a")}
        assert int(z[f"{tag}_step"]) == steps
        out[tag] = errors(got, ref, L)
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    mode, case, path = sys.argv[1], sys.argv[2], sys.argv[3]
    if mode == "gpu":
        run_gpu(case, path)
    else:
        run_oracle(case, path, sys.argv[4] if len(sys.argv) > 4 else None)
