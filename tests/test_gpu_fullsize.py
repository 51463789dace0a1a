"""Parity at the full sizes of the benchmark workloads: 128^3 grid with 2^23 particles (float32
and float64 forms) and 256^3 with 2^25 particles (float32), and at the largest grid the
library takes, 512^3 (2^18 particles, both forms), the simulation stepped through the
captured step graph as the benchmark steps it.

The oracle cannot take whole steps at these sizes within test time, so each case checks
what it can compute on its own from the same seeded initial state:
* the initial deposit ubar^0 on the whole grid (Alg. p2g, trilinear R_h);
* the gradient of v^0 that drove the first push, on the whole grid (eq. gradv), within a
  bound derived from the rounding of the working precision (gradient_tolerance);
* the first step's v^1, m^1, w^1 on the whole grid (reaction and implicit solves of the
  oracle's field update, fed by the oracle's own deposit);
* the first step's positions and masses of a sample of particles: the first and last 64
  indices and 2^16 random ones, advanced by the oracle's particle update from the initial
  state (the noise is keyed by particle index, so any subset can be advanced alone);
* after 24 more steps (two re-binnings inside the captured graph), the properties that hold
  at any size: partition of unity h^3 sum ubar = sum_p a_p, the per-step mass bounds of
  Lemma mass (e^{-tau} <= a^{n+1} / a^n <= e^{tau}, so e^{-n tau} <= a^n / a^0 <= e^{n tau}),
  positivity of ubar, v and a, and no non-finite values.
Tolerances as in the other parity tests: 1e-10 (float64 form), 1e-4 (float32 form).
"""
import numpy as np
import pytest

from oracle import pic, spectral
from oracle import step as S
from paper_2605_20140_amd import workloads as W

from _parity import (gpu_sim, gradient_tolerance, min_image, oracle_params, oracle_state,
                     rel_errors)

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-4}
_cache = {}


def _oracle_first_step(name, **over):
    """Initial state, oracle deposit, gradient, first-step fields and sampled particles."""
    key = (name, tuple(sorted(over.items())))
    if key in _cache:
        return _cache[key]
    _cache.clear()
    ic = W.make_initial_state(name, **over)
    prm = oracle_params(ic["params"])
    st = oracle_state(ic)
    P, N, L = st.X.shape[0], prm.N, prm.L
    ubar = pic.deposit(st.X, st.a, N, L)
    grad = spectral.gradient(st.v, L)
    v1, m1, w1 = S.field_update(ubar, st.v, st.m, st.w, prm)
    rng = np.random.default_rng(7)
    ids = np.unique(np.concatenate([np.arange(64), np.arange(P - 64, P),
                                    rng.choice(P, 1 << 16, replace=False)]))
    g = pic.gather(list(grad) + [st.w], st.X[ids], N, L)
    X1, a1, _ = S.particle_update(st.X[ids], st.a[ids], ids, g, st.n, prm)
    ref = dict(ic=ic, prm=prm, ubar=ubar, grad=grad, v=v1, m=m1, w=w1, ids=ids, X=X1, a=a1)
    _cache[key] = ref
    return ref


def _check_fields(got, ref, tol, what):
    for k in got:
        assert np.all(np.isfinite(got[k])), (what, k)
        l2, mx = rel_errors(got[k], ref[k])
        assert max(l2, mx) <= tol, f"{what} {k}: relative L2 {l2:.3g}, max {mx:.3g} > {tol}"


# the benchmark workloads, and the largest grid the library takes (512^3) with 2^18
# particles in one blob
CASES = [("blobs128", {}, 1), ("blobs128", {}, 0), ("blobs256", {}, 1),
         ("blob16", dict(N=512, P=1 << 18), 1), ("blob16", dict(N=512, P=1 << 18), 0)]


@pytest.mark.parametrize("name,over,precision", CASES,
                         ids=[f"{c[0]}-{c[1].get('N', '')}-{'fp32' if c[2] else 'fp64'}"
                              for c in CASES])
def test_full_size_first_step_and_invariants(name, over, precision):
    ref = _oracle_first_step(name, **over)
    ic, prm, tol = ref["ic"], ref["prm"], TOL[precision]
    N, L, dt = prm.N, prm.L, prm.dt
    P = ic["X0"].shape[0]
    print(f"full-size case {name} {over} precision {precision}: N {N} P {P}", flush=True)
    sim = gpu_sim(ic, precision=precision)
    try:
        u0, _ = sim.aux()
        _check_fields(dict(ubar=u0), ref, tol, "initial deposit")
        sim.step(1)
        out = sim.fields(particles=True)
        _, grad = sim.aux()
        tol_g = gradient_tolerance(ic["v0"], ref["grad"], L, precision)
        _check_fields(dict(g0=grad[0], g1=grad[1], g2=grad[2]),
                      dict(g0=ref["grad"][0], g1=ref["grad"][1], g2=ref["grad"][2]), tol_g,
                      "gradient of v^0")
        _check_fields(dict(v=out["v"], m=out["m"], w=out["w"]), ref, tol, "first step")
        ids = ref["ids"]
        Xg, ag = out["X"][ids], out["a"][ids]
        assert np.all(np.isfinite(Xg)) and np.all(np.isfinite(ag))
        ex = np.abs(min_image(Xg - ref["X"], L)).max() / L
        ea = np.abs(ag / ref["a"] - 1.0).max()
        assert ex <= tol and ea <= tol, f"sampled particles: X {ex:.3g}, a {ea:.3g} > {tol}"
        assert out["diag"]["step"] == 1

        # invariants after 24 more steps (two re-binnings at the default period)
        a0_sum = float(np.sum(ic["a0"]))
        a_prev = out["a"]
        n = 25
        sim.step(n - 1)
        out = sim.fields(particles=True)
        u, _ = sim.aux()
        a = out["a"]
        assert np.all(np.isfinite(out["X"])) and np.all(np.isfinite(a))
        assert np.all(np.isfinite(u)) and np.all(np.isfinite(out["v"]))
        assert np.all(np.isfinite(out["m"])) and np.all(np.isfinite(out["w"]))
        assert u.min() >= 0.0 and out["v"].min() > 0.0 and a.min() > 0.0
        assert np.all((out["X"] >= 0.0) & (out["X"] < L))
        mass = float(np.sum(a))
        gap = abs(float(np.sum(u)) * (L / N) ** 3 - mass) / mass
        assert gap <= tol, f"partition of unity: relative gap {gap:.3g}"
        # Lemma mass per particle over steps 1 .. n (premise w >= 0, so 0 <= rho(w) < 2), with
        # one rounding of the factor per step
        assert out["w"].min() >= 0.0
        r = a / a_prev
        slack = (n - 1) * (1e-6 if precision else 1e-14)
        assert r.min() >= np.exp(-(n - 1) * dt) - slack and r.max() <= np.exp((n - 1) * dt) + slack
        assert np.exp(-n * dt) - n * 1e-6 <= mass / a0_sum <= np.exp(n * dt) + n * 1e-6
        assert out["diag"]["step"] == n and out["diag"]["n_nan"] == 0
    finally:
        sim.close()
