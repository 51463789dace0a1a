"""Residual resampling (Alg. res_res) through the C ABI against the oracle.

On identical seeded inputs (a fresh state with unequal masses) the particle list is a
function of the input alone on both sides, so it must agree bit for bit: positions, masses,
and the counts.  After steps taken on the GPU the state differs from the oracle's in the last
bits, so there the checks are the properties the algorithm fixes, computed from the GPU's own
state before the call.
"""
import math

import numpy as np
import pytest

from oracle import resample as RS
from oracle import step as S
from paper_2605_20140_amd import sipf
from paper_2605_20140_amd import workloads as W

from _parity import compare_state, gpu_sim, oracle_params, oracle_state

pytestmark = pytest.mark.gpu


def _weighted(N, P, spread=1.0, **kw):
    ic = W.make_initial_state("blob16", N=N, P=P, mass_spread=spread, **kw)
    assert np.all((ic["X0"] >= 0) & (ic["X0"] < 1.0))
    return ic


@pytest.mark.parametrize("N,P,spread", [(16, 4096, 1.0), (32, 4096 * 3 + 77, 0.3),
                                        (8, 1, 1.0), (16, 5000, 3.0)])
def test_fresh_state_bit_exact_fp64(N, P, spread):
    ic = _weighted(N, P, spread)
    sim = gpu_sim(ic, sim_id=7)
    info = sim.resample()
    out = sim.fields()
    sim.close()
    Xr, ar, ref = RS.residual_resample(ic["X0"], ic["a0"], n=0, sim_id=7,
                                       seed=ic["params"]["seed"])
    assert info["a0"] == ref["a0"]
    assert info["n_det"] == ref["n_det"] and info["n_stoch"] == ref["n_stoch"]
    assert np.array_equal(out["a"], ar)
    assert np.array_equal(out["X"], Xr)
    d = out["diag"]
    assert d["step"] == 0
    assert d["mass_particles"] == pytest.approx(P * ref["a0"], rel=1e-13)
    assert d["mass_grid"] == pytest.approx(d["mass_particles"], rel=1e-12)


def test_fresh_state_bit_exact_fp32_positions():
    ic = _weighted(16, 4096, 1.0)
    sim = gpu_sim(ic, precision=1)
    info = sim.resample()
    out = sim.fields()
    sim.close()
    _, ar, ref = RS.residual_resample(ic["X0"], ic["a0"], n=0, sim_id=0,
                                      seed=ic["params"]["seed"])
    X32 = ic["X0"].astype(np.float32).astype(np.float64)
    assert info["a0"] == ref["a0"] and info["n_stoch"] == ref["n_stoch"]
    assert np.array_equal(out["a"], ar)
    assert np.array_equal(out["X"], X32[ref["src"]])


def test_large_fresh_state_bit_exact():
    """2^20 particles on 64^3: many scan blocks and a long draw list."""
    ic = _weighted(64, 1 << 20, 0.5)
    sim = gpu_sim(ic, sim_id=3)
    info = sim.resample()
    out = sim.fields()
    sim.close()
    Xr, ar, ref = RS.residual_resample(ic["X0"], ic["a0"], n=0, sim_id=3,
                                       seed=ic["params"]["seed"])
    assert info["n_stoch"] == ref["n_stoch"] and info["n_stoch"] > 1000
    assert np.array_equal(out["a"], ar)
    assert np.array_equal(out["X"], Xr)


def test_steps_after_resampling_match_oracle():
    ic = _weighted(16, 4096, 1.0)
    sim = gpu_sim(ic)
    sim.resample()
    sim.step(20)
    out = sim.fields()
    sim.close()
    Xr, ar, _ = RS.residual_resample(ic["X0"], ic["a0"], n=0, sim_id=0,
                                     seed=ic["params"]["seed"])
    st = oracle_state(ic)
    st = S.State(Xr, ar, st.v, st.m, st.w, 0)
    ref = S.run(st, oracle_params(ic["params"]), 20)
    compare_state(out, ref, 1e-10)


@pytest.mark.parametrize("precision", [0, 1])
def test_properties_after_gpu_steps(precision):
    """Resampling at step n > 0 of a GPU run: checked against the GPU's own state."""
    ic = W.make_initial_state("blob16", P=6000)
    sim = gpu_sim(ic, precision=precision, sim_id=2)
    sim.step(37)
    before = sim.fields()
    info = sim.resample()
    after = sim.fields()
    a, X = before["a"], before["X"]
    P = a.shape[0]
    a0 = math.fsum(a.tolist()) / P
    assert info["a0"] == a0
    assert np.all(after["a"] == a0)
    assert after["diag"]["step"] == 37 == before["diag"]["step"]
    for f in ("v", "m", "w"):
        assert np.array_equal(after[f], before[f])
    # every output particle is a copy of an input particle; count the copies
    index = {tuple(x): p for p, x in enumerate(X)}
    assert len(index) == P
    src = np.array([index[tuple(x)] for x in after["X"]])
    cnt = np.bincount(src, minlength=P)
    k = np.floor(a / a0).astype(np.int64)
    assert np.all(cnt >= k) and cnt.sum() == P
    assert info["n_det"] == k.sum() and info["n_stoch"] == P - k.sum()
    # deterministic copies come first, in particle order
    assert np.array_equal(src[:k.sum()], np.repeat(np.arange(P), k))
    frac = a / a0 - k
    assert np.all(frac[np.bincount(src[k.sum():], minlength=P) > 0] > 0)
    # the state keeps stepping
    sim.step(10)
    d = sim.fields()["diag"]
    sim.close()
    assert d["step"] == 47 and d["n_nan"] == 0
    assert d["mass_grid"] == pytest.approx(d["mass_particles"], rel=1e-5)


def test_empty_particle_set_is_a_no_op():
    ic = W.make_initial_state("blob16", P=0)
    sim = gpu_sim(ic)
    assert sim.resample() == dict(a0=0.0, n_det=0, n_stoch=0)
    sim.step(2)
    assert sim.fields()["diag"]["step"] == 2
    sim.close()


def test_out_of_range_masses_rejected_and_state_kept():
    ic = W.make_initial_state("blob16", P=100)
    a = np.full(100, 1e-2)
    a[3] = 1e-55                       # 2^-160 of the largest mass is about 6.8e-51
    ic["a0"] = a
    sim = gpu_sim(ic)
    before = sim.fields()
    with pytest.raises(sipf.SipfError) as e:
        sim.resample()
    assert e.value.code == -1
    after = sim.fields()
    sim.close()
    assert np.array_equal(after["X"], before["X"]) and np.array_equal(after["a"], before["a"])
