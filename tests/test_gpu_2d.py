"""Two-dimensional form (the paper's 2D example, dim = 2) through the C ABI against the FP64
oracle on identical seeded inputs: deposit, gradient, whole steps on both particle paths
(global atomics below 32^2, LDS tiles from 32^2), float32, the step variants, the low-pass
filter and resampling.  Tolerances as in 3D: 1e-10 (float64), 1e-4 (float32)."""
import numpy as np
import pytest

from oracle import pic
from oracle import resample as RS
from oracle import step as S
from paper_2605_20140_amd import workloads as W

from _parity import compare_state, flags_of, gpu_sim, oracle_params, oracle_state, rel_errors

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-4


def _run(ic, steps, precision=0, **kw):
    sim = gpu_sim(ic, precision=precision, flags=flags_of(**kw),
                  **{k: v for k, v in kw.items() if k == "H0"})
    sim.step(steps)
    out = sim.fields()
    u, g = sim.aux()
    sim.close()
    prm = oracle_params(ic["params"], **kw)
    st = oracle_state(ic)
    aux = None
    for _ in range(steps):
        st, aux = S.step(st, prm, return_aux=True)
    return out, u, g, st, aux


@pytest.mark.parametrize("N,P", [(8, 300), (32, 4096 * 2 + 77), (128, 50000)])
def test_2d_initial_deposit(N, P):
    ic = W.blob2d_initial_state(N=N, P=P)
    sim = gpu_sim(ic)
    u, _ = sim.aux()
    d = sim.fields(particles=False)["diag"]
    sim.close()
    assert u.shape == (N, N)
    assert max(rel_errors(u, pic.deposit(ic["X0"], ic["a0"], N, 1.0))) < 1e-12
    assert d["mass_grid"] == pytest.approx(d["mass_particles"], rel=1e-12)


@pytest.mark.parametrize("N,P,steps", [(8, 300, 7), (32, 4096 + 77, 25), (64, 20000, 5),
                                       (256, 30000, 2)])
def test_2d_steps_fp64(N, P, steps):
    ic = W.blob2d_initial_state(N=N, P=P)
    out, u, g, ref, aux = _run(ic, steps)
    compare_state(out, ref, TOL64)
    for j in range(2):
        assert max(rel_errors(g[j], aux["grad"][j])) < 1e-11, j
    assert max(rel_errors(u, pic.deposit(ref.X, ref.a, N, 1.0))) < 1e-10
    assert out["diag"]["step"] == steps and out["diag"]["n_nan"] == 0


@pytest.mark.parametrize("resort_every", [1, 0])
def test_2d_rebinning_period(resort_every):
    """Every step, and the library's default period (four-cell tile margins in 2D)."""
    ic = W.blob2d_initial_state(N=64, P=20000)
    sim = gpu_sim(ic, resort_every=resort_every)
    sim.step(12)
    out = sim.fields()
    sim.close()
    ref = S.run(oracle_state(ic), oracle_params(ic["params"]), 12)
    compare_state(out, ref, TOL64)


def test_2d_fp32():
    ic = W.blob2d_initial_state(N=64, P=20000)
    out, _, _, ref, _ = _run(ic, 30, precision=1)
    compare_state(out, ref, TOL32)


def test_2d_fp32_largest_grid():
    """1024^2, float32 (the finest grid of the paper's 2D refinement)."""
    ic = W.blob2d_initial_state(N=1024, P=1 << 16)
    out, _, _, ref, _ = _run(ic, 2, precision=1)
    compare_state(out, ref, TOL32)


@pytest.mark.parametrize("kw", [dict(no_noise=True), dict(linear_mass=True),
                                dict(implicit_v=True), dict(diffusion="exp"),
                                dict(freeze_w=True), dict(H0=16.0)])
def test_2d_variants_fp64(kw):
    ic = W.blob2d_initial_state(N=32, P=3000)
    out, _, _, ref, _ = _run(ic, 10, **kw)
    compare_state(out, ref, TOL64)


def test_2d_aliased_kernel_fp64():
    ic = W.blob2d_initial_state(N=16, P=3000, D_m=5.0, D_w=8.0)
    out, _, _, ref, _ = _run(ic, 10, diffusion="aliased")
    compare_state(out, ref, TOL64)


def test_2d_lowpass_fp32_largest_grid():
    ic = W.blob2d_initial_state(N=512, P=20000)
    out, _, _, ref, _ = _run(ic, 2, precision=1, H0=256.0)
    compare_state(out, ref, TOL32)


def test_2d_resample_bit_exact():
    ic = W.blob2d_initial_state(N=64, P=10000, mass_spread=1.0)
    sim = gpu_sim(ic, sim_id=4)
    info = sim.resample()
    out = sim.fields()
    sim.step(5)
    after = sim.fields()
    sim.close()
    Xr, ar, ref = RS.residual_resample(ic["X0"], ic["a0"], n=0, sim_id=4,
                                       seed=ic["params"]["seed"])
    assert info["n_stoch"] == ref["n_stoch"] and info["a0"] == ref["a0"]
    assert np.array_equal(out["X"], Xr) and np.array_equal(out["a"], ar)
    st = oracle_state(ic)
    st = S.State(Xr, ar, st.v, st.m, st.w, 0)
    compare_state(after, S.run(st, oracle_params(dict(ic["params"], sim_id=4)), 5), TOL64)


def test_2d_batch_rejected():
    from paper_2605_20140_amd import sipf
    ic = W.blob2d_initial_state(N=16, P=100)
    sim = gpu_sim(ic)
    with pytest.raises(sipf.SipfError):
        sipf.step_batch([sim], 1)
    sim.close()


def test_2d_fp64_largest_grid():
    """1024^2 in float64: two rows per block in the row passes (raised LDS limit)."""
    ic = W.blob2d_initial_state(N=1024, P=1 << 16)
    out, _, g, ref, aux = _run(ic, 2)
    compare_state(out, ref, TOL64)
    for j in range(2):
        assert max(rel_errors(g[j], aux["grad"][j])) < 1e-11, j
