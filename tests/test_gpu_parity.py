"""Parity of the HIP path (through the C ABI) with the FP64 oracle on identical seeded
inputs.  Tolerances: float64 form 1e-10 relative (fields: relative L2 and max norms; particle
positions: max minimum-image distance / L; masses: max relative error); float32 form 1e-4 on
the same measures (the FP32 bound is checked over the lengths below, where rounding of
float32 positions and fields accumulates)."""
import numpy as np
import pytest

from oracle import pic, spectral
from oracle import step as S
from paper_2605_20140_amd import workloads as W

from _parity import (compare_state, flags_of, gpu_sim, gradient_tolerance, oracle_params,
                     oracle_state, rel_errors)

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-4


def _run_both(ic, nsteps, precision=0, sim_id=0, **kw):
    sim = gpu_sim(ic, precision=precision, flags=flags_of(**kw), sim_id=sim_id)
    sim.step(nsteps)
    out = sim.fields()
    sim.close()
    prm = oracle_params(dict(ic["params"], sim_id=sim_id), **kw)
    ref = S.run(oracle_state(ic), prm, nsteps)
    return out, ref, prm


def test_init_deposit_matches_oracle():
    ic = W.make_initial_state("blob16")
    sim = gpu_sim(ic)
    u, _ = sim.aux()
    out = sim.fields()
    ref = pic.deposit(ic["X0"], ic["a0"], 16, 1.0)
    assert max(rel_errors(u, ref)) < 1e-12
    d = out["diag"]
    assert d["mass_grid"] == pytest.approx(1.0, rel=1e-12)
    assert d["mass_particles"] == pytest.approx(1.0, rel=1e-13)
    assert d["step"] == 0


def test_one_step_gradient_and_deposit():
    ic = W.make_initial_state("modes64", N=32, P=50000)
    sim = gpu_sim(ic)
    sim.step(1)
    u, g = sim.aux()
    out = sim.fields()
    prm = oracle_params(ic["params"])
    ref, aux = S.step(oracle_state(ic), prm, return_aux=True)
    for j in range(3):
        assert max(rel_errors(g[j], aux["grad"][j])) < 1e-11, j
    u_ref = pic.deposit(ref.X, ref.a, 32, 1.0)
    assert max(rel_errors(u, u_ref)) < 1e-10
    compare_state(out, ref, TOL64)


def test_blob16_full_length_fp64():
    """16^3 grid, 4096 particles, 100 steps of dt = 1e-3."""
    ic = W.make_initial_state("blob16")
    out, ref, prm = _run_both(ic, 100)
    errs = compare_state(out, ref, TOL64)
    d = out["diag"]
    assert d["step"] == 100 and d["n_nan"] == 0
    assert d["mass_grid"] == pytest.approx(d["mass_particles"], rel=1e-12)
    od = S.diagnostics(ref, prm)
    for k in ("mass_particles", "mass_grid", "mass_m", "min_v", "min_m", "min_w", "max_m",
              "max_w", "min_a", "max_a", "min_u"):
        assert d[k] == pytest.approx(od[k], rel=1e-9, abs=1e-12), k
    for k in ("n_nan", "n_neg_m", "n_neg_w"):
        assert d[k] == od[k], k
    print("blob16 fp64 errors", errs)


@pytest.mark.parametrize("N,P,steps", [(4, 300, 5), (8, 257, 7), (32, 4096 + 77, 5),
                                       (64, 20000, 3)])
def test_sizes_and_ragged_tails_fp64(N, P, steps):
    ic = W.make_initial_state("blob16", N=N, P=P)
    out, ref, _ = _run_both(ic, steps)
    compare_state(out, ref, TOL64)


@pytest.mark.parametrize("resort_every", [1, 3, 7, 0])
def test_rebinning_period_changes_only_summation_order(resort_every):
    """Any tile re-binning period (0: the library's default from the diffusive step size)
    gives the oracle's state: the period reorders the particles in memory and the deposit's
    sums, nothing else."""
    ic = W.make_initial_state("blob16", N=32, P=4096 * 3 + 77)
    sim = gpu_sim(ic, resort_every=resort_every)
    sim.step(25)
    out = sim.fields()
    sim.close()
    ref = S.run(oracle_state(ic), oracle_params(ic["params"]), 25)
    compare_state(out, ref, TOL64)


def test_empty_particle_set_fp64():
    ic = W.make_initial_state("blob16", P=0)
    out, ref, _ = _run_both(ic, 10)
    compare_state(out, ref, TOL64)
    assert out["diag"]["mass_particles"] == 0.0


@pytest.mark.parametrize("kw", [dict(freeze_w=True), dict(freeze_v=True, freeze_m=True),
                                dict(no_noise=True), dict(linear_mass=True),
                                dict(implicit_v=True), dict(diffusion="exp")])
def test_variants_fp64(kw):
    ic = W.make_initial_state("blob16", P=3000)
    out, ref, _ = _run_both(ic, 20, **kw)
    compare_state(out, ref, TOL64)


@pytest.mark.parametrize("diffusion", ["exp", "aliased"])
def test_resolved_heat_kernel_variants_fp64(diffusion):
    """Exponential and aliased multipliers where the grid resolves the heat kernel
    (dt D (pi N / L)^2 > 10, the regime of Lemma kernel)."""
    ic = W.make_initial_state("blob16", P=3000, D_m=5.0, D_w=8.0)
    out, ref, _ = _run_both(ic, 10, diffusion=diffusion)
    compare_state(out, ref, TOL64)


def test_sim_id_and_seed_select_streams():
    ic = W.make_initial_state("blob16", P=2000)
    out, ref, _ = _run_both(ic, 3, sim_id=(7 << 32) + 5)
    compare_state(out, ref, TOL64)


def test_restart_from_checkpoint_matches_uninterrupted():
    ic = W.make_initial_state("blob16", P=2000)
    sim = gpu_sim(ic)
    sim.step(6)
    mid = sim.fields()
    sim.step(4)
    full = sim.fields()
    sim.close()
    ic2 = dict(ic, X0=mid["X"], a0=mid["a"], v0=mid["v"], m0=mid["m"], w0=mid["w"])
    sim2 = gpu_sim(ic2, step0=6)
    sim2.step(4)
    res = sim2.fields()
    sim2.close()
    for f in ("v", "m", "w"):
        assert max(rel_errors(res[f], full[f])) < 1e-12
    assert np.abs(res["X"] - full["X"]).max() < 1e-13
    assert res["diag"]["step"] == 10


def test_blob16_full_length_fp32():
    ic = W.make_initial_state("blob16")
    out, ref, _ = _run_both(ic, 100, precision=1)
    errs = compare_state(out, ref, TOL32)
    print("blob16 fp32 errors", errs)


def test_mass_update_outside_the_polynomial_range():
    """Steps of tau = 1/2 (the largest the library takes) from w0 = -0.2, a negative lobe such
    as the implicit solve leaves: rho(w) = 2w / (1 + w) = -1/2 there, so tau |rho - 1| = 3/4
    passes 1/2 at the first step (eq. u_hat_update) and the float32 form's mass update takes
    its wide-range path (2^k 2^f in place of the Taylor polynomial) for every particle.  Both
    forms against the oracle over three steps."""
    ic = W.make_initial_state("blob16", dt=0.5)
    w0 = -0.2
    ic["w0"] = np.full_like(ic["w0"], w0)
    tau, rho = ic["params"]["dt"], 2 * w0 / (1 + w0)
    assert tau == 0.5 and abs(tau * (rho - 1)) > 0.5
    for precision, tol in ((0, TOL64), (1, TOL32)):
        out, ref, _ = _run_both(ic, 3, precision=precision)
        errs = compare_state(out, ref, tol)
        print("wide-range mass update, precision", precision, errs)


def test_modes64_fp64_and_fp32_prefix():
    """64^3 grid, 2^20 particles: the first 5 steps in both forms."""
    ic = W.make_initial_state("modes64")
    prm = oracle_params(ic["params"])
    ref = S.run(oracle_state(ic), prm, 5)
    for precision, tol in ((0, TOL64), (1, TOL32)):
        sim = gpu_sim(ic, precision=precision)
        sim.step(5)
        out = sim.fields()
        sim.close()
        errs = compare_state(out, ref, tol)
        print("modes64 precision", precision, errs)


# ---- fourth-order assignment R_h^(4) (Sec. 2.2.1) ----

@pytest.mark.parametrize("N,P", [(8, 500), (16, 4096), (32, 4096 * 3 + 77)])
def test_init_deposit_order4_matches_oracle(N, P):
    """N = 8 takes the global-atomic path; N >= 16 the LDS tile regions with a 2-node margin."""
    ic = W.make_initial_state("blob16", N=N, P=P)
    sim = gpu_sim(ic, deposit_order=4)
    u, _ = sim.aux()
    out = sim.fields()
    sim.close()
    ref = pic.deposit(ic["X0"], ic["a0"], N, 1.0, order=4)
    assert max(rel_errors(u, ref)) < 1e-12
    # partition of unity: h^3 sum ubar is the particle mass for either order
    assert out["diag"]["mass_grid"] == pytest.approx(out["diag"]["mass_particles"], rel=1e-12)


@pytest.mark.parametrize("N,P,steps", [(8, 257, 7), (16, 4096, 30), (32, 4096 + 77, 5)])
def test_order4_steps_fp64(N, P, steps):
    ic = W.make_initial_state("blob16", N=N, P=P)
    sim = gpu_sim(ic, deposit_order=4)
    sim.step(steps)
    out = sim.fields()
    u, _ = sim.aux()
    sim.close()
    prm = oracle_params(ic["params"], deposit_order=4)
    ref = S.run(oracle_state(ic), prm, steps)
    compare_state(out, ref, TOL64)
    assert max(rel_errors(u, pic.deposit(ref.X, ref.a, N, 1.0, order=4))) < 1e-10


def test_order4_fp32():
    ic = W.make_initial_state("blob16")
    sim = gpu_sim(ic, precision=1, deposit_order=4)
    sim.step(50)
    out = sim.fields()
    sim.close()
    ref = S.run(oracle_state(ic), oracle_params(ic["params"], deposit_order=4), 50)
    compare_state(out, ref, TOL32)


# ---- the three-pass FFT path (planes too large for the LDS) without the filter ----

def test_three_pass_path_several_steps():
    """Float64 at N = 128, where a plane of a half spectrum no longer fits the LDS: the
    three-pass path, which forms grad v as one round trip per axis after the z transform
    (eq. gradv): y in the forward y pass, x in the x pass, z in the inverse z pass.  Three
    steps, so that gradients formed by the step's own field passes (not only by the
    initialisation's) drive the push."""
    ic = W.make_initial_state("modes64", N=128, P=20000)
    sim = gpu_sim(ic, precision=0)
    sim.step(3)
    out = sim.fields()
    _, g = sim.aux()
    sim.close()
    prm = oracle_params(ic["params"])
    st = oracle_state(ic)
    ref, aux = None, None
    for _ in range(3):
        ref, aux = S.step(st, prm, return_aux=True)
        st = ref
    compare_state(out, ref, TOL64)
    for j in range(3):
        assert max(rel_errors(g[j], aux["grad"][j])) < 1e-11, j


_ic256 = {}


@pytest.mark.parametrize("H0", [0.0, 128.0])
def test_three_pass_path_float32(H0):
    """Float32 at N = 256, the smallest grid whose planes no longer fit the LDS in float32:
    two steps of the three-pass path without the filter (grad v as per-axis round trips) and
    with it (full transforms of v, eq. gradv with the low-pass factor), state at the float32
    bound and each gradient component within the bound of its rounding (gradient_tolerance)."""
    if not _ic256:
        _ic256["ic"] = W.make_initial_state("modes64", N=256, P=1 << 15)
    ic = _ic256["ic"]
    sim = gpu_sim(ic, precision=1, H0=H0)
    sim.step(2)
    out = sim.fields()
    _, g = sim.aux()
    sim.close()
    prm = oracle_params(ic["params"], H0=H0)
    st = oracle_state(ic)
    ref, aux = None, None
    for _ in range(2):
        ref, aux = S.step(st, prm, return_aux=True)
        st = ref
    errs = compare_state(out, ref, TOL32)
    tol_g = gradient_tolerance(ref.v, aux["grad"], prm.L, 1)
    gerr = [max(rel_errors(g[j], aux["grad"][j])) for j in range(3)]
    print(f"three-pass float32 H0 {H0}: state {errs}, gradient {gerr} (bound {tol_g:.3g})")
    assert max(gerr) < tol_g, (gerr, tol_g)


# ---- low-pass filter exp(-2 pi^2 |q|^2 / H0^2) (Alg. p2g text, Alg. sipf-pic) ----

@pytest.mark.parametrize("N,P,steps,precision", [(16, 4096, 20, 0), (64, 30000, 3, 0),
                                                 (128, 20000, 2, 0), (32, 4096, 20, 1)])
def test_lowpass_filter(N, P, steps, precision):
    """N <= 64 (float64) and N <= 128 (float32) take the plane kernel; N = 128 in float64 the
    three-pass path."""
    ic = W.make_initial_state("modes64", N=N, P=P)
    H0 = N / 2
    sim = gpu_sim(ic, precision=precision, H0=H0)
    sim.step(steps)
    out = sim.fields()
    _, g = sim.aux()
    sim.close()
    prm = oracle_params(ic["params"], H0=H0)
    ref, aux = None, None
    st = oracle_state(ic)
    for _ in range(steps):
        ref, aux = S.step(st, prm, return_aux=True)
        st = ref
    compare_state(out, ref, TOL64 if precision == 0 else TOL32)
    if precision == 0:
        for j in range(3):
            assert max(rel_errors(g[j], aux["grad"][j])) < 1e-11, j
