"""Parity with the FP64 oracle on the paper's own examples and on paths the small-drift
workloads do not reach.

* The paper's 3D and 2D examples (Sec. three-dimensional simulation, Sec. two-dimensional
  simulation): L = 6, chi = 0.4, D_u = D_m = D_w = 0.01, alpha = 5, beta = 0.01, gamma = 5, a
  ball (3D) or paraboloid (2D) of cells, a non-periodic v0.  These exercise every
  L-dependent quantity of the kernels (1/h, 2 pi / L, the wrap at L, the cell volume).
* Particles drifting past the margin of their tile's LDS region (one cell in 3D, four in
  2D; Alg. g2p and Alg. p2g for every particle): the gather and deposit of such particles go
  through global memory from a block that uses a region.
* The strict positivity check (positivity lemma): a state with v = 0 at one node makes
  sipf_fields return SIPF_EPOS.
"""
import numpy as np
import pytest

from oracle import step as S
from paper_2605_20140_amd import workloads as W

from _parity import compare_state, gpu_sim, oracle_params, oracle_state

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-4


def _paper_case(ic, nsteps, precision):
    sim = gpu_sim(ic, precision=precision)
    sim.step(nsteps)
    out = sim.fields()
    sim.close()
    return out


@pytest.mark.parametrize("precision,tol", [(0, TOL64), (1, TOL32)])
def test_paper3d_example(precision, tol):
    """The paper's 3D example at N = 32, P = 2^14, 10 steps of tau = 1e-3 on [0, 6)^3."""
    ic = W.paper3d_initial_state(32, P=1 << 14)
    out = _paper_case(ic, 10, precision)
    ref = S.run(oracle_state(ic), oracle_params(ic["params"]), 10)
    errs = compare_state(out, ref, tol, L=6.0)
    print("paper3d precision", precision, errs)


@pytest.mark.parametrize("precision,tol", [(0, TOL64), (1, TOL32)])
def test_paper2d_example(precision, tol):
    """The paper's 2D example at N = 64, P = 2^15, 10 steps on [0, 6)^2."""
    ic = W.paper2d_initial_state(64, P=1 << 15)
    prm = dict(ic["params"])
    sim = gpu_sim(ic, precision=precision)
    sim.step(10)
    out = sim.fields()
    sim.close()
    ref = S.run(oracle_state(ic), oracle_params(prm), 10)
    errs = compare_state(out, ref, tol, L=6.0)
    print("paper2d precision", precision, errs)


def _past_margin_fraction(traj, N, L, period, tile=8, margin=1):
    """Fraction of (particle, step) pairs whose stencil, for the gather at X^n or the deposit
    at X^{n+1}, leaves the LDS region of the tile the particle was binned into.  Binning
    happens at initialisation and then on every step with since_bin >= period, i.e. at steps
    0, period, 2 period, ...; the region of a tile holds the stencils of the cells
    tile*T - margin .. tile*T + T - 1 + margin on each axis (T = tile cells per axis: 8 with
    a one-cell margin in 3D, 16 with a four-cell margin in 2D)."""
    h = L / N
    cells = [np.floor(X / h).astype(np.int64) % N for X in traj]
    out = []
    for n in range(len(traj) - 1):
        b = (n // period) * period
        origin = (cells[b] // tile) * tile - margin
        for c in (cells[n], cells[n + 1]):
            lrel = (c - origin) % N
            out.append(np.any(lrel > tile + 2 * margin - 1, axis=1))
    return float(np.mean(out))


@pytest.mark.parametrize("precision,tol,order", [(0, TOL64, 2), (1, TOL32, 2), (0, TOL64, 4),
                                                 (1, TOL32, 4)])
def test_particles_past_the_drift_margin(precision, tol, order):
    """N = 32, D_u raised to 0.044 (a diffusive step of 0.3 cell), binning every 8 steps, 24
    steps: about 1.4 % of the particle-steps (some 8000 gathers and deposits) go through global
    memory (float32: after the early region loads of the same particle).  The fourth-order
    deposit's region holds the 4^3 stencils of the same cells (two nodes of margin below the
    tile, three above), so the same particles deposit through global memory."""
    D_u, period, nsteps = 0.044, 8, 24
    ic = W.make_initial_state("blob16", N=32, P=4096 * 3 + 77, D_u=D_u)
    prm = oracle_params(ic["params"], deposit_order=order)
    assert abs(np.sqrt(2 * D_u * prm.dt) * prm.N - 0.3) < 0.01
    sim = gpu_sim(ic, precision=precision, resort_every=period, deposit_order=order)
    sim.step(nsteps)
    out = sim.fields()
    sim.close()
    st = oracle_state(ic)
    traj = [st.X]
    for _ in range(nsteps):
        st = S.step(st, prm)
        traj.append(st.X)
    frac = _past_margin_fraction(traj, prm.N, prm.L, period)
    print(f"particle-steps past the region margin: {frac:.4f}")
    assert frac > 0.005
    compare_state(out, st, tol)


@pytest.mark.parametrize("precision,tol", [(0, TOL64), (1, TOL32)])
def test_2d_particles_past_the_drift_margin(precision, tol):
    """The 2D pass (16 x 16 tiles, four-cell margins): N = 64, D_u = 0.2 (a diffusive step of
    1.3 cells), binning every 8 steps, 24 steps; the particles that leave their tile's region
    gather and deposit through global memory."""
    D_u, period, nsteps = 0.2, 8, 24
    ic = W.blob2d_initial_state(N=64, P=20000, D_u=D_u)
    prm = oracle_params(ic["params"])
    assert abs(np.sqrt(2 * D_u * prm.dt) * prm.N - 1.28) < 0.01
    sim = gpu_sim(ic, precision=precision, resort_every=period)
    sim.step(nsteps)
    out = sim.fields()
    sim.close()
    st = oracle_state(ic)
    traj = [st.X]
    for _ in range(nsteps):
        st = S.step(st, prm)
        traj.append(st.X)
    frac = _past_margin_fraction(traj, prm.N, prm.L, period, tile=16, margin=4)
    print(f"particle-steps past the region margin: {frac:.4f}")
    assert frac > 0.005
    compare_state(out, st, tol)


def test_strict_flag_reports_violated_positivity():
    """SIPF_FLAG_STRICT: a state with v = 0 at one node violates v > 0 (the hard invariant of
    the positivity lemma); sipf_fields fills its outputs and returns SIPF_EPOS.  The same
    state without the zero passes."""
    from paper_2605_20140_amd import sipf
    ic = W.make_initial_state("blob16", P=2000)
    sim = gpu_sim(ic, flags=sipf.FLAG_STRICT)
    sim.step(3)
    good = sim.fields()
    sim.close()
    assert good["rc"] == 0 and good["diag"]["min_v"] > 0
    v0 = ic["v0"].copy()
    v0[3, 4, 5] = 0.0
    bad_ic = dict(ic, v0=v0)
    sim = gpu_sim(bad_ic, flags=sipf.FLAG_STRICT)
    first = sim.fields()
    sim.step(3)
    later = sim.fields()
    sim.close()
    for o in (first, later):
        assert o["rc"] == -4, o["rc"]
        assert o["diag"]["min_v"] == 0.0
        assert np.all(np.isfinite(o["v"])) and o["v"][3, 4, 5] == 0.0
    # without the flag the same state is reported, not rejected
    sim = gpu_sim(bad_ic)
    sim.step(3)
    plain = sim.fields()
    sim.close()
    assert plain["rc"] == 0 and plain["diag"]["min_v"] == 0.0
