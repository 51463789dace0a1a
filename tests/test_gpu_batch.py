"""Served form: one batched launch set over several resident simulations gives, for each,
the result it gets alone (up to the order of floating-point atomic additions)."""
import numpy as np
import pytest

from paper_2605_20140_amd import workloads as W

from _parity import gpu_sim, rel_errors

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_batch_equals_solo(precision, tol):
    from paper_2605_20140_amd import sipf
    ics = [W.make_initial_state("blob16", N=N, P=P, ic_seed=k)
           for k, (N, P) in enumerate([(16, 3000), (32, 20000), (8, 700)])]
    solo = []
    for k, ic in enumerate(ics):
        s = gpu_sim(ic, precision=precision, sim_id=k)
        s.step(7)
        solo.append(s.fields())
        s.close()
    sims = [gpu_sim(ic, precision=precision, sim_id=k) for k, ic in enumerate(ics)]
    sipf.step_batch(sims, 3)
    sipf.step_batch(sims[:2], 2)
    sipf.step_batch(sims, 2)
    sipf.step_batch([sims[2]], 2)
    for k, s in enumerate(sims):
        out = s.fields()
        for f in ("v", "m", "w"):
            assert max(rel_errors(out[f], solo[k][f])) < tol, (k, f)
        d = out["X"] - solo[k]["X"]
        assert np.abs(d - np.round(d)).max() < tol
        assert np.abs(out["a"] / solo[k]["a"] - 1).max() < tol
        assert out["diag"]["step"] == 7
        s.close()


def test_batch_mixes_fft_paths():
    """A float64 batch holding a 128^3 simulation (three-pass FFT path: grad v as one round
    trip per axis) and a 16^3 one (plane path): each equals its solo run."""
    from paper_2605_20140_amd import sipf
    ics = [W.make_initial_state("modes64", N=128, P=20000),
           W.make_initial_state("blob16", N=16, P=3000, ic_seed=3)]
    solo = []
    for k, ic in enumerate(ics):
        s = gpu_sim(ic, precision=0, sim_id=k)
        s.step(4)
        solo.append(s.fields())
        s.close()
    sims = [gpu_sim(ic, precision=0, sim_id=k) for k, ic in enumerate(ics)]
    sipf.step_batch(sims, 4)
    for k, s in enumerate(sims):
        out = s.fields()
        for f in ("v", "m", "w"):
            assert max(rel_errors(out[f], solo[k][f])) < 1e-12, (k, f)
        d = out["X"] - solo[k]["X"]
        assert np.abs(d - np.round(d)).max() < 1e-12
        assert np.abs(out["a"] / solo[k]["a"] - 1).max() < 1e-12
        assert out["diag"]["step"] == 4
        s.close()


def test_batch_fourth_order():
    """A float64 batch with the fourth-order deposit (an 8^3 and a 32^3 simulation: the
    global-atomic and LDS region paths of that deposit): each equals its solo run."""
    from paper_2605_20140_amd import sipf
    ics = [W.make_initial_state("blob16", N=8, P=700, ic_seed=5),
           W.make_initial_state("blob16", N=32, P=20000, ic_seed=6)]
    solo = []
    for k, ic in enumerate(ics):
        s = gpu_sim(ic, precision=0, sim_id=k, deposit_order=4)
        s.step(5)
        solo.append(s.fields())
        s.close()
    sims = [gpu_sim(ic, precision=0, sim_id=k, deposit_order=4) for k, ic in enumerate(ics)]
    sipf.step_batch(sims, 5)
    for k, s in enumerate(sims):
        out = s.fields()
        for f in ("v", "m", "w"):
            assert max(rel_errors(out[f], solo[k][f])) < 1e-12, (k, f)
        d = out["X"] - solo[k]["X"]
        assert np.abs(d - np.round(d)).max() < 1e-12
        assert np.abs(out["a"] / solo[k]["a"] - 1).max() < 1e-12
        assert out["diag"]["step"] == 5
        s.close()
