"""sipf_step_batch_noalloc, the allocation-free batched step, against sipf_step_batch (the
entry point it is a variant of) through the C ABI: two calls in a row, the second with a
smaller batch (a smaller launch table in the library's per-GPU array), then a third with the
same batch (the table is reused as it stands)."""
import numpy as np
import pytest

from oracle import step as S
from paper_2605_20140_amd import workloads as W

from _parity import compare_state, gpu_sim, oracle_params, oracle_state, rel_errors

pytestmark = pytest.mark.gpu

CASES = [(16, 3000), (32, 20000), (8, 700), (64, 9000)]


def _sims(precision):
    ics = [W.make_initial_state("blob16", N=N, P=P, ic_seed=k) for k, (N, P) in enumerate(CASES)]
    return ics, [gpu_sim(ic, precision=precision, sim_id=k) for k, ic in enumerate(ics)]


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-4)])
def test_noalloc_batch_equals_batch(precision, tol):
    from paper_2605_20140_amd import sipf
    ics, ref = _sims(precision)
    sipf.step_batch(ref, 4)
    sipf.step_batch(ref[1:3], 3)
    sipf.step_batch(ref[1:3], 2)
    ics, got = _sims(precision)
    sipf.step_batch_noalloc(got, 4)
    sipf.step_batch_noalloc(got[1:3], 3)
    sipf.step_batch_noalloc(got[1:3], 2)
    steps = [4, 9, 9, 4]
    for k, (a, b) in enumerate(zip(got, ref)):
        oa, ob = a.fields(), b.fields()
        assert oa["diag"]["step"] == ob["diag"]["step"] == steps[k]
        for f in ("v", "m", "w"):
            assert max(rel_errors(oa[f], ob[f])) < tol, (k, f)
        d = oa["X"] - ob["X"]
        assert np.abs(d - np.round(d)).max() < tol, k
        assert np.abs(oa["a"] / ob["a"] - 1).max() < tol, k
        if precision == 0 and CASES[k][0] <= 32:
            # and the oracle's state for the same schedule
            st = S.run(oracle_state(ics[k]), oracle_params(dict(ics[k]["params"], sim_id=k)),
                       steps[k])
            compare_state(oa, st, 1e-10)
        a.close()
        b.close()


def test_noalloc_rejects_oversized_batch():
    from paper_2605_20140_amd import sipf
    ics, sims = _sims(1)
    with pytest.raises(sipf.SipfError) as e:
        sipf.step_batch_noalloc(sims * 17, 1)   # 68 entries: over the 64-simulation limit
    assert e.value.code == -1 and "at most 64" in str(e.value)
    for s in sims:
        s.close()
