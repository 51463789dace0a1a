"""Served form on the GPU: simulations of mixed grid and particle sizes admitted while others
run, stepped together in batched launches, give each the result it gets alone and the
oracle's (Alg. sipf-pic per request), within the stated tolerances."""
import numpy as np
import pytest

from oracle import step as S

from _parity import compare_state, oracle_params, oracle_state, rel_errors

pytestmark = pytest.mark.gpu


def _mix(precision):
    from paper_2605_20140_amd import serve, workloads as W
    q = W.served_mix(nreq=7, rate=None, steps=23, sizes=(16, 32), logp=(11, 15), seed=11)
    for i, r in enumerate(q):
        r["steps"] = 15 + 4 * i     # different lengths: slots free up while others still run
    # one 64^3 request, so that a tick holds FFT groups of three grid sizes
    q[1]["N"], q[1]["P"] = 64, 20000
    return serve.make_requests(q)


@pytest.mark.parametrize("precision,tol,tol_oracle", [(0, 1e-11, 1e-10), (1, 1e-5, 1e-4)])
def test_served_results_equal_solo_and_oracle(precision, tol, tol_oracle):
    from paper_2605_20140_amd import serve, sipf
    reqs = _mix(precision)
    assert sorted({r.N for r in reqs}) == [16, 32, 64]
    be = serve.GpuBackend(precision=precision)
    srv = serve.Server(be, hbm_budget=1 << 30, max_slots=3, tick_steps=5, keep_outputs=True)
    recs, summ = srv.run(reqs)
    assert summ["requests"] == len(reqs)
    # requests 3.. wait for a slot and join simulations that are still running
    late = [r.rid for r in reqs[3:]]
    assert all(any(recs[e].t_admit < recs[l].t_admit < recs[e].t_done for e in recs if e != l)
               for l in late)
    for r in reqs:
        out = recs[r.rid].output
        p = sipf.make_params(precision=precision, **r.params)
        solo = sipf.Simulation(p, r.ic["X0"], r.ic["a0"], r.ic["v0"], r.ic["m0"], r.ic["w0"])
        solo.step(r.steps)
        ref = solo.fields()
        solo.close()
        for f in ("v", "m", "w"):
            assert max(rel_errors(out[f], ref[f])) < tol, (r.rid, f)
        d = out["X"] - ref["X"]
        assert np.abs(d - np.round(d)).max() < tol, r.rid
        assert np.abs(out["a"] / ref["a"] - 1).max() < tol, r.rid
        assert out["diag"]["step"] == r.steps
        # the oracle, run on the request's own inputs and parameters (sim_id keys its noise)
        orc = S.run(oracle_state(r.ic), oracle_params(r.params), r.steps)
        compare_state(out, orc, tol_oracle)
