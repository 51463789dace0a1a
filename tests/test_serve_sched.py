"""Scheduling logic of the served form, on the CPU with a simulated clock and device:
admission by HBM budget and slots, first-come-first-served order, continuous batching
(admission while others run), retirement and the latency summary."""
import numpy as np
import pytest

from paper_2605_20140_amd.serve import Request, Server


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeBackend:
    """Step cost proportional to the resident work; bytes proportional to N^3 + P."""

    def __init__(self, clock):
        self.clock = clock
        self.resident = set()
        self.steps_taken = {}
        self.batches = []

    def state_bytes(self, r):
        return 100 * r.N ** 3 + 40 * r.P

    def admit(self, r):
        self.resident.add(r.rid)
        self.steps_taken[r.rid] = 0
        self.clock.t += 1e-4
        return r.rid

    def step(self, handles, k):
        assert set(handles) <= self.resident
        self.batches.append(tuple(handles))
        work = sum(self._req[h].P for h in handles)
        self.clock.t += k * (2e-5 + work * 1e-10)
        for h in handles:
            self.steps_taken[h] += k

    def fence(self):
        return None

    def wait(self, token):
        pass

    def finish(self, h, keep):
        return dict(steps=self.steps_taken[h])

    def release(self, h):
        self.resident.remove(h)


def _requests(n=40, seed=0, rate=200.0):
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        N = int(rng.choice([16, 32, 64]))
        P = int(2 ** rng.uniform(10, 16))
        out.append(Request(i, t, N, P, int(rng.integers(5, 60)), {}))
    return out


@pytest.mark.parametrize("budget,slots", [(10 ** 9, 64), (4 * 10 ** 7, 8), (3 * 10 ** 7, 3)])
def test_all_served_within_budget_and_slots(budget, slots):
    clk = FakeClock()
    be = FakeBackend(clk)
    reqs = _requests()
    be._req = {r.rid: r for r in reqs}
    srv = Server(be, budget, max_slots=slots, tick_steps=7, clock=clk, sleep=clk.sleep)
    recs, summ = srv.run(reqs)
    assert summ["requests"] == len(reqs)
    for r in reqs:
        rec = recs[r.rid]
        assert rec.output["steps"] == r.steps          # every step taken, none extra
        assert rec.t_admit >= r.t_arrive and rec.t_done > rec.t_admit
    for _, kind, _, resident, used in srv.events:
        assert used <= budget and resident <= slots
    assert summ["latency_p99_s"] >= summ["latency_p50_s"] > 0
    assert summ["particle_steps"] == sum(r.P * r.steps for r in reqs)


def test_first_come_first_served_and_continuous_batching():
    clk = FakeClock()
    be = FakeBackend(clk)
    reqs = _requests(n=30, rate=500.0)
    be._req = {r.rid: r for r in reqs}
    srv = Server(be, 5 * 10 ** 7, max_slots=6, tick_steps=5, clock=clk, sleep=clk.sleep)
    recs, _ = srv.run(reqs)
    admits = [rid for _, kind, rid, _, _ in srv.events if kind == "admit"]
    assert admits == sorted(admits, key=lambda i: (reqs[i].t_arrive, i))
    # some request joins while others are resident, and batches mix simulations
    assert any(res > 1 for _, kind, _, res, _ in srv.events if kind == "admit")
    assert max(len(b) for b in be.batches) > 1
    # a request is admitted before an earlier-admitted one retires (not a queue alone)
    t_done = {rid: recs[rid].t_done for rid in recs}
    assert any(recs[b].t_admit < t_done[a] for a in recs for b in recs
               if recs[a].t_admit < recs[b].t_admit)


def test_request_larger_than_budget_is_rejected():
    clk = FakeClock()
    be = FakeBackend(clk)
    r = Request(0, 0.0, 64, 1 << 20, 10, {})
    be._req = {0: r}
    with pytest.raises(ValueError):
        Server(be, 1000, clock=clk, sleep=clk.sleep).run([r])
