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
    """Step cost proportional to the resident work; bytes proportional to N^3 + P.
    Admission and retirement complete after admit_delay / retire_delay seconds of the
    (simulated) clock, as the GPU backend's worker threads do."""

    def __init__(self, clock, admit_delay=0.0, retire_delay=0.0):
        self.clock = clock
        self.admit_delay = admit_delay
        self.retire_delay = retire_delay
        self.resident = set()
        self.steps_taken = {}
        self.batches = []
        self.admitting, self.retiring = set(), set()
        self.ticks_while_admitting = 0
        self.ticks_while_retiring = 0

    def state_bytes(self, r):
        return 100 * r.N ** 3 + 40 * r.P

    def admit_start(self, r):
        self.clock.t += 1e-5
        self.admitting.add(r.rid)
        return (r.rid, self.clock.t + self.admit_delay)

    def admit_poll(self, ticket):
        rid, ready = ticket
        if self.clock.t < ready:
            return None
        self.admitting.remove(rid)
        self.resident.add(rid)
        self.steps_taken[rid] = 0
        return rid

    def step(self, handles, k):
        assert set(handles) <= self.resident and not set(handles) & self.retiring
        self.ticks_while_admitting += bool(self.admitting)
        self.ticks_while_retiring += bool(self.retiring)
        self.batches.append(tuple(handles))
        work = sum(self._req[h].P for h in handles)
        self.clock.t += k * (2e-5 + work * 1e-10)
        for h in handles:
            self.steps_taken[h] += k

    def fence(self):
        return None

    def wait(self, token):
        pass

    def retire_start(self, h, keep):
        assert h in self.resident
        self.retiring.add(h)
        return (h, self.clock.t + self.retire_delay)

    def retire_poll(self, ticket):
        h, ready = ticket
        if self.clock.t < ready:
            return None
        self.retiring.remove(h)
        self.resident.remove(h)
        return self.clock.t, dict(steps=self.steps_taken[h])


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


def test_ticks_continue_while_admission_and_retirement_run():
    """Slow initialisation and slow copies to the host do not stall the resident
    simulations: ticks keep being issued while other requests are admitted or retired, and a
    simulation joins the batch only once it is initialised."""
    clk = FakeClock()
    be = FakeBackend(clk, admit_delay=2e-3, retire_delay=3e-3)
    reqs = _requests(n=30, rate=2000.0)
    be._req = {r.rid: r for r in reqs}
    srv = Server(be, 10 ** 9, max_slots=8, tick_steps=5, clock=clk, sleep=clk.sleep)
    recs, summ = srv.run(reqs)
    assert summ["requests"] == len(reqs)
    for r in reqs:
        rec = recs[r.rid]
        assert rec.output["steps"] == r.steps
        assert rec.t_join >= rec.t_admit + 2e-3 - 1e-12
        assert rec.t_done > rec.t_join
    # batches were stepped while some request was still initialising or being copied out
    assert be.ticks_while_admitting > 0 and be.ticks_while_retiring > 0
    assert set(summ["host_ms_per_tick"]) == {"admit", "join", "launch", "wait", "retire", "idle"}
    assert summ["ticks"] > 0
