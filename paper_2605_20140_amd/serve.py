"""Served form of the SIPF-W step: continuous batching of many simulations on one GPU.

Requests (a simulation: grid, particles, parameters, number of steps, initial state) arrive
over time.  The server keeps every admitted simulation resident in its own device workspace
and advances all of them together: each tick is one set of batched launches (one launch per
kernel covers every resident simulation, captured once per batch composition as a HIP
graph).  A request that arrives while others are running is admitted as soon as a slot is
free and its workspace fits the HBM budget; it is initialised on an admission stream, so its
upload overlaps the ticks already running, and joins the batch at the next tick.  A
simulation that has taken all its steps is retired: its fields are copied out and its
workspace is freed.  Latency is measured from arrival to the end of that copy.

Admission is first come, first served: the oldest waiting request is admitted first, and a
request that does not fit blocks the ones behind it (no starvation of large requests).

The scheduling logic (``Server``) only talks to a backend object, so it can be tested
without a GPU; ``GpuBackend`` is the backend that drives libsipf.
"""
from dataclasses import dataclass, field
import time

import numpy as np


@dataclass
class Request:
    rid: int
    t_arrive: float          # seconds after the start of the run
    N: int
    P: int
    steps: int
    params: dict             # physical parameters and dt, seed, sim_id
    ic: dict = None          # X0, a0, v0, m0, w0 (host float64)


@dataclass
class Record:
    rid: int
    t_arrive: float
    t_admit: float = None
    t_done: float = None
    steps: int = 0
    P: int = 0
    N: int = 0
    output: dict = None

    @property
    def latency(self):
        return self.t_done - self.t_arrive


@dataclass
class _Active:
    req: Request
    handle: object
    nbytes: int
    remaining: int
    record: Record


class Server:
    """Continuous-batching scheduler.

    backend: object with state_bytes(req), admit(req) -> handle, step(handles, nsteps),
    fence() -> token, wait(token), finish(handle, keep_output) -> output, release(handle).
    hbm_budget: bytes of device workspace the resident simulations may use together.
    max_slots: most simulations resident at once.  tick_steps: steps per batched tick.
    inflight: ticks that may be queued on the device ahead of the host.
    """

    def __init__(self, backend, hbm_budget, max_slots=64, tick_steps=10, inflight=2,
                 keep_outputs=False, clock=time.perf_counter, sleep=time.sleep):
        self.backend = backend
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.tick_steps = int(tick_steps)
        self.inflight = max(1, int(inflight))
        self.keep = keep_outputs
        self.clock = clock
        self.sleep = sleep
        self.events = []   # (time, kind, rid, resident count, bytes in use) for tests/traces

    def run(self, requests):
        reqs = sorted(requests, key=lambda r: (r.t_arrive, r.rid))
        for r in reqs:
            need = self.backend.state_bytes(r)
            if need > self.budget:
                raise ValueError(f"request {r.rid} needs {need} bytes, budget {self.budget}")
        records = {r.rid: Record(r.rid, r.t_arrive, steps=r.steps, P=r.P, N=r.N) for r in reqs}
        pending = list(reqs)
        active = []
        used = 0
        fences = []
        t0 = self.clock()
        now = lambda: self.clock() - t0
        total_ps = 0
        while pending or active:
            # admission, oldest first
            while (pending and pending[0].t_arrive <= now() and len(active) < self.max_slots
                   and used + self.backend.state_bytes(pending[0]) <= self.budget):
                r = pending.pop(0)
                nb = self.backend.state_bytes(r)
                h = self.backend.admit(r)
                used += nb
                rec = records[r.rid]
                rec.t_admit = now()
                active.append(_Active(r, h, nb, r.steps, rec))
                self.events.append((rec.t_admit, "admit", r.rid, len(active), used))
            if not active:
                if pending:
                    wait = pending[0].t_arrive - now()
                    if wait > 0:
                        self.sleep(min(wait, 0.01))
                continue
            # one tick of batched steps over every resident simulation
            k = min(self.tick_steps, min(a.remaining for a in active))
            self.backend.step([a.handle for a in active], k)
            fences.append(self.backend.fence())
            for a in active:
                a.remaining -= k
                total_ps += a.req.P * k
            if len(fences) > self.inflight:
                self.backend.wait(fences.pop(0))
            # retirement
            done = [a for a in active if a.remaining == 0]
            if done:
                active = [a for a in active if a.remaining > 0]
                for a in done:
                    out = self.backend.finish(a.handle, self.keep)
                    a.record.t_done = now()
                    a.record.output = out
                    self.backend.release(a.handle)
                    used -= a.nbytes
                    self.events.append((a.record.t_done, "retire", a.req.rid, len(active), used))
        wall = now()
        return records, summarize(records, wall, total_ps)


def summarize(records, wall, particle_steps):
    lat = np.array([r.latency for r in records.values()])
    return dict(
        requests=len(lat), wall_s=wall,
        particle_steps=int(particle_steps),
        particle_steps_per_s=particle_steps / wall if wall > 0 else None,
        latency_p50_s=float(np.percentile(lat, 50)) if lat.size else None,
        latency_p99_s=float(np.percentile(lat, 99)) if lat.size else None,
        latency_mean_s=float(lat.mean()) if lat.size else None,
    )


class GpuBackend:
    """libsipf backend: workspaces are torch tensors; admission on its own stream, batched
    ticks on a compute stream (both default priority)."""

    def __init__(self, precision=1, device="cuda:0"):
        import torch
        from . import sipf
        self.torch = torch
        self.sipf = sipf
        self.precision = precision
        self.device = device
        self.admit_stream = torch.cuda.Stream(device=device)
        self.compute_stream = torch.cuda.Stream(device=device)

    def _params(self, req):
        return self.sipf.make_params(precision=self.precision, **req.params)

    def state_bytes(self, req):
        return self.sipf.state_bytes(self._params(req))

    def admit(self, req):
        ic = req.ic
        sim = self.sipf.Simulation(self._params(req), ic["X0"], ic["a0"], ic["v0"], ic["m0"],
                                   ic["w0"], device=self.device, stream=self.admit_stream)
        sim.set_stream(self.compute_stream)
        return sim

    def step(self, handles, nsteps):
        self.sipf.step_batch(handles, nsteps)

    def fence(self):
        ev = self.torch.cuda.Event()
        ev.record(self.compute_stream)
        return ev

    def wait(self, token):
        token.synchronize()

    def finish(self, handle, keep_output):
        out = handle.fields(particles=keep_output)
        return out if keep_output else dict(diag=out["diag"])

    def release(self, handle):
        handle.close()
        handle.workspace = None


def make_requests(reqs, lazy=False):
    """Request objects from the served workload list (paper_2605_20140_amd.workloads)."""
    from . import workloads as W
    out = []
    for q in reqs:
        prm = dict(W.BASE_PARAMS)
        prm.update(N=q["N"], P=q["P"], dt=q["dt"], chi=q["chi"], seed=q["seed"],
                   sim_id=q["sim_id"])
        r = Request(q["sim_id"], q["t_arrive"], q["N"], q["P"], q["steps"], prm)
        if not lazy:
            r.ic = W.served_initial_state(q)
        out.append(r)
    return out
