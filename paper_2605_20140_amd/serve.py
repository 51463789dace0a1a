"""Served form of the SIPF-W step: continuous batching of many simulations on one GPU.

Requests (a simulation: grid, particles, parameters, number of steps, initial state) arrive
over time.  The server keeps every admitted simulation resident in its own device workspace
and advances all of them together: each tick is one set of batched launches (one launch per
kernel covers every resident simulation).

The tick loop never waits for admission or retirement:
* a request that arrives while others are running is admitted as soon as a slot is free and
  its workspace fits the HBM budget; its initialisation (upload of the initial state) runs on
  a worker thread and its own stream, and the simulation joins the batch at the first tick
  after it is ready;
* a simulation that has taken all its steps leaves the batch at once; the copy of its fields
  to the host runs on a worker thread, on a stream that waits (on the device) for the
  simulation's last tick only, and its workspace is freed when the copy is done.
Latency is measured from arrival to the end of that copy.

Admission is first come, first served: the oldest waiting request is admitted first, and a
request that does not fit blocks the ones behind it (no starvation of large requests).

The scheduling logic (``Server``) only talks to a backend object, so it can be tested
without a GPU; ``GpuBackend`` is the backend that drives libsipf.
"""
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass
import threading
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
    t_admit: float = None    # admission started (slot and bytes reserved)
    t_join: float = None     # initialised: in the batch from the next tick on
    t_done: float = None     # fields copied to the host
    steps: int = 0
    P: int = 0
    N: int = 0
    output: dict = None

    @property
    def latency(self):
        return self.t_done - self.t_arrive


@dataclass
class _Entry:
    req: Request
    nbytes: int
    record: Record
    ticket: object = None    # admission or retirement in progress
    handle: object = None
    remaining: int = 0


class Server:
    """Continuous-batching scheduler.

    backend: object with
      state_bytes(req) -> bytes of device workspace;
      admit_start(req) -> ticket, admit_poll(ticket) -> handle or None (non-blocking);
      step(handles, nsteps) (enqueues one tick; returns without waiting);
      fence() -> token, wait(token) (bounds the ticks queued ahead of the host);
      retire_start(handle, keep_output) -> ticket,
      retire_poll(ticket) -> None while running, else (t_done, output) with t_done on
      the server's clock (the workspace is released by then).
    hbm_budget: bytes of device workspace the simulations may hold together (admitting,
    resident and retiring).  max_slots: most simulations admitting or resident at once.
    tick_steps: steps per batched tick.  inflight: ticks that may be queued on the device
    ahead of the host.
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
        self.events = []   # (time, kind, rid, slots in use, bytes in use) for tests/traces
        # host seconds spent by the tick loop, per activity
        self.host = dict(admit=0.0, join=0.0, launch=0.0, wait=0.0, retire=0.0, idle=0.0)
        self.ticks = 0

    def run(self, requests):
        reqs = sorted(requests, key=lambda r: (r.t_arrive, r.rid))
        for r in reqs:
            need = self.backend.state_bytes(r)
            if need > self.budget:
                raise ValueError(f"request {r.rid} needs {need} bytes, budget {self.budget}")
        records = {r.rid: Record(r.rid, r.t_arrive, steps=r.steps, P=r.P, N=r.N) for r in reqs}
        pending = list(reqs)
        admitting, active, retiring = [], [], []
        used = 0
        fences = []
        be, clk, host = self.backend, self.clock, self.host
        t0 = clk()
        now = lambda: clk() - t0
        total_ps = 0
        while pending or admitting or active or retiring:
            progressed = False
            # admission, oldest first
            t = clk()
            while (pending and pending[0].t_arrive <= now()
                   and len(admitting) + len(active) < self.max_slots
                   and used + be.state_bytes(pending[0]) <= self.budget):
                r = pending.pop(0)
                e = _Entry(r, be.state_bytes(r), records[r.rid], remaining=r.steps)
                used += e.nbytes
                e.record.t_admit = now()
                e.ticket = be.admit_start(r)
                admitting.append(e)
                self.events.append((e.record.t_admit, "admit", r.rid,
                                    len(admitting) + len(active), used))
                progressed = True
            host["admit"] += clk() - t
            # initialised simulations join the batch
            t = clk()
            for e in list(admitting):
                h = be.admit_poll(e.ticket)
                if h is not None:
                    e.handle, e.ticket = h, None
                    e.record.t_join = now()
                    admitting.remove(e)
                    active.append(e)
                    self.events.append((e.record.t_join, "join", e.req.rid,
                                        len(admitting) + len(active), used))
                    progressed = True
            host["join"] += clk() - t
            if active:
                # one tick of batched steps over every resident simulation
                t = clk()
                k = min(self.tick_steps, min(a.remaining for a in active))
                be.step([a.handle for a in active], k)
                fences.append(be.fence())
                self.ticks += 1
                for a in active:
                    a.remaining -= k
                    total_ps += a.req.P * k
                host["launch"] += clk() - t
                t = clk()
                if len(fences) > self.inflight:
                    be.wait(fences.pop(0))
                host["wait"] += clk() - t
                # simulations that took all their steps leave the batch
                t = clk()
                for a in [a for a in active if a.remaining == 0]:
                    active.remove(a)
                    a.ticket = be.retire_start(a.handle, self.keep)
                    retiring.append(a)
                host["retire"] += clk() - t
                progressed = True
            # finished copies: record the latency, return the bytes
            t = clk()
            for a in list(retiring):
                res = be.retire_poll(a.ticket)
                if res is not None:
                    t_done, out = res
                    a.record.t_done = t_done - t0
                    a.record.output = out
                    retiring.remove(a)
                    used -= a.nbytes
                    self.events.append((a.record.t_done, "retire", a.req.rid,
                                        len(admitting) + len(active), used))
                    progressed = True
            host["retire"] += clk() - t
            if not progressed:
                t = clk()
                wait = pending[0].t_arrive - now() if pending else 1e-3
                self.sleep(min(max(wait, 0.0), 1e-3) if (admitting or retiring or pending)
                           else 0.0)
                host["idle"] += clk() - t
        wall = now()
        summ = summarize(records, wall, total_ps)
        summ["ticks"] = self.ticks
        summ["host_ms_per_tick"] = {k: 1e3 * v / max(self.ticks, 1) for k, v in host.items()}
        return records, summ


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
    """libsipf backend.  Workspaces are torch tensors.  Initialisation runs on admission
    worker threads, each with a stream of its own; ticks run on one compute stream through
    the allocation-free batched step (launch table in the library's per-GPU array, no graph
    per batch composition) or, with graphs=True, through sipf_step_batch's captured graphs;
    copies to the host run on retirement worker threads and a retirement stream.  All
    streams have the default priority."""

    def __init__(self, precision=1, device="cuda:0", graphs=False, admit_workers=2,
                 retire_workers=2, clock=time.perf_counter):
        import torch
        from . import sipf
        self.torch = torch
        self.sipf = sipf
        self.precision = precision
        self.device = device
        self.graphs = graphs
        self.clock = clock
        self.compute_stream = torch.cuda.Stream(device=device)
        self.retire_stream = torch.cuda.Stream(device=device)
        self._tls = threading.local()
        # With graphs, a tick may capture a new batch graph; a capture on one thread has
        # failed here while other threads initialised or read out simulations, so on that path
        # the library calls of the three threads take turns.  (The allocation-free step
        # captures nothing.)
        self._lock = threading.Lock() if graphs else None
        self._admit = ThreadPoolExecutor(admit_workers, thread_name_prefix="sipf-admit")
        self._retire = ThreadPoolExecutor(retire_workers, thread_name_prefix="sipf-retire")

    def _params(self, req):
        return self.sipf.make_params(precision=self.precision, **req.params)

    def state_bytes(self, req):
        return self.sipf.state_bytes(self._params(req))

    def _init(self, req):
        torch = self.torch
        torch.cuda.set_device(self.device)
        st = getattr(self._tls, "stream", None)
        if st is None:
            st = self._tls.stream = torch.cuda.Stream(device=self.device)
        ic = req.ic
        with self._locked():
            sim = self.sipf.Simulation(self._params(req), ic["X0"], ic["a0"], ic["v0"],
                                       ic["m0"], ic["w0"], device=self.device, stream=st)
            sim.set_stream(self.compute_stream)   # ordered on the device, no host wait
        return sim

    def _locked(self):
        import contextlib
        return self._lock if self._lock is not None else contextlib.nullcontext()

    def admit_start(self, req):
        return self._admit.submit(self._init, req)

    def admit_poll(self, fut):
        return fut.result() if fut.done() else None

    def step(self, handles, nsteps):
        if self.graphs:
            with self._lock:
                self.sipf.step_batch(handles, nsteps)
        else:
            self.sipf.step_batch_noalloc(handles, nsteps)

    def fence(self):
        ev = self.torch.cuda.Event()
        ev.record(self.compute_stream)
        return ev

    def wait(self, token):
        token.synchronize()

    def _finish(self, handle, keep_output):
        self.torch.cuda.set_device(self.device)
        with self._locked():
            out = handle.fields(particles=keep_output)
            t_done = self.clock()
            handle.close()
            handle.workspace = None
        return t_done, (out if keep_output else dict(diag=out["diag"]))

    def retire_start(self, handle, keep_output):
        # the retirement stream waits (on the device) for the work queued so far, which ends
        # with this simulation's last tick; the copy then needs no wait on the compute stream
        with self._locked():
            handle.set_stream(self.retire_stream)
        return self._retire.submit(self._finish, handle, keep_output)

    def retire_poll(self, fut):
        return fut.result() if fut.done() else None

    def close(self):
        self._admit.shutdown(wait=True)
        self._retire.shutdown(wait=True)


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
