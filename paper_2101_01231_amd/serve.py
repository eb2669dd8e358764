"""Continuous-batching server for independent RIDG runs on one GPU.

Requests (independent periodic constant-velocity advection problems of any dimension, mesh size and
order, each with its own number of steps and step size) arrive over time. The server

  * admits a request as soon as it has arrived and its device footprint (libridg workspace) fits
    the memory budget, creating its handle and uploading its initial state;
  * keeps every admitted request's state resident on the device;
  * on each tick advances all active requests by one step with shared launches
    (`ridg_step_batch`: one prediction and one correction launch per (dimension, order) family);
    requests with large space-time bases (theta_T >= MFMA_MIN_THETA_T) run on the FP64 matrix
    cores, the others on the vector kernels (the same choice is made when a request runs alone);
  * keeps the device fed: tick k + 1 is queued before tick k has finished (at most two ticks in
    flight); a request leaves the active set when its last step has been queued, and is retired
    (state copied back, workspace freed) once that tick's event has completed. Uploads of admitted
    requests go on a separate stream, so admission does not wait for queued ticks.

Per-step latency is measured with HIP events on the server's stream, from when a request's step
becomes eligible (the end of its previous step, or the start of its first tick) to the end of the
tick that computes it. Busy time is the sum of the ticks' execution intervals. A request that cannot
be served (invalid, or larger than the whole budget) is rejected alone; the others continue.
"""

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import inputs, ridg

# measured on MI355X: the MFMA tap kernels win from theta_T ~ 30 up (2D order 5, 3D orders 4-5)
MFMA_MIN_THETA_T = 30


@dataclass
class Request:
    id: int
    arrival: float
    d: int
    n: tuple
    M: int
    steps: int
    velocity: tuple
    dt: float
    seed: int
    q0: np.ndarray = field(default=None, repr=False)

    def problem(self):
        return ridg.make_problem(self.d, self.n, self.M, velocity=self.velocity)

    def initial_state(self):
        if self.q0 is None:
            self.q0 = inputs.gaussian_bump_state(self.d, self.n, self.M, self.seed)
        return self.q0

    @property
    def theta_t(self):
        from math import comb
        return comb(self.M + self.d, self.d + 1)

    def configure(self, sim):
        """Kernel choice of the serving policy (applied alone and in the mix alike)."""
        if self.theta_t >= MFMA_MIN_THETA_T:
            sim.set_option(ridg.OPT_MFMA, 1)

    @property
    def st_dofs_per_step(self):
        from math import comb
        return int(np.prod(self.n)) * comb(self.M + self.d, self.d + 1)


def requests_from_mix(specs):
    return [Request(s["id"], s["arrival"], s["d"], tuple(s["n"]), s["M"], s["steps"], tuple(s["velocity"]),
                    s["dt"], s["seed"]) for s in specs]


class Server:
    def __init__(self, device="cuda:0", mem_budget_bytes=32 << 30, max_active=256):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(self.device)  # batched steps (default priority)
        self.upload = torch.cuda.Stream(self.device)  # handles' own stream: uploads and read-backs
        self.budget = int(mem_budget_bytes)
        self.max_active = max_active
        self.used = 0

    def _admit(self, req):
        prob = req.problem()
        need = ridg.workspace_bytes(prob)
        if need > self.budget:
            raise ridg.RidgError(ridg.RIDG_E_NOMEM, f"request {req.id} needs {need} bytes, budget {self.budget}")
        if self.used + need > self.budget:
            return None
        sim = ridg.Simulation(prob, device=self.device, stream=self.upload)
        req.configure(sim)
        sim.set_state(req.initial_state())  # synchronous on the upload stream only
        self.used += need
        return dict(req=req, sim=sim, bytes=need, issued=0, last_end=None)

    def run(self, requests, time_scale=1.0, keep_results=True):
        """Serve the requests (arrival times in seconds, divided by time_scale); returns stats."""
        torch = self.torch
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting = deque()
        active, retiring = [], []  # retiring: (slot, end event of its last tick)
        inflight = deque()  # ticks queued, not yet accounted: (start, end, [(slot, eligible event)])
        results, rejected = {}, {}
        lat_ms, tick_ms, active_counts = [], [], []
        st_updates = 0
        idle = 0.0  # wall time with no request in the system (waiting for the next arrival)
        t0 = time.perf_counter()

        def account(tick):
            ev0, ev1, members = tick
            ev1.synchronize()
            ms = ev0.elapsed_time(ev1)
            tick_ms.append(ms)
            for slot, eligible in members:
                lat_ms.append(eligible.elapsed_time(ev1) if eligible is not None else ms)

        def retire_ready(block=False):
            nonlocal retiring
            keep = []
            for slot, ev in retiring:
                if block or ev.query():
                    ev.synchronize()
                    q = slot["sim"].get_state()
                    if keep_results:
                        results[slot["req"].id] = q
                    slot["sim"].close()
                    self.used -= slot["bytes"]
                else:
                    keep.append((slot, ev))
            retiring = keep

        while pending or waiting or active or retiring or inflight:
            now = (time.perf_counter() - t0) * time_scale
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            retire_ready()
            while waiting and len(active) < self.max_active:
                try:
                    slot = self._admit(waiting[0])
                except ridg.RidgError as err:
                    rejected[waiting.popleft().id] = str(err)
                    continue
                if slot is None:
                    break
                waiting.popleft()
                active.append(slot)
            if active:
                ev0 = torch.cuda.Event(enable_timing=True)
                ev1 = torch.cuda.Event(enable_timing=True)
                ev0.record(self.stream)
                ridg.step_batch([a["sim"] for a in active], [a["req"].dt for a in active], 1, self.stream)
                ev1.record(self.stream)
                inflight.append((ev0, ev1, [(a, a["last_end"]) for a in active]))
                active_counts.append(len(active))
                still = []
                for a in active:
                    a["issued"] += 1
                    a["last_end"] = ev1
                    st_updates += a["req"].st_dofs_per_step
                    if a["issued"] >= a["req"].steps:
                        retiring.append((a, ev1))
                    else:
                        still.append(a)
                active = still
                while len(inflight) > 2:  # at most two ticks queued ahead of the host
                    account(inflight.popleft())
                continue
            # nothing to launch: drain what is queued, then wait for retirements or arrivals
            while inflight:
                account(inflight.popleft())
            if retiring:
                retire_ready(block=not (pending or waiting))
                continue
            if pending and not waiting:
                ts = time.perf_counter()
                time.sleep(max(0.0, (pending[0].arrival - now) / time_scale))
                idle += time.perf_counter() - ts
            elif waiting and not retiring:
                # nothing active and the head of the queue does not fit: it never will
                rejected[waiting.popleft().id] = "does not fit the memory budget"
        wall = time.perf_counter() - t0
        busy = sum(tick_ms) * 1e-3
        lat = np.array(lat_ms) if lat_ms else np.zeros(1)
        return dict(results=results, rejected=rejected, wall_s=wall, busy_s=busy, idle_s=idle, ticks=len(tick_ms),
                    p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                    latency_samples=int(lat.size),
                    mean_active=float(np.mean(active_counts)) if active_counts else 0.0,
                    st_dof_updates=st_updates,
                    st_dof_updates_per_s_busy=st_updates / busy if busy else 0.0,
                    st_dof_updates_per_s_wall=st_updates / wall if wall else 0.0)


def run_alone(req, device="cuda:0"):
    """The same request advanced on its own handle with ridg_step (reference for the mix)."""
    sim = ridg.Simulation(req.problem(), device=device)
    req.configure(sim)
    sim.set_state(req.initial_state())
    sim.step(req.steps, req.dt)
    out = sim.get_state()
    sim.close()
    return out
