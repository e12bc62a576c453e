"""Continuous-batching request loop for two-level LBM simulations.

Requests (a grid description, an initial state and a number of coarse steps)
arrive over time.  The server admits a waiting request as soon as a batch slot
and enough device memory (by footprint) are free and keeps its populations
resident on the device until it leaves.  Admitted requests are grouped by
(lattice, collision, precision, size class); each group is one batch of the
library, stepped by replaying its captured launch sequence on its own stream,
so every member of a group advances in lock-step.  A request leaves when it
has taken its steps; its macroscopic fields are read back and its slot and
memory freed.  FP32 requests whose result is not finite are run again in FP64
(fallback).

Scheduling between groups ("srpt", the default): each round steps the group
whose shortest member has the least estimated remaining time, for at most
one time slice.  Other groups ride along on their own streams only if their
memory traffic fits in a fraction (`backfill`) of that round, so small,
launch-bound groups overlap with it for free while a large group waits with
its state resident: long requests are preempted in favour of short ones at
no copy cost.  Policy "share" steps every group by the same number of steps
each round (processor sharing).

Everything device-side goes through an executor; ``DeviceExecutor`` drives
the C-ABI batches of the HIP library.  The scheduling logic itself is plain
host code and is tested on the CPU with a fake executor.
"""
from __future__ import annotations

import math
import threading
import time
from concurrent.futures import FIRST_COMPLETED, ThreadPoolExecutor
from concurrent.futures import wait as futures_wait
from dataclasses import dataclass, field

import numpy as np

from . import inputs as I

# step-time model of a group, seconds per coarse step: a floor for the ~15
# launches of a step plus its lattice updates at a sustained rate
STEP_FLOOR_S = 60e-6
UPDATE_RATE = 20e9
# size classes of a batch group: bins of this factor in updates per step.
# Coarser bins make fewer, larger batches (fewer launch-bound rounds):
# factor 16 measured 13.8 GLUPS against 12.3-13.1 with factor 4 on a
# small-grid trace, and 18.9 against 18.6-18.7 on a large-grid one.
SIZE_BIN = 16


@dataclass
class Request:
    rid: int
    workload: I.Workload
    steps: int
    arrival: float          # seconds from trace start
    fp64: bool = False      # run in FP64 from the start
    collision: str = "RR"
    tau_coarse: float = 0.51
    sigma: float = 0.995
    payload: dict = None    # level -> (rho, u) initial fields, prepared by the client
    # filled by the server
    admitted: float = math.nan
    finished: float = math.nan
    result: dict = field(default_factory=dict)
    fell_back: bool = False

    @property
    def lattice(self) -> int:
        return 0 if self.workload.geom.D == 2 else 1

    def key(self, fp64=None):
        return (self.lattice, self.collision, "fp64" if (self.fp64 if fp64 is None else fp64) else "fp32")

    def ups(self) -> int:
        """Lattice updates per coarse step."""
        return self.workload.geom.updates_per_step()

    def group(self, fp64=None):
        """Batch key: the library batch key plus a size class (SIZE_BIN-factor
        bins of the updates per step), so lock-stepped members are of
        comparable size."""
        return self.key(fp64) + (int(math.log(max(self.ups(), 1), SIZE_BIN)),)

    def updates(self) -> int:
        return self.ups() * self.steps

    def prepare(self):
        """Samples the initial fields (client side, before submission)."""
        self.payload = {lv: I.fields(self.workload, lv) for lv in (0, 1)}
        return self

    def fields(self, level):
        return self.payload[level] if self.payload is not None else I.fields(self.workload, level)


def poisson_trace(n: int, rate: float, seed: int = 0, mix_3d: float = 0.5, d2_side=(128, 2048), d3_side=(64, 256),
                  steps=(100, 2000), fp64_frac: float = 0.1, collision: str = "RR"):
    """Seeded request stream: Poisson arrivals at `rate` per second; half
    D2Q9 (side log-uniform in d2_side) and half D3Q19 (side log-uniform in
    d3_side); fine patch over the central half of each side; steps uniform in
    `steps`; a fraction flagged FP64; a convected vortex (2D) or an acoustic
    pulse (3D) as initial state."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    U = 0.1 * I.CS
    for k in range(n):
        t += rng.exponential(1.0 / rate)
        three = rng.uniform() < mix_3d
        lo_s, hi_s = d3_side if three else d2_side
        N = int(4 * round(math.exp(rng.uniform(math.log(lo_s), math.log(hi_s))) / 4))
        a, b = N // 4, 3 * N // 4
        if three:
            geom = I.Geometry(3, (N, N, N), (a, a, a), (b, b, b))
            c = tuple(float(x) for x in rng.uniform(a, b, 3))
            wl = I.Workload(geom=geom, U=(U, 0.0, 0.0), pulses=[I.Pulse(center=c, A=1e-3)])
        else:
            geom = I.Geometry(2, (N, N, 1), (a, a, 0), (b, b, 0))
            c = (float(rng.uniform(a, b)), float(rng.uniform(a, b)))
            wl = I.Workload(geom=geom, U=(U, 0.0, 0.0),
                            vortices=[I.Vortex(center=c, eps=0.15 * U * rng.uniform(0.5, 1.5), U=(U, 0.0, 0.0))])
        st = int(rng.integers(steps[0], steps[1] + 1))
        out.append(Request(rid=k, workload=wl, steps=st, arrival=t, fp64=bool(rng.uniform() < fp64_frac),
                           collision=collision))
    return out


class Server:
    """Continuous batching over an executor.

    Admission in arrival order, skipping a request that does not fit yet: it
    is admitted when its footprint fits the free memory budget and its group
    has a free slot.

    executor interface:
      footprint(req, fp64) -> bytes
      free_slots(group) -> int
      admit(req, fp64, group) -> handle      (allocates and sets the state)
      step({group: n})                      (advances each listed group n steps, then waits)
      read(handle) -> dict                   (macroscopic fields)
      release(handle)
    overlap_host (attribute, default False): admit, read and release may run
    on another thread for a group while other groups step; then
      open(group)                           (optional, on the main thread before
                                             a group's first admission there)
      settle(group)                         (optional, after each job on the worker)
    """

    def __init__(self, executor, hbm_budget: int, clock=time.perf_counter, max_chunk: int = 32,
                 policy: str = "srpt", slice_s: float = 0.02, backfill: float = 0.25):
        if policy not in ("srpt", "share"):
            raise ValueError(f"unknown policy {policy!r}")
        self.ex = executor
        self.budget = hbm_budget
        self.clock = clock
        self.max_chunk = max_chunk
        self.policy = policy
        self.slice_s = slice_s
        self.backfill = backfill

    @staticmethod
    def step_cost(members):
        """Modelled seconds per coarse step of a group stepped alone."""
        return STEP_FLOOR_S + sum(m.req.ups() for m in members) / UPDATE_RATE

    def plan(self, groups):
        """{group: n} for this round; groups maps a group to its members."""
        left = {g: min(m.left for m in ms) for g, ms in groups.items()}
        if self.policy == "share":
            n = min(self.max_chunk, min(left.values()))
            return {g: n for g in groups}
        cost = {g: self.step_cost(ms) for g, ms in groups.items()}
        order = sorted(groups, key=lambda g: (left[g] * cost[g], g))
        g0 = order[0]
        n0 = max(1, min(left[g0], int(self.slice_s / cost[g0])))
        T = n0 * cost[g0]
        out = {g0: n0}
        extra = 0.0
        for g in order[1:]:
            n = max(1, min(left[g], math.ceil(T / cost[g])))
            bw = n * sum(m.req.ups() for m in groups[g]) / UPDATE_RATE
            if extra + bw <= self.backfill * T:
                out[g] = n
                extra += bw
        return out

    def run(self, requests, realtime: bool = True):
        """Runs the trace; returns the requests with admission and finish
        times (seconds from the start).  With realtime=False arrival times are
        ignored (every request is waiting from the start).

        With an executor that allows host work on one group while others step
        (overlap_host = True), the slow host work runs on a worker thread
        beside the rounds: admitting requests into groups with no member
        stepping (allocation, upload of the initial state) and reading back
        and releasing groups whose members all finished.  A group with such a
        job in progress is held: not stepped and not touched until it ends.
        A request that joins a group with members stepping is admitted on the
        main thread between rounds, once the worker is idle (a blocking call
        there would wait for the worker's); the read of a finished member
        whose group steps on is made there too, or, while the worker is busy,
        queued to it with the group held.  After each job the executor may
        settle the group (autotune it) on the worker."""
        pending = sorted(requests, key=lambda r: r.arrival)
        waiting = []                # arrived, not admitted (arrival order)
        active = {}                 # handle -> _Active, still stepping
        used = 0
        t0 = self.clock()
        now = lambda: self.clock() - t0
        i = 0
        done = []
        overlap = getattr(self.ex, "overlap_host", False)
        pool = ThreadPoolExecutor(max_workers=1) if overlap else None
        jobs = {}                   # future -> (kind, group, payload)
        held = set()                # groups with a job in progress

        def deliver(items, res):
            for h, a in items:
                r = a.req
                ok = all(np.isfinite(v).all() for v in res[h].values())
                if not ok and not a.fp64:
                    # FP64 fallback: the request is run again from its start
                    r.fell_back = True
                    r.fp64 = True
                    waiting.insert(0, r)
                    continue
                r.result = res[h]
                r.finished = now()
                done.append(r)

        def read_release(items):
            res = {h: self.ex.read(h) for h, _ in items}
            for h, _ in items:
                self.ex.release(h)
            return res

        settle = getattr(self.ex, "settle", lambda g: None)

        def admit_job(g, items):
            hs = [self.ex.admit(r, r.fp64, g) for r, _ in items]
            settle(g)
            return hs

        def read_job(g, items):
            res = read_release(items)
            settle(g)
            return res

        def collect(timeout):
            nonlocal used
            if not jobs:
                return
            if timeout != 0:
                futures_wait(list(jobs), timeout=timeout, return_when=FIRST_COMPLETED)
            for f in [f for f in jobs if f.done()]:
                kind, g, payload = jobs.pop(f)
                held.discard(g)
                out = f.result()
                if kind == "admit":
                    for (r, fp), h in zip(payload, out):
                        r.admitted = now()
                        active[h] = _Active(r, r.steps, r.fp64, fp, g)
                else:
                    used -= sum(a.bytes for _, a in payload)
                    deliver(payload, out)

        try:
            while i < len(pending) or waiting or active or jobs:
                t = now()
                while i < len(pending) and (not realtime or pending[i].arrival <= t):
                    waiting.append(pending[i])
                    i += 1
                collect(0)
                live = {a.group for a in active.values()}
                new = {}
                for r in list(waiting):
                    fp = self.ex.footprint(r, r.fp64)
                    if fp > self.budget:
                        raise ValueError(f"request {r.rid} needs {fp} bytes, more than the whole budget")
                    g = r.group()
                    if g in held or used + fp > self.budget:
                        continue
                    if self.ex.free_slots(g) - len(new.get(g, ())) <= 0:
                        continue
                    if overlap and g in live and jobs:
                        continue                   # joins once the worker is idle
                    waiting.remove(r)
                    used += fp
                    if overlap and g not in live:
                        new.setdefault(g, []).append((r, fp))
                        continue
                    h = self.ex.admit(r, r.fp64, g)
                    r.admitted = now()
                    active[h] = _Active(r, r.steps, r.fp64, fp, g)
                for g, items in new.items():
                    held.add(g)
                    if hasattr(self.ex, "open"):
                        self.ex.open(g)          # device objects of a group are made on this thread
                    jobs[pool.submit(admit_job, g, items)] = ("admit", g, items)
                groups = {}
                for a in active.values():
                    if a.group not in held:
                        groups.setdefault(a.group, []).append(a)
                if not groups:
                    nxt = pending[i].arrival - now() if i < len(pending) and realtime else None
                    if jobs:
                        collect(None if nxt is None else max(nxt, 1e-4))
                    elif nxt is not None and nxt > 0:
                        time.sleep(min(nxt, 0.05))
                    continue
                plan = self.plan(groups)
                self.ex.step(plan)
                for a in active.values():
                    if a.group in plan:
                        a.left -= plan[a.group]
                now_done = [(h, a) for h, a in active.items() if a.left <= 0]
                for h, _ in now_done:
                    del active[h]
                still = {a.group for a in active.values()}
                # finished members are read before their group steps again:
                # here if the worker is idle and the group steps on, else on
                # the worker with the group held (a group that is all done is
                # read there while other groups step)
                collect(0)
                inline = [(h, a) for h, a in now_done if not overlap or (a.group in still and not jobs)]
                if inline:
                    used -= sum(a.bytes for _, a in inline)
                    deliver(inline, read_release(inline))
                later = {}
                for h, a in now_done:
                    if overlap and not (a.group in still and not jobs):
                        later.setdefault(a.group, []).append((h, a))
                for g, items in later.items():
                    held.add(g)
                    jobs[pool.submit(read_job, g, items)] = ("read", g, items)
        finally:
            if pool is not None:
                pool.shutdown(wait=True)
        return done


@dataclass
class _Active:
    req: Request
    left: int
    fp64: bool
    bytes: int
    group: tuple


def latency_stats(done):
    lat = np.array([r.finished - r.arrival for r in done])
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max()), "n": int(lat.size)}


class DeviceExecutor:
    """Runs requests on the HIP library: one batch per group, each stepped on
    its own stream.  Library calls on one batch wait for that batch's work
    only, so a worker thread can admit into or read from one group while the
    main thread steps others (overlap_host).  A group whose membership
    changed is autotuned before it is stepped again if its work per step is
    at least `tune_min` lattice updates (kernel variants give bitwise the
    same results)."""

    def __init__(self, capacity: int = 64, device: int = 0, tune_min: float = 4e6):
        import torch
        from . import lbm
        self.torch = torch
        self.lbm = lbm
        self.capacity = capacity
        self.device = device
        self.batches = {}
        self.streams = {}
        self.where = {}
        self.next = 0
        self.tune_min = tune_min
        self.changed = set()
        self.lock = threading.Lock()   # handle counter and maps, shared with the worker thread
        from .tuning import TuneCache
        self.tunings = TuneCache(None)  # in memory: variants per batch membership

    overlap_host = True

    def _code(self, key):
        lat, col, prec = key[:3]
        lbm = self.lbm
        return (lat, {"BGK": lbm.LBM_BGK, "RR": lbm.LBM_RR, "HRR": lbm.LBM_HRR}[col],
                lbm.LBM_FP64 if prec == "fp64" else lbm.LBM_FP32_DEV)

    def open(self, group):
        self.batch(group)

    def batch(self, group):
        if group not in self.batches:
            lat, col, prec = self._code(group)
            self.batches[group] = self.lbm.Batch(lat, col, prec, self.capacity, self.device)
            self.streams[group] = self.torch.cuda.Stream(device=self.device)
        return self.batches[group]

    def footprint(self, req, fp64):
        g = req.workload.geom
        D = g.D
        lat, col, prec = self._code(req.key(fp64))
        d = self.lbm.make_desc(lat, col, prec, g.n[:D], g.lo[:D], g.hi[:D], req.tau_coarse, req.sigma)
        return self.lbm.lbm_footprint(d)

    def free_slots(self, group):
        b = self.batches.get(group)
        return self.capacity if b is None else self.capacity - b.info()["grids"]

    def admit(self, req, fp64, group):
        b = self.batch(group)
        g = req.workload.geom
        D = g.D
        sl = b.add(g.n[:D], g.lo[:D], g.hi[:D], req.tau_coarse, req.sigma)
        for lv in (0, 1):
            rho, u = req.fields(lv)
            b.set_state(sl, lv, rho, u)
        with self.lock:
            h = self.next
            self.next += 1
            self.where[h] = (group, sl)
            self.changed.add(group)
        return h

    def settle(self, group):
        """Autotunes a group whose membership changed, if it is large enough
        (a membership seen before reuses its stored variants)."""
        with self.lock:
            tune = group in self.changed
            self.changed.discard(group)
        b = self.batches.get(group)
        if tune and b is not None and b.info()["updates_per_step"] >= self.tune_min:
            self.tunings.apply(b, reps=2)

    def step(self, plan):
        for g in plan:
            self.settle(g)
        for g, n in plan.items():
            self.batches[g].step(n, self.streams[g].cuda_stream)
        for g in plan:
            self.streams[g].synchronize()

    def read(self, h):
        group, sl = self.where[h]
        b = self.batches[group]
        out = {}
        for lv in (0, 1):
            rho, u = b.get_macros(sl, lv)
            out[f"rho{lv}"] = rho
            out[f"u{lv}"] = u
        return out

    def release(self, h):
        with self.lock:
            group, sl = self.where.pop(h)
        self.batches[group].remove(sl)
        with self.lock:
            self.changed.add(group)

    def close(self):
        for b in self.batches.values():
            b.close()
        self.batches.clear()
        self.streams.clear()


def run_alone(req, fp64=None, device: int = 0):
    """The plain per-instance path for one request: its own grid, stepped
    alone; returns the same fields as DeviceExecutor.read."""
    from . import lbm
    g = req.workload.geom
    D = g.D
    col = {"BGK": lbm.LBM_BGK, "RR": lbm.LBM_RR, "HRR": lbm.LBM_HRR}[req.collision]
    use64 = req.fp64 if fp64 is None else fp64
    grid = lbm.Grid(req.lattice, col, lbm.LBM_FP64 if use64 else lbm.LBM_FP32_DEV, g.n[:D], g.lo[:D], g.hi[:D],
                    req.tau_coarse, req.sigma, device)
    for lv in (0, 1):
        grid.set_state(lv, *req.fields(lv))
    grid.step(req.steps)
    out = {}
    for lv in (0, 1):
        rho, u = grid.get_macros(lv)
        out[f"rho{lv}"] = rho
        out[f"u{lv}"] = u
    grid.close()
    return out


def fifo_loop(requests, realtime: bool = True, clock=time.perf_counter):
    """Plain per-instance loop: one request at a time in arrival order."""
    t0 = clock()
    done = []
    for r in sorted(requests, key=lambda q: q.arrival):
        if realtime:
            wait = r.arrival - (clock() - t0)
            if wait > 0:
                time.sleep(wait)
        r.admitted = clock() - t0
        r.result = run_alone(r)
        r.finished = clock() - t0
        done.append(r)
    return done
