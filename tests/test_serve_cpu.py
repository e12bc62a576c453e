"""Host logic of the continuous-batching server, on the CPU with a fake
executor that runs each request on the CPU oracle (tiny grids)."""
import math
import threading
import time

import numpy as np
import pytest

import oracle as O
from paper_2004_11863_amd import inputs as I
from paper_2004_11863_amd import serve


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Oracle grids per request.  On the virtual clock a round costs the
    longest launch floor of its groups (they overlap on their streams) plus
    the memory time of all of their updates (bandwidth is shared)."""

    def __init__(self, capacity=3, nan_fp32=False, clock=None):
        self.clock = clock
        self.plans = []
        self.capacity = capacity
        self.nan_fp32 = nan_fp32
        self.grids = {}
        self.next = 0
        self.used_slots = {}
        self.max_used = 0
        self.bytes_used = 0
        self.max_bytes = 0
        self.admit_order = []
        self.steps_seen = {}

    def footprint(self, req, fp64):
        return req.workload.geom.nodes(0) * (16 if fp64 else 8)

    def free_slots(self, group):
        return self.capacity - self.used_slots.get(group, 0)

    def admit(self, req, fp64, group):
        g = req.workload.geom
        D = g.D
        grid = O.Grid(O.D2Q9 if D == 2 else O.D3Q19, O.RR, g.n[:D], g.lo[:D], g.hi[:D], tau_c=req.tau_coarse)
        for lv in (0, 1):
            grid.set_state(lv, *req.fields(lv))
        h = self.next
        self.next += 1
        key = group
        assert group == req.group(fp64)
        self.grids[h] = (grid, req, fp64, key)
        self.used_slots[key] = self.used_slots.get(key, 0) + 1
        self.bytes_used += self.footprint(req, fp64)
        self.max_bytes = max(self.max_bytes, self.bytes_used)
        self.admit_order.append(req.rid)
        self.steps_seen[h] = 0
        return h

    def step(self, plan):
        self.plans.append(dict(plan))
        for h, (grid, req, _, key) in self.grids.items():
            if key in plan:
                grid.step(plan[key])
                self.steps_seen[h] += plan[key]
        if self.clock is not None:
            floor, mem = 0.0, 0.0
            for g, n in plan.items():
                ms = [req for (_, req, _, key) in self.grids.values() if key == g]
                floor = max(floor, n * serve.STEP_FLOOR_S)
                mem += n * sum(r.ups() for r in ms) / serve.UPDATE_RATE
            self.clock.t += floor + mem

    def read(self, h):
        grid, req, fp64, _ = self.grids[h]
        out = {}
        for lv in (0, 1):
            rho, u = grid.get_macros(lv)
            if self.nan_fp32 and not fp64 and req.rid % 2 == 0:
                rho = rho * np.nan
            out[f"rho{lv}"] = rho
            out[f"u{lv}"] = u
        assert self.steps_seen[h] == req.steps
        return out

    def release(self, h):
        grid, req, fp64, key = self.grids.pop(h)
        self.used_slots[key] -= 1
        self.bytes_used -= self.footprint(req, fp64)


def _trace(n=7, seed=3):
    return serve.poisson_trace(n, rate=50.0, seed=seed, d2_side=(24, 40), d3_side=(12, 16), steps=(3, 9),
                               fp64_frac=0.3)


def test_trace_is_seeded_and_shaped():
    a, b = _trace(), _trace()
    assert [r.arrival for r in a] == [r.arrival for r in b]
    assert all(r2.arrival > r1.arrival for r1, r2 in zip(a, a[1:]))
    assert {r.workload.geom.D for r in a} == {2, 3}
    for r in a:
        g = r.workload.geom
        assert all(h - l == n // 2 for l, h, n in zip(g.lo[:g.D], g.hi[:g.D], g.n[:g.D]))


def test_every_request_completes_within_budget_and_slots():
    reqs = _trace()
    ex = FakeExecutor(capacity=2)
    budget = 3 * max(ex.footprint(r, True) for r in reqs)
    done = serve.Server(ex, budget, max_chunk=4, policy="share").run(reqs, realtime=False)
    assert sorted(r.rid for r in done) == list(range(len(reqs)))
    assert ex.max_bytes <= budget
    for r in done:
        assert r.finished >= r.admitted
    st = serve.latency_stats(done)
    assert st["p50_s"] <= st["p99_s"]


@pytest.mark.parametrize("policy", ["srpt", "share"])
def test_admission_in_arrival_order_within_budget(policy):
    reqs = _trace()
    ex = FakeExecutor(capacity=2)
    budget = 3 * max(ex.footprint(r, True) for r in reqs)
    done = serve.Server(ex, budget, max_chunk=4, policy=policy).run(reqs, realtime=False)
    assert sorted(r.rid for r in done) == list(range(len(reqs)))
    assert ex.max_bytes <= budget
    assert max(ex.used_slots.values()) == 0
    for r in done:
        assert r.finished >= r.admitted
        assert np.isfinite(r.result["rho0"]).all()
    st = serve.latency_stats(done)
    assert st["p50_s"] <= st["p99_s"]


def test_results_equal_running_alone():
    reqs = _trace(n=4, seed=5)
    ex = FakeExecutor(capacity=4)
    done = serve.Server(ex, 10 ** 12, max_chunk=2).run(reqs, realtime=False)
    for r in done:
        g = r.workload.geom
        D = g.D
        alone = O.Grid(O.D2Q9 if D == 2 else O.D3Q19, O.RR, g.n[:D], g.lo[:D], g.hi[:D], tau_c=r.tau_coarse)
        for lv in (0, 1):
            alone.set_state(lv, *I.fields(r.workload, lv))
        alone.step(r.steps)
        for lv in (0, 1):
            rho, u = alone.get_macros(lv)
            assert np.array_equal(rho, r.result[f"rho{lv}"]) and np.array_equal(u, r.result[f"u{lv}"])


def test_fp64_fallback_reruns_unstable_fp32_requests():
    reqs = _trace(n=5, seed=7)
    for r in reqs:
        r.fp64 = False
    ex = FakeExecutor(capacity=3, nan_fp32=True)
    done = serve.Server(ex, 10 ** 12, max_chunk=3).run(reqs, realtime=False)
    assert len(done) == len(reqs)
    for r in done:
        assert r.fell_back == (r.rid % 2 == 0)
        assert np.isfinite(r.result["rho0"]).all()


def test_request_larger_than_budget_is_rejected():
    reqs = _trace(n=2)
    ex = FakeExecutor()
    with pytest.raises(ValueError):
        serve.Server(ex, 10, max_chunk=2).run(reqs, realtime=False)


def test_groups_split_by_key_and_size_class():
    reqs = _trace(n=7, seed=3)
    for r in reqs:
        lat, col, prec, sc = r.group()
        assert (lat, col, prec) == r.key()
        assert serve.SIZE_BIN ** sc <= r.ups() < serve.SIZE_BIN ** (sc + 1)
    r = reqs[0]
    assert r.group(fp64=True)[2] == "fp64" and r.group(fp64=False)[2] == "fp32"


def test_srpt_runs_shortest_remaining_first():
    reqs = _trace(n=8, seed=4)
    for k, r in enumerate(reqs):
        r.steps = 30 if k == 0 else 3
        r.fp64 = False
    clock = VirtualClock()
    ex = FakeExecutor(capacity=8, clock=clock)
    done = serve.Server(ex, 10 ** 12, clock=clock, max_chunk=4, policy="srpt").run(reqs, realtime=False)
    fin = {r.rid: r.finished for r in done}
    assert all(fin[0] >= fin[k] for k in fin)            # the long request leaves last


class _R:
    """Stand-in request for plan(): only its size matters."""

    def __init__(self, ups):
        self._u = ups

    def ups(self):
        return self._u


def _members(ups, lefts):
    return [serve._Active(_R(ups), n, False, 0, None) for n in lefts]


def test_plan_pauses_a_large_group_for_a_short_one():
    srv = serve.Server(None, 0, policy="srpt", slice_s=0.02, backfill=0.25)
    groups = {"big": _members(50e6, [1000]), "small": _members(1e5, [100, 300])}
    plan = srv.plan(groups)
    cost_small = serve.STEP_FLOOR_S + 2e5 / serve.UPDATE_RATE
    assert plan == {"small": min(100, int(0.02 / cost_small))}


def test_plan_backfills_small_groups_and_caps_the_slice():
    srv = serve.Server(None, 0, policy="srpt", slice_s=0.02, backfill=0.25)
    groups = {"big": _members(50e6, [1000]), "a": _members(1e4, [60000]), "b": _members(2e4, [50000])}
    plan = srv.plan(groups)
    # the big group has the least remaining time (1000 steps) and takes one slice
    cost_big = serve.STEP_FLOOR_S + 50e6 / serve.UPDATE_RATE
    n0 = int(0.02 / cost_big)
    assert plan["big"] == n0
    # the small, launch-bound groups ride along for about the same time
    T = n0 * cost_big
    for g, u in (("a", 1e4), ("b", 2e4)):
        assert plan[g] == math.ceil(T / (serve.STEP_FLOOR_S + u / serve.UPDATE_RATE))


def test_plan_share_steps_every_group_alike():
    srv = serve.Server(None, 0, policy="share", max_chunk=8)
    groups = {"big": _members(50e6, [1000]), "small": _members(1e5, [5, 300])}
    assert srv.plan(groups) == {"big": 5, "small": 5}


def test_srpt_preempts_a_running_long_request():
    pool = _trace(n=8, seed=6)
    long_ = next(r for r in pool if r.workload.geom.D == 3)
    short = next(r for r in pool if r.workload.geom.D == 2)   # another group
    long_.steps, short.steps = 200, 2
    long_.fp64 = short.fp64 = False
    long_.arrival = 0.0
    c_long = serve.STEP_FLOOR_S + long_.ups() / serve.UPDATE_RATE
    short.arrival = 10.5 * c_long                        # arrives while the long one runs
    clock = VirtualClock()
    ex = FakeExecutor(capacity=2, clock=clock)
    srv = serve.Server(ex, 10 ** 12, clock=clock, policy="srpt", slice_s=2 * c_long)
    done = srv.run([long_, short], realtime=True)
    fin = {r.rid: r.finished for r in done}
    assert fin[short.rid] < fin[long_.rid]
    assert long_.group() in ex.plans[0] and short.group() not in ex.plans[0]
    assert any(short.group() in p for p in ex.plans)


def test_srpt_mean_latency_not_worse_than_sharing():
    def run(policy):
        reqs = _trace(n=8, seed=4)
        for k, r in enumerate(reqs):
            r.steps = 30 if k % 4 == 0 else 3
            r.fp64 = False
        clock = VirtualClock()
        ex = FakeExecutor(capacity=8, clock=clock)
        done = serve.Server(ex, 10 ** 12, clock=clock, max_chunk=4, policy=policy).run(reqs, realtime=False)
        return serve.latency_stats(done)["mean_s"]
    assert run("srpt") <= run("share") + 1e-12


def test_unknown_policy_rejected():
    with pytest.raises(ValueError):
        serve.Server(FakeExecutor(), 1, policy="lifo")


def test_prepared_payload_is_used():
    r = _trace(n=1)[0].prepare()
    assert set(r.payload) == {0, 1}
    rho, u = r.fields(0)
    assert rho.shape[0] == r.workload.geom.nodes(0)


class ThreadedFakeExecutor(FakeExecutor):
    """Host jobs on a worker thread beside the rounds.  Stepping a group while
    a host call works on it, or two host calls on one group at once, is an
    error (on the device it would race with the batch's work)."""

    overlap_host = True

    def __init__(self, **kw):
        super().__init__(**kw)
        self.lock = threading.Lock()
        self.flight = set()           # groups of the round being stepped
        self.touch = {}               # group -> host calls in progress
        self.overlapped = {"admit": 0, "read": 0, "release": 0, "settle": 0}

    def _enter(self, key, what):
        with self.lock:
            assert key not in self.flight, f"{what} on group {key} while it steps"
            assert self.touch.get(key, 0) == 0, f"two host calls on group {key}"
            self.touch[key] = 1
            if self.flight:
                self.overlapped[what] += 1

    def _leave(self, key):
        with self.lock:
            self.touch[key] = 0

    def admit(self, req, fp64, group):
        self._enter(group, "admit")
        try:
            with self.lock:
                h = self.next
                self.next += 1
                self.steps_seen[h] = 0
            g = req.workload.geom
            D = g.D
            grid = O.Grid(O.D2Q9 if D == 2 else O.D3Q19, O.RR, g.n[:D], g.lo[:D], g.hi[:D], tau_c=req.tau_coarse)
            for lv in (0, 1):
                grid.set_state(lv, *req.fields(lv))
            time.sleep(0.002)                           # an upload takes a while
            with self.lock:
                self.grids[h] = (grid, req, fp64, group)
                self.used_slots[group] = self.used_slots.get(group, 0) + 1
                self.bytes_used += self.footprint(req, fp64)
                self.max_bytes = max(self.max_bytes, self.bytes_used)
                self.admit_order.append(req.rid)
            return h
        finally:
            self._leave(group)

    def read(self, h):
        key = self.grids[h][3]
        self._enter(key, "read")
        try:
            time.sleep(0.002)
            return super().read(h)
        finally:
            self._leave(key)

    def release(self, h):
        key = self.grids[h][3]
        self._enter(key, "release")
        try:
            with self.lock:
                super().release(h)
        finally:
            self._leave(key)

    def settle(self, group):
        self._enter(group, "settle")
        self.settled = getattr(self, "settled", 0) + 1
        self._leave(group)

    def step(self, plan):
        with self.lock:
            assert not any(self.touch.get(g, 0) for g in plan), "stepping a group a host call works on"
            self.flight = set(plan)
            members = [(h, v) for h, v in self.grids.items() if v[3] in plan]
        self.plans.append(dict(plan))
        for h, (grid, req, _, key) in members:
            grid.step(plan[key])
            self.steps_seen[h] += plan[key]
        time.sleep(0.003)
        with self.lock:
            self.flight = set()


def _alone_equal(r):
    g = r.workload.geom
    D = g.D
    alone = O.Grid(O.D2Q9 if D == 2 else O.D3Q19, O.RR, g.n[:D], g.lo[:D], g.hi[:D], tau_c=r.tau_coarse)
    for lv in (0, 1):
        alone.set_state(lv, *I.fields(r.workload, lv))
    alone.step(r.steps)
    for lv in (0, 1):
        rho, u = alone.get_macros(lv)
        assert np.array_equal(rho, r.result[f"rho{lv}"]) and np.array_equal(u, r.result[f"u{lv}"])


@pytest.mark.parametrize("policy", ["srpt", "share"])
def test_host_jobs_beside_rounds_equal_running_alone(policy):
    reqs = _trace(n=8, seed=5)
    ex = ThreadedFakeExecutor(capacity=2)
    budget = 3 * max(ex.footprint(r, True) for r in reqs)
    done = serve.Server(ex, budget, max_chunk=3, policy=policy).run(reqs, realtime=False)
    assert sorted(r.rid for r in done) == list(range(len(reqs)))
    assert ex.max_bytes <= budget and max(ex.used_slots.values()) == 0
    assert ex.overlapped["admit"] + ex.overlapped["read"] > 0     # some host work ran beside a round
    assert ex.settled > 0
    for r in done:
        assert r.finished >= r.admitted
        _alone_equal(r)


def test_host_jobs_beside_rounds_keep_the_fp64_fallback():
    reqs = _trace(n=6, seed=7)
    for r in reqs:
        r.fp64 = False
    ex = ThreadedFakeExecutor(capacity=3, nan_fp32=True)
    done = serve.Server(ex, 10 ** 12, max_chunk=3).run(reqs, realtime=False)
    assert len(done) == len(reqs)
    for r in done:
        assert r.fell_back == (r.rid % 2 == 0)
        assert np.isfinite(r.result["rho0"]).all()
        _alone_equal(r)


def test_host_jobs_beside_rounds_in_real_time():
    reqs = _trace(n=6, seed=9)
    ex = ThreadedFakeExecutor(capacity=2)
    done = serve.Server(ex, 10 ** 12, max_chunk=3).run(reqs, realtime=True)
    assert sorted(r.rid for r in done) == list(range(len(reqs)))
    for r in done:
        assert r.admitted >= r.arrival - 1e-9 and r.finished >= r.admitted
