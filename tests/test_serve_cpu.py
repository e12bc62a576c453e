"""Host logic of the continuous-batching server, on the CPU with a fake
executor that runs each request on the CPU oracle (tiny grids)."""
import numpy as np
import pytest

import oracle as O
from paper_2004_11863_amd import inputs as I
from paper_2004_11863_amd import serve


class FakeExecutor:
    def __init__(self, capacity=3, nan_fp32=False):
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

    def free_slots(self, key):
        return self.capacity - self.used_slots.get(key, 0)

    def admit(self, req, fp64):
        g = req.workload.geom
        D = g.D
        grid = O.Grid(O.D2Q9 if D == 2 else O.D3Q19, O.RR, g.n[:D], g.lo[:D], g.hi[:D], tau_c=req.tau_coarse)
        for lv in (0, 1):
            grid.set_state(lv, *req.fields(lv))
        h = self.next
        self.next += 1
        key = req.key(fp64)
        self.grids[h] = (grid, req, fp64, key)
        self.used_slots[key] = self.used_slots.get(key, 0) + 1
        self.bytes_used += self.footprint(req, fp64)
        self.max_bytes = max(self.max_bytes, self.bytes_used)
        self.admit_order.append(req.rid)
        self.steps_seen[h] = 0
        return h

    def step(self, n):
        for h, (grid, _, _, _) in self.grids.items():
            grid.step(n)
            self.steps_seen[h] += n

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
    done = serve.Server(ex, budget, max_chunk=4, policy="fifo").run(reqs, realtime=False)
    assert sorted(r.rid for r in done) == list(range(len(reqs)))
    assert ex.max_bytes <= budget
    assert ex.admit_order == sorted(ex.admit_order)      # FIFO admission
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


def test_sjf_admits_shortest_work_first_and_saturation_caps_concurrency():
    reqs = _trace(n=6, seed=9)
    ex = FakeExecutor(capacity=6)
    sat = min(r.workload.geom.updates_per_step() for r in reqs)
    done = serve.Server(ex, 10 ** 12, max_chunk=2, policy="sjf", saturation=sat).run(reqs, realtime=False)
    assert len(done) == len(reqs)
    order = [r.rid for r in sorted(reqs, key=lambda q: (q.updates(), q.arrival))]
    assert ex.admit_order == order
    # with the cap at the smallest request's load, one request runs at a time
    spans = sorted((r.admitted, r.finished) for r in done)
    for (a0, f0), (a1, f1) in zip(spans, spans[1:]):
        assert a1 >= f0 - 1e-9


def test_prepared_payload_is_used():
    r = _trace(n=1)[0].prepare()
    assert set(r.payload) == {0, 1}
    rho, u = r.fields(0)
    assert rho.shape[0] == r.workload.geom.nodes(0)
