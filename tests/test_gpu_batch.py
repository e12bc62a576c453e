"""Batched persistent launches: a grid advanced inside a batch (captured
hipGraph, continuous joining and leaving) computes exactly what it computes
alone, and FP64 batches match the CPU oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2004_11863_amd import inputs as I
from parity_util import make_pair

pytestmark = pytest.mark.gpu


def _lbm():
    from paper_2004_11863_amd import lbm
    return lbm


def _geoms2d():
    return [I.Geometry(2, (64, 64, 1), (16, 16, 0), (48, 48, 0)),
            I.Geometry(2, (71, 37, 1), (6, 5, 0), (33, 30, 0)),
            I.Geometry(2, (40, 24, 1), (0, 0, 0), (0, 0, 0)),
            I.Geometry(2, (96, 80, 1), (20, 30, 0), (70, 50, 0))]


def _wl(geom, k):
    c = tuple(0.5 * (l + h) + 1.3 * k if l != h else 0.4 * n for l, h, n in zip(geom.lo[:geom.D], geom.hi[:geom.D],
                                                                                 geom.n[:geom.D]))
    return I.Workload(geom=geom, U=(0.05, 0.01, 0.0), vortices=[I.Vortex(center=c[:2], eps=0.01, U=(0.05, 0.01, 0.0))],
                      pulses=[I.Pulse(center=c, A=1e-3, R=3.0)])


def _alone(wl, model, prec, steps, variants=None):
    gpu, _, levels = make_pair(wl, model, prec, with_oracle=False)
    if variants is not None:
        gpu.set_variants(variants)
    gpu.step(steps)
    out = [gpu.get_populations(lv) for lv in levels]
    live = gpu.class_map(0) != _lbm().LBM_C_COVERED
    gpu.close()
    return out, live


def _add(batch, wl):
    g = wl.geom
    D = g.D
    lo = g.lo[:D] if g.has_fine else None
    hi = g.hi[:D] if g.has_fine else None
    sl = batch.add(g.n[:D], lo, hi, tau_coarse=0.51)
    for lv in ((0, 1) if g.has_fine else (0,)):
        batch.set_state(sl, lv, *I.fields(wl, lv))
    return sl


def _check_same(batch, sl, alone):
    out, live = alone
    b0 = batch.get_populations(sl, 0)
    # every stored value of the batch member is finite, covered nodes included
    assert np.isfinite(b0).all()
    if len(out) > 1:
        assert np.isfinite(out[1]).all()
    assert np.array_equal(b0[:, live], out[0][:, live])
    if len(out) > 1:
        assert np.array_equal(batch.get_populations(sl, 1), out[1])


def _geoms3d():
    return [I.Geometry(3, (40, 36, 34), (5, 4, 6), (35, 20, 28)),   # fine 61 x 33 x 45
            I.Geometry(3, (27, 21, 22), (4, 5, 3), (19, 14, 17)),   # fine 31 x 19 x 29
            I.Geometry(3, (20, 18, 16), (0, 0, 0), (0, 0, 0))]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("model", ["BGK", "RR"])
def test_batch_equals_alone_d3q19(prec, model):
    """A single D3Q19 grid runs both fine substeps either as two launches
    (fine-role variants 0, 1) or in one marching kernel with the half-step
    state on chip (variants 2, 3); a batch runs them as two launches.  All
    are bitwise equal, over several tiles, z-runs and ragged row ends."""
    lbm = _lbm()
    mcode = {"BGK": lbm.LBM_BGK, "RR": lbm.LBM_RR}[model]
    p = lbm.LBM_FP32_DEV if prec == "fp32" else lbm.LBM_FP64
    batch = lbm.Batch(lbm.LBM_D3Q19, mcode, p, capacity=3)
    wls = [_wl(g, k) for k, g in enumerate(_geoms3d())]
    slots = [_add(batch, w) for w in wls]
    batch.step(7)
    for w, sl in zip(wls, slots):
        for v in (0, 2, 3):
            _check_same(batch, sl, _alone(w, model, p, 7, variants=[0, v, 0, 0]))
    batch.close()


@pytest.mark.parametrize("model", ["BGK", "RR", "HRR"])
@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_alone_fp32(model, graph):
    lbm = _lbm()
    mcode = {"BGK": lbm.LBM_BGK, "RR": lbm.LBM_RR, "HRR": lbm.LBM_HRR}[model]
    batch = lbm.Batch(lbm.LBM_D2Q9, mcode, lbm.LBM_FP32_DEV, capacity=8)
    batch.use_graph(graph)
    wls = [_wl(g, k) for k, g in enumerate(_geoms2d())]
    slots = [_add(batch, w) for w in wls]
    batch.step(9)
    for w, sl in zip(wls, slots):
        assert batch.slot_steps(sl) == 9
        _check_same(batch, sl, _alone(w, model, lbm.LBM_FP32_DEV, 9))
    batch.close()


def test_continuous_batching_join_and_leave():
    lbm = _lbm()
    batch = lbm.Batch(lbm.LBM_D2Q9, lbm.LBM_RR, lbm.LBM_FP32_DEV, capacity=4)
    g = _geoms2d()
    wa, wb, wc = _wl(g[0], 0), _wl(g[1], 1), _wl(g[3], 2)
    a = _add(batch, wa)
    batch.step(5)
    b = _add(batch, wb)
    batch.step(4)
    batch.remove(a)
    c = _add(batch, wc)
    batch.step(6)
    assert batch.slot_steps(b) == 10 and batch.slot_steps(c) == 6
    _check_same(batch, b, _alone(wb, "RR", lbm.LBM_FP32_DEV, 10))
    _check_same(batch, c, _alone(wc, "RR", lbm.LBM_FP32_DEV, 6))
    info = batch.info()
    assert info["grids"] == 2
    batch.close()


@pytest.mark.parametrize("model", ["RR", "HRR"])
def test_batch_d3q19_fp64_matches_oracle(model):
    lbm = _lbm()
    mcode = {"RR": lbm.LBM_RR, "HRR": lbm.LBM_HRR}[model]
    batch = lbm.Batch(lbm.LBM_D3Q19, mcode, lbm.LBM_FP64, capacity=3)
    geoms = [I.Geometry(3, (22, 20, 24), (5, 4, 6), (15, 14, 17)), I.Geometry(3, (18, 18, 18), (4, 4, 4), (12, 12, 12))]
    wls = [I.Workload(geom=gm, U=(0.05, 0.01, -0.01), pulses=[I.Pulse(center=(9.0, 8.5, 10.2), A=1e-3, R=2.5)])
           for gm in geoms]
    slots = [_add(batch, w) for w in wls]
    batch.tune(reps=1)
    batch.step(7)
    for w, sl in zip(wls, slots):
        g = w.geom
        ref = O.Grid(O.D3Q19, {"RR": O.RR, "HRR": O.HRR}[model], g.n[:3], g.lo[:3], g.hi[:3], tau_c=0.51)
        for lv in (0, 1):
            ref.set_state(lv, *I.fields(w, lv))
        ref.step(7)
        for lv in (0, 1):
            r1, u1 = batch.get_macros(sl, lv)
            r0, u0 = ref.get_macros(lv)
            assert np.abs(r1 - r0).max() <= 1e-12 * np.abs(r0).max()
            assert np.abs(u1 - u0).max() <= 1e-12 * np.abs(u0).max()
    batch.close()


def test_batch_rejects_mismatched_descriptor_and_overflow():
    lbm = _lbm()
    batch = lbm.Batch(lbm.LBM_D2Q9, lbm.LBM_RR, lbm.LBM_FP32_DEV, capacity=1)
    batch.add((32, 32), (8, 8), (24, 24))
    with pytest.raises(lbm.LbmError) as e:
        batch.add((32, 32), (8, 8), (24, 24))
    assert e.value.code == lbm.LBM_ENOMEM
    batch.close()
    batch = lbm.Batch(lbm.LBM_D2Q9, lbm.LBM_RR, lbm.LBM_FP32_DEV, capacity=2)
    with pytest.raises(lbm.LbmError) as e:
        batch.add((32, 32), (8, 8), (40, 24))  # patch outside the grid
    assert e.value.code == lbm.LBM_EINVAL
    batch.close()


def test_batch_calls_from_two_threads_beside_graph_capture():
    """One thread steps a batch whose step graph is captured again every
    round while another thread adds, fills, steps, reads and removes grids of
    a second batch: a blocking call there must not invalidate the capture,
    and the first batch's grids still compute what they compute alone."""
    import threading

    import torch
    lbm = _lbm()
    geoms = _geoms2d()
    wls = [_wl(geoms[0], 0), _wl(geoms[3], 1)]
    rounds, per = 10, 2
    a = lbm.Batch(lbm.LBM_D2Q9, lbm.LBM_RR, lbm.LBM_FP32_DEV, capacity=4)
    slots = [_add(a, w) for w in wls]
    b = lbm.Batch(lbm.LBM_D2Q9, lbm.LBM_RR, lbm.LBM_FP32_DEV, capacity=4)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    stop = threading.Event()
    errors, cycles = [], [0]

    def other():
        try:
            while not stop.is_set():
                sl = _add(b, _wl(geoms[1], cycles[0]))
                b.step(1, sb.cuda_stream)
                rho, u = b.get_macros(sl, 0)
                assert np.isfinite(rho).all()
                b.remove(sl)
                cycles[0] += 1
        except Exception as e:            # reported by the main thread
            errors.append(e)

    th = threading.Thread(target=other)
    th.start()
    try:
        for _ in range(rounds):
            a.use_graph(False)            # drops the graph: the next step captures it again
            a.use_graph(True)
            a.step(per, sa.cuda_stream)
            sa.synchronize()
    finally:
        stop.set()
        th.join()
    assert not errors, errors
    assert cycles[0] > 0
    for sl, w in zip(slots, wls):
        _check_same(a, sl, _alone(w, "RR", lbm.LBM_FP32_DEV, rounds * per))
    a.close()
    b.close()


def _oracle_run(w, model, steps, tau_c=0.51, sigma=0.995):
    g = w.geom
    D = g.D
    lo = g.lo[:D] if g.has_fine else None
    hi = g.hi[:D] if g.has_fine else None
    ref = O.Grid(O.D2Q9 if D == 2 else O.D3Q19, {"BGK": O.BGK, "RR": O.RR, "HRR": O.HRR}[model], g.n[:D], lo, hi,
                 tau_c=tau_c, sigma=sigma)
    for lv in ((0, 1) if g.has_fine else (0,)):
        ref.set_state(lv, *I.fields(w, lv))
    ref.step(steps)
    return ref


@pytest.mark.parametrize("model", ["RR", "HRR"])
def test_batch_d2q9_fp32_matches_oracle(model):
    """Four D2Q9 grids (three two-level of different shapes, one uniform) in
    one FP32 batch (graph replay, fused fine phase for RR), each against the
    FP64 oracle at the FP32 bar: density max-abs < 1e-5, velocity relative
    L2 < 1e-4."""
    lbm = _lbm()
    mcode = {"RR": lbm.LBM_RR, "HRR": lbm.LBM_HRR}[model]
    batch = lbm.Batch(lbm.LBM_D2Q9, mcode, lbm.LBM_FP32_DEV, capacity=4)
    wls = [_wl(g, k) for k, g in enumerate(_geoms2d())]
    assert sum(not w.geom.has_fine for w in wls) == 1
    slots = [_add(batch, w) for w in wls]
    batch.tune(reps=1)
    steps = 60
    batch.step(steps)
    for w, sl in zip(wls, slots):
        ref = _oracle_run(w, model, steps)
        for lv in ((0, 1) if w.geom.has_fine else (0,)):
            r1, u1 = batch.get_macros(sl, lv)
            r0, u0 = ref.get_macros(lv)
            assert np.isfinite(r1).all() and np.isfinite(u1).all()
            assert np.abs(r1 - r0).max() < 1e-5, (sl, lv)
            assert np.linalg.norm(u1 - u0) / np.linalg.norm(u0) < 1e-4, (sl, lv)
    batch.close()


@pytest.mark.parametrize("model", ["BGK", "RR", "HRR"])
def test_batch_d2q9_fp64_matches_oracle(model):
    """The same four D2Q9 grids in one FP64 batch: 1e-12 relative on rho and
    u of both levels against the oracle."""
    lbm = _lbm()
    mcode = {"BGK": lbm.LBM_BGK, "RR": lbm.LBM_RR, "HRR": lbm.LBM_HRR}[model]
    batch = lbm.Batch(lbm.LBM_D2Q9, mcode, lbm.LBM_FP64, capacity=4)
    wls = [_wl(g, k) for k, g in enumerate(_geoms2d())]
    slots = [_add(batch, w) for w in wls]
    steps = 40
    batch.step(steps)
    for w, sl in zip(wls, slots):
        ref = _oracle_run(w, model, steps)
        for lv in ((0, 1) if w.geom.has_fine else (0,)):
            r1, u1 = batch.get_macros(sl, lv)
            r0, u0 = ref.get_macros(lv)
            assert np.abs(r1 - r0).max() <= 1e-12 * np.abs(r0).max(), (sl, lv)
            assert np.abs(u1 - u0).max() <= 1e-12 * np.abs(u0).max(), (sl, lv)
    batch.close()
