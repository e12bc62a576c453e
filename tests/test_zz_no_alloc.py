"""The allocation-free totals entry point against lbm_get_totals, through the
C ABI: two calls in a row on one GPU, the second on a smaller grid, each
bitwise equal to the allocating entry point (same kernels, same order) and
within 1e-12 of the oracle's FP64 totals; a level beyond its scratch is
rejected before any device work."""
import numpy as np
import pytest

from paper_2004_11863_amd import inputs as I
from parity_util import make_pair

pytestmark = pytest.mark.gpu


def _geom(D, n, lo, hi):
    return I.Geometry(D, tuple(n) + (1,) * (3 - D), tuple(lo) + (0,) * (3 - D), tuple(hi) + (0,) * (3 - D))


def _check(gpu, ref, steps):
    from paper_2004_11863_amd import lbm
    gpu.step(steps)
    ref.step(steps)
    m0, p0 = lbm.lbm_get_totals(gpu.h)
    m1, p1 = lbm.lbm_get_totals_noalloc(gpu.h)
    assert np.array_equal(m0, m1) and np.array_equal(p0, p1)
    mo, po = ref.totals()
    assert np.abs(m1 - mo).max() <= 1e-12 * np.abs(mo).max()
    assert np.abs(p1 - po).max() <= 1e-12 * np.abs(mo).max()
    # a second call on the same grid returns the same bits
    m2, p2 = lbm.lbm_get_totals_noalloc(gpu.h)
    assert np.array_equal(m1, m2) and np.array_equal(p1, p2)


def test_noalloc_totals_two_calls_then_smaller():
    from paper_2004_11863_amd import lbm
    # first call: D3Q19 two-level, FP32 deviation storage (both levels near 2^18 nodes)
    wl = I.pulse_cube_384(seed=0, n=64)
    print("noalloc: D3Q19 64^3 RR FP32", flush=True)
    gpu, ref, _ = make_pair(wl, "RR", lbm.LBM_FP32_DEV)
    gpu.step(0)
    m0, p0 = lbm.lbm_get_totals(gpu.h)
    m1, p1 = lbm.lbm_get_totals_noalloc(gpu.h)
    assert np.array_equal(m0, m1) and np.array_equal(p0, p1)
    gpu.step(5)
    m0, p0 = lbm.lbm_get_totals(gpu.h)
    m1, p1 = lbm.lbm_get_totals_noalloc(gpu.h)
    assert np.array_equal(m0, m1) and np.array_equal(p0, p1)
    gpu.close()
    # second call: a smaller D2Q9 FP64 grid; the scratch still holds the
    # larger grid's partial sums, which must not leak into this one
    print("noalloc: D2Q9 64^2 H-RR FP64", flush=True)
    gpu, ref, _ = make_pair(I.vortex_crossing_64(seed=1), "HRR", lbm.LBM_FP64)
    _check(gpu, ref, 7)
    gpu.close()


def test_noalloc_totals_rejects_levels_beyond_scratch():
    from paper_2004_11863_amd import lbm
    print("noalloc: uniform D2Q9 8192 x 8193 (2^26 + 8192 nodes) FP32", flush=True)
    g = lbm.Grid(lbm.LBM_D2Q9, lbm.LBM_RR, lbm.LBM_FP32_DEV, (8192, 8193))
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_get_totals_noalloc(g.h)
    assert e.value.code == lbm.LBM_EINVAL
    # the allocating entry point still works on it
    m, p = lbm.lbm_get_totals(g.h)
    assert np.isfinite(m).all()
    g.close()
