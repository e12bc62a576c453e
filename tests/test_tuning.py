"""Stored autotuning results: keys, the JSON round trip and apply() (host
logic on stand-in objects); on the GPU, that stored variants applied to a new
grid or batch give bitwise the results of its default variants."""
import numpy as np
import pytest

from paper_2004_11863_amd import lbm, tuning


def test_keys_name_the_configuration():
    k = tuning.grid_key(lbm.LBM_D3Q19, lbm.LBM_RR, lbm.LBM_FP32_DEV, ((384,) * 3, (96,) * 3, (288,) * 3))
    assert k == "grid/D3Q19/RR/fp32/384x384x384[96,96,96:288,288,288]"
    assert tuning.grid_key(0, 0, 0, ((64, 64), None, None)) == "grid/D2Q9/BGK/fp64/64x64"
    a = ((64, 64), (16, 16), (48, 48))
    b = ((128, 64), (32, 16), (96, 48))
    k1 = tuning.batch_key(0, 1, 1, [a, b, a])
    assert k1 == tuning.batch_key(0, 1, 1, [b, a, a])          # a multiset: order does not matter
    assert "2*64x64" in k1 and k1 != tuning.batch_key(0, 1, 1, [a, b])
    many = [((64 + i, 64), None, None) for i in range(100)]
    km = tuning.batch_key(0, 1, 1, many)
    assert km.startswith("batch/D2Q9/RR/fp32/100 grids sha1 ") and len(km) < 80


class _Obj:
    def __init__(self, shape, best):
        self.lattice, self.collision, self.precision, self.device = 0, 1, 1, 0
        self.shape = shape
        self.best = best
        self.tuned = 0
        self.applied = None

    def tune(self, reps=3):
        self.tuned += 1
        return list(self.best)

    def set_variants(self, v):
        self.applied = list(v)


def test_apply_tunes_once_then_reuses(tmp_path):
    path = str(tmp_path / "t.json")
    c = tuning.TuneCache(path, arch="gfx950")
    o = _Obj(((64, 64), (16, 16), (48, 48)), [2, 1, 3, 0])
    assert c.apply(o) == ([2, 1, 3, 0], False) and o.tuned == 1 and o.applied is None
    o2 = _Obj(o.shape, [0, 0, 0, 0])
    assert c.apply(o2) == ([2, 1, 3, 0], True) and o2.tuned == 0 and o2.applied == [2, 1, 3, 0]
    c.save()
    c2 = tuning.TuneCache(path, arch="gfx950")
    assert c2.get(tuning.key_of(o)) == [2, 1, 3, 0]
    assert tuning.TuneCache(path, arch="gfx942").get(tuning.key_of(o)) is None   # per architecture
    o3 = _Obj(((96, 64), (16, 16), (48, 48)), [1, 1, 1, 1])                      # another geometry
    assert c2.apply(o3) == ([1, 1, 1, 1], False)


def test_unreadable_or_foreign_file_is_ignored(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text("{not json")
    assert tuning.TuneCache(str(p), arch="x").entries == {}
    p.write_text('{"format": 99, "entries": {"x": {}}}')
    assert tuning.TuneCache(str(p), arch="x").entries == {}


def test_committed_file_is_well_formed():
    c = tuning.TuneCache(tuning.FILE, arch="gfx950")
    for arch, ents in c.entries.items():
        for k, e in ents.items():
            assert k.startswith(("grid/", "batch/"))
            n = 4 if k.startswith("grid/") else 2
            assert len(e["variants"]) == n and all(0 <= v < lbm.LBM_N_VARIANTS for v in e["variants"])


def _grid(fp32):
    from paper_2004_11863_amd import inputs as I
    wl = I.scaled(I.pulse_cube_384, 48, seed=2)
    g = wl.geom
    gr = lbm.Grid(lbm.LBM_D3Q19, lbm.LBM_RR, lbm.LBM_FP32_DEV if fp32 else lbm.LBM_FP64, g.n[:3], g.lo[:3], g.hi[:3])
    for lv in (0, 1):
        gr.set_state(lv, *I.fields(wl, lv))
    return gr, wl


@pytest.mark.gpu
def test_stored_variants_give_the_same_bits(tmp_path):
    c = tuning.TuneCache(str(tmp_path / "t.json"))
    a, _ = _grid(True)
    v, hit = c.apply(a, reps=1)
    assert not hit
    a.close()
    b, _ = _grid(True)
    v2, hit2 = c.apply(b, reps=1)
    assert hit2 and v2 == v
    b.step(6)
    ref, _ = _grid(True)
    ref.set_variants([0, 0, 0, 0])
    ref.step(6)
    for lv in (0, 1):
        for x, y in zip(b.get_macros(lv), ref.get_macros(lv)):
            assert np.array_equal(x, y)


@pytest.mark.gpu
def test_batch_set_variants_checks_range_and_keeps_results():
    from paper_2004_11863_amd import inputs as I
    wls = [I.batch_instance(3, i) for i in range(3)]
    outs = []
    for v in (None, [3, 1], [1, 0]):
        b = lbm.Batch(lbm.LBM_D2Q9, lbm.LBM_RR, lbm.LBM_FP32_DEV, capacity=4)
        for w in wls:
            g = w.geom
            sl = b.add(g.n[:2], g.lo[:2], g.hi[:2], 0.51)
            for lv in (0, 1):
                b.set_state(sl, lv, *I.fields(w, lv))
        if v is not None:
            b.set_variants(v)
        with pytest.raises(lbm.LbmError):
            b.set_variants([lbm.LBM_N_VARIANTS, 0])
        b.step(5)
        outs.append([b.get_macros(s, lv) for s in range(3) for lv in (0, 1)])
        b.close()
    for o in outs[1:]:
        for (r0, u0), (r1, u1) in zip(outs[0], o):
            assert np.array_equal(r0, r1) and np.array_equal(u0, u1)
