"""Stored autotuning results.

The library's autotuner (lbm_tune for a grid, lbm_batch_tune for a batch)
times the launch variants of the bulk kernels and keeps the fastest.  The
choice depends on the lattice, collision model, precision, geometry and
device, never on the state, and every variant computes the same bits, so a
stored choice can be applied to a later run (lbm_set_variants /
lbm_batch_set_variants) instead of timing again; a stale entry can only cost
time.  TuneCache keeps the choices in a JSON file, keyed by the device's
architecture and the configuration.

    python -m paper_2004_11863_amd.tuning --sweep [PATH]

tunes the standard configurations on the current device and writes them
(default: tuning.json beside this module).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import tempfile

FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
FORMAT = 1

_LAT = {0: "D2Q9", 1: "D3Q19"}
_COL = {0: "BGK", 1: "RR", 2: "HRR"}
_PREC = {0: "fp64", 1: "fp32"}


def _shape_txt(shape):
    n, lo, hi = shape
    txt = "x".join(str(v) for v in n)
    if lo is not None and hi is not None and any(a != b for a, b in zip(lo, hi)):
        txt += "[" + ",".join(str(v) for v in lo) + ":" + ",".join(str(v) for v in hi) + "]"
    return txt


def grid_key(lattice, collision, precision, shape) -> str:
    """Key of a single grid: lattice/collision/precision/geometry."""
    return f"grid/{_LAT[lattice]}/{_COL[collision]}/{_PREC[precision]}/{_shape_txt(shape)}"


def batch_key(lattice, collision, precision, shapes) -> str:
    """Key of a batch: its members' geometries as a multiset."""
    count = {}
    for s in shapes:
        t = _shape_txt(s)
        count[t] = count.get(t, 0) + 1
    members = ";".join(f"{c}*{t}" if c > 1 else t for t, c in sorted(count.items()))
    if len(members) > 160:   # many distinct members: a digest of the multiset
        members = f"{sum(count.values())} grids sha1 " + hashlib.sha1(members.encode()).hexdigest()[:16]
    return f"batch/{_LAT[lattice]}/{_COL[collision]}/{_PREC[precision]}/{members}"


def key_of(obj) -> str:
    """Key of an lbm.Grid or lbm.Batch."""
    if hasattr(obj, "shapes"):
        return batch_key(obj.lattice, obj.collision, obj.precision, obj.shapes.values())
    return grid_key(obj.lattice, obj.collision, obj.precision, obj.shape)


def device_arch(device: int = 0) -> str:
    import torch
    if not torch.cuda.is_available():
        return "none"
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


class TuneCache:
    """Variants per (architecture, key), loaded from and saved to `path`."""

    def __init__(self, path: str | None = FILE, arch: str | None = None):
        self.path = path
        self.arch = arch
        self.entries = {}
        if path and os.path.exists(path):
            try:
                with open(path) as fh:
                    d = json.load(fh)
            except (OSError, ValueError):
                d = {}
            if d.get("format") == FORMAT and isinstance(d.get("entries"), dict):
                self.entries = d["entries"]

    def _arch(self, obj=None):
        if self.arch is None:
            self.arch = device_arch(getattr(obj, "device", 0) or 0)
        return self.arch

    def get(self, key, arch=None):
        e = self.entries.get(arch or self._arch(), {}).get(key)
        return None if e is None else list(e["variants"])

    def put(self, key, variants, arch=None, **meta):
        self.entries.setdefault(arch or self._arch(), {})[key] = dict(meta, variants=[int(v) for v in variants])

    def save(self, path=None):
        path = path or self.path
        d = os.path.dirname(os.path.abspath(path))
        fd, tmp = tempfile.mkstemp(dir=d, suffix=".tmp")
        with os.fdopen(fd, "w") as fh:
            json.dump({"format": FORMAT, "entries": self.entries}, fh, indent=1, sort_keys=True)
            fh.write("\n")
        os.replace(tmp, path)

    def apply(self, obj, reps: int = 3):
        """Applies the stored variants to a grid or batch, or tunes it and
        stores the result.  Returns (variants, True if they were stored)."""
        key = key_of(obj)
        v = self.get(key, self._arch(obj))
        if v is not None:
            obj.set_variants(v)
            return v, True
        v = obj.tune(reps=reps)
        self.put(key, v, self._arch(obj))
        return list(v), False


def sweep(path: str = FILE, reps: int = 5, log=print):
    """Tunes the standard configurations on device 0 and saves them: the
    D2Q9 4096^2 and D3Q19 384^3 two-level grids with every collision model
    and precision, and the batch of 256 D2Q9 grids."""
    import numpy as np
    from . import inputs as I
    from . import lbm
    cache = TuneCache(path)
    for wl in (I.vortex_pulse_4096(n=4096), I.pulse_cube_384(n=384)):
        g = wl.geom
        D = g.D
        lat = lbm.LBM_D2Q9 if D == 2 else lbm.LBM_D3Q19
        states = {}
        for col in (lbm.LBM_BGK, lbm.LBM_RR, lbm.LBM_HRR):
            for prec in (lbm.LBM_FP32_DEV, lbm.LBM_FP64):
                grid = lbm.Grid(lat, col, prec, g.n[:D], g.lo[:D], g.hi[:D], tau_coarse=0.51)
                for lv in (0, 1):
                    N = grid.nodes(lv)
                    if lv not in states:
                        states[lv] = (np.ones(N), np.zeros((D, N)))
                    grid.set_state(lv, *states[lv])
                key = key_of(grid)
                v = grid.tune(reps=reps)
                cache.put(key, v)
                log(f"{key}: {v}")
                grid.close()
                del grid
    wls = [I.batch_instance(0, i) for i in range(256)]
    b = lbm.Batch(lbm.LBM_D2Q9, lbm.LBM_RR, lbm.LBM_FP32_DEV, capacity=256)
    for w in wls:
        g = w.geom
        sl = b.add(g.n[:2], g.lo[:2], g.hi[:2], 0.51)
        for lv in (0, 1):
            N = b.nodes(sl, lv)
            b.set_state(sl, lv, np.ones(N), np.zeros((2, N)))
    key = key_of(b)
    v = b.tune(reps=reps)
    cache.put(key, v)
    log(f"{key}: {v}")
    b.close()
    cache.save(path)
    return cache


def main(argv=None):
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    p.add_argument("--sweep", action="store_true", help="tune the standard configurations and save them")
    p.add_argument("path", nargs="?", default=FILE)
    p.add_argument("--reps", type=int, default=5)
    a = p.parse_args(argv)
    if a.sweep:
        sweep(a.path, a.reps, log=lambda s: print(s, flush=True))
    else:
        c = TuneCache(a.path)
        for arch, ents in c.entries.items():
            for k, e in sorted(ents.items()):
                print(arch, k[:100], e["variants"])


if __name__ == "__main__":
    main()
