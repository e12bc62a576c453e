#!/usr/bin/env python3
"""Throughput benchmark of the two-level lattice-Boltzmann hot path on one
MI355X.

A step is one coarse time step of the two-level scheme (one coarse update and
two fine substeps with the full interface treatment).  The default workload
is the D3Q19 two-level problem with a 384^3 periodic coarse grid and a
centred 385^3-node fine cube (patch [96, 288]^3 in coarse vertices),
recursive regularised collision, tau_c = 0.51, populations stored in FP32 as
deviations from the lattice weights; input: a Gaussian acoustic pulse
(amplitude 1e-3) near the interface on a uniform flow at Mach 0.1, seeded.

Prints ONE JSON line.  value = MLUPS = (evolving coarse nodes + 2 x fine
nodes) x steps / seconds / 1e6, inputs resident in HBM.  The roofline object
prices the dominant kernel (the fine-level pull-stream + collide) with the
bytes it must move -- one read and one write of the Q populations of every
node it updates, once per launch, also when one launch performs both fine
substeps -- over its mean launch duration measured with HIP events on its
launch stream during the timed region.  cpu_baseline times the FP64 CPU
oracle on a bounded sample of the same workload (for the D3Q19 grid: the
64^3 subcase of the same configuration) and error_vs_oracle compares the GPU
run of that sample with it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_dominant_kernel.json")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1000)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--workload", default="d3q19-384", choices=["d3q19-384", "d2q9-4096", "d2q9-1024"])
    p.add_argument("--collision", default="RR", choices=["BGK", "RR", "HRR"])
    p.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    p.add_argument("--no-extra", action="store_true", help="skip the secondary measurements")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-steps", type=int, default=None,
                   help="coarse steps of the CPU oracle sample (default: 300 of the D3Q19 64^3 subcase, "
                        "24 of the D2Q9 grids; about 10-20 s on 16 host cores)")
    p.add_argument("--no-batch", action="store_true", help="skip the batched-instances measurement")
    p.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    p.add_argument("--no-paper", action="store_true",
                   help="skip the paper's cases (acoustic wave, sensors, dynamic sigma)")
    p.add_argument("--batch-n", type=int, default=256)
    p.add_argument("--batch-steps", type=int, default=200)
    p.add_argument("--serve-n", type=int, default=16, help="arrivals of the full-size serving trace")
    p.add_argument("--serve-small-n", type=int, default=128, help="arrivals of the small-grid serving trace")
    p.add_argument("--serve-reps", type=int, default=3, help="repeats of the small-grid trace (spread)")
    p.add_argument("--variants", default=None,
                   help="launch variants of the headline grid as r0,r1,r2,r3 instead of autotuning")
    p.add_argument("--three-levels", action="store_true",
                   help="only run the three-nested-levels case (D3Q19 256^3, RR and H-RR) and print its JSON")
    p.add_argument("--copy-probe", type=int, default=0,
                   help="only run a plain device copy of this many MiB (counter calibration)")
    return p.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("lattice.hpp", "geometry.hpp", "kernels.hpp", "lbm.hip"):
        with open(os.path.join(ROOT, "paper_2004_11863_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_label(D, collision, variants=None):
    """The fine-level kernel lbm_profile_enable times for this grid with the
    autotuner's variants (D3Q19: the fine role's variants 2 and 3 select the
    one-pass kernels)."""
    v = list(variants) if variants is not None else [0, 0, 0, 0]
    if D == 2 and collision != "HRR":
        return ("k_fine2: both fine substeps of a coarse step (pull + collide twice, the t+1/2 state in LDS); "
                "one read and one write of every fine node's populations per launch, 2 updates per node")
    if collision == "HRR" and D == 2:
        return "k_hrr2: one H-RR fine substep in one pass (pull, velocities of the tile in LDS, strain rate, collide)"
    if collision == "HRR":
        if v[3] == 2:
            return "k_hrr3: one H-RR fine substep in one marching pass (velocity planes in LDS, strain rate, collide)"
        if v[3] == 3:
            return ("k_hrr3s: one H-RR fine substep in one marching pass, one node per lane (velocity planes in "
                    "LDS, strain rate, collide)")
        return "k_collide_hrr: fine-level pull + H-RR collide (second pass)"
    if v[1] >= 2:
        return ("k_fine3s: both fine substeps of a coarse step in one marching pass, one node per lane; one read "
                "and one write of every fine node's populations per launch, 2 updates per node")
    return "k_stream: fine-level pull + collide"


def fine_middle_nodes(geom):
    """Fine nodes the bulk fine kernels update (the patch without its ring)."""
    m = 1
    for d in range(geom.D):
        m *= 2 * (geom.hi[d] - geom.lo[d]) + 1 - 2
    return m


def roofline_of(kt, Q, pb, geom):
    """Roofline figures of the timed fine kernel from (launches, mean ms,
    updates per launch): bytes it must move = one read + one write of Q
    populations per node it updates, once per launch (a launch that does
    both fine substeps updates every node twice but moves it once)."""
    launches, mean_ms, updates = kt
    nodes = fine_middle_nodes(geom)
    per_node = 2 * Q * pb
    moved = per_node * nodes
    achieved = moved / (mean_ms * 1e-3) / 1e9
    upd_eq = per_node * updates / (mean_ms * 1e-3) / 1e9
    return {"achieved": round(achieved, 1), "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_launch": moved,
            "nodes_per_launch": nodes, "updates_per_launch": updates, "launches": launches,
            "mean_launch_ms": mean_ms,
            # 2 Q P_b per lattice update: above `achieved` when a launch
            # updates each node twice
            "update_equivalent_GBs": round(upd_eq, 1), "update_equivalent_frac": round(upd_eq / HBM_PEAK_GBS, 4)}


def workload(name, seed=0):
    from paper_2004_11863_amd import inputs as I
    if name == "d2q9-4096":
        return I.vortex_pulse_4096(seed=seed, n=4096)
    if name == "d2q9-1024":
        return I.vortex_pulse_4096(seed=seed, n=1024)
    return I.pulse_cube_384(seed=seed, n=384)


def make_gpu(wl, collision, precision, tau_coarse=0.51):
    from paper_2004_11863_amd import inputs as I
    from paper_2004_11863_amd import lbm
    g = wl.geom
    D = g.D
    lat = lbm.LBM_D2Q9 if D == 2 else lbm.LBM_D3Q19
    col = {"BGK": lbm.LBM_BGK, "RR": lbm.LBM_RR, "HRR": lbm.LBM_HRR}[collision]
    prec = lbm.LBM_FP32_DEV if precision == "fp32" else lbm.LBM_FP64
    grid = lbm.Grid(lat, col, prec, g.n[:D], g.lo[:D], g.hi[:D], tau_coarse=tau_coarse, sigma=0.995)
    for lv in (0, 1):
        rho, u = I.fields(wl, lv)
        grid.set_state(lv, rho, u)
        del rho, u
    return grid


def timed_run(grid, steps, warmup, profile, tune=True):
    import torch
    from paper_2004_11863_amd import lbm
    stream = torch.cuda.current_stream().cuda_stream
    if tune:
        grid.variants = grid.tune(reps=3)
    grid.step(warmup, stream)
    torch.cuda.synchronize()
    if profile:
        lbm.lbm_profile_enable(grid.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grid.step(steps, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = None
    if profile:
        kt = lbm.lbm_kernel_time(grid.h)
        lbm.lbm_profile_enable(grid.h, False)
    return t1 - t0, kt


def stored_traffic(kernel_hash, key, variant=None):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None if it was taken on other code.  Where
    the launch variants are distinct kernels (the fused D2Q9 fine kernel's
    tile shapes) the entry holds one figure per variant."""
    try:
        with open(TRAFFIC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_hash:
        return None
    e = d.get("entries", {}).get(key)
    if e is not None and "by_variant" in e:
        e = e["by_variant"].get(str(variant))
    return None if e is None else e.get("hbm_bytes_per_launch")


def cpu_sample(name, seed=0):
    """The workload the CPU oracle is timed on: the D3Q19 grid's 64^3
    subcase (same configuration at 64^3), or the D2Q9 grid itself."""
    from paper_2004_11863_amd import inputs as I
    if name == "d3q19-384":
        return I.pulse_cube_384(seed=seed, n=64), "D3Q19 64^3 subcase of the same configuration (patch [16, 48]^3)"
    return workload(name, seed), "the same grid"


def cpu_baseline(wl, collision, steps):
    import oracle as O
    from paper_2004_11863_amd import inputs as I
    g = wl.geom
    D = g.D
    ref = O.Grid(O.D2Q9 if D == 2 else O.D3Q19, {"BGK": O.BGK, "RR": O.RR, "HRR": O.HRR}[collision],
                 g.n[:D], g.lo[:D], g.hi[:D], tau_c=0.51, sigma=0.995)
    for lv in (0, 1):
        rho, u = I.fields(wl, lv)
        ref.set_state(lv, rho, u)
        del rho, u
    t0 = time.perf_counter()
    ref.step(steps)
    dt = time.perf_counter() - t0
    return g.updates_per_step() * steps / dt / 1e6, O.threads(), dt, ref


def error_vs_oracle(wl, collision, precision, steps, ref):
    """Density max-abs and velocity relative L2 error of the GPU run against
    the FP64 oracle after the same number of steps, worst over the levels."""
    import numpy as np
    grid = make_gpu(wl, collision, precision)
    grid.step(steps)
    err = {"rho_maxabs": 0.0, "u_relL2": 0.0, "steps": steps,
           "grid": "x".join(str(x) for x in wl.geom.n[:wl.geom.D])}
    for lv in (0, 1):
        r1, u1 = grid.get_macros(lv)
        r0, u0 = ref.get_macros(lv)
        err["rho_maxabs"] = max(err["rho_maxabs"], float(np.abs(r1 - r0).max()))
        err["u_relL2"] = max(err["u_relL2"], float(np.linalg.norm(u1 - u0) / np.linalg.norm(u0)))
    grid.close()
    err["within_bar"] = bool(err["rho_maxabs"] < 1e-5 and err["u_relL2"] < 1e-4)
    return err


def paper_cases():
    """The paper's own diagnostics and cases on one GPU:
    * the acoustic wave of Sec. 8.2 (eq init_Pulse, A = 1e-4, nu = 1e-6) on its
      full set-up (fine band 500 < x < 1000, 2620 coarse steps, FP64), RR and
      H-RR: throughput, the waves RR emits at t = 2620 as fractions of A (the
      paper reports about A/25 upstream and A/100 downstream), H-RR's, and the
      fine-level SpuriousAc detections (divergence product below -1e-18);
    * the NH sensors and the probe switched on over a D2Q9 4096^2 RR FP32
      run, and dynamic sigma over a D2Q9 4096^2 H-RR FP32 run: throughput
      against the same runs without them."""
    import numpy as np
    import torch
    from paper_2004_11863_amd import inputs as I
    from paper_2004_11863_amd import lbm
    out = {}
    T = 2620
    A = 1e-4
    for col in ("RR", "HRR"):
        wl = I.acoustic_wave_case(height=2 * T + 64, left=1500, A=A)
        g = wl.geom
        gr = make_gpu(wl, col, "fp64", tau_coarse=0.5 + 1e-6 / I.CS2)
        ups = gr.updates_per_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gr.step(T - 1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        lbm.lbm_sensors_enable(gr.h, True)
        gr.step(1)
        nxc, nyc = g.n[0], g.n[1]
        nxf, nyf = g.fine_shape()
        jm = (nyf - 1) // 2
        ym = g.lo[1] + jm // 2
        shift = wl.plane_pulses[0].xc - 750.0
        rc = gr.get_macros(0)[0].reshape(nyc, nxc)[ym] - 1.0
        rf = gr.get_macros(1)[0].reshape(nyf, nxf)[jm] - 1.0
        _, dg = gr.sensors(1, 0.0)
        dprod = dg[0].reshape(nyf, nxf)[jm]
        gr.close()
        del gr
        torch.cuda.empty_cache()
        xc = np.arange(nxc) - shift
        up = np.abs(rc[(xc > 0) & (xc < 500)]).max()
        dn = np.abs(rf).max()
        out[f"acoustic_wave_{col.lower()}_fp64"] = {
            "mlups": round(ups * (T - 1) / dt / 1e6, 1), "steps": T, "updates_per_step": ups,
            "emitted_upstream_over_A": float(up / A), "emitted_downstream_over_A": float(dn / A),
            "fine_spurious_ac_detections": int((dprod < -1e-18).sum())}
        print(f"# paper case acoustic {col}: {out[f'acoustic_wave_{col.lower()}_fp64']}", file=sys.stderr, flush=True)
    for name, col, switch in (("sensors_probe", "RR", "sensors"), ("dynamic_sigma", "HRR", "dyn")):
        wl = workload("d2q9-4096")
        res = {}
        for on in (False, True):
            gr = make_gpu(wl, col, "fp32")
            gr.variants = gr.tune(reps=2)
            if on and switch == "sensors":
                lbm.lbm_sensors_enable(gr.h, True)
                lbm.lbm_probe_enable(gr.h, 1, (100, 100, 0), 1000)
            elif on:
                gr.set_dynamic_sigma(True, 0.0, 1e-12)
            gr.step(5)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gr.step(200)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res["on" if on else "off"] = round(gr.updates_per_step() * 200 / dt / 1e6, 1)
            if on and switch == "sensors":
                # one step per call: every step records (a read-out after
                # each step); a call of many steps records its last ones only
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(200):
                    gr.step(1)
                torch.cuda.synchronize()
                res["on_every_step"] = round(gr.updates_per_step() * 200 / (time.perf_counter() - t0) / 1e6, 1)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                gr.sensors(1, 1e-8)
                res["readout_fine_s"] = round(time.perf_counter() - t0, 4)
            gr.close()
            del gr
            torch.cuda.empty_cache()
        out[f"d2q9_4096_{col.lower()}_fp32_{name}"] = {
            "mlups_off": res["off"], "mlups_on": res["on"],
            **({"mlups_on_recording_every_step": res["on_every_step"], "readout_fine_s": res["readout_fine_s"]}
               if "readout_fine_s" in res else {})}
        print(f"# paper case {name}: {out[f'd2q9_4096_{col.lower()}_fp32_{name}']}", file=sys.stderr, flush=True)
    out["d3q19_256_three_levels_fp32"] = three_levels()
    print(f"# paper case three levels: {out['d3q19_256_three_levels_fp32']}", file=sys.stderr, flush=True)
    return out


def three_levels(steps=40):
    """Nested refinement (Sec. 10): D3Q19 FP32, RR and H-RR, coarse 256^3 with the
    level-1 patch [64, 192]^3 (257^3 nodes) and the level-2 patch [64, 192]^3
    of level-1 vertices (257^3 nodes, coarse [96, 160]^3); a plane-wave
    pulse crossing both interfaces on a uniform flow.  Throughput in lattice
    updates (level l counts 2^l per coarse step) against the two-level grid
    of the same coarse grid and level-1 patch, and its fraction of the
    per-update roofline (one read and one write of the populations)."""
    import numpy as np
    import torch
    from paper_2004_11863_amd import lbm
    n, lo, hi, lo2, hi2 = 256, 64, 192, 64, 192
    U, A, R = 0.05, 1e-3, 6.0

    def level_x(lv):
        if lv == 0:
            return np.arange(n, dtype=np.float64)
        x1 = lo + 0.5 * np.arange(2 * (hi - lo) + 1)
        return x1 if lv == 1 else lo + 0.5 * (lo2 + 0.5 * np.arange(2 * (hi2 - lo2) + 1))

    def state(g, lv):
        x = level_x(lv)
        m = x.size
        rho1 = 1.0 + A * np.exp(-((x - 80.0) ** 2) / (2 * R * R))  # varies along x only
        rho = np.broadcast_to(rho1[None, None, :], (m, m, m)).reshape(-1).copy()
        u = np.zeros((3, m ** 3))
        u[0] = U
        g.set_state(lv, rho, u)

    res = {}
    for col, levels in (("RR", 3), ("RR", 2), ("HRR", 3), ("HRR", 2)):
        cid = lbm.LBM_RR if col == "RR" else lbm.LBM_HRR
        if levels == 3:
            g = lbm.Nested(lbm.LBM_D3Q19, cid, lbm.LBM_FP32_DEV, (n,) * 3, (lo,) * 3, (hi,) * 3, (lo2,) * 3,
                           (hi2,) * 3, tau_coarse=0.51)
        else:
            g = lbm.Grid(lbm.LBM_D3Q19, cid, lbm.LBM_FP32_DEV, (n,) * 3, (lo,) * 3, (hi,) * 3, tau_coarse=0.51)
            g.variants = g.tune(reps=2)
        for lv in range(levels):
            state(g, lv)
        g.step(3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ups = g.updates_per_step()
        mlups = ups * steps / dt / 1e6
        r, _ = g.get_macros(levels - 1)
        finite = bool(np.isfinite(r).all())
        g.close()
        del g
        torch.cuda.empty_cache()
        res[f"{col.lower()}_levels{levels}"] = {"mlups": round(mlups, 1), "updates_per_step": ups,
                                  "ms_per_step": round(dt / steps * 1e3, 3),
                                  "frac_of_update_roofline": round(mlups * 1e6 * 2 * 19 * 4 / 1e9 / HBM_PEAK_GBS, 4),
                                  "finite": finite}
    return {"steps": steps, **res}


def batched(n_inst, steps):
    """n_inst independent D2Q9 two-level grids (sides log-uniform in
    [64, 1024], patch over the central half of each side, FP32, RR), all in
    one batch: one persistent launch per phase, one hipGraph replay per
    coarse step, autotuned tiles; against the plain per-instance loop (each
    grid stepped on its own, one after the other)."""
    import torch
    from paper_2004_11863_amd import inputs as I
    from paper_2004_11863_amd import lbm
    wls = [I.batch_instance(0, i) for i in range(n_inst)]
    b = lbm.Batch(lbm.LBM_D2Q9, lbm.LBM_RR, lbm.LBM_FP32_DEV, capacity=n_inst)
    for w in wls:
        g = w.geom
        sl = b.add(g.n[:2], g.lo[:2], g.hi[:2], 0.51)
        for lv in (0, 1):
            b.set_state(sl, lv, *I.fields(w, lv))
    ups = b.info()["updates_per_step"]
    variants = b.tune(reps=2)
    b.step(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    info = b.info()
    b.close()
    # plain per-instance loop on the same grids
    grids = []
    for w in wls:
        g = w.geom
        gr = lbm.Grid(lbm.LBM_D2Q9, lbm.LBM_RR, lbm.LBM_FP32_DEV, g.n[:2], g.lo[:2], g.hi[:2], 0.51)
        for lv in (0, 1):
            gr.set_state(lv, *I.fields(w, lv))
        grids.append(gr)
    loop_steps = max(5, steps // 10)
    for gr in grids:
        gr.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for gr in grids:
        gr.step(loop_steps)
    torch.cuda.synchronize()
    dl = time.perf_counter() - t0
    for gr in grids:
        gr.close()
    torch.cuda.empty_cache()
    return {"instances": n_inst, "updates_per_step": ups, "steps": steps, "device_bytes": info["bytes"],
            "batched_mlups": round(ups * steps / dt / 1e6, 1), "batched_ms_per_step": dt / steps * 1e3,
            "per_instance_loop_mlups": round(ups * loop_steps / dl / 1e6, 1),
            "per_instance_loop_steps": loop_steps, "variants": variants,
            "speedup": round((ups * steps / dt) / (ups * loop_steps / dl), 2)}


def _served(reqs, realtime=True):
    """One run of the continuous-batching server over prepared requests."""
    import torch
    from paper_2004_11863_amd import serve
    free, total = torch.cuda.mem_get_info()
    ex = serve.DeviceExecutor(capacity=64)
    srv = serve.Server(ex, int(0.8 * free), policy="srpt")
    t0 = time.perf_counter()
    done = srv.run(reqs, realtime=realtime)
    span = time.perf_counter() - t0
    ex.close()
    torch.cuda.empty_cache()
    return done, span


def _fifo(reqs, realtime=True):
    import torch
    from paper_2004_11863_amd import serve
    t0 = time.perf_counter()
    done = serve.fifo_loop(reqs, realtime=realtime)
    span = time.perf_counter() - t0
    torch.cuda.empty_cache()
    return done, span


def _run_stats(done, span, work):
    from paper_2004_11863_amd import serve
    st = serve.latency_stats(done)
    return {"p50_s": round(st["p50_s"], 3), "p99_s": round(st["p99_s"], 3), "max_s": round(st["max_s"], 3),
            "n": st["n"], "aggregate_mlups": round(work / span / 1e6, 1), "makespan_s": round(span, 3),
            "fp64_fallbacks": sum(getattr(r, "fell_back", False) for r in done)}


def serve_trace(n_req, rate, realtime=True, seed=5, reps=1, **shape):
    """Served (continuous batching) and FIFO one-at-a-time runs of one trace,
    `reps` times each, alternating; latency statistics and aggregate
    throughput of every run."""
    from paper_2004_11863_amd import serve
    served, fifo = [], []
    work = first = last = None
    for _ in range(reps):
        reqs = [r.prepare() for r in serve.poisson_trace(n_req, rate=rate, seed=seed, **shape)]
        work = sum(r.updates() for r in reqs)
        first, last = reqs[0].arrival, reqs[-1].arrival
        done, span = _served(reqs, realtime)
        served.append(_run_stats(done, span, work))
        reqs = [r.prepare() for r in serve.poisson_trace(n_req, rate=rate, seed=seed, **shape)]
        done, span = _fifo(reqs, realtime)
        fifo.append(_run_stats(done, span, work))
    return {"served_runs": served, "fifo_runs": fifo, "total_updates": work, "first_arrival_s": first,
            "last_arrival_s": last}


def _spread(runs, key):
    v = sorted(r[key] for r in runs)
    return {"min": v[0], "median": v[len(v) // 2], "max": v[-1]}


def serving(n_full, n_small, reps, rate=200.0, utilization=0.7):
    """A seeded Poisson stream (mean 200 requests/s) of two-level problems,
    half D2Q9 and half D3Q19, 100-2000 coarse steps each, FP32 with 10 %
    flagged FP64, RR.  Initial fields are sampled before the trace starts
    (client side).  Continuous batching (size-class groups, shortest
    remaining time first with backfill) against the plain FIFO per-instance
    loop on the same requests.

    small_requests: n_small arrivals with small grids (D2Q9 sides 64-512,
    D3Q19 sides 32-96), where per-request launches and host work matter,
    repeated `reps` times for the spread, then the same requests arriving at
    the rate that offers `utilization` of the served throughput.
    full_size: the first n_full arrivals of the full-size generator (D2Q9
    sides 128-2048, D3Q19 sides 64-256), one run each; with so few arrivals
    its p99 is close to the maximum."""
    import inspect
    from paper_2004_11863_amd import serve
    SERVER_DEFAULTS = {k: v.default for k, v in inspect.signature(serve.Server).parameters.items()}
    out = {"rate_per_s": rate, "policy": "srpt", "slice_s": SERVER_DEFAULTS["slice_s"],
           "backfill": SERVER_DEFAULTS["backfill"]}
    shape = dict(d2_side=(64, 512), d3_side=(32, 96))
    sm = serve_trace(n_small, rate, seed=11, reps=reps, **shape)
    work = sm["total_updates"]
    offered = work / (sm["last_arrival_s"] - sm["first_arrival_s"] + 1e-9)
    srv_thr, fifo_thr = _spread(sm["served_runs"], "aggregate_mlups"), _spread(sm["fifo_runs"], "aggregate_mlups")
    small = {"requests": n_small, "seed": 11, "d2_side": [64, 512], "d3_side": [32, 96], "total_updates": work,
             "offered_mlups": round(offered / 1e6, 1), "reps": reps,
             "served_runs": sm["served_runs"], "fifo_runs": sm["fifo_runs"],
             "served_mlups_spread": srv_thr, "fifo_mlups_spread": fifo_thr,
             "served_p50_spread": _spread(sm["served_runs"], "p50_s"),
             "served_p99_spread": _spread(sm["served_runs"], "p99_s"),
             "fifo_p50_spread": _spread(sm["fifo_runs"], "p50_s"),
             "fifo_p99_spread": _spread(sm["fifo_runs"], "p99_s"),
             "throughput_ratio_median": round(srv_thr["median"] / fifo_thr["median"], 3),
             # the served and FIFO throughput ranges over the repeats overlap
             "throughput_tie": bool(srv_thr["min"] <= fifo_thr["max"] and fifo_thr["min"] <= srv_thr["max"])}
    small["saturated"] = bool(offered > srv_thr["median"] * 1e6)
    rate_u = utilization * srv_thr["median"] * 1e6 / (work / n_small)
    sub = serve_trace(n_small, rate_u, seed=11, **shape)
    small["sub_saturation"] = {"utilization_target": utilization, "rate_per_s": round(rate_u, 4),
                               "served": sub["served_runs"][0], "fifo_per_instance": sub["fifo_runs"][0]}
    out["small_requests"] = small
    print(f"# serving small: {small}", file=sys.stderr, flush=True)
    full = serve_trace(n_full, rate, seed=5)
    fw = full["total_updates"]
    out["full_size"] = {"requests": n_full, "seed": 5, "d2_side": [128, 2048], "d3_side": [64, 256],
                        "total_updates": fw,
                        "offered_mlups": round(fw / (full["last_arrival_s"] - full["first_arrival_s"] + 1e-9) / 1e6, 1),
                        "served": full["served_runs"][0], "fifo_per_instance": full["fifo_runs"][0]}
    return out


def d2d_copy_GBs(mib=2048, reps=10):
    """Device-to-device copy bandwidth (bytes read + written per second) of a
    plain `copy_` of mib MiB, timed with HIP events on the current stream."""
    import torch
    a = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    gbs = 2 * a.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def copy_probe(mib):
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "launches": 5}))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    from paper_2004_11863_amd import lbm
    lbm.load()
    if args.three_levels:
        print(json.dumps({"three_levels_d3q19_256_fp32": three_levels()}), flush=True)
        return

    copy_gbs = (d2d_copy_GBs(), lbm.lbm_copy_probe(2 << 30, 10))
    wl = workload(args.workload)
    grid = make_gpu(wl, args.collision, args.precision)
    ups = grid.updates_per_step()
    if args.variants:
        grid.variants = [int(x) for x in args.variants.split(",")]
        grid.set_variants(grid.variants)
    dt, kt = timed_run(grid, args.steps, args.warmup, profile=True, tune=not args.variants)
    mlups = ups * args.steps / dt / 1e6
    m, p = grid.totals()  # finite check
    Q = grid.Q
    pb = 4 if args.precision == "fp32" else 8
    g = wl.geom
    D = g.D
    variants = getattr(grid, "variants", None)
    roof = roofline_of(kt, Q, pb, g)
    khash = kernel_source_hash()
    key = f"{args.workload}/{args.collision}/{args.precision}"
    traffic = stored_traffic(khash, key, None if variants is None else variants[1])
    grid.close()
    del grid
    torch.cuda.empty_cache()

    mean_ms = roof["mean_launch_ms"]
    result = {
        "metric": "MLUPS & % HBM roofline, FP32 vs FP64 two-level; batched p50/p99 solve latency",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": ("D2Q9 two-level, coarse %dx%d periodic, fine patch %dx%d nodes, %s, %s storage"
                         % (g.n[0], g.n[1], 2 * (g.hi[0] - g.lo[0]) + 1, 2 * (g.hi[1] - g.lo[1]) + 1,
                            args.collision, "FP32-deviation" if args.precision == "fp32" else "FP64")
                         if D == 2 else
                         "D3Q19 two-level, coarse %d^3 periodic, fine cube %d^3 nodes, %s, %s storage"
                         % (g.n[0], 2 * (g.hi[0] - g.lo[0]) + 1, args.collision,
                            "FP32-deviation" if args.precision == "fp32" else "FP64")),
            "lattice": "D2Q9" if D == 2 else "D3Q19",
            "coarse": list(g.n[:D]),
            "patch_lo": list(g.lo[:D]),
            "patch_hi": list(g.hi[:D]),
            "collision": args.collision,
            "tau_coarse": 0.51,
            "updates_per_step": ups,
            "parallelism": "single GPU",
        },
        "roofline": dict({
            "bound": "hbm",
            "kernel": kernel_label(D, args.collision, variants),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "traffic": traffic,
            # HBM bandwidth the kernel actually drew (counter traffic over the
            # live launch time)
            "hbm_achieved": None if traffic is None else round(traffic / (mean_ms * 1e-3) / 1e9, 1),
            "hbm_frac": None if traffic is None else round(traffic / (mean_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            # the same against the faster of two device-to-device copies
            # measured in this run (hipMemcpy through torch, and the
            # library's streaming copy kernel), bytes read + written
            "copy_GBs": {"memcpy": round(copy_gbs[0], 1), "streaming_kernel": round(copy_gbs[1], 1)},
            "frac_of_copy": round(roof["achieved"] / max(copy_gbs), 4),
        }, **roof),
        # whole step against the per-update roofline (2 Q P_b bytes per lattice update at 8 TB/s)
        "step_frac_of_update_roofline": round(mlups * 1e6 * 2 * Q * pb / 1e9 / HBM_PEAK_GBS, 4),
        "kernel_variants": variants,
        "totals_finite": bool(all(map(lambda v: v == v, list(m) + list(p.ravel())))),
        "kernel_source_hash": khash,
    }
    print(f"# headline: {result['value']} MLUPS, {result['ms_per_step']:.3f} ms/step, roofline "
          f"{result['roofline']['frac']}", file=sys.stderr, flush=True)

    if not args.no_extra:
        extra = {}
        for name, wname, col, prec, steps in (
                ("d3q19_384_rr_fp64", "d3q19-384", "RR", "fp64", 30),
                ("d3q19_384_hrr_fp32", "d3q19-384", "HRR", "fp32", 40),
                ("d2q9_4096_rr_fp32", "d2q9-4096", "RR", "fp32", 400),
                ("d2q9_4096_rr_fp64", "d2q9-4096", "RR", "fp64", 200),
                ("d2q9_4096_hrr_fp32", "d2q9-4096", "HRR", "fp32", 200)):
            if (wname, col, prec) == (args.workload, args.collision, args.precision):
                continue
            w2 = workload(wname)
            gr = make_gpu(w2, col, prec)
            u2 = gr.updates_per_step()
            d2, k2 = timed_run(gr, steps, 5, profile=True)
            q2, pb2 = gr.Q, (4 if prec == "fp32" else 8)
            r2 = roofline_of(k2, q2, pb2, w2.geom)
            mlu = u2 * steps / d2 / 1e6
            extra[name] = {"mlups": round(mlu, 1), "steps": steps,
                           "ms_per_step": d2 / steps * 1e3,
                           "fine_kernel": kernel_label(w2.geom.D, col, getattr(gr, "variants", None)).split(":")[0],
                           "variants": getattr(gr, "variants", None),
                           "fine_kernel_GBs": r2["achieved"], "fine_kernel_frac": r2["frac"],
                           "fine_kernel_update_equivalent_GBs": r2["update_equivalent_GBs"],
                           "fine_kernel_mean_ms": r2["mean_launch_ms"],
                           "step_frac_of_update_roofline": round(mlu * 1e6 * 2 * q2 * pb2 / 1e9 / HBM_PEAK_GBS, 4)}
            gr.close()
            del gr, w2
            torch.cuda.empty_cache()
            print(f"# extra {name}: {extra[name]}", file=sys.stderr, flush=True)
        result["extra"] = extra

    if not args.no_paper:
        result["paper_cases"] = paper_cases()
    if not args.no_batch:
        result["batched"] = batched(args.batch_n, args.batch_steps)
        print(f"# batched: {result['batched']}", file=sys.stderr, flush=True)
    if not args.no_serve:
        result["serving"] = serving(args.serve_n, args.serve_small_n, args.serve_reps)
        print(f"# serving: {result['serving']}", file=sys.stderr, flush=True)

    if not args.no_cpu:
        sw, what = cpu_sample(args.workload)
        steps = args.cpu_steps if args.cpu_steps is not None else (300 if D == 3 else 24)
        v, cores, t, ref = cpu_baseline(sw, args.collision, steps)
        result["cpu_baseline"] = {"value": round(v, 2), "unit": "MLUPS", "cores": cores, "kind": "oracle",
                                  "sample": "%d coarse steps of the %s in FP64 (%.1f s)" % (steps, what, t)}
        result["error_vs_oracle"] = error_vs_oracle(sw, args.collision, args.precision, steps, ref)
        result["error_vs_oracle"]["sample"] = what
        del ref
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
