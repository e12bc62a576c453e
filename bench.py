#!/usr/bin/env python3
"""Throughput benchmark of the two-level lattice-Boltzmann hot path on one
MI355X.

A step is one coarse time step of the two-level scheme (one coarse update and
two fine substeps with the full interface treatment).  The default workload
is the D2Q9 two-level problem with a 4096^2 periodic coarse grid and a
4097 x 2049-node fine band (patch [1024, 3072] x [1536, 2560] in coarse
vertices), recursive regularised collision, tau_c = 0.51, populations stored
in FP32 as deviations from the lattice weights; input: a convected vortex
plus a Gaussian acoustic pulse (amplitude 1e-3), seeded.

Prints ONE JSON line.  value = MLUPS = (evolving coarse nodes + 2 x fine
nodes) x steps / seconds / 1e6, inputs resident in HBM.  The roofline object
prices the dominant kernel (the fine-level pull-stream + collide) with its
algorithmic bytes (one read and one write of Q populations per node) over its
mean launch duration measured with HIP events on its launch stream during
the timed region.  cpu_baseline times the FP64 CPU oracle on a bounded sample
of the same workload.
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
    p.add_argument("--workload", default="d2q9-4096", choices=["d2q9-4096", "d3q19-384", "d2q9-1024"])
    p.add_argument("--collision", default="RR", choices=["BGK", "RR", "HRR"])
    p.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    p.add_argument("--no-extra", action="store_true", help="skip the secondary measurements")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-steps", type=int, default=24,
                   help="coarse steps of the CPU oracle sample (about 10 s on 16 host cores at D2Q9 4096^2)")
    p.add_argument("--no-batch", action="store_true", help="skip the batched-instances measurement")
    p.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    p.add_argument("--batch-n", type=int, default=256)
    p.add_argument("--batch-steps", type=int, default=200)
    p.add_argument("--serve-n", type=int, default=16)
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
                "algorithmic bytes count 2 Q P_b per lattice update, 2 updates per node per launch")
    if collision == "HRR" and D == 2:
        return "k_hrr2: one H-RR fine substep in one pass (pull, velocities of the tile in LDS, strain rate, collide)"
    if collision == "HRR":
        if v[3] >= 2:
            return "k_hrr3: one H-RR fine substep in one marching pass (velocity planes in LDS, strain rate, collide)"
        return "k_collide_hrr: fine-level pull + H-RR collide (second pass)"
    if v[1] >= 2:
        return "k_fine3: both fine substeps of a coarse step in one marching pass (2 updates per node per launch)"
    return "k_stream: fine-level pull + collide"


def workload(name, seed=0):
    from paper_2004_11863_amd import inputs as I
    if name == "d2q9-4096":
        return I.config2(seed=seed, n=4096)
    if name == "d2q9-1024":
        return I.config2(seed=seed, n=1024)
    return I.config3(seed=seed, n=384)


def make_gpu(wl, collision, precision):
    from paper_2004_11863_amd import inputs as I
    from paper_2004_11863_amd import lbm
    g = wl.geom
    D = g.D
    lat = lbm.LBM_D2Q9 if D == 2 else lbm.LBM_D3Q19
    col = {"BGK": lbm.LBM_BGK, "RR": lbm.LBM_RR, "HRR": lbm.LBM_HRR}[collision]
    prec = lbm.LBM_FP32_DEV if precision == "fp32" else lbm.LBM_FP64
    grid = lbm.Grid(lat, col, prec, g.n[:D], g.lo[:D], g.hi[:D], tau_coarse=0.51, sigma=0.995)
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
    err = {"rho_maxabs": 0.0, "u_relL2": 0.0, "steps": steps}
    for lv in (0, 1):
        r1, u1 = grid.get_macros(lv)
        r0, u0 = ref.get_macros(lv)
        err["rho_maxabs"] = max(err["rho_maxabs"], float(np.abs(r1 - r0).max()))
        err["u_relL2"] = max(err["u_relL2"], float(np.linalg.norm(u1 - u0) / np.linalg.norm(u0)))
    grid.close()
    return err


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


def serve_trace(n_req, rate, realtime=True, seed=5, **shape):
    """Served (continuous batching) and FIFO one-at-a-time runs of one trace;
    latency statistics and aggregate throughput of each."""
    import torch
    from paper_2004_11863_amd import serve
    reqs = [r.prepare() for r in serve.poisson_trace(n_req, rate=rate, seed=seed, **shape)]
    work = sum(r.updates() for r in reqs)
    free, total = torch.cuda.mem_get_info()
    ex = serve.DeviceExecutor(capacity=64)
    srv = serve.Server(ex, int(0.8 * free), policy="srpt")
    t0 = time.perf_counter()
    done = srv.run(reqs, realtime=realtime)
    span = time.perf_counter() - t0
    ex.close()
    torch.cuda.empty_cache()
    st = serve.latency_stats(done)
    reqs2 = [r.prepare() for r in serve.poisson_trace(n_req, rate=rate, seed=seed, **shape)]
    t0 = time.perf_counter()
    done2 = serve.fifo_loop(reqs2, realtime=realtime)
    span2 = time.perf_counter() - t0
    st2 = serve.latency_stats(done2)
    torch.cuda.empty_cache()
    return {"served": {"p50_s": round(st["p50_s"], 3), "p99_s": round(st["p99_s"], 3),
                       "aggregate_mlups": round(work / span / 1e6, 1), "makespan_s": round(span, 3),
                       "fp64_fallbacks": sum(r.fell_back for r in done)},
            "fifo_per_instance": {"p50_s": round(st2["p50_s"], 3), "p99_s": round(st2["p99_s"], 3),
                                  "aggregate_mlups": round(work / span2 / 1e6, 1), "makespan_s": round(span2, 3)},
            "total_updates": work, "first_arrival_s": reqs[0].arrival, "last_arrival_s": reqs[-1].arrival}


def serving(n_req, rate=200.0, utilization=0.7):
    """A seeded Poisson stream (mean 200 requests/s) mixing D2Q9 (sides
    128-2048) and D3Q19 (sides 64-256) two-level problems with 100-2000 coarse
    steps, FP32 with 10 % flagged FP64, RR; first n_req arrivals.  Initial
    fields are sampled before the trace starts (client side).  Continuous
    batching (size-class groups, shortest remaining time first with backfill)
    against the plain FIFO per-instance loop on the same trace; then the same
    requests arriving at the rate that offers `utilization` of the measured
    served throughput (the request mix is the same: the seed fixes it); and
    64 arrivals of the same generator with small grids."""
    import inspect
    from paper_2004_11863_amd import serve
    SERVER_DEFAULTS = {k: v.default for k, v in inspect.signature(serve.Server).parameters.items()}
    sat = serve_trace(n_req, rate)
    work = sat["total_updates"]
    offered = work / (sat["last_arrival_s"] - sat["first_arrival_s"] + 1e-9)
    out = {"requests": n_req, "rate_per_s": rate, "total_updates": work,
           "policy": "srpt", "slice_s": SERVER_DEFAULTS["slice_s"], "backfill": SERVER_DEFAULTS["backfill"],
           "served": sat["served"], "fifo_per_instance": sat["fifo_per_instance"],
           "offered_mlups": round(offered / 1e6, 1), "saturated": bool(offered > sat["served"]["aggregate_mlups"] * 1e6)}
    capacity = sat["served"]["aggregate_mlups"] * 1e6
    mean_work = work / n_req
    rate_u = utilization * capacity / mean_work
    sub = serve_trace(n_req, rate_u)
    out["sub_saturation"] = {"utilization_target": utilization, "rate_per_s": round(rate_u, 4),
                             "served": sub["served"], "fifo_per_instance": sub["fifo_per_instance"]}
    # the same generator with small grids (64 requests: D2Q9 sides 64-512,
    # D3Q19 sides 32-96), where per-request launches dominate and batching pays
    small = serve_trace(64, rate, seed=11, d2_side=(64, 512), d3_side=(32, 96))
    out["small_requests"] = {"requests": 64, "rate_per_s": rate, "d2_side": [64, 512], "d3_side": [32, 96],
                             "seed": 11, "total_updates": small["total_updates"],
                             "served": small["served"], "fifo_per_instance": small["fifo_per_instance"]}
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

    copy_gbs = (d2d_copy_GBs(), lbm.lbm_copy_probe(2 << 30, 10))
    wl = workload(args.workload)
    grid = make_gpu(wl, args.collision, args.precision)
    ups = grid.updates_per_step()
    dt, kt = timed_run(grid, args.steps, args.warmup, profile=True)
    mlups = ups * args.steps / dt / 1e6
    m, p = grid.totals()  # finite check
    launches, mean_ms, nodes = kt
    Q = grid.Q
    pb = 4 if args.precision == "fp32" else 8
    alg_bytes = 2 * Q * pb * nodes
    achieved = alg_bytes / (mean_ms * 1e-3) / 1e9
    variants = getattr(grid, "variants", None)
    khash = kernel_source_hash()
    key = f"{args.workload}/{args.collision}/{args.precision}"
    traffic = stored_traffic(khash, key, None if variants is None else variants[1])
    grid.close()
    del grid
    torch.cuda.empty_cache()

    g = wl.geom
    D = g.D
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
        "roofline": {
            "bound": "hbm",
            "kernel": kernel_label(D, args.collision, variants),
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch": alg_bytes,
            "updates_per_launch": nodes,
            "launches": launches,
            "mean_launch_ms": mean_ms,
            # HBM bandwidth the kernel actually drew (counter traffic over the
            # live launch time); differs from `achieved` when one launch
            # performs several lattice updates per node
            "hbm_achieved": None if traffic is None else round(traffic / (mean_ms * 1e-3) / 1e9, 1),
            "hbm_frac": None if traffic is None else round(traffic / (mean_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            # the same against the faster of two device-to-device copies
            # measured in this run (hipMemcpy through torch, and the
            # library's streaming copy kernel), bytes read + written
            "copy_GBs": {"memcpy": round(copy_gbs[0], 1), "streaming_kernel": round(copy_gbs[1], 1)},
            "hbm_frac_of_copy": None if traffic is None else round(traffic / (mean_ms * 1e-3) / 1e9 / max(copy_gbs), 4),
        },
        "kernel_variants": variants,
        "totals_finite": bool(all(map(lambda v: v == v, list(m) + list(p.ravel())))),
        "kernel_source_hash": khash,
    }

    if not args.no_extra:
        extra = {}
        for name, wname, col, prec, steps in (
                ("d2q9_4096_rr_fp64", "d2q9-4096", "RR", "fp64", 200),
                ("d2q9_4096_hrr_fp32", "d2q9-4096", "HRR", "fp32", 200),
                ("d3q19_384_rr_fp32", "d3q19-384", "RR", "fp32", 60),
                ("d3q19_384_rr_fp64", "d3q19-384", "RR", "fp64", 30),
                ("d3q19_384_hrr_fp32", "d3q19-384", "HRR", "fp32", 40)):
            if (wname, col, prec) == (args.workload, args.collision, args.precision):
                continue
            w2 = workload(wname)
            gr = make_gpu(w2, col, prec)
            u2 = gr.updates_per_step()
            d2, k2 = timed_run(gr, steps, 5, profile=True)
            q2, pb2 = gr.Q, (4 if prec == "fp32" else 8)
            a2 = 2 * q2 * pb2 * k2[2] / (k2[1] * 1e-3) / 1e9
            extra[name] = {"mlups": round(u2 * steps / d2 / 1e6, 1), "steps": steps,
                           "ms_per_step": d2 / steps * 1e3,
                           "fine_kernel": kernel_label(2 if wname.startswith("d2q9") else 3, col,
                                                       getattr(gr, "variants", None)).split(":")[0],
                           "variants": getattr(gr, "variants", None),
                           "fine_kernel_alg_GBs": round(a2, 1), "fine_kernel_alg_frac": round(a2 / HBM_PEAK_GBS, 4)}
            gr.close()
            del gr, w2
            torch.cuda.empty_cache()
            print(f"# extra {name}: {extra[name]}", file=sys.stderr, flush=True)
        result["extra"] = extra

    if not args.no_batch:
        result["batched"] = batched(args.batch_n, args.batch_steps)
        print(f"# batched: {result['batched']}", file=sys.stderr, flush=True)
    if not args.no_serve:
        result["serving"] = serving(args.serve_n)
        print(f"# serving: {result['serving']}", file=sys.stderr, flush=True)

    if not args.no_cpu:
        v, cores, t, ref = cpu_baseline(wl, args.collision, args.cpu_steps)
        result["cpu_baseline"] = {"value": round(v, 2), "unit": "MLUPS", "cores": cores, "kind": "oracle",
                                  "sample": "%d coarse steps of the same grid and input in FP64 (%.1f s)"
                                            % (args.cpu_steps, t)}
        result["error_vs_oracle"] = error_vs_oracle(wl, args.collision, args.precision, args.cpu_steps, ref)
        del ref
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
