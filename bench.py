"""Benchmark of the fused stream-and-collide sweep on one MI355X.

Default workload: D3Q27 regularized cumulant method, 512^3 periodic box, Taylor-Green vortex
(u0 = 0.05, Re = 1600 -> omega_s = 1.969902, all other rates 1), pull pattern, FP32 storage
and compute (value).  Reported beside it, on the same GPU: the plain FP64 single-box form,
the batched ensemble form (256 D3Q27 central-moment boxes of edge 32..96, one launch per
step, a 100-step hipGraph, FP32), the copy-kernel ceiling and the FP64 CPU oracle timed on a
bounded sample.  One step = one fused stream + collide sweep over all cells.  Inputs are
resident in HBM before timing; the hipGraph of the timed steps is recorded before timing.

Prints one JSON line.  `roofline.achieved` = algorithmic bytes per launch (2 Q sizeof per
lattice update) / average launch duration from HIP events on the library's stream.

  python bench.py [--gpus 1] [--steps 200] [--warmup 10]
  python bench.py --workload d3q19_raw_256 | swe_d2q9_4096 | d2q9_central_64 | batch_d3q27_central
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import lbm_workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_{workload}.json")
SBYTES = {"f64": 8, "f32": 4, "f16": 2}


def measured_traffic(workload, layout):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken on the
    current kernel sources and the same storage layout; else None."""
    path = TRAFFIC_FILE.format(workload=workload)
    if not os.path.exists(path):
        return None
    from paper_2211_02435_amd.rocprof_summary import kernel_source_hash
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha") != kernel_source_hash() or t.get("layout") != layout:
        return None
    return t.get("bytes_per_launch")


def workload_fields(name, cfg, n):
    if name == "swe_d2q9_4096":
        return W.swe_bumps(n, seed=0), (n, n, 1)
    if name == "d2q9_central_64":
        return W.tgv2d_fields(n, n, 1, u0=cfg["u0"]), (n, n, 1)
    return W.tgv3d_fields(n, u0=cfg["u0"]), (n, n, n)


def workload_rates(cfg, general=False):
    """Regularized rates of the workload; with general=True every rate of order >= 3 is 1.3
    instead of 1, which selects the general (non-regularized) kernels."""
    from paper_2211_02435_amd import lbm
    om = lbm.regularized_rates(cfg["stencil"], cfg["omega_shear"])
    if general:
        for k, order in enumerate(lbm.BASIS_ORDERS[cfg["stencil"]]):
            if order >= 3:
                om[k] = 1.3
    return om


def measure_box(lbm, cfg, storage, fields, dims, steps, warmup, autotune, streaming, layout, transform="chimera",
                general=False):
    """Run one box: init, autotune, warm-up, record the graph, time `steps` sweeps."""
    import torch
    stencil, space = cfg["stencil"], cfg["space"]
    om = workload_rates(cfg, general)
    q = lbm.Q[stencil]
    kw = {}
    if cfg.get("equilibrium") == "swe":
        kw = {"equilibrium": "swe", "gravity": cfg["gravity"]}
    lat = lbm.Lattice(stencil, space, om, dims, storage=storage, streaming=streaming, layout=layout, **kw)
    lat.lbm_init_equilibrium(*fields)
    if autotune:
        lat.lbm_autotune()
    if transform != "chimera":
        bx, by, _ = lat.lbm_get_launch()
        if bx * by > 256:  # the ablation kernel takes at most four waves per block
            nbx = min(bx, 256)
            lat.lbm_set_launch(nbx, max(1, 256 // nbx), 1)
        lat.lbm_set_transform(transform)
    lat.lbm_step(warmup)
    lat.lbm_graph_prepare(steps)
    lat.lbm_synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_events = lat.lbm_time_steps(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cells = dims[0] * dims[1] * dims[2]
    t_launch = ms_events / 1e3 / steps
    gbs = 2 * q * SBYTES[storage] * cells / t_launch / 1e9
    res = {"mlups": cells * steps / wall / 1e6, "ms_per_step": wall * 1e3 / steps,
           "avg_launch_ms": t_launch * 1e3, "achieved_GBps": gbs, "frac": gbs / HBM_PEAK_GBS,
           "bytes_per_lup": 2 * q * SBYTES[storage],
           "launch_bx_by_swizzle_vec_lds": list(lat.lbm_get_launch()) + [int(lat.lbm_get_vectorized()),
                                                                        lat.lbm_get_lds_reserve()],
           "transform": lat.lbm_get_transform(), "layout": lat.lbm_get_layout()}
    return lat, res


def measure_batch(lbm, steps, warmup):
    """The ensemble of 256 D3Q27 central-moment boxes (FP32), one launch per step, graph."""
    import torch
    boxes = W.batch_ensemble(256, seed=0)
    dims = [(b["edge"],) * 3 for b in boxes]
    rates = [lbm.regularized_rates("D3Q27", b["omega_shear"]) for b in boxes]
    fields = [W.batch_fields(b) for b in boxes]
    rho = np.concatenate([f[0].ravel() for f in fields])
    u = np.concatenate([f[1].ravel() for f in fields])
    del fields
    bat = lbm.Batch("D3Q27", "central", dims, rates, storage="f32")
    bat.lbm_batch_init_equilibrium(rho, u)
    del rho, u
    launch = bat.lbm_batch_autotune()
    bat.lbm_batch_step(warmup)
    bat.lbm_batch_graph_prepare(steps)
    bat.lbm_batch_synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = bat.lbm_batch_time_steps(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cells = bat.lbm_batch_cells()
    gbs = 216 * cells / (ms / 1e3 / steps) / 1e9
    return {"boxes": len(boxes), "cells": cells, "steps": steps, "graph_steps": steps,
            "mlups": cells * steps / wall / 1e6, "ms_per_step": wall * 1e3 / steps,
            "avg_launch_ms": ms / steps, "achieved_GBps": gbs, "frac": gbs / HBM_PEAK_GBS,
            "storage": "f32", "space": "central", "launch_threads_swizzle_lds": list(launch)}


def cpu_baseline(cfg, n, steps):
    """The FP64 oracle, single-threaded, on an n^3 copy of the Taylor-Green workload."""
    from threadpoolctl import threadpool_limits
    import oracle as O
    with threadpool_limits(limits=1):
        m = O.Method(cfg["stencil"], cfg["space"], O.regularized_rates(cfg["stencil"], cfg["omega_shear"]))
        rho, u = W.tgv3d_fields(n, u0=cfg["u0"])
        df = O.init_equilibrium(m, rho, u)
        t0 = time.perf_counter()
        O.step(m, df, steps)
        dt = time.perf_counter() - t0
    return {"value": n ** 3 * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": "FP64 numpy oracle (dense K(u), set-partition cumulants), %d^3 copy of the same "
                      "Taylor-Green workload, %d steps, %.1f s" % (n, steps, dt)}


def copy_ceiling(lbm):
    import torch
    nbytes = 4 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    ms = lbm.lbm_copy_bandwidth(b, a, nbytes, 20)
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes * 20 / (ms / 1e3) / 1e9


def velocity_rel_diff(lbm, lat_a, lat_b):
    import torch
    n = lat_a.ncells
    us = []
    for lat in (lat_a, lat_b):
        r = torch.empty(n, dtype=torch.float64, device="cuda")
        v = torch.empty(3 * n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        lbm.check(lat.lib.lbm_macroscopic(lat.ctx, lbm._dptr(r), lbm._dptr(v)))
        us.append(v)
        del r
    return float(torch.linalg.norm(us[0] - us[1]) / torch.linalg.norm(us[1]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="d3q27_cumulant_512", choices=sorted(W.WORKLOADS))
    ap.add_argument("--size", type=int, default=0, help="override the edge length (smaller boxes)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--layout", default="auto", choices=["auto", "planes", "rows"])
    ap.add_argument("--streaming", default="pull", choices=["pull", "push", "aa", "esoteric", "twist"])
    ap.add_argument("--rates", default="regularized", choices=["regularized", "general"],
                    help="general: every rate of order >= 3 set to 1.3 (non-regularized kernels)")
    ap.add_argument("--transform", default="chimera", choices=["chimera", "dense_mfma"],
                    help="dense_mfma: the measured ablation of the raw-moment transform on MFMA")
    ap.add_argument("--cpu-size", type=int, default=32)
    ap.add_argument("--cpu-steps", type=int, default=40)
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (a box would shard "
              "as z-slabs with one halo exchange per step; not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2211_02435_amd import lbm

    name = args.workload
    cfg = W.WORKLOADS[name]
    if name == "batch_d3q27_central":
        res = measure_batch(lbm, args.steps, args.warmup)
        out = {"metric": "MLUPS and % of HBM roofline, batched ensemble of 256 D3Q27 central-moment boxes",
               "value": res["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic Taylor-Green boxes",
               "config": {"workload": "256 periodic D3Q27 central-moment boxes, edges 32..96, seed 0"},
               "roofline": {"bound": "hbm", "achieved": res["achieved_GBps"], "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": res["frac"], "traffic": None}, "batch": res}
        print(json.dumps(out), flush=True)
        return

    n = args.size or cfg["dims"][0]
    fields, dims = workload_fields(name, cfg, n)
    storages = {"swe_d2q9_4096": ["f16", "f64"], "d2q9_central_64": ["f64"]}.get(name, ["f32", "f64"])
    if args.no_fp64:
        storages = [s for s in storages if s != "f64"] or storages[:1]
    print("[bench] %s %s dims %s, steps %d, warmup %d" % (name, storages, dims, args.steps, args.warmup),
          file=sys.stderr, flush=True)
    runs, lats = {}, {}
    for st in storages:
        lat, res = measure_box(lbm, cfg, st, fields, dims, args.steps, args.warmup,
                               not args.no_autotune, args.streaming, args.layout, args.transform,
                               args.rates == "general")
        runs[st], lats[st] = res, lat
        print("[bench] %s: %.0f MLUPS, %.1f GB/s" % (st, res["mlups"], res["achieved_GBps"]),
              file=sys.stderr, flush=True)
    del fields
    main_st = storages[0]
    vel = None
    if "f64" in lats and main_st != "f64":
        vel = velocity_rel_diff(lbm, lats[main_st], lats["f64"])
    for lat in lats.values():
        lat.close()
    lats.clear()
    torch.cuda.empty_cache()

    is_metric = name == "d3q27_cumulant_512" and n == cfg["dims"][0]
    batch = None
    if is_metric and not args.no_batch:
        batch = measure_batch(lbm, 100, args.warmup)
        print("[bench] batch: %.0f MLUPS" % batch["mlups"], file=sys.stderr, flush=True)
    ceiling = copy_ceiling(lbm)
    cpu = None
    if is_metric and not args.no_cpu:
        cpu = cpu_baseline(cfg, args.cpu_size, args.cpu_steps)

    r = runs[main_st]
    fields_desc = ("shallow water g 0.1, 16 Gaussian bumps" if name == "swe_d2q9_4096"
                   else "Taylor-Green u0 %.2f" % cfg["u0"])
    workload = "%s %s %s periodic, %s, omega_s %.6f, %s, %s" % (
        cfg["stencil"], cfg["space"], "x".join(str(d) for d in dims), fields_desc, cfg["omega_shear"],
        "other rates 1" if args.rates == "regularized" else "orders >= 3 at 1.3, bulk 1", args.streaming)
    out = {
        "metric": ("MLUPS and % of HBM roofline, D3Q27 cumulant 512^3, FP32 vs FP64" if is_metric
                   else "MLUPS and % of HBM roofline, " + name),
        "value": r["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_st,
        "data": "synthetic initial fields (Taylor-Green vortex / Gaussian water bumps)",
        "config": {"workload": workload, "cells": int(np.prod(dims)), "storage": main_st,
                   "layout": r.get("layout", args.layout), "streaming": args.streaming, "transform": args.transform,
                   "rates": args.rates,
                   "launch_bx_by_swizzle_vec_lds": r["launch_bx_by_swizzle_vec_lds"]},
        "roofline": {"bound": "hbm", "achieved": r["achieved_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r["frac"],
                     "traffic": measured_traffic(name, r.get("layout")) if (n == cfg["dims"][0] and main_st == "f32"
                                                           and args.streaming == "pull"
                                                           and args.transform == "chimera"
                                                           and args.rates == "regularized") else None,
                     "kernel": "sweep_kernel<%s, %s, %s, %s, %s>" % (cfg["stencil"], cfg["space"], args.rates,
                                                                     main_st, args.streaming),
                     "bytes_per_lup": r["bytes_per_lup"], "avg_launch_ms": r["avg_launch_ms"]},
        "fp64": runs.get("f64") if main_st != "f64" else None,
        "velocity_rel_l2_vs_fp64": vel,
        "batched": batch,
        "copy_ceiling_GBps": ceiling,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
