"""Benchmark of the fused stream-and-collide sweep on one MI355X.

Default workload: D3Q27 regularized cumulant method, 512^3 periodic box, Taylor-Green vortex
(u0 = 0.05, Re = 1600 -> omega_s = 1.969902, all other rates 1), pull pattern, FP32 storage
and compute (value) with the FP64 form on the same GPU beside it.  One step = one fused
stream + collide sweep over all 134 M cells.  Inputs are resident in HBM before timing.

Prints one JSON line: MLUPS, roofline of the sweep kernel (algorithmic bytes 2 Q sizeof per
lattice update over its HIP-event-timed average launch), the measured copy-kernel ceiling,
the FP32-vs-FP64 velocity difference and the FP64 CPU oracle timed on a bounded sample.

  python bench.py [--gpus 1] [--steps 200] [--warmup 10] [--workload d3q27_cumulant_512]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import lbm_workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_{workload}.json")


def measured_traffic(workload, lups_per_launch):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken on the
    current kernel source; else None."""
    path = TRAFFIC_FILE.format(workload=workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    from paper_2211_02435_amd.rocprof_summary import kernel_source_hash
    if t.get("kernel_source_sha") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def build_workload(name):
    cfg = W.WORKLOADS[name]
    return cfg


def run_box(lbm, stencil, space, om, dims, storage, rho, u, steps, warmup, autotune, streaming="pull",
            layout="auto"):
    import torch
    lat = lbm.Lattice(stencil, space, om, dims, storage=storage, streaming=streaming, layout=layout)
    lat.lbm_init_equilibrium(rho, u)
    if autotune:
        lat.lbm_autotune()
    lat.lbm_step(warmup)
    lat.lbm_graph_prepare(steps)  # record the hipGraph outside the timed region
    lat.lbm_synchronize()
    # the timed region: graph replay of `steps` sweeps, bracketed by full synchronisation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_events = lat.lbm_time_steps(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return lat, wall, ms_events


def velocity_device(lat, lbm):
    import torch
    nx, ny, nz = lat.dims
    rho = torch.empty(nx * ny * nz, dtype=torch.float64, device="cuda")
    u = torch.empty(3 * nx * ny * nz, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    lbm.check(lat.lib.lbm_macroscopic(lat.ctx, lbm._dptr(rho), lbm._dptr(u)))
    return rho, u


def cpu_baseline(stencil, space, om, n, steps):
    """The FP64 oracle, single-threaded, on an n^3 copy of the Taylor-Green workload."""
    from threadpoolctl import threadpool_limits
    import oracle as O
    with threadpool_limits(limits=1):
        m = O.Method(stencil, space, om)
        rho, u = W.tgv3d_fields(n, u0=0.05)
        df = O.init_equilibrium(m, rho, u)
        t0 = time.perf_counter()
        O.step(m, df, steps)
        dt = time.perf_counter() - t0
    return {"value": n ** 3 * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": "FP64 numpy oracle (dense K(u), set-partition cumulants), %d^3 copy of the same "
                      "Taylor-Green workload, %d steps, %.1f s" % (n, steps, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="d3q27_cumulant_512")
    ap.add_argument("--size", type=int, default=0, help="override the edge length (smaller boxes)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--layout", default="auto", choices=["auto", "planes", "rows"])
    ap.add_argument("--streaming", default="pull", choices=["pull", "aa"])
    ap.add_argument("--cpu-size", type=int, default=32)
    ap.add_argument("--cpu-steps", type=int, default=40)
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (the sweep would shard "
              "as z-slabs with one halo exchange per step; not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2211_02435_amd import lbm
    import oracle as O  # rates helper for the workload definition and the cpu baseline

    cfg = build_workload(args.workload)
    stencil, space = cfg["stencil"], cfg["space"]
    n = args.size or cfg["dims"][0]
    dims = (n, n, n)
    om = O.regularized_rates(stencil, cfg["omega_shear"])
    q = O.stencil(stencil).q
    rho, u = W.tgv3d_fields(n, u0=cfg["u0"])
    cells = n ** 3
    print("[bench] %s %s %d^3, steps %d, warmup %d" % (stencil, space, n, args.steps, args.warmup),
          file=sys.stderr, flush=True)

    # FP32 (value)
    lat32, wall32, ev32 = run_box(lbm, stencil, space, om, dims, "f32", rho, u, args.steps, args.warmup,
                                  not args.no_autotune, args.streaming, args.layout)
    mlups32 = cells * args.steps / wall32 / 1e6
    bytes32 = 2 * q * 4 * cells
    t_launch32 = ev32 / 1e3 / args.steps
    achieved32 = bytes32 / t_launch32 / 1e9
    launch32 = list(lat32.lbm_get_launch()) + [int(lat32.lbm_get_vectorized())]
    print("[bench] fp32 done: %.0f MLUPS, %.1f GB/s" % (mlups32, achieved32), file=sys.stderr, flush=True)

    result_fp64 = None
    vel_err = None
    if not args.no_fp64:
        lat64, wall64, ev64 = run_box(lbm, stencil, space, om, dims, "f64", rho, u, args.steps, args.warmup,
                                      not args.no_autotune, args.streaming, args.layout)
        t_launch64 = ev64 / 1e3 / args.steps
        result_fp64 = {"mlups": cells * args.steps / wall64 / 1e6,
                       "ms_per_step": wall64 * 1e3 / args.steps,
                       "achieved_GBps": 2 * q * 8 * cells / t_launch64 / 1e9,
                       "frac": 2 * q * 8 * cells / t_launch64 / 1e9 / HBM_PEAK_GBS,
                       "launch": list(lat64.lbm_get_launch()) + [int(lat64.lbm_get_vectorized())]}
        _, u32 = velocity_device(lat32, lbm)
        _, u64 = velocity_device(lat64, lbm)
        vel_err = float(torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64))
        del u32, u64
        lat64.close()
        print("[bench] fp64 done: %.0f MLUPS" % result_fp64["mlups"], file=sys.stderr, flush=True)
    lat32.close()
    torch.cuda.empty_cache()

    # copy-kernel ceiling on 4 GiB
    nbytes = 4 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    ms = lbm.lbm_copy_bandwidth(b, a, nbytes, 20)
    copy_gbs = 2 * nbytes * 20 / (ms / 1e3) / 1e9
    del a, b

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(stencil, space, om, args.cpu_size, args.cpu_steps)

    workload = "%s %s %d^3 periodic Taylor-Green (u0 %.2f, omega_s %.6f, other rates 1), %s" % (
        stencil, space, n, cfg["u0"], cfg["omega_shear"], args.streaming)
    out = {
        "metric": "MLUPS and % of HBM roofline, D3Q27 cumulant 512^3, FP32 vs FP64",
        "value": mlups32,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall32 * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic Taylor-Green vortex initial fields",
        "config": {"workload": workload, "cells": cells, "stencil": stencil, "space": space,
                   "storage": "f32", "streaming": args.streaming,
                   "layout": args.layout if args.layout != "auto" else "planes (auto for f32)",
                   "launch_bx_by_swizzle_vec": launch32},
        "roofline": {"bound": "hbm", "achieved": achieved32, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved32 / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload if n == cfg["dims"][0] else "none", cells),
                     "kernel": "sweep_kernel<D3Q27, CUMULANT, regularized, f32, pull>",
                     "bytes_per_lup": 2 * q * 4,
                     "avg_launch_ms": t_launch32 * 1e3},
        "fp64": result_fp64,
        "fp32_vs_fp64_velocity_rel_l2": vel_err,
        "copy_ceiling_GBps": copy_gbs,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
