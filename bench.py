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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_{workload}_{storage}.json")
SBYTES = {"f64": 8, "f32": 4, "f16": 2}


def measured_traffic(workload, layout, storage="f32"):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken on the
    current kernel sources (device code, runtime, build flags) and the same storage layout;
    else None."""
    path = TRAFFIC_FILE.format(workload=workload, storage=storage)
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


def apply_launch(lat, spec):
    """Set a launch given as "bx,by,swizzle,variant,lds" (variant 0 per-cell, 1 vectorised,
    2 LDS-staged)."""
    bx, by, swz, var, lds = (int(v) for v in spec.split(","))
    lat.lbm_set_launch(bx, by, swz)
    lat.lbm_set_vectorized(var == 1)
    lat.lbm_set_staged(var == 2)
    lat.lbm_set_lds_reserve(lds)


def measure_box(lbm, cfg, storage, fields, dims, steps, warmup, autotune, streaming, layout, transform="chimera",
                general=False, launch=None):
    """Run one box: init, autotune (or the given launch), warm-up, record the graph, time
    `steps` sweeps."""
    import torch
    stencil, space = cfg["stencil"], cfg["space"]
    om = workload_rates(cfg, general)
    q = lbm.Q[stencil]
    kw = {}
    if cfg.get("equilibrium") == "swe":
        kw = {"equilibrium": "swe", "gravity": cfg["gravity"]}
    lat = lbm.Lattice(stencil, space, om, dims, storage=storage, streaming=streaming, layout=layout, **kw)
    lat.lbm_init_equilibrium(*fields)
    if launch:
        apply_launch(lat, launch)
    elif autotune:
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
           "launch_bx_by_swizzle_variant_lds": list(lat.lbm_get_launch()) + [
               1 if lat.lbm_get_vectorized() else (2 if lat.lbm_get_staged() else 0), lat.lbm_get_lds_reserve()],
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
    res = {"boxes": len(boxes), "cells": cells, "steps": steps, "graph_steps": steps,
           "mlups": cells * steps / wall / 1e6, "ms_per_step": wall * 1e3 / steps,
           "avg_launch_ms": ms / steps, "achieved_GBps": gbs, "frac": gbs / HBM_PEAK_GBS,
           "storage": "f32", "space": "central",
           "launch_threads_swizzle_lds_persistent": list(launch) + [int(bat.lbm_batch_get_persistent())]}
    res["vs_oracle"] = batch_accuracy(lbm, bat, boxes, dims, rho, u)
    return res


def batch_accuracy(lbm, bat, boxes, dims, rho, u):
    """Outside the timed region: the ensemble re-initialised and advanced by one replay of the
    100-step graph; the velocity of its sampled edge-32 boxes against the FP64 oracle's values
    at their sampled cells (tests/golden/ensemble32_oracle.npz, written from the oracle alone)."""
    import torch
    path = os.path.join(ROOT, "tests", "golden", "ensemble32_oracle.npz")
    if not os.path.exists(path):
        return None
    ref = np.load(path)
    steps = int(ref["steps"])
    bat.lbm_batch_init_equilibrium(rho, u)
    bat.lbm_batch_graph_prepare(steps)
    bat.lbm_batch_step(steps)
    n = bat.lbm_batch_cells()
    rg = torch.empty(n, dtype=torch.float64, device="cuda")
    ug = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    lbm.check(lbm.load().lbm_batch_macroscopic(bat.b, lbm._dptr(rg), lbm._dptr(ug)))
    offs = np.concatenate([[0], np.cumsum([d[0] * d[1] * d[2] for d in dims])])
    worst = 0.0
    per_box = {}
    for k in (int(v) for v in ref["boxes"]):
        e = dims[k][0]
        uk = ug[3 * int(offs[k]):3 * int(offs[k + 1])].view(3, e, e, e).cpu().numpy()
        pts = ref["u_pts_%d" % k]
        got = uk[:, pts[:, 2], pts[:, 1], pts[:, 0]].T
        rel = float(np.linalg.norm(got - ref["u_%d" % k]) / np.linalg.norm(ref["u_%d" % k]))
        per_box[str(k)] = rel
        worst = max(worst, rel)
    del rg, ug
    torch.cuda.empty_cache()
    return {"velocity_rel_l2_vs_oracle_max": worst, "per_box": per_box, "steps": steps,
            "sample": "edge-32 boxes %s of the ensemble, %d sampled cells each, after one replay of the "
                      "%d-step graph" % (list(per_box), len(ref["u_pts_%d" % int(ref["boxes"][0])]), steps)}


def oracle_accuracy(lbm, cfg):
    """Outside the timed region: the 128^3 copy of the metric workload (same u0 and rates) in
    FP32 and FP64 against the FP64 oracle's values at sampled cells
    (tests/golden/tgv128_cumulant_oracle.npz, written from the oracle alone): max |d df| after
    100 steps and the relative L2 velocity error after 200 steps."""
    path = os.path.join(ROOT, "tests", "golden", "tgv128_cumulant_oracle.npz")
    if not os.path.exists(path):
        return None
    ref = np.load(path)
    n, u0, k1, k2 = int(ref["n"]), float(ref["u0"]), int(ref["df_step"]), int(ref["steps"])
    fields = W.tgv3d_fields(n, u0=u0)
    pts = ref["df_pts"]
    zz, yy, xx = np.meshgrid(ref["z"], ref["y"], ref["x"], indexing="ij")
    out = {"copy": "%d^3, u0 %.2f, omega_s %.6f" % (n, u0, cfg["omega_shear"]),
           "df_step": k1, "velocity_step": k2, "df_cells": len(pts), "velocity_cells": int(zz.size)}
    for st in ("f32", "f64"):
        lat = lbm.Lattice(cfg["stencil"], cfg["space"], workload_rates(cfg), (n, n, n), storage=st)
        lat.lbm_init_equilibrium(*fields)
        lat.lbm_autotune()
        lat.lbm_step(k1)
        df = lat.lbm_get_populations()
        err = float(np.abs(df[:, pts[:, 2], pts[:, 1], pts[:, 0]].T - ref["df"]).max())
        del df
        lat.lbm_step(k2 - k1)
        _, ug = lat.lbm_macroscopic()
        lat.close()
        us = ug[:, zz, yy, xx]
        out[st] = {"max_abs_df_vs_oracle": err,
                   "velocity_rel_l2_vs_oracle": float(np.linalg.norm(us - ref["u"]) / np.linalg.norm(ref["u"]))}
    return out


def swe_instance_accuracy(lbm, cfg, storages, name="swe1024"):
    """Outside the timed region: an n x n instance of the shallow-water workload (same
    generator, rates and gravity) over the workload's 1000 steps in every storage of the line,
    against the FP64 oracle's values at sampled cells (tests/golden/<name>_oracle.npz, written
    from the oracle alone): max |d df| after 100 steps, the relative L2 error of the in-plane
    velocity and max |d h| after 1000 steps."""
    path = os.path.join(ROOT, "tests", "golden", name + "_oracle.npz")
    if not os.path.exists(path):
        return None
    ref = np.load(path)
    n, k1, k2 = int(ref["n"]), int(ref["df_step"]), int(ref["steps"])
    h, u = W.swe_bumps(n, seed=0)
    pts, upts = ref["df_pts"], ref["u_pts"]
    sel = (upts[:, 2], upts[:, 1], upts[:, 0])
    out = {"instance": "%d^2, 16 bumps, seed 0" % n, "df_step": k1, "velocity_step": k2,
           "df_cells": int(len(pts)), "velocity_cells": int(len(upts))}
    for st in storages:
        lat = lbm.Lattice(cfg["stencil"], cfg["space"], workload_rates(cfg), (n, n, 1), storage=st,
                          equilibrium="swe", gravity=cfg["gravity"])
        lat.lbm_init_equilibrium(h, u)
        lat.lbm_autotune()
        lat.lbm_step(k1)
        df = lat.lbm_get_populations()
        err = float(np.abs(df[:, pts[:, 2], pts[:, 1], pts[:, 0]].T - ref["df"]).max())
        del df
        lat.lbm_step(k2 - k1)
        hg, ug = lat.lbm_macroscopic()
        lat.close()
        want = ref["u"][:, :2]
        got = ug[(slice(0, 2),) + sel].T
        out[st] = {"max_abs_df_vs_oracle": err,
                   "velocity_rel_l2_vs_oracle": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
                   "max_abs_dh_vs_oracle": float(np.abs(hg[sel] - ref["h"]).max())}
    return out


FULL_SIZE_REFERENCES = {"d3q19_raw_256": "d3q19_raw256", "swe_d2q9_4096": "swe4096"}


def full_size_accuracy(lbm, name, cfg, storages, fields, dims):
    """Outside the timed region: the workload at its full size, run for as many steps as the
    FP64 oracle's reference (tests/golden/<ref>_oracle.npz, written from the oracle alone) in
    every storage of the line, compared at the reference's sampled cells: max |d df| and the
    relative L2 error of the velocity (in-plane for the 2-D workload)."""
    import torch
    ref_name = FULL_SIZE_REFERENCES.get(name)
    path = ref_name and os.path.join(ROOT, "tests", "golden", ref_name + "_oracle.npz")
    if not path or not os.path.exists(path):
        return None
    ref = np.load(path)
    if tuple(int(v) for v in ref["dims"]) != tuple(dims):
        return None
    steps = int(ref["steps"])
    nx, ny, nz = dims
    n = nx * ny * nz
    d = 2 if cfg["stencil"] == "D2Q9" else 3
    kw = {"equilibrium": "swe", "gravity": cfg["gravity"]} if cfg.get("equilibrium") == "swe" else {}
    out = {"steps": steps, "df_cells": int(len(ref["df_pts"])), "velocity_cells": int(len(ref["u_pts"]))}

    def cells(pts):
        return torch.as_tensor((pts[:, 2] * ny + pts[:, 1]) * nx + pts[:, 0], device="cuda")

    for st in storages:
        lat = lbm.Lattice(cfg["stencil"], cfg["space"], workload_rates(cfg), dims, storage=st, **kw)
        lat.lbm_init_equilibrium(*fields)
        lat.lbm_autotune()
        lat.lbm_step(steps)
        q = lat.q
        dev = torch.empty(q * n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        lbm.check(lat.lib.lbm_get_populations(lat.ctx, lbm._dptr(dev)))
        c = cells(ref["df_pts"])
        df = dev[torch.arange(q, device="cuda")[None, :] * n + c[:, None]].cpu().numpy()
        del dev
        r = torch.empty(n, dtype=torch.float64, device="cuda")
        u = torch.empty(3 * n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        lbm.check(lat.lib.lbm_macroscopic(lat.ctx, lbm._dptr(r), lbm._dptr(u)))
        c = cells(ref["u_pts"])
        uc = u[torch.arange(d, device="cuda")[None, :] * n + c[:, None]].cpu().numpy()
        del r, u
        lat.close()
        torch.cuda.empty_cache()
        want = ref["u"][:, :d]
        out[st] = {"max_abs_df_vs_oracle": float(np.abs(df - ref["df"]).max()),
                   "velocity_rel_l2_vs_oracle": float(np.linalg.norm(uc - want) / np.linalg.norm(want))}
    return out


_ORACLE_METHODS = {}


def _oracle_method(spec):
    import oracle as O
    if spec not in _ORACLE_METHODS:
        stencil, space, omega = spec
        _ORACLE_METHODS[spec] = O.Method(stencil, space, O.regularized_rates(stencil, omega))
    return _ORACLE_METHODS[spec]


def _oracle_collide_slab(args):
    import oracle as O
    spec, slab = args
    return O.collide(_oracle_method(spec), slab)


def _oracle_init_slab(args):
    import oracle as O
    spec, rho, u = args
    return O.init_equilibrium(_oracle_method(spec), rho, u)


def _oracle_rate(spec, fields, steps, procs):
    """Oracle MLUPS of `steps` steps from the equilibrium of `fields`: collide on `procs` slabs in
    a process pool (procs > 1) or in this process, then stream; init is not timed."""
    import oracle as O
    m = _oracle_method(spec)
    rho, u = fields
    cells = rho.size
    if procs == 1:
        df = O.init_equilibrium(m, rho, u)
        t0 = time.perf_counter()
        O.step(m, df, steps)
        return cells * steps / (time.perf_counter() - t0) / 1e6
    from multiprocessing import get_context
    with get_context("fork").Pool(procs) as pool:
        axis = 0 if rho.shape[0] > 1 else 1  # z-slabs (y-slabs of a 2-D box)
        parts = zip(np.array_split(rho, procs, axis=axis), np.array_split(u, procs, axis=axis + 1))
        df = np.concatenate(pool.map(_oracle_init_slab, [(spec, r, v) for r, v in parts]), axis=axis + 1)
        axis = 1 if df.shape[1] > 1 else 2
        t0 = time.perf_counter()
        for _ in range(steps):
            slabs = np.array_split(df, procs, axis=axis)
            df = O.stream(m, np.concatenate(pool.map(_oracle_collide_slab, [(spec, s) for s in slabs]), axis=axis))
        dt = time.perf_counter() - t0
    return cells * steps / dt / 1e6


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, n_all=128, steps_all=2, n_one=64, steps_one=2, d2q9_steps=250):
    """The FP64 oracle on the host cores, before the GPU is touched (its process pool forks):
    the D3Q27 cumulant Taylor-Green workload on a 128^3 copy with every usable core (one worker
    process per core, at most 16) and on a 64^3 copy with one core, and the D2Q9 central-moment
    64^2 Taylor-Green run (the small workload) with one core.  One BLAS thread per process."""
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    from threadpoolctl import threadpool_limits
    cores = min(16, len(os.sched_getaffinity(0)))
    spec = (cfg["stencil"], cfg["space"], cfg["omega_shear"])
    c2 = W.WORKLOADS["d2q9_central_64"]
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        all_cores = _oracle_rate(spec, W.tgv3d_fields(n_all, u0=cfg["u0"]), steps_all, cores)
        one_core = _oracle_rate(spec, W.tgv3d_fields(n_one, u0=cfg["u0"]), steps_one, 1)
        d2q9 = _oracle_rate((c2["stencil"], c2["space"], c2["omega_shear"]),
                            W.tgv2d_fields(64, 64, 1, u0=c2["u0"]), d2q9_steps, 1)
    wall = time.perf_counter() - t0
    return {"value": all_cores, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": "FP64 numpy oracle (dense K(u), set-partition cumulants) on the D3Q27 cumulant "
                      "Taylor-Green workload: %d^3 copy, %d steps, %d worker processes; %.1f s for all "
                      "three legs" % (n_all, steps_all, cores, wall),
            "single_core": {"value": one_core, "unit": "MLUPS", "cores": 1,
                            "sample": "%d^3 copy, %d steps" % (n_one, steps_one)},
            "d2q9_central_64": {"value": d2q9, "unit": "MLUPS", "cores": 1,
                                "sample": "D2Q9 central-moment 64^2 Taylor-Green (u0 0.01, omega_s 1.6), "
                                          "%d of its 1000 steps" % d2q9_steps},
            "nproc": os.cpu_count(), "usable_cores": len(os.sched_getaffinity(0)), "cpu_model": _cpu_model()}


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
    ap.add_argument("--launch", default=None,
                    help="bx,by,swizzle,variant,lds for every storage instead of autotuning (variant 0 "
                         "per-cell, 1 vectorised, 2 LDS-staged)")
    ap.add_argument("--fp64-launch", default=None, help="the same for the FP64 run (default: --launch)")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the checks against the oracle's reference values (outside the timed region)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (a box would shard "
              "as z-slabs with one halo exchange per step; not built).", file=sys.stderr)
        sys.exit(2)

    name = args.workload
    cfg = W.WORKLOADS[name]
    n = args.size or cfg.get("dims", (0,))[0]
    is_metric = name == "d3q27_cumulant_512" and n == cfg["dims"][0]
    cpu = None
    if is_metric and not args.no_cpu:
        # before the GPU is touched: the oracle's worker processes are forked
        print("[bench] cpu baseline (FP64 oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfg)

    import torch
    from paper_2211_02435_amd import lbm

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

    fields, dims = workload_fields(name, cfg, n)
    full_accuracy = swe_accuracy = None
    storages = {"swe_d2q9_4096": ["f16", "f64"], "d2q9_central_64": ["f64"]}.get(name, ["f32", "f64"])
    if args.no_fp64:
        storages = [s for s in storages if s != "f64"] or storages[:1]
    print("[bench] %s %s dims %s, steps %d, warmup %d" % (name, storages, dims, args.steps, args.warmup),
          file=sys.stderr, flush=True)
    runs, lats = {}, {}
    for st in storages:
        launch = (args.fp64_launch or args.launch) if st == "f64" else args.launch
        lat, res = measure_box(lbm, cfg, st, fields, dims, args.steps, args.warmup,
                               not args.no_autotune, args.streaming, args.layout, args.transform,
                               args.rates == "general", launch)
        runs[st], lats[st] = res, lat
        print("[bench] %s: %.0f MLUPS, %.1f GB/s" % (st, res["mlups"], res["achieved_GBps"]),
              file=sys.stderr, flush=True)
    if not args.no_accuracy and name in FULL_SIZE_REFERENCES and args.streaming == "pull" \
            and args.transform == "chimera" and args.rates == "regularized":
        full_accuracy = full_size_accuracy(lbm, name, cfg, storages, fields, dims)
        print("[bench] accuracy vs oracle: %s" % json.dumps(full_accuracy), file=sys.stderr, flush=True)
        if name == "swe_d2q9_4096":
            swe_accuracy = swe_instance_accuracy(lbm, cfg, storages)
            print("[bench] accuracy vs oracle, 1000 steps: %s" % json.dumps(swe_accuracy), file=sys.stderr,
                  flush=True)
    del fields
    main_st = storages[0]
    vel = None
    if "f64" in lats and main_st != "f64":
        vel = velocity_rel_diff(lbm, lats[main_st], lats["f64"])
    for lat in lats.values():
        lat.close()
    lats.clear()
    torch.cuda.empty_cache()

    batch = None
    if is_metric and not args.no_batch:
        batch = measure_batch(lbm, 100, args.warmup)
        print("[bench] batch: %.0f MLUPS" % batch["mlups"], file=sys.stderr, flush=True)
    ceiling = copy_ceiling(lbm)
    accuracy = None
    if is_metric and not args.no_accuracy:
        accuracy = oracle_accuracy(lbm, cfg)
        print("[bench] accuracy vs oracle: %s" % json.dumps(accuracy), file=sys.stderr, flush=True)

    r = runs[main_st]
    cells = int(np.prod(dims))
    plain = (n == cfg["dims"][0] and args.streaming == "pull" and args.transform == "chimera"
             and args.rates == "regularized" and not args.launch)
    if "f64" in runs and main_st != "f64":
        runs["f64"]["traffic"] = measured_traffic(name, runs["f64"].get("layout"), "f64") if plain else None
        runs["f64"]["traffic_bytes_per_lup"] = runs["f64"]["traffic"] / cells if runs["f64"]["traffic"] else None
    traffic = measured_traffic(name, r.get("layout"), main_st) if plain else None
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
        "config": {"workload": workload, "cells": cells, "storage": main_st,
                   "layout": r.get("layout", args.layout), "streaming": args.streaming, "transform": args.transform,
                   "rates": args.rates,
                   "launch_bx_by_swizzle_variant_lds": r["launch_bx_by_swizzle_variant_lds"]},
        "roofline": {"bound": "hbm", "achieved": r["achieved_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r["frac"],
                     "traffic": traffic,
                     "traffic_bytes_per_lup": traffic / cells if traffic else None,
                     "kernel": "sweep_kernel<%s, %s, %s, %s, %s>" % (cfg["stencil"], cfg["space"], args.rates,
                                                                     main_st, args.streaming),
                     "bytes_per_lup": r["bytes_per_lup"], "avg_launch_ms": r["avg_launch_ms"]},
        "fp64": runs.get("f64") if main_st != "f64" else None,
        "velocity_rel_l2_vs_fp64": vel,
        "vs_oracle_128_copy": accuracy,
        "vs_oracle_full_size": full_accuracy,
        "vs_oracle_1024_instance_1000_steps": swe_accuracy,
        "batched": batch,
        "copy_ceiling_GBps": ceiling,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
