"""Writes the FP64 oracle references of the reduced copies of the benchmark workloads.

Only oracle/ and the seeded input generators (lbm_workloads) are used.  The collision is per
cell, so each step collides slabs of the box in a process pool (oracle.collide on each slab)
and then streams the whole box (oracle.stream): the same arithmetic as oracle.step.

Targets (each writes tests/golden/<name>_oracle.npz):

  tgv128_cumulant   D3Q27 cumulant, 128^3 copy of the 512^3 Taylor-Green workload (u0 = 0.05,
                    omega_s = 1.969902 from Re = 1600 at 512^3, every other rate 1), 200 steps:
                    velocity and density at a 16^3 grid of cells after 200 steps, df at 1024
                    sampled cells after 100 steps
  d3q19_raw64       D3Q19 raw moments, delta-equilibrium, 64^3 copy of the 256^3 Taylor-Green
                    workload (u0 = 0.02, omega_s = 1.993907 from Re = 1600 at 256^3), 500 steps:
                    df at 1024 sampled cells after 100 steps, velocity and density at 4096
                    sampled cells after 500 steps
  ensemble32        D3Q27 central moments: four edge-32 boxes of the seed-0 ensemble of 256
                    boxes (those with the smallest omega_s, the one a quarter and the one half
                    way up the sorted omega_s of the edge-32 boxes, and the largest), each with
                    its own u0, phase and omega_s, 100 steps: df at 256 sampled cells and the
                    velocity at 2048 sampled cells after 100 steps
  swe512            D2Q9 shallow water (Zhou's equilibrium, central moments, g = 0.1,
                    omega_s = 0.695652), a 512^2 instance of the 16-bump workload (same
                    generator, amplitude and bump widths, seed 0), 1000 steps: df at 1024
                    sampled cells after 100 steps, velocity and height at 4096 sampled cells
                    after 1000 steps
  swe4096           the shallow-water workload at its full size, 4096^2, 100 steps: df at 1024
                    sampled cells, velocity and height at 4096 sampled cells
  d3q19_raw256      the D3Q19 raw-moment workload at its full size, 256^3, 100 steps: df at
                    1024 sampled cells, velocity and density at 4096 sampled cells
  swe1024           a 1024^2 instance of the shallow-water workload (as swe512), over the
                    workload's full length of 1000 steps: df at 1024 sampled cells after 100
                    steps, velocity and height at 4096 sampled cells after 1000 steps

    python tests/golden/make_oracle_references.py [--procs 8] [target ...]
"""
import argparse
import os
import sys
import time
from functools import lru_cache
from multiprocessing import Pool

# one BLAS thread per worker: the pool supplies the parallelism
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import lbm_workloads as W  # noqa: E402
import oracle as O  # noqa: E402


def ensemble32_boxes():
    """Indices of the four edge-32 boxes of the seed-0 ensemble used as sampled boxes."""
    boxes = W.batch_ensemble(256, seed=0)
    e32 = sorted((b["omega_shear"], k) for k, b in enumerate(boxes) if b["edge"] == 32)
    n = len(e32)
    return [e32[j][1] for j in (0, n // 4, n // 2, n - 1)]


# method specifications (picklable keys for the pool workers)
def _spec(key):
    kind, arg = key
    if kind == "tgv128_cumulant":
        return ("D3Q27", "cumulant", O.regularized_rates("D3Q27", W.re_to_omega(0.05, 512, 1600.0)), {})
    if kind == "d3q19_raw64":  # the D3Q19 method of every D3Q19 target (the 256^3 rates)
        return ("D3Q19", "raw", O.regularized_rates("D3Q19", W.re_to_omega(0.02, 256, 1600.0)), {})
    if kind == "ensemble32":
        b = W.batch_ensemble(256, seed=0)[arg]
        return ("D3Q27", "central", O.regularized_rates("D3Q27", b["omega_shear"]), {})
    if kind == "swe512":  # the shallow-water method of every shallow-water target
        cfg = W.WORKLOADS["swe_d2q9_4096"]
        return ("D2Q9", "central", O.regularized_rates("D2Q9", cfg["omega_shear"]),
                {"equilibrium": "swe", "gravity": cfg["gravity"]})
    raise KeyError(kind)


@lru_cache(maxsize=None)
def method(key):
    st, sp, om, kw = _spec(key)
    return O.Method(st, sp, om, **kw)


def _collide_slab(args):
    key, slab = args
    return O.collide(method(key), slab)


def run(pool, procs, key, df, steps, snapshots, label):
    """Advance df by `steps` oracle steps, calling snapshots[t](df) after step t."""
    m = method(key)
    axis = 1 if df.shape[1] > 1 else 2  # split along z, or along y for a 2-D box
    t0 = time.time()
    for t in range(1, steps + 1):
        slabs = np.array_split(df, procs, axis=axis)
        df = O.stream(m, np.concatenate(pool.map(_collide_slab, [(key, s) for s in slabs]), axis=axis))
        if t in snapshots:
            snapshots[t](df)
        if t % 50 == 0 or t == steps:
            print("%s: step %d, %.0f s" % (label, t, time.time() - t0), flush=True)
    return df


def _cells_df(df, pts):
    return df[:, pts[:, 2], pts[:, 1], pts[:, 0]].T  # (m, q)


def make_tgv128(pool, procs):
    n, steps, u0 = 128, 200, 0.05
    key = ("tgv128_cumulant", None)
    m = method(key)
    rho, u = W.tgv3d_fields(n, u0=u0)
    df = O.init_equilibrium(m, rho, u)
    del rho, u
    pts_df = W.sample_cells((n, n, n), 1024, seed=11)
    snap = {}
    df = run(pool, procs, key, df, steps, {100: lambda d: snap.__setitem__("df100", _cells_df(d, pts_df))},
             "tgv128")
    rho, u = O.macroscopic(m, df)
    k = np.arange(16)  # 16^3 cells off the vortex's symmetry planes
    z, y, x = 8 * k + 3, 8 * k + 5, 8 * k + 1
    zz, yy, xx = np.meshgrid(z, y, x, indexing="ij")
    np.savez_compressed(os.path.join(HERE, "tgv128_cumulant_oracle.npz"), u=u[:, zz, yy, xx],
                        rho=rho[zz, yy, xx], z=z, y=y, x=x, u_l2=np.linalg.norm(u), steps=steps, n=n, u0=u0,
                        df_step=100, df_pts=pts_df, df=snap["df100"])


def make_d3q19(pool, procs):
    n, steps, u0 = 64, 500, 0.02
    key = ("d3q19_raw64", None)
    m = method(key)
    rho, u = W.tgv3d_fields(n, u0=u0)
    df = O.init_equilibrium(m, rho, u)
    pts_df = W.sample_cells((n, n, n), 1024, seed=12)
    pts_u = W.sample_cells((n, n, n), 4096, seed=13)
    snap = {}
    df = run(pool, procs, key, df, steps, {100: lambda d: snap.__setitem__("df100", _cells_df(d, pts_df))},
             "d3q19_raw64")
    rho, u = O.macroscopic(m, df)
    sel = (pts_u[:, 2], pts_u[:, 1], pts_u[:, 0])
    np.savez_compressed(os.path.join(HERE, "d3q19_raw64_oracle.npz"), n=n, steps=steps, u0=u0,
                        omega_shear=W.re_to_omega(u0, 256, 1600.0), df_step=100, df_pts=pts_df,
                        df=snap["df100"], u_pts=pts_u, u=u[(slice(None),) + sel].T, rho=rho[sel])


def make_ensemble32(pool, procs):
    steps = 100
    boxes = W.batch_ensemble(256, seed=0)
    out = {"steps": steps, "boxes": np.array(ensemble32_boxes())}
    for k in ensemble32_boxes():
        b = boxes[k]
        key = ("ensemble32", k)
        m = method(key)
        rho, u = W.batch_fields(b)
        df = O.init_equilibrium(m, rho, u)
        n = b["edge"]
        pts_df = W.sample_cells((n, n, n), 256, seed=100 + k)
        pts_u = W.sample_cells((n, n, n), 2048, seed=200 + k)
        df = run(pool, procs, key, df, steps, {}, "ensemble box %d" % k)
        rho, u = O.macroscopic(m, df)
        sel = (pts_u[:, 2], pts_u[:, 1], pts_u[:, 0])
        out.update({"df_pts_%d" % k: pts_df, "df_%d" % k: _cells_df(df, pts_df),
                    "u_pts_%d" % k: pts_u, "u_%d" % k: u[(slice(None),) + sel].T})
    np.savez_compressed(os.path.join(HERE, "ensemble32_oracle.npz"), **out)


def _swe_instance(pool, procs, n, seeds):
    """An n x n instance of the shallow-water workload over its 1000 steps."""
    steps = 1000
    key = ("swe512", None)
    m = method(key)
    h, u = W.swe_bumps(n, seed=0)
    df = O.init_equilibrium(m, h, u)
    pts_df = W.sample_cells((n, n, 1), 1024, seed=seeds[0])
    pts_u = W.sample_cells((n, n, 1), 4096, seed=seeds[1])
    snap = {}
    df = run(pool, procs, key, df, steps, {100: lambda d: snap.__setitem__("df100", _cells_df(d, pts_df))},
             "swe%d" % n)
    h, u = O.macroscopic(m, df)
    sel = (pts_u[:, 2], pts_u[:, 1], pts_u[:, 0])
    np.savez_compressed(os.path.join(HERE, "swe%d_oracle.npz" % n), n=n, steps=steps, df_step=100,
                        df_pts=pts_df, df=snap["df100"], u_pts=pts_u, u=u[(slice(None),) + sel].T, h=h[sel])


def make_swe512(pool, procs):
    _swe_instance(pool, procs, 512, (14, 15))


def make_swe1024(pool, procs):
    _swe_instance(pool, procs, 1024, (18, 19))


def _full_size(pool, procs, name, key, fields, dims, steps):
    """df at 1024 and the macroscopic fields at 4096 sampled cells of a full-size workload."""
    m = method(key)
    df = O.init_equilibrium(m, *fields)
    del fields
    pts_df = W.sample_cells(dims, 1024, seed=16)
    pts_u = W.sample_cells(dims, 4096, seed=17)
    df = run(pool, procs, key, df, steps, {}, name)
    sel = (pts_u[:, 2], pts_u[:, 1], pts_u[:, 0])
    r, u = O.macroscopic(m, df)
    np.savez_compressed(os.path.join(HERE, name + "_oracle.npz"), dims=np.array(dims), steps=steps,
                        df_pts=pts_df, df=_cells_df(df, pts_df), u_pts=pts_u, u=u[(slice(None),) + sel].T,
                        rho=r[sel])


def make_swe4096(pool, procs):
    n = 4096
    _full_size(pool, procs, "swe4096", ("swe512", None), W.swe_bumps(n, seed=0), (n, n, 1), 100)


def make_d3q19_256(pool, procs):
    n, u0 = 256, 0.02
    _full_size(pool, procs, "d3q19_raw256", ("d3q19_raw64", None), W.tgv3d_fields(n, u0=u0), (n, n, n), 100)


TARGETS = {"tgv128_cumulant": make_tgv128, "d3q19_raw64": make_d3q19, "ensemble32": make_ensemble32,
           "swe512": make_swe512, "swe4096": make_swe4096, "d3q19_raw256": make_d3q19_256,
           "swe1024": make_swe1024}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    ap.add_argument("targets", nargs="*", default=sorted(TARGETS))
    a = ap.parse_args(argv)
    with Pool(a.procs) as pool:
        for t in a.targets:
            t0 = time.time()
            TARGETS[t](pool, a.procs)
            print("wrote %s (%.0f s)" % (t, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
