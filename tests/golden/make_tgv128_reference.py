"""Writes tests/golden/tgv128_cumulant_oracle.npz: the FP64 oracle's velocity and density at
4096 sampled cells of the 128^3 copy of the D3Q27 cumulant Taylor-Green workload (u0 = 0.05,
the 512^3 rates: omega_s = 1.969902, every other rate 1) after 200 steps.

Only oracle/ and the seeded input generators are used.  The collision is per cell, so each
step collides z-slabs in a process pool (oracle.collide on each slab) and then streams the
whole box (oracle.stream); the result is the same arithmetic as oracle.step.

    python tests/golden/make_tgv128_reference.py [--procs 8]
"""
import argparse
import os
import sys
import time
from multiprocessing import Pool

# one BLAS thread per worker: the pool supplies the parallelism
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lbm_workloads as W  # noqa: E402
import oracle as O  # noqa: E402

N, STEPS, U0 = 128, 200, 0.05
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tgv128_cumulant_oracle.npz")


def method():
    return O.Method("D3Q27", "cumulant", O.regularized_rates("D3Q27", W.re_to_omega(U0, 512, 1600.0)))


def sample_points():
    """16^3 cells off the vortex's symmetry planes: z = 8k + 3, y = 8j + 5, x = 8i + 1."""
    k = np.arange(16)
    return 8 * k + 3, 8 * k + 5, 8 * k + 1


def _collide_slab(slab):
    return O.collide(method(), slab)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    a = ap.parse_args(argv)
    m = method()
    rho, u = W.tgv3d_fields(N, u0=U0)
    df = O.init_equilibrium(m, rho, u)
    del rho, u
    t0 = time.time()
    with Pool(a.procs) as pool:
        for t in range(STEPS):
            slabs = np.array_split(df, a.procs, axis=1)
            df = O.stream(m, np.concatenate(pool.map(_collide_slab, slabs), axis=1))
            if t % 20 == 19:
                print("step %d, %.0f s" % (t + 1, time.time() - t0), flush=True)
    rho, u = O.macroscopic(m, df)
    z, y, x = sample_points()
    zz, yy, xx = np.meshgrid(z, y, x, indexing="ij")
    np.savez_compressed(OUT, u=u[:, zz, yy, xx], rho=rho[zz, yy, xx], z=z, y=y, x=x,
                        u_l2=np.linalg.norm(u), steps=STEPS, n=N, u0=U0)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
