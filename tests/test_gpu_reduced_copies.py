"""Reduced copies of the benchmark workloads against the FP64 oracle over many steps.

Each copy keeps its workload's velocity amplitude and relaxation rates (so the kernel
constants are those of the full-size run) and runs in the autotuned launch.  The references
are the oracle's own outputs at sampled cells, written by tests/golden/make_oracle_references.py
from oracle/ and the seeded input generators alone.

Bars (the Taylor-Green configuration of sec. 5.1 and the shallow-water case of sec. 5.2):
  FP64 storage: max |df_gpu - df_oracle| <= 1e-12 after 100 steps;
  FP32 storage: relative L2 velocity error <= 1e-5 at the end of the run;
  FP16 storage (shallow water): the velocity error at step 1000 is stated and bounded.
Relative L2 errors are taken over the sampled cells.  The D3Q19 and shallow-water workloads
are also checked at their full sizes (256^3, 4096^2) for 100 steps.
"""
import os

import numpy as np
import pytest

import lbm_workloads as W
from paper_2211_02435_amd import lbm

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _ref(name):
    path = os.path.join(GOLDEN, name + "_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("oracle reference %s not generated (tests/golden/make_oracle_references.py %s)" % (path, name))
    return np.load(path)


def _df_at(df, pts):
    return df[:, pts[:, 2], pts[:, 1], pts[:, 0]].T


def _u_at(u, pts):
    return u[:, pts[:, 2], pts[:, 1], pts[:, 0]].T


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ------------------------------------------------------------------------------------------
# D3Q19 raw moments, 64^3 copy of the 256^3 Taylor-Green workload (u0 = 0.02, omega_s from
# Re = 1600 at 256^3), 500 steps
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_d3q19_raw_64_copy_against_oracle(storage):
    ref = _ref("d3q19_raw64")
    n, steps, u0 = int(ref["n"]), int(ref["steps"]), float(ref["u0"])
    cfg = W.WORKLOADS["d3q19_raw_256"]
    assert abs(float(ref["omega_shear"]) - cfg["omega_shear"]) < 1e-15
    om = lbm.regularized_rates("D3Q19", cfg["omega_shear"])
    rho, u = W.tgv3d_fields(n, u0=u0)
    lat = lbm.Lattice("D3Q19", "raw", om, (n, n, n), storage=storage)
    lat.lbm_init_equilibrium(rho, u)
    lat.lbm_autotune()
    lat.lbm_step(int(ref["df_step"]))
    err_df = float(np.abs(_df_at(lat.lbm_get_populations(), ref["df_pts"]) - ref["df"]).max())
    lat.lbm_step(steps - int(ref["df_step"]))
    rg, ug = lat.lbm_macroscopic()
    pts = ref["u_pts"]
    rel = _rel(_u_at(ug, pts), ref["u"])
    drho = float(np.abs(rg[pts[:, 2], pts[:, 1], pts[:, 0]] - ref["rho"]).max())
    print("D3Q19 raw 64^3 %s: max|d df| at step 100 = %.3e; step %d: relative L2 velocity error %.3e, "
          "max|d rho| %.3e" % (storage, err_df, steps, rel, drho))
    if storage == "f64":
        assert err_df <= 1e-12
        assert rel <= 1e-10
        assert drho <= 1e-12
    elif storage == "f32":
        assert rel <= 1e-5
        assert drho <= 1e-6
    else:
        assert rel <= F16_VELOCITY_BAR


# FP16 storage in 3-D (an extension of the precision layer beyond the shallow-water case):
# binary16 keeps 11 significant bits, so every stored deviation carries a relative rounding error
# of up to 2^-11 = 4.9e-4 each step.  The velocity is a sum of such deviations divided by rho;
# its error stays of the order of that unit roundoff relative to u0, times the growth over the
# run's few hundred steps.  Bar: 1e-2 relative L2; measured 6.4e-4 (D3Q27 cumulant 128^3,
# 200 steps), 1.0e-3 (D3Q19 raw 64^3, 500 steps) and at most 2.4e-4 (ensemble boxes, 100 steps).
F16_VELOCITY_BAR = 1e-2


def test_tgv128_fp16_storage_against_oracle():
    """The 128^3 copy of the metric workload with FP16 population storage (FP32 compute), 200
    steps, against the oracle's velocity at its 16^3 sampled cells."""
    ref = _ref("tgv128_cumulant")
    n, u0, steps = int(ref["n"]), float(ref["u0"]), int(ref["steps"])
    om = lbm.regularized_rates("D3Q27", W.re_to_omega(u0, 512, 1600.0))
    rho, u = W.tgv3d_fields(n, u0=u0)
    lat = lbm.Lattice("D3Q27", "cumulant", om, (n, n, n), storage="f16")
    lat.lbm_init_equilibrium(rho, u)
    lat.lbm_autotune()
    lat.lbm_step(int(ref["df_step"]))
    err_df = float(np.abs(_df_at(lat.lbm_get_populations(), ref["df_pts"]) - ref["df"]).max())
    lat.lbm_step(steps - int(ref["df_step"]))
    rg, ug = lat.lbm_macroscopic()
    lat.close()
    zz, yy, xx = np.meshgrid(ref["z"], ref["y"], ref["x"], indexing="ij")
    rel = _rel(ug[:, zz, yy, xx], ref["u"])
    drho = float(np.abs(rg[zz, yy, xx] - ref["rho"]).max())
    print("TGV 128^3 f16: max|d df| at step %d = %.3e; step %d: relative L2 velocity error %.3e, "
          "max|d rho| %.3e" % (int(ref["df_step"]), err_df, steps, rel, drho))
    assert rel <= F16_VELOCITY_BAR


# ------------------------------------------------------------------------------------------
# Ensemble: four edge-32 boxes of the seed-0 ensemble (their own u0, phase and omega_s) in a
# batch with four boxes of other edges, 100 steps replayed from one recorded graph
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("storage", ["f32", "f64", "f16"])
def test_ensemble_boxes_graph_against_oracle(storage):
    ref = _ref("ensemble32")
    steps = int(ref["steps"])
    boxes = W.batch_ensemble(256, seed=0)
    sampled = [int(k) for k in ref["boxes"]]
    members = [0, 1, 3, 4] + sampled          # edges 96, 64, 48, 48 and the four of edge 32
    dims = [(boxes[k]["edge"],) * 3 for k in members]
    rates = [lbm.regularized_rates("D3Q27", boxes[k]["omega_shear"]) for k in members]
    fields = [W.batch_fields(boxes[k]) for k in members]
    rho_cat = np.concatenate([f[0].ravel() for f in fields])
    u_cat = np.concatenate([f[1].ravel() for f in fields])
    bat = lbm.Batch("D3Q27", "central", dims, rates, storage=storage)
    bat.lbm_batch_init_equilibrium(rho_cat, u_cat)
    print("batch launch", bat.lbm_batch_autotune())
    bat.lbm_batch_graph_prepare(steps)
    bat.lbm_batch_step(steps)
    _, u_all = bat.lbm_batch_macroscopic()
    off = 0
    worst_rel, worst_df = 0.0, 0.0
    for j, k in enumerate(members):
        nc = int(np.prod(dims[j]))
        if k in sampled:
            e = dims[j][0]
            u = u_all[3 * off:3 * (off + nc)].reshape(3, e, e, e)
            rel = _rel(_u_at(u, ref["u_pts_%d" % k]), ref["u_%d" % k])
            df = bat.lbm_batch_get_box_populations(j)
            err = float(np.abs(_df_at(df, ref["df_pts_%d" % k]) - ref["df_%d" % k]).max())
            print("box %d (omega_s %.6f, u0 %.4f) %s: relative L2 velocity error %.3e, max|d df| %.3e"
                  % (k, boxes[k]["omega_shear"], boxes[k]["u0"], storage, rel, err))
            worst_rel, worst_df = max(worst_rel, rel), max(worst_df, err)
        off += nc
    if storage == "f64":
        assert worst_df <= 1e-12
        assert worst_rel <= 1e-10
    elif storage == "f32":
        assert worst_rel <= 1e-5
    else:
        assert worst_rel <= F16_VELOCITY_BAR


# ------------------------------------------------------------------------------------------
# Shallow water: 512^2 and 1024^2 instances of the 16-bump workload, 1000 steps
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["swe512", "swe1024"])
def test_swe_instance_against_oracle(name):
    ref = _ref(name)
    n, steps, k100 = int(ref["n"]), int(ref["steps"]), int(ref["df_step"])
    cfg = W.WORKLOADS["swe_d2q9_4096"]
    om = lbm.regularized_rates("D2Q9", cfg["omega_shear"])
    h, u = W.swe_bumps(n, seed=0)
    pts = ref["u_pts"]
    out = {}
    for storage in ("f64", "f16"):
        lat = lbm.Lattice("D2Q9", "central", om, (n, n, 1), storage=storage, equilibrium="swe",
                          gravity=cfg["gravity"])
        lat.lbm_init_equilibrium(h, u)
        lat.lbm_autotune()
        lat.lbm_step(k100)
        err_df = float(np.abs(_df_at(lat.lbm_get_populations(), ref["df_pts"]) - ref["df"]).max())
        lat.lbm_step(steps - k100)
        hg, ug = lat.lbm_macroscopic()
        lat.close()
        rel = _rel(_u_at(ug[:2], pts), ref["u"][:, :2])
        dh = float(np.abs(hg[pts[:, 2], pts[:, 1], pts[:, 0]] - ref["h"]).max())
        out[storage] = (err_df, rel, dh)
        print("SWE %d^2 %s: max|d df| at step %d = %.3e; step %d: relative L2 velocity error %.3e, "
              "max|d h| %.3e" % (n, storage, k100, err_df, steps, rel, dh))
    assert out["f64"][0] <= 1e-12
    assert out["f64"][1] <= 1e-10
    assert out["f64"][2] <= 1e-12
    # FP16 storage of the zero-centred populations (11-bit significand; the rest population's
    # deviation reaches 0.08 where the bumps stand, an FP16 spacing of 6e-5): after 1000 steps the
    # velocity field is within a few percent of the oracle's (measured relative L2 3.3e-2 at 512^2
    # and 2.8e-2 at 1024^2, with max |d h| = 1.1e-2 and 5.5e-3 over the sampled cells)
    assert out["f16"][1] <= 6e-2
    assert out["f16"][2] <= 2e-2


# ------------------------------------------------------------------------------------------
# The 128^3 copy of the metric workload: populations after 100 steps
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_tgv128_populations_at_step_100_against_oracle(storage):
    ref = _ref("tgv128_cumulant")
    n, u0 = int(ref["n"]), float(ref["u0"])
    om = lbm.regularized_rates("D3Q27", W.re_to_omega(u0, 512, 1600.0))
    rho, u = W.tgv3d_fields(n, u0=u0)
    lat = lbm.Lattice("D3Q27", "cumulant", om, (n, n, n), storage=storage)
    lat.lbm_init_equilibrium(rho, u)
    lat.lbm_autotune()
    lat.lbm_graph_prepare(int(ref["df_step"]))
    lat.lbm_step(int(ref["df_step"]))
    err = float(np.abs(_df_at(lat.lbm_get_populations(), ref["df_pts"]) - ref["df"]).max())
    print("TGV 128^3 %s after %d steps, %d sampled cells: max|d df| = %.3e"
          % (storage, int(ref["df_step"]), len(ref["df_pts"]), err))
    assert err <= (1e-12 if storage == "f64" else 1e-6)


# ------------------------------------------------------------------------------------------
# Two workloads at their full size for 100 steps (the oracle's sampled cells)
# ------------------------------------------------------------------------------------------
def _gpu_cells(lat, pts):
    """df and the macroscopic fields of the sampled cells, gathered on the device."""
    import torch
    nx, ny, nz = lat.dims
    n = nx * ny * nz
    cells = torch.as_tensor((pts[:, 2] * ny + pts[:, 1]) * nx + pts[:, 0], device="cuda")
    dev = torch.empty(lat.q * n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    lbm.check(lat.lib.lbm_get_populations(lat.ctx, lbm._dptr(dev)))
    df = dev[torch.arange(lat.q, device="cuda")[None, :] * n + cells[:, None]].cpu().numpy()
    del dev
    r = torch.empty(n, dtype=torch.float64, device="cuda")
    u = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    lbm.check(lat.lib.lbm_macroscopic(lat.ctx, lbm._dptr(r), lbm._dptr(u)))
    uc = u[torch.arange(3, device="cuda")[None, :] * n + cells[:, None]].cpu().numpy()
    rc = r[cells].cpu().numpy()
    del r, u
    torch.cuda.empty_cache()
    return df, rc, uc


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_d3q19_raw_256_full_size_100_steps_against_oracle(storage):
    ref = _ref("d3q19_raw256")
    dims, steps = tuple(int(v) for v in ref["dims"]), int(ref["steps"])
    cfg = W.WORKLOADS["d3q19_raw_256"]
    om = lbm.regularized_rates("D3Q19", cfg["omega_shear"])
    rho, u = W.tgv3d_fields(dims[0], u0=cfg["u0"])
    lat = lbm.Lattice("D3Q19", "raw", om, dims, storage=storage)
    lat.lbm_init_equilibrium(rho, u)
    del rho, u
    lat.lbm_autotune()
    lat.lbm_graph_prepare(steps)
    lat.lbm_step(steps)
    df, _, _ = _gpu_cells(lat, ref["df_pts"])
    _, rg, ug = _gpu_cells(lat, ref["u_pts"])
    err = float(np.abs(df - ref["df"]).max())
    rel = _rel(ug, ref["u"])
    print("D3Q19 raw 256^3 %s, %d steps: max|d df| = %.3e, relative L2 velocity error %.3e, max|d rho| %.3e"
          % (storage, steps, err, rel, float(np.abs(rg - ref["rho"]).max())))
    if storage == "f64":
        assert err <= 1e-12
        assert rel <= 1e-10
    else:
        assert rel <= 1e-5


@pytest.mark.parametrize("storage", ["f64", "f16"])
def test_swe_4096_full_size_100_steps_against_oracle(storage):
    ref = _ref("swe4096")
    dims, steps = tuple(int(v) for v in ref["dims"]), int(ref["steps"])
    cfg = W.WORKLOADS["swe_d2q9_4096"]
    om = lbm.regularized_rates("D2Q9", cfg["omega_shear"])
    h, u = W.swe_bumps(dims[0], seed=0)
    lat = lbm.Lattice("D2Q9", "central", om, dims, storage=storage, equilibrium="swe", gravity=cfg["gravity"])
    lat.lbm_init_equilibrium(h, u)
    del h, u
    lat.lbm_autotune()
    lat.lbm_step(steps)
    df, _, _ = _gpu_cells(lat, ref["df_pts"])
    _, hg, ug = _gpu_cells(lat, ref["u_pts"])
    err = float(np.abs(df - ref["df"]).max())
    rel = _rel(ug[:, :2], ref["u"][:, :2])
    dh = float(np.abs(hg - ref["rho"]).max())
    print("SWE 4096^2 %s, %d steps: max|d df| = %.3e, relative L2 velocity error %.3e, max|d h| %.3e"
          % (storage, steps, err, rel, dh))
    if storage == "f64":
        assert err <= 1e-12
        assert rel <= 1e-10
    else:
        # FP16 storage after 100 steps (the 512^2 instance: 1.6e-3 in df at step 100)
        assert err <= 5e-3
        assert rel <= 5e-2
