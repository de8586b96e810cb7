"""Parity at the full workload sizes, in the launch configuration bench.py times (autotuned,
cached in LBM_AUTOTUNE_CACHE when set).

The oracle cannot run 512^3 cells, so after one step from the equilibrium initial state each
sampled output df_i(x, 1) = Omega(df(x - xi_i, 0))_i is computed by the oracle from its own
equilibrium of the 27 (or 19, 9) neighbours.  Over several steps, properties that hold at any
size are checked: mass and momentum conservation and the mirror symmetry of the vortex.
"""
import math

import numpy as np
import pytest

import lbm_workloads as W
import oracle as O
import sampled_oracle as SO
from paper_2211_02435_amd import lbm

pytestmark = pytest.mark.gpu


def _gpu_samples(lat, pts):
    import torch
    nx, ny, nz = lat.dims
    n = nx * ny * nz
    dev = torch.empty(lat.q * n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    lbm.check(lat.lib.lbm_get_populations(lat.ctx, lbm._dptr(dev)))
    cells = torch.as_tensor((pts[:, 2] * ny + pts[:, 1]) * nx + pts[:, 0], device="cuda")
    idx = torch.arange(lat.q, device="cuda")[None, :] * n + cells[:, None]
    out = dev[idx].cpu().numpy()
    del dev
    torch.cuda.empty_cache()
    return out


@pytest.mark.parametrize("storage,tol", [("f32", 2e-8), ("f64", 1e-15)])
def test_d3q27_cumulant_512_one_step_sampled(storage, tol):
    cfg = W.WORKLOADS["d3q27_cumulant_512"]
    n = cfg["dims"][0]
    om = O.regularized_rates("D3Q27", cfg["omega_shear"])
    rho, u = W.tgv3d_fields(n, u0=cfg["u0"])
    lat = lbm.Lattice("D3Q27", "cumulant", om, (n, n, n), storage=storage)
    lat.lbm_init_equilibrium(rho, u)
    del rho, u
    lat.lbm_autotune()
    print("launch", lat.lbm_get_launch(), "vec", lat.lbm_get_vectorized(), "lds", lat.lbm_get_lds_reserve())
    lat.lbm_step(1)
    pts = W.sample_cells((n, n, n), 48, seed=1)
    got = _gpu_samples(lat, pts)
    m = O.Method("D3Q27", "cumulant", om)
    want = SO.one_step_samples(m, pts, (n, n, n), lambda x, y, z: W.tgv3d_points(x, y, z, n, cfg["u0"]))
    err = np.abs(got - want).max()
    print("D3Q27 cumulant 512^3 %s one step, %d sampled cells: max|d df| = %.3e" % (storage, len(pts), err))
    assert err <= tol


@pytest.mark.parametrize("storage,streaming,tol", [("f32", "pull", 6e-8), ("f64", "pull", 3e-15),
                                                    ("f32", "aa", 6e-8), ("f32", "esoteric", 6e-8),
                                                    ("f32", "twist", 6e-8), ("f32", "push", 6e-8)])
def test_d3q27_cumulant_512_three_steps_sampled(storage, streaming, tol):
    """The timed sequence at full size: one eager step, then two steps replayed from a recorded
    graph, so that both buffers (or both phases of an in-place pattern) are written by the
    timed launch.  Bars: three times the one-step bars."""
    cfg = W.WORKLOADS["d3q27_cumulant_512"]
    n = cfg["dims"][0]
    om = O.regularized_rates("D3Q27", cfg["omega_shear"])
    rho, u = W.tgv3d_fields(n, u0=cfg["u0"])
    lat = lbm.Lattice("D3Q27", "cumulant", om, (n, n, n), storage=storage, streaming=streaming)
    lat.lbm_init_equilibrium(rho, u)
    del rho, u
    lat.lbm_autotune()
    lat.lbm_step(1)
    lat.lbm_graph_prepare(2)
    lat.lbm_time_steps(2)
    assert lat.lib.lbm_time(lat.ctx) == 3
    pts = W.sample_cells((n, n, n), 48, seed=4)
    got = _gpu_samples(lat, pts)
    del lat
    m = O.Method("D3Q27", "cumulant", om)
    want = SO.k_step_samples(m, pts, (n, n, n), lambda x, y, z: W.tgv3d_points(x, y, z, n, cfg["u0"]), 3)
    err = np.abs(got - want).max()
    print("D3Q27 cumulant 512^3 %s %s three steps, %d sampled cells: max|d df| = %.3e"
          % (storage, streaming, len(pts), err))
    assert err <= tol


@pytest.mark.parametrize("storage,bx", [("f32", 256), ("f64", 128)])
def test_d3q27_512_streaming_only_sweeps_move_populations_exactly(storage, bx):
    """The pull index maps at the metric size in the metric launches (blocks of 256 x 1 threads
    for FP32 and 128 x 1 for FP64, XCD order, 53248 bytes of LDS reserved, rows layout): 20
    sweeps with the collision replaced by the identity (lbm_debug_stream_only) must leave
    df_i(x, 20) = df_i(x - 20 xi_i, 0) bit for bit at every sampled cell, box faces and corners
    included."""
    import torch
    cfg = W.WORKLOADS["d3q27_cumulant_512"]
    n = cfg["dims"][0]
    steps = 20
    om = O.regularized_rates("D3Q27", cfg["omega_shear"])
    rho, u = W.tgv3d_fields(n, u0=cfg["u0"])
    lat = lbm.Lattice("D3Q27", "cumulant", om, (n, n, n), storage=storage)
    lat.lbm_init_equilibrium(rho, u)
    del rho, u
    lat.lbm_set_launch(bx, 1, 1)
    lat.lbm_set_lds_reserve(53248)
    pts = W.sample_cells((n, n, n), 512, seed=8)
    c = np.asarray(O.stencil("D3Q27").xi, dtype=np.int64)  # (q, 3)
    # source cell of population i of every sampled cell, steps cells upstream
    src = (pts[:, None, :] - steps * c[None, :, :]) % n  # (m, q, 3)
    ncell = n ** 3
    idx0 = torch.as_tensor(np.arange(lat.q)[None, :] * ncell + (src[..., 2] * n + src[..., 1]) * n + src[..., 0],
                           device="cuda")
    dev = torch.empty(lat.q * ncell, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    lbm.check(lat.lib.lbm_get_populations(lat.ctx, lbm._dptr(dev)))
    want = dev[idx0].cpu().numpy()
    del dev
    torch.cuda.empty_cache()
    lat.lbm_debug_stream_only(steps)
    got = _gpu_samples(lat, pts)
    lat.close()
    mism = int((got != want).sum())
    print("D3Q27 512^3 %s, %d streaming-only sweeps, %d sampled cells: %d mismatches"
          % (storage, steps, len(pts), mism))
    assert mism == 0


@pytest.mark.parametrize("storage,tol", [("f32", 2e-8), ("f64", 1e-15)])
def test_d3q27_cumulant_512_general_rates_sampled(storage, tol):
    """The general-rate kernel at full size (every rate of order >= 3 set to 1.3, so no
    order is pinned to its equilibrium), one step, sampled."""
    cfg = W.WORKLOADS["d3q27_cumulant_512"]
    n = cfg["dims"][0]
    st = O.stencil("D3Q27")
    om = O.regularized_rates("D3Q27", cfg["omega_shear"])
    om[[j for j in range(st.q) if st.order(j) >= 3]] = 1.3
    rho, u = W.tgv3d_fields(n, u0=cfg["u0"])
    lat = lbm.Lattice("D3Q27", "cumulant", om, (n, n, n), storage=storage)
    lat.lbm_init_equilibrium(rho, u)
    del rho, u
    lat.lbm_autotune()
    lat.lbm_step(1)
    pts = W.sample_cells((n, n, n), 48, seed=5)
    got = _gpu_samples(lat, pts)
    del lat
    m = O.Method("D3Q27", "cumulant", om)
    want = SO.one_step_samples(m, pts, (n, n, n), lambda x, y, z: W.tgv3d_points(x, y, z, n, cfg["u0"]))
    err = np.abs(got - want).max()
    print("D3Q27 cumulant 512^3 general rates %s one step: max|d df| = %.3e" % (storage, err))
    assert err <= tol


@pytest.mark.parametrize("storage,tol", [("f32", 2e-8), ("f64", 1e-15)])
def test_d3q15_raw_512_three_steps_sampled(storage, tol):
    """D3Q15 raw moments at 512^3 (the stencil's bench workload): one eager step and two
    graph-replayed steps, sampled."""
    cfg = W.WORKLOADS["d3q15_raw_512"]
    n = cfg["dims"][0]
    om = O.regularized_rates("D3Q15", cfg["omega_shear"])
    rho, u = W.tgv3d_fields(n, u0=cfg["u0"])
    lat = lbm.Lattice("D3Q15", "raw", om, (n, n, n), storage=storage)
    lat.lbm_init_equilibrium(rho, u)
    del rho, u
    lat.lbm_autotune()
    lat.lbm_step(1)
    lat.lbm_graph_prepare(2)
    lat.lbm_time_steps(2)
    pts = W.sample_cells((n, n, n), 48, seed=6)
    got = _gpu_samples(lat, pts)
    del lat
    m = O.Method("D3Q15", "raw", om)
    want = SO.k_step_samples(m, pts, (n, n, n), lambda x, y, z: W.tgv3d_points(x, y, z, n, cfg["u0"]), 3)
    err = np.abs(got - want).max()
    print("D3Q15 raw 512^3 %s three steps: max|d df| = %.3e" % (storage, err))
    assert err <= 3 * tol


def test_d3q27_cumulant_512_conservation_and_symmetry():
    """FP32, 20 steps at 512^3: mass and momentum stay at their initial sums and the velocity
    keeps the vortex's mirror symmetry u_x(-x) = -u_x(x), u_y(-x) = u_y(x)."""
    import torch
    cfg = W.WORKLOADS["d3q27_cumulant_512"]
    n = cfg["dims"][0]
    om = O.regularized_rates("D3Q27", cfg["omega_shear"])
    rho, u = W.tgv3d_fields(n, u0=cfg["u0"])
    lat = lbm.Lattice("D3Q27", "cumulant", om, (n, n, n), storage="f32")
    lat.lbm_init_equilibrium(rho, u)
    del rho, u
    lat.lbm_autotune()
    d0 = lat.lbm_diagnostics()
    lat.lbm_step(20)
    d1 = lat.lbm_diagnostics()
    print("diagnostics t=0", d0, "t=20", d1)
    # FP32 storage rounds every population each step: bound the drift by 1e-9 of the total mass
    assert abs(d1[0] - d0[0]) <= 1e-9 * n ** 3
    assert np.abs(d1[1:4] - d0[1:4]).max() <= 1e-9 * n ** 3
    assert d1[4] < d0[4]  # kinetic energy decays
    rg = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    ug = torch.empty(3 * n ** 3, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    lbm.check(lat.lib.lbm_macroscopic(lat.ctx, lbm._dptr(rg), lbm._dptr(ug)))
    ux = ug[: n ** 3].view(n, n, n)
    uy = ug[n ** 3: 2 * n ** 3].view(n, n, n)
    mirror = (-torch.arange(n, device="cuda")) % n
    ux_m = ux[:, :, mirror]
    uy_m = uy[:, :, mirror]
    scale = float(ux.abs().max())
    e1 = float((ux + ux_m).abs().max()) / scale
    e2 = float((uy - uy_m).abs().max()) / scale
    print("mirror symmetry residuals (relative to max |u_x|): %.3e %.3e" % (e1, e2))
    assert e1 <= 1e-5 and e2 <= 1e-5


@pytest.mark.parametrize("storage,tol", [("f32", 2e-8), ("f64", 1e-15)])
def test_d3q19_raw_256_one_step_sampled(storage, tol):
    cfg = W.WORKLOADS["d3q19_raw_256"]
    n = cfg["dims"][0]
    om = O.regularized_rates("D3Q19", cfg["omega_shear"])
    rho, u = W.tgv3d_fields(n, u0=cfg["u0"])
    lat = lbm.Lattice("D3Q19", "raw", om, (n, n, n), storage=storage)
    lat.lbm_init_equilibrium(rho, u)
    lat.lbm_autotune()
    lat.lbm_step(1)
    pts = W.sample_cells((n, n, n), 48, seed=2)
    got = _gpu_samples(lat, pts)
    m = O.Method("D3Q19", "raw", om)
    want = SO.one_step_samples(m, pts, (n, n, n), lambda x, y, z: W.tgv3d_points(x, y, z, n, cfg["u0"]))
    err = np.abs(got - want).max()
    print("D3Q19 raw 256^3 %s one step: max|d df| = %.3e" % (storage, err))
    assert err <= tol


@pytest.mark.parametrize("storage,tol", [("f16", 5e-4), ("f64", 1e-15)])
def test_swe_4096_one_step_sampled(storage, tol):
    cfg = W.WORKLOADS["swe_d2q9_4096"]
    n = cfg["dims"][0]
    om = O.regularized_rates("D2Q9", cfg["omega_shear"])
    h, u = W.swe_bumps(n, seed=0)
    lat = lbm.Lattice("D2Q9", "central", om, (n, n, 1), storage=storage, equilibrium="swe",
                      gravity=cfg["gravity"])
    lat.lbm_init_equilibrium(h, u)
    lat.lbm_autotune()
    lat.lbm_step(1)
    pts = W.sample_cells((n, n, 1), 48, seed=3)
    got = _gpu_samples(lat, pts)
    m = O.Method("D2Q9", "central", om, equilibrium="swe", gravity=cfg["gravity"])
    hh = h[0]

    def fields_at(x, y, z):
        return hh[y, x], np.zeros((len(x), 3))
    want = SO.one_step_samples(m, pts, (n, n, 1), fields_at)
    err = np.abs(got - want).max()
    print("SWE 4096^2 %s one step: max|d df| = %.3e" % (storage, err))
    assert err <= tol


def test_batch_256_boxes_one_step_sampled():
    """The 256-box ensemble (FP32, central moments, one launch per step): sampled outputs of
    every 16th box after one step against the oracle."""
    boxes = W.batch_ensemble(256, seed=0)
    dims = [(b["edge"],) * 3 for b in boxes]
    rates = [O.regularized_rates("D3Q27", b["omega_shear"]) for b in boxes]
    rho_cat = np.concatenate([W.batch_fields(b)[0].ravel() for b in boxes])
    u_cat = np.concatenate([W.batch_fields(b)[1].ravel() for b in boxes])
    bat = lbm.Batch("D3Q27", "central", dims, rates, storage="f32")
    print("ensemble cells", bat.lbm_batch_cells())
    bat.lbm_batch_init_equilibrium(rho_cat, u_cat)
    bat.lbm_batch_step(1)
    worst = 0.0
    rng = np.random.default_rng(5)
    for k, (b, d, om) in enumerate(zip(boxes, dims, rates)):
        if k % 16 == 0:
            box = bat.lbm_batch_get_box_populations(k)
            pts = W.sample_cells(d, 4, seed=int(rng.integers(1 << 30)))
            got = box[:, pts[:, 2], pts[:, 1], pts[:, 0]].T
            m = O.Method("D3Q27", "central", om)
            want = SO.one_step_samples(
                m, pts, d, lambda x, y, z, b=b, e=d[0]: W.tgv3d_points(x, y, z, e, b["u0"], b["phase"]))
            worst = max(worst, float(np.abs(got - want).max()))
    print("ensemble one step, 16 boxes sampled: max|d df| = %.3e" % worst)
    assert worst <= 2e-8
