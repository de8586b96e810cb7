"""Edge cases of the sweep on the GPU against the FP64 oracle, through the C ABI.

* Degenerate periodic boxes: a single cell, two cells along one axis (x - 1 and x + 1 are the
  same cell), one-cell-thick slabs, for every streaming pattern.
* The limits of the rate range: omega = 0 on every non-conserved polynomial (the collision is
  the identity) and omega = 2 (the zero-viscosity limit of eq. MrtUpdateGeneral).
* lbm_step(0) changes nothing; lbm_step rejects a negative count.
* The rest state (df = 0) and the shallow-water lake at rest are exact fixed points in every
  precision (bit-exact zero after 50 steps); a uniform flow stays bit-identical across cells
  and at its equilibrium.
* The largest z-plane the 32-bit lane offsets admit: boxes whose z-plane of population
  storage sits just under 4 GiB (rows layout, FP32 and FP64, ragged x), two steps of pull and
  of AA, sampled against the oracle (one- and two-step bars of the full-size tests).

Bars: FP64 max |df_gpu - df_oracle| <= 1e-13 after 5 steps from a non-equilibrium state.
"""
import os

import numpy as np
import pytest

import lbm_workloads as W
import oracle as O
import sampled_oracle as SO
from paper_2211_02435_amd import lbm

pytestmark = pytest.mark.gpu

STREAMING = ["pull", "push", "aa", "esoteric", "twist"]


def _state(m, dims, seed=3):
    nx, ny, nz = dims
    rho, u = W.random_near_equilibrium_fields((nz, ny, nx), seed=seed, drho=5e-3, umax=0.04)
    if m.st.d == 2:
        u[2] = 0.0
    df = O.init_equilibrium(m, rho, u)
    return df + W.random_perturbation(m.st.q, (nz, ny, nx), seed=seed + 1, scale=2e-4)


def _general(stencil, seed=5):
    st = O.stencil(stencil)
    om = np.random.default_rng(seed).uniform(0.7, 1.9, st.q)
    om[st.conserved] = 0.0
    return om


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 1, 1), (1, 2, 1), (1, 1, 2), (3, 2, 1), (2, 2, 2), (1, 5, 3)])
@pytest.mark.parametrize("streaming", STREAMING)
def test_degenerate_boxes_d3q27(dims, streaming):
    om = _general("D3Q27")
    m = O.Method("D3Q27", "cumulant", om)
    df0 = _state(m, dims)
    lat = lbm.Lattice("D3Q27", "cumulant", om, dims, storage="f64", streaming=streaming)
    lat.lbm_set_populations(df0)
    lat.lbm_step(5)
    err = np.abs(lat.lbm_get_populations() - O.step(m, df0, 5)).max()
    print("D3Q27 %s %s max|d df| = %.3e" % (dims, streaming, err))
    assert err <= 1e-13


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 1, 1), (1, 2, 1), (5, 1, 1)])
@pytest.mark.parametrize("streaming", STREAMING)
def test_degenerate_boxes_d2q9(dims, streaming):
    om = _general("D2Q9")
    m = O.Method("D2Q9", "central", om)
    df0 = _state(m, dims)
    lat = lbm.Lattice("D2Q9", "central", om, dims, storage="f64", streaming=streaming)
    lat.lbm_set_populations(df0)
    lat.lbm_step(5)
    err = np.abs(lat.lbm_get_populations() - O.step(m, df0, 5)).max()
    assert err <= 1e-13


@pytest.mark.parametrize("space", ["raw", "central", "cumulant", "srt"])
@pytest.mark.parametrize("omega", [0.0, 2.0])
def test_rate_limits(space, omega):
    st = O.stencil("D3Q27")
    om = np.full(st.q, omega)
    om[st.conserved] = 0.0
    dims = (9, 4, 3)
    m = O.Method("D3Q27", space, om)
    df0 = _state(m, dims)
    lat = lbm.Lattice("D3Q27", space, om, dims, storage="f64")
    lat.lbm_set_populations(df0)
    lat.lbm_step(5)
    got = lat.lbm_get_populations()
    want = O.step(m, df0, 5)
    err = np.abs(got - want).max()
    print("omega %.1f %s max|d df| = %.3e" % (omega, space, err))
    assert err <= 1e-13
    if omega == 0.0:  # identity collision: five steps of pure streaming, up to the round-off
        pure = df0   # of five transform round trips (a few ulps of |df| ~ 0.05 each)
        for _ in range(5):
            pure = O.stream(O.Method("D3Q27", "raw", np.zeros(27)), pure)
        assert np.abs(got - pure).max() <= 1e-14


@pytest.mark.parametrize("streaming", STREAMING)
def test_zero_steps_is_a_no_op(streaming):
    om = _general("D3Q27")
    m = O.Method("D3Q27", "cumulant", om)
    dims = (6, 5, 4)
    df0 = _state(m, dims)
    lat = lbm.Lattice("D3Q27", "cumulant", om, dims, storage="f64", streaming=streaming)
    lat.lbm_set_populations(df0)
    lat.lbm_step(1)
    before = lat.lbm_get_populations()
    t = lat.lib.lbm_time(lat.ctx)
    lat.lbm_step(0)
    assert lat.lib.lbm_time(lat.ctx) == t
    np.testing.assert_array_equal(lat.lbm_get_populations(), before)
    with pytest.raises(lbm.LbmError):
        lat.lbm_step(-1)


@pytest.mark.parametrize("stencil,space", [(st, sp) for st in ("D2Q9", "D3Q15", "D3Q19", "D3Q27")
                                           for sp in ("raw", "central", "cumulant", "srt")])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("streaming", ["pull", "aa"])
def test_rest_state_is_an_exact_fixed_point(stencil, space, storage, streaming):
    """The fluid at rest (rho = 1, u = 0) is stored as df = 0 in zero-centred storage, and every
    collision maps it to itself: after 50 steps each stored deviation is still exactly zero,
    in every precision (no background value ever enters the stored numbers)."""
    st = O.stencil(stencil)
    om = _general(stencil)
    if space == "srt":
        om[[j for j in range(st.q) if st.order(j) >= 2]] = 1.4
    dims = (9, 7, 1) if stencil == "D2Q9" else (9, 7, 5)
    nx, ny, nz = dims
    lat = lbm.Lattice(stencil, space, om, dims, storage=storage, streaming=streaming)
    lat.lbm_init_equilibrium(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    lat.lbm_step(50)
    df = lat.lbm_get_populations()
    print("%s %s %s %s: max|df| = %.3e" % (stencil, space, storage, streaming, np.abs(df).max()))
    assert not np.any(df)
    rho, u = lat.lbm_macroscopic()
    assert np.all(rho == 1.0) and not np.any(u)


@pytest.mark.parametrize("storage", ["f64", "f16"])
def test_lake_at_rest_is_an_exact_fixed_point(storage):
    """Shallow water: a flat surface at rest (h = 1, u = 0) stays exactly flat and still."""
    om = O.regularized_rates("D2Q9", 1.8)
    lat = lbm.Lattice("D2Q9", "central", om, (33, 17, 1), storage=storage, equilibrium="swe", gravity=0.1)
    lat.lbm_init_equilibrium(np.ones((1, 17, 33)), np.zeros((3, 1, 17, 33)))
    lat.lbm_step(50)
    assert not np.any(lat.lbm_get_populations())


@pytest.mark.parametrize("space", ["raw", "central", "cumulant", "srt"])
@pytest.mark.parametrize("storage,tol", [("f64", 5e-15), ("f32", 2e-6)])
@pytest.mark.parametrize("streaming", ["pull", "aa", "twist", "push"])
def test_uniform_flow_stays_uniform_and_at_equilibrium(space, storage, tol, streaming):
    """A uniform flow (rho = 1.01, u = (0.05, -0.03, 0.02)) is the equilibrium everywhere, a
    fixed point of every collision.  Every cell does the same arithmetic on the same inputs,
    so after 50 steps all cells hold bit-identical populations (whatever the launch tiling
    or streaming pattern), and those stay within rounding of the oracle's equilibrium.
    Bars: the conserved moments do not relax, so their rounding can accumulate; at most
    half an ulp of |df| <= 0.03 per population and step gives 50 * 27 * ulp / 2, about 2.4e-15
    in FP64 and 1.3e-6 in FP32."""
    st = O.stencil("D3Q27")
    om = _general("D3Q27")
    if space == "srt":
        om[[j for j in range(st.q) if st.order(j) >= 2]] = 1.4
    dims = (70, 9, 5)
    nx, ny, nz = dims
    u0 = np.array([0.05, -0.03, 0.02])
    lat = lbm.Lattice("D3Q27", space, om, dims, storage=storage, streaming=streaming)
    lat.lbm_init_equilibrium(np.full((nz, ny, nx), 1.01), np.broadcast_to(u0[:, None, None, None], (3, nz, ny, nx)).copy())
    lat.lbm_step(50)
    df = lat.lbm_get_populations().reshape(st.q, -1)
    assert np.all(df == df[:, :1])
    m = O.Method("D3Q27", space, om)
    want = O.init_equilibrium(m, np.full((1, 1, 1), 1.01), u0[:, None, None, None]).reshape(st.q)
    err = np.abs(df[:, 0] - want).max()
    print("uniform flow %s %s %s: max|df - df_eq| = %.3e" % (space, storage, streaming, err))
    assert err <= tol


# (storage, dims, bar after two steps): the rows layout pads x to 256 bytes, so the z-plane of
# D3Q27 populations is ny * 27 * nxp * sizeof(storage) bytes, nxp = 6272 (F32) or 4448 (F64);
# one more row along y would reach 4 GiB and is refused (tests/test_abi_cpu.py)
LARGEST_PLANE = [("f32", (6250, 6340, 2), 4e-8), ("f64", (4420, 4470, 2), 2e-15)]


@pytest.mark.parametrize("storage,dims,tol", LARGEST_PLANE)
@pytest.mark.parametrize("streaming", ["pull", "aa"])
def test_largest_z_plane_two_steps_sampled(storage, dims, tol, streaming):
    import torch
    nx, ny, nz = dims
    esize = 4 if storage == "f32" else 8
    align = 256 // esize
    nxp = (nx + align - 1) // align * align
    plane = ny * 27 * nxp * esize
    assert 0.9999 * 2 ** 32 < plane < 2 ** 32 - 1
    u0 = 0.05
    om = O.regularized_rates("D3Q27", 1.9)
    rho, u = W.tgv3d_fields(nx, ny, nz, u0=u0, period=nx)
    lat = lbm.Lattice("D3Q27", "cumulant", om, dims, storage=storage, streaming=streaming, layout="rows")
    assert lat.lbm_get_layout() == "rows"
    lat.lbm_init_equilibrium(rho, u)
    del rho, u
    lat.lbm_set_launch(256, 1, 1)
    lat.lbm_step(2)
    pts = W.sample_cells(dims, 48, seed=9)
    n = nx * ny * nz
    dev = torch.empty(27 * n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    lbm.check(lat.lib.lbm_get_populations(lat.ctx, lbm._dptr(dev)))
    cells = torch.as_tensor((pts[:, 2] * ny + pts[:, 1]) * nx + pts[:, 0], device="cuda")
    got = dev[torch.arange(27, device="cuda")[None, :] * n + cells[:, None]].cpu().numpy()
    del dev
    lat.close()
    torch.cuda.empty_cache()
    m = O.Method("D3Q27", "cumulant", om)
    want = SO.k_step_samples(m, pts, dims, lambda x, y, z: W.tgv3d_points(x, y, z, nx, u0), 2)
    err = float(np.abs(got - want).max())
    print("D3Q27 %s %s, z-plane of %d bytes, two steps, %d sampled cells: max|d df| = %.3e"
          % (storage, dims, plane, len(pts), err))
    assert err <= tol


def test_allocation_failure_reports_enomem_and_leaves_the_device_usable():
    """A box that passes validation but needs more device memory than the GPU holds (2^31
    D3Q27 cells in FP64 with two library-owned buffers, 2 x 464 GB): lbm_create compares the
    request with the free device memory before allocating and returns LBM_ENOMEM with both
    sizes in the message; a context created afterwards steps and matches the oracle."""
    om = O.regularized_rates("D3Q27", 1.9)
    big = (2048, 2048, 512)
    assert lbm.lbm_validate(lbm.make_params("D3Q27", "cumulant", om, big, storage="f64")) == 0
    with pytest.raises(lbm.LbmError) as err:
        lbm.Lattice("D3Q27", "cumulant", om, big, storage="f64", torch_buffers=False)
    print("lbm_create of %s FP64: %s" % (big, err.value))
    assert err.value.status == lbm.LBM_ENOMEM
    assert "bytes of device memory are free" in str(err.value)
    dims = (20, 12, 9)
    m = O.Method("D3Q27", "cumulant", om)
    df0 = _state(m, dims, seed=31)
    lat = lbm.Lattice("D3Q27", "cumulant", om, dims, storage="f64", torch_buffers=False)
    lat.lbm_set_populations(df0)
    lat.lbm_step(5)
    err = np.abs(lat.lbm_get_populations() - O.step(m, df0, 5)).max()
    lat.close()
    assert err <= 1e-13


def test_library_loaded_before_torch_shares_its_runtime(tmp_path):
    """A fresh process that loads the library (through a host-only call) before it imports
    torch, then creates a context with library-owned buffers and steps it: the binding imports
    torch before loading the library, so one HIP runtime serves both."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2211_02435_amd import lbm\n"
        "import oracle as O\n"
        "om = O.regularized_rates('D3Q27', 1.9)\n"
        "assert lbm.lbm_validate(lbm.make_params('D3Q27', 'cumulant', om, (16, 16, 16))) == 0\n"
        "lat = lbm.Lattice('D3Q27', 'cumulant', om, (16, 16, 16), storage='f64', torch_buffers=False)\n"
        "lat.lbm_init_equilibrium(*__import__('lbm_workloads').tgv3d_fields(16, u0=0.05))\n"
        "lat.lbm_step(3)\n"
        "print('ok', lat.lbm_time())\n" % root)
    print("fresh process: library loaded before torch", flush=True)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=root)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr[-2000:])
    assert r.stdout.split()[-2:] == ["ok", "3"]
