"""GPU parity of the HIP sweep against the FP64 oracle, through the C ABI.

Bars: FP64 populations within max |df_gpu - df_oracle| <= 1e-12 (after 100 steps where
stated); integer index maps (streaming only) bit-exact; AA == pull, graph == host loop and
checkpoint/resume bit-exact; FP32 relative L2 velocity error <= 1e-5 against the oracle.
Grids span several launch tiles with ragged tails in x and y.
"""
import math

import numpy as np
import pytest

import lbm_workloads as W
import oracle as O
from paper_2211_02435_amd import lbm

pytestmark = pytest.mark.gpu

RAGGED3 = (70, 9, 5)     # two x-tiles of 64 with a tail of 6, y tail, 5 planes
RAGGED2 = (70, 37, 1)


def _rates(stencil, kind, seed=0):
    if kind == "reg":
        return O.regularized_rates(stencil, 1.7, omega_bulk=1.2)
    rng = np.random.default_rng(seed)
    om = rng.uniform(0.7, 1.9, O.stencil(stencil).q)
    om[O.stencil(stencil).conserved] = 0.0
    return om


def _noisy_state(m, dims, seed=0, noise=2e-4):
    nx, ny, nz = dims
    rho, u = W.random_near_equilibrium_fields((nz, ny, nx), seed=seed, drho=5e-3, umax=0.04)
    if m.st.d == 2:
        u[2] = 0.0
    df = O.init_equilibrium(m, rho, u)
    return df + W.random_perturbation(m.st.q, (nz, ny, nx), seed=seed + 1, scale=noise)


def _lattice(stencil, space, om, dims, **kw):
    return lbm.Lattice(stencil, space, om, dims, **kw)


# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("stencil,space", [("D2Q9", "raw"), ("D2Q9", "central"), ("D2Q9", "cumulant"),
                                           ("D3Q19", "raw"), ("D3Q19", "central"), ("D3Q19", "cumulant"),
                                           ("D3Q27", "raw"), ("D3Q27", "central"), ("D3Q27", "cumulant")])
@pytest.mark.parametrize("streaming", ["pull", "push", "aa", "esoteric", "twist"])
def test_init_equilibrium_matches_oracle(stencil, space, streaming):
    dims = RAGGED2 if stencil == "D2Q9" else RAGGED3
    om = _rates(stencil, "reg")
    rho, u = W.tgv3d_fields(dims[0], dims[1], dims[2], u0=0.05, period=16) if stencil != "D2Q9" \
        else W.tgv2d_fields(dims[0], dims[1], 1, u0=0.05)
    lat = _lattice(stencil, space, om, dims, storage="f64", streaming=streaming)
    lat.lbm_init_equilibrium(rho, u)
    got = lat.lbm_get_populations()
    m = O.Method(stencil, space, om)
    want = O.init_equilibrium(m, rho, u)
    assert np.abs(got - want).max() <= 4e-15
    r2, u2 = lat.lbm_macroscopic()
    assert np.abs(r2 - rho).max() <= 1e-15
    d = 3 if stencil != "D2Q9" else 2
    assert np.abs(u2[:d] - u[:d]).max() <= 1e-15


@pytest.mark.parametrize("stencil,space", [("D2Q9", "raw"), ("D2Q9", "central"), ("D2Q9", "cumulant"),
                                           ("D3Q19", "raw"), ("D3Q19", "central"), ("D3Q19", "cumulant"),
                                           ("D3Q27", "raw"), ("D3Q27", "central"), ("D3Q27", "cumulant")])
@pytest.mark.parametrize("kind", ["reg", "gen"])
@pytest.mark.parametrize("layout", ["planes", "rows"])
def test_sweep_fp64_matches_oracle(stencil, space, kind, layout):
    """Non-equilibrium start (equilibrium + noise from the oracle), 4 steps, FP64."""
    dims = RAGGED2 if stencil == "D2Q9" else RAGGED3
    om = _rates(stencil, kind, seed=3)
    m = O.Method(stencil, space, om)
    df0 = _noisy_state(m, dims, seed=11)
    lat = _lattice(stencil, space, om, dims, storage="f64", layout=layout)
    lat.lbm_set_populations(df0)
    lat.lbm_step(4)
    got = lat.lbm_get_populations()
    want = O.step(m, df0, 4)
    err = np.abs(got - want).max()
    print("%s %s %s max|d df| = %.3e" % (stencil, space, kind, err))
    assert err <= 1e-13


@pytest.mark.parametrize("stencil,space,kind", [("D2Q9", "central", "reg"), ("D3Q19", "raw", "reg"),
                                                ("D3Q27", "cumulant", "reg"), ("D3Q27", "cumulant", "gen"),
                                                ("D3Q27", "central", "reg")])
def test_sweep_fp64_100_steps(stencil, space, kind):
    """Taylor-Green start, 100 steps, FP64: max |d df| <= 1e-12."""
    dims = (20, 12, 9) if stencil != "D2Q9" else RAGGED2
    om = _rates(stencil, kind, seed=5) if kind == "gen" else O.regularized_rates(stencil, 1.9699)
    if stencil == "D2Q9":
        rho, u = W.tgv2d_fields(dims[0], dims[1], 1, u0=0.02)
    else:
        rho, u = W.tgv3d_fields(dims[0], dims[1], dims[2], u0=0.05, period=12)
    lat = _lattice(stencil, space, om, dims, storage="f64")
    lat.lbm_init_equilibrium(rho, u)
    lat.lbm_step(100)
    got = lat.lbm_get_populations()
    m = O.Method(stencil, space, om)
    want = O.step(m, O.init_equilibrium(m, rho, u), 100)
    err = np.abs(got - want).max()
    print("%s %s %s 100 steps max|d df| = %.3e" % (stencil, space, kind, err))
    assert err <= 1e-12


def test_config_d2q9_central_64_taylor_green():
    """D2Q9 central moments, 64^2, u0 = 0.01, omega_s = 1.6, other rates 1, FP64: parity with
    the oracle at step 100 and over the configuration's full 1000 steps, and the velocity
    amplitude decays as exp(-2 nu k^2 t) over the 1000 steps."""
    n = 64
    om = O.regularized_rates("D2Q9", 1.6)
    rho, u = W.tgv2d_fields(n, n, 1, u0=0.01)
    lat = _lattice("D2Q9", "central", om, (n, n, 1), storage="f64")
    lat.lbm_init_equilibrium(rho, u)
    lat.lbm_step(100)
    m = O.Method("D2Q9", "central", om)
    df = O.step(m, O.init_equilibrium(m, rho, u), 100)
    assert np.abs(lat.lbm_get_populations() - df).max() <= 1e-12
    lat.lbm_step(900)
    df = O.step(m, df, 900)
    err = np.abs(lat.lbm_get_populations() - df).max()
    _, ug = lat.lbm_macroscopic()
    _, uo = O.macroscopic(m, df)
    rel = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    print("D2Q9 central 64^2 FP64, 1000 steps: max|d df| = %.3e, relative L2 velocity error %.3e" % (err, rel))
    assert err <= 1e-12
    assert rel <= 1e-10
    k = 2 * math.pi / n
    x = np.arange(n)
    ref = np.cos(k * x)[None, :] * np.sin(k * x)[:, None]
    amp = (ug[0, 0] * ref).sum() / (ref * ref).sum() / 0.01
    nu = O.omega_to_viscosity(1.6)
    want = math.exp(-2 * nu * k * k * 1000)
    assert abs(amp / want - 1) < 1e-2, (amp, want)


# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19", "D3Q27"])
@pytest.mark.parametrize("streaming", ["pull", "push", "aa", "esoteric", "twist"])
@pytest.mark.parametrize("n", [1, 2, 5])
@pytest.mark.parametrize("layout", ["planes", "rows"])
def test_streaming_index_maps_bit_exact(stencil, streaming, n, layout):
    """Identity collision: n steps of streaming equal numpy.roll bit for bit."""
    dims = RAGGED2 if stencil == "D2Q9" else RAGGED3
    q = O.stencil(stencil).q
    rng = np.random.default_rng(7)
    df = rng.integers(-1000, 1000, size=(q, dims[2], dims[1], dims[0])).astype(np.float64) / 1024.0
    lat = _lattice(stencil, "raw", _rates(stencil, "reg"), dims, storage="f32", streaming=streaming,
                   layout=layout)
    lat.lbm_set_populations(df)
    lat.lbm_debug_stream_only(n)
    got = lat.lbm_get_populations()
    m = O.Method(stencil, "raw", np.zeros(q))
    want = df
    for _ in range(n):
        want = O.stream(m, want)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("n", [3, 4])
def test_aa_equals_pull_in_both_layouts(storage, n):
    """Pull, push, AA, Esoteric Pull and Esoteric Twist, planes and rows: ten kernels sharing
    one collision, bit-equal results."""
    dims = RAGGED3
    om = _rates("D3Q27", "reg")
    rho, u = W.tgv3d_fields(*dims, u0=0.05, period=16)
    outs = []
    for streaming in ("pull", "push", "aa", "esoteric", "twist"):
        for layout in ("planes", "rows"):
            lat = _lattice("D3Q27", "cumulant", om, dims, storage=storage, streaming=streaming, layout=layout)
            lat.lbm_init_equilibrium(rho, u)
            lat.lbm_step(n)
            outs.append(lat.lbm_get_populations())
    for o in outs[1:]:
        np.testing.assert_array_equal(outs[0], o)


@pytest.mark.parametrize("streaming", ["pull", "push", "aa", "esoteric", "twist"])
def test_graph_equals_host_loop_and_checkpoint(streaming):
    dims = RAGGED3
    om = _rates("D3Q27", "gen", seed=9)
    rho, u = W.tgv3d_fields(*dims, u0=0.05, period=16)
    a = _lattice("D3Q27", "cumulant", om, dims, storage="f32", streaming=streaming)
    b = _lattice("D3Q27", "cumulant", om, dims, storage="f32", streaming=streaming)
    for lat in (a, b):
        lat.lbm_init_equilibrium(rho, u)
    a.lbm_set_graphs(True)
    b.lbm_set_graphs(False)
    a.lbm_step(7)
    b.lbm_step(7)
    pa = a.lbm_get_populations()
    np.testing.assert_array_equal(pa, b.lbm_get_populations())
    # replay the cached graph twice more, with host work in between
    a.lbm_step(7)
    _ = a.lbm_diagnostics()
    a.lbm_step(7)
    b.lbm_step(14)
    np.testing.assert_array_equal(a.lbm_get_populations(), b.lbm_get_populations())
    assert a.lbm_time() == 21
    # checkpoint / resume: restore step 7 into a fresh context and advance 14 more
    c = _lattice("D3Q27", "cumulant", om, dims, storage="f32", streaming=streaming)
    c.lbm_set_populations(pa)
    c.lbm_set_time(7)
    c.lbm_step(14)
    np.testing.assert_array_equal(c.lbm_get_populations(), a.lbm_get_populations())


def test_diagnostics_match_oracle_and_detect_nonfinite():
    dims = (20, 12, 9)
    om = _rates("D3Q27", "reg")
    rho, u = W.tgv3d_fields(*dims, u0=0.05, period=12)
    lat = _lattice("D3Q27", "cumulant", om, dims, storage="f64")
    lat.lbm_init_equilibrium(rho, u)
    lat.lbm_step(3)
    d = lat.lbm_diagnostics()
    m = O.Method("D3Q27", "cumulant", om)
    want = O.diagnostics(m, O.step(m, O.init_equilibrium(m, rho, u), 3))
    # mass is conserved exactly up to round-off: compare with the input fields themselves;
    # the oracle's dense solves in absolute populations drift by ~1e-16 per cell and step
    assert abs(d[0] - math.fsum((rho - 1.0).ravel())) <= 1e-13
    np.testing.assert_allclose(d[0], want[0], rtol=1e-11)
    np.testing.assert_allclose(d[4], want[4], rtol=1e-12)
    np.testing.assert_allclose(d[1:4], want[1:4], rtol=0, atol=1e-12)
    assert d[5] == 0
    df = lat.lbm_get_populations()
    df[3, 1, 2, 3] = np.nan
    df[0, 0, 0, 0] = np.inf
    lat.lbm_set_populations(df)
    d2 = lat.lbm_diagnostics(allow_nonfinite=True)
    assert d2[5] == 2
    with pytest.raises(lbm.LbmError):
        lat.lbm_diagnostics()


def test_fp32_velocity_error_cumulant():
    """D3Q27 cumulant, Taylor-Green u0 = 0.05, omega_s = 1.969902 (the 512^3 constants), 16^3,
    200 steps, FP32 storage and compute: relative L2 velocity error vs the FP64 oracle <= 1e-5."""
    n, steps = 16, 200
    om = O.regularized_rates("D3Q27", W.re_to_omega(0.05, 512, 1600.0))
    rho, u = W.tgv3d_fields(n, u0=0.05)
    lat = _lattice("D3Q27", "cumulant", om, (n, n, n), storage="f32")
    lat.lbm_init_equilibrium(rho, u)
    lat.lbm_step(steps)
    _, ug = lat.lbm_macroscopic()
    m = O.Method("D3Q27", "cumulant", om)
    _, uo = O.macroscopic(m, O.step(m, O.init_equilibrium(m, rho, u), steps))
    rel = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    print("FP32 cumulant 16^3 x 200: relative L2 velocity error %.3e" % rel)
    assert rel <= 1e-5


def test_swe_fp64_parity_and_fp16_error():
    """Shallow water (Zhou equilibrium, central moments), 96 x 80, g = 0.1, omega_s = 0.695652."""
    dims = (96, 80, 1)
    om = O.regularized_rates("D2Q9", 1.0 / (3 * 0.3125 + 0.5))
    h, u = W.swe_bumps(96, seed=0, sigma=(4.0, 12.0))
    h, u = h[:, :80, :], u[:, :, :80, :]
    h, u = np.ascontiguousarray(h), np.ascontiguousarray(u)
    m = O.Method("D2Q9", "central", om, equilibrium="swe", gravity=0.1)
    want = O.step(m, O.init_equilibrium(m, h, u), 100)
    lat = _lattice("D2Q9", "central", om, dims, storage="f64", equilibrium="swe", gravity=0.1)
    lat.lbm_init_equilibrium(h, u)
    lat.lbm_step(100)
    assert np.abs(lat.lbm_get_populations() - want).max() <= 1e-12
    l16 = _lattice("D2Q9", "central", om, dims, storage="f16", equilibrium="swe", gravity=0.1)
    l16.lbm_init_equilibrium(h, u)
    l16.lbm_step(100)
    h16, u16 = l16.lbm_macroscopic()
    ho, uo = O.macroscopic(m, want)
    rel = np.linalg.norm(u16[:2] - uo[:2]) / np.linalg.norm(uo[:2])
    print("SWE FP16 storage relative L2 velocity error after 100 steps: %.3e" % rel)
    assert rel <= 2e-2
    assert np.abs(h16 - ho).max() <= 2e-3


# ------------------------------------------------------------------------------------------
def test_batch_matches_single_boxes_and_oracle():
    boxes = [(16, 16, 16), (12, 12, 12), (20, 20, 20)]
    rates = [O.regularized_rates("D3Q27", w) for w in (1.9, 1.3, 1.6)]
    fields = [W.tgv3d_fields(d[0], u0=0.03 + 0.01 * k, phase=(0.1 * k, 0.2, 0.3)) for k, d in enumerate(boxes)]
    rho_cat = np.concatenate([f[0].ravel() for f in fields])
    u_cat = np.concatenate([f[1].ravel() for f in fields])
    for storage in ("f64", "f32"):
        bat = lbm.Batch("D3Q27", "central", boxes, rates, storage=storage)
        bat.lbm_batch_init_equilibrium(rho_cat, u_cat)
        bat.lbm_batch_step(5)
        got = bat.lbm_batch_get_populations()
        off = 0
        for d, om, (rho, u) in zip(boxes, rates, fields):
            lat = _lattice("D3Q27", "central", om, d, storage=storage)
            lat.lbm_init_equilibrium(rho, u)
            lat.lbm_step(5)
            single = lat.lbm_get_populations().ravel()
            mine = got[off:off + single.size]
            assert np.abs(mine - single).max() <= (1e-15 if storage == "f64" else 1e-7)
            if storage == "f64":
                m = O.Method("D3Q27", "central", om)
                want = O.step(m, O.init_equilibrium(m, rho, u), 5).ravel()
                assert np.abs(mine - want).max() <= 1e-13
            off += single.size


def test_batch_launch_shapes_and_autotune_leave_results_unchanged():
    """Every tile size, tile order and LDS reserve of the ensemble sweep gives bit-identical
    populations; the autotuner leaves the state and the step counter alone and picks one of
    the candidates; out-of-range shapes are rejected."""
    dims = [(20, 12, 9), (16, 16, 16), (9, 7, 5)]
    om = [_rates("D3Q27", "reg"), O.regularized_rates("D3Q27", 1.3), _rates("D3Q27", "gen", seed=4)]
    rhos, us = [], []
    for k, (nx, ny, nz) in enumerate(dims):
        r, u = W.random_near_equilibrium_fields((nz, ny, nx), seed=20 + k, drho=5e-3, umax=0.04)
        rhos.append(r.ravel())
        us.append(u.ravel())  # box by box, each (3, nz, ny, nx)
    rho = np.concatenate(rhos)
    u = np.concatenate(us)
    ref = None
    for threads, swz, lds in ((256, 1, 0), (128, 0, 0), (512, 1, 32768), (64, 1, 16384), (128, 1, 65536),
                              (256, 0, 53248)):
        bat = lbm.Batch("D3Q27", "central", dims, om, storage="f32")
        bat.lbm_batch_set_launch(threads, swz, lds)
        assert bat.lbm_batch_get_launch() == (threads, swz, lds)
        bat.lbm_batch_init_equilibrium(rho, u)
        bat.lbm_batch_step(3)
        got = bat.lbm_batch_get_populations()
        if ref is None:
            ref = got
        np.testing.assert_array_equal(got, ref)
    bat = lbm.Batch("D3Q27", "central", dims, om, storage="f32")
    bat.lbm_batch_init_equilibrium(rho, u)
    bat.lbm_batch_step(1)
    before = bat.lbm_batch_get_populations()
    threads, swz, lds = bat.lbm_batch_autotune()
    assert threads in (64, 128, 256, 512) and swz in (0, 1)
    assert lds in (0, 16384, 20480, 26624, 32768, 40960, 53248, 65536)
    np.testing.assert_array_equal(bat.lbm_batch_get_populations(), before)
    bat.lbm_batch_step(2)
    np.testing.assert_array_equal(bat.lbm_batch_get_populations(), ref)
    for bad in ((96, 1, 0), (1024, 1, 0), (256, 1, -1), (256, 1, 70000)):
        with pytest.raises(lbm.LbmError):
            bat.lbm_batch_set_launch(*bad)


@pytest.mark.parametrize("streaming", ["pull", "aa", "twist"])
def test_occupancy_cap_and_autotune_leave_results_unchanged(streaming):
    """The LDS reserve only limits how many blocks share a CU: every cap gives bit-identical
    populations, and the autotuner (which times the caps on each block size) keeps the state."""
    dims = (70, 9, 5)
    om = _rates("D3Q27", "reg")
    rho, u = W.random_near_equilibrium_fields(dims[::-1], seed=8, drho=5e-3, umax=0.04)
    ref = None
    for bx, by, lds in ((64, 2, 0), (64, 1, 53248), (128, 1, 65536), (256, 1, 20480)):
        lat = lbm.Lattice("D3Q27", "cumulant", om, dims, storage="f32", streaming=streaming)
        lat.lbm_set_launch(bx, by, 1)
        lat.lbm_set_lds_reserve(lds)
        assert lat.lbm_get_lds_reserve() == lds
        lat.lbm_init_equilibrium(rho, u)
        lat.lbm_step(3)
        got = lat.lbm_get_populations()
        if ref is None:
            ref = got
        np.testing.assert_array_equal(got, ref)
    lat = lbm.Lattice("D3Q27", "cumulant", om, dims, storage="f32", streaming=streaming)
    lat.lbm_init_equilibrium(rho, u)
    lat.lbm_step(1)
    before = lat.lbm_get_populations()
    lat.lbm_autotune()
    assert lat.lbm_get_lds_reserve() in (0, 16384, 20480, 26624, 32768, 40960, 53248, 65536)
    np.testing.assert_array_equal(lat.lbm_get_populations(), before)
    lat.lbm_step(2)
    np.testing.assert_array_equal(lat.lbm_get_populations(), ref)
    with pytest.raises(lbm.LbmError):
        lat.lbm_set_lds_reserve(65537)


def test_autotune_cache_round_trip(tmp_path, monkeypatch):
    """LBM_AUTOTUNE_CACHE: the first autotune writes the chosen launch under a key of the
    method, precision, pattern, layout and size; a second context of the same configuration
    takes it from the file; another configuration adds its own key and keeps the first."""
    import json
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("LBM_AUTOTUNE_CACHE", str(cache))
    dims = (70, 9, 5)
    om = _rates("D3Q27", "reg")
    rho, u = W.random_near_equilibrium_fields(dims[::-1], seed=9, drho=5e-3, umax=0.04)

    def tuned(streaming="pull", basis="graded"):
        lat = lbm.Lattice("D3Q27", "raw" if basis != "graded" else "cumulant", om, dims, storage="f32",
                          streaming=streaming, basis=basis)
        lat.lbm_init_equilibrium(rho, u)
        lat.lbm_autotune()
        return lat, list(lat.lbm_get_launch()) + [int(lat.lbm_get_vectorized()), lat.lbm_get_lds_reserve()]

    a, la = tuned()
    data = json.loads(cache.read_text())
    assert len(data) == 1 and list(data.values())[0][:5] == la
    # a hand-edited entry is what the next context of this configuration takes
    key = list(data)[0]
    edited = [64, 2, 0, 0, 26624]
    cache.write_text(json.dumps({key: edited + [1.0]}))
    b, lb = tuned()
    assert lb == edited
    a.lbm_step(3)
    b.lbm_step(3)
    np.testing.assert_array_equal(a.lbm_get_populations(), b.lbm_get_populations())
    tuned("aa")
    tuned("pull", "weighted_orthogonal")
    data = json.loads(cache.read_text())
    assert len(data) == 3 and data[key][:5] == edited
    assert any("_cross" in k for k in data)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("streaming", ["pull", "aa"])
@pytest.mark.parametrize("layout", ["planes", "rows"])
def test_vectorized_sweep_equals_per_cell_sweep(storage, streaming, layout):
    """The vectorised kernel (V cells per lane, wave-shift neighbours) gives bit-identical
    populations to the per-cell kernel, including the periodic wrap at both row ends."""
    dims = (256, 6, 5)
    om = _rates("D3Q27", "reg")
    rho, u = W.tgv3d_fields(*dims, u0=0.05, period=16)
    outs = []
    for vec in (False, True):
        lat = _lattice("D3Q27", "cumulant", om, dims, storage=storage, streaming=streaming, layout=layout)
        lat.lbm_set_launch(64, 2, 0)
        lat.lbm_set_vectorized(vec)
        assert lat.lbm_get_vectorized() == vec
        lat.lbm_init_equilibrium(rho, u)
        lat.lbm_step(3)
        outs.append(lat.lbm_get_populations())
    np.testing.assert_array_equal(outs[0], outs[1])


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19", "D3Q27"])
def test_vectorized_stream_only_bit_exact(stencil):
    dims = (256, 7, 3) if stencil != "D2Q9" else (256, 7, 1)
    q = O.stencil(stencil).q
    rng = np.random.default_rng(3)
    df = rng.integers(-1000, 1000, size=(q, dims[2], dims[1], dims[0])).astype(np.float64) / 1024.0
    lat = _lattice(stencil, "raw", _rates(stencil, "reg"), dims, storage="f32")
    lat.lbm_set_launch(64, 1, 0)
    lat.lbm_set_vectorized(True)
    lat.lbm_set_populations(df)
    lat.lbm_debug_stream_only(2)
    m = O.Method(stencil, "raw", np.zeros(q))
    np.testing.assert_array_equal(lat.lbm_get_populations(), O.stream(m, O.stream(m, df)))


def test_vectorized_fp64_matches_oracle():
    dims = (128, 5, 4)
    om = _rates("D3Q27", "gen", seed=2)
    m = O.Method("D3Q27", "cumulant", om)
    df0 = _noisy_state(m, dims, seed=4)
    lat = _lattice("D3Q27", "cumulant", om, dims, storage="f64")
    lat.lbm_set_launch(64, 1, 0)
    lat.lbm_set_vectorized(True)
    lat.lbm_set_populations(df0)
    lat.lbm_step(3)
    assert np.abs(lat.lbm_get_populations() - O.step(m, df0, 3)).max() <= 1e-13


@pytest.mark.parametrize("space", ["raw", "central", "cumulant"])
@pytest.mark.parametrize("kind", ["reg", "gen"])
def test_mfma_ablation_fp64_matches_oracle(space, kind):
    """Dense M df / M^-1 dm* on the matrix cores (ablation) against the oracle, FP64, on a
    ragged grid whose last tiles have idle lanes that still join the wave-wide products."""
    dims = RAGGED3
    om = _rates("D3Q27", kind, seed=7)
    m = O.Method("D3Q27", space, om)
    df0 = _noisy_state(m, dims, seed=13)
    lat = _lattice("D3Q27", space, om, dims, storage="f64")
    lat.lbm_set_launch(64, 4, 0)
    lat.lbm_set_transform("dense_mfma")
    assert lat.lbm_get_transform() == "dense_mfma"
    lat.lbm_set_populations(df0)
    lat.lbm_step(3)
    err = np.abs(lat.lbm_get_populations() - O.step(m, df0, 3)).max()
    print("MFMA ablation %s %s FP64: max|d df| = %.3e" % (space, kind, err))
    assert err <= 1e-13


@pytest.mark.parametrize("storage,tol", [("f32", 2e-8), ("f16", 1e-2)])
def test_mfma_ablation_close_to_chimera(storage, tol):
    dims = (128, 9, 5)
    om = _rates("D3Q27", "reg")
    rho, u = W.tgv3d_fields(*dims, u0=0.05, period=16)
    outs = []
    for tr in ("chimera", "dense_mfma"):
        lat = _lattice("D3Q27", "cumulant", om, dims, storage=storage)
        lat.lbm_set_launch(128, 2, 0)
        lat.lbm_set_transform(tr)
        lat.lbm_init_equilibrium(rho, u)
        lat.lbm_step(5)
        outs.append(lat.lbm_get_populations())
    err = np.abs(outs[0] - outs[1]).max()
    print("MFMA vs Chimera %s: max|d df| = %.3e" % (storage, err))
    assert err <= tol


@pytest.mark.parametrize("space", ["raw", "central", "cumulant"])
@pytest.mark.parametrize("streaming", ["pull", "push", "aa", "esoteric", "twist"])
def test_absolute_storage_fp64_matches_oracle(space, streaming):
    """Absolute storage (f = df + w in the buffers, eq. MrtUpdateGeneral's storage format):
    FP64 populations after 5 steps against the oracle."""
    dims = RAGGED3
    om = _rates("D3Q27", "gen", seed=8)
    m = O.Method("D3Q27", space, om)
    df0 = _noisy_state(m, dims, seed=21)
    lat = _lattice("D3Q27", space, om, dims, storage="f64", streaming=streaming, zero_centered=False)
    lat.lbm_set_populations(df0)
    lat.lbm_step(5)
    err = np.abs(lat.lbm_get_populations() - O.step(m, df0, 5)).max()
    print("absolute storage %s %s: max|d df| = %.3e" % (space, streaming, err))
    assert err <= 1e-13


def test_tgv128_fp32_and_fp64_against_the_oracle_reference():
    """The 128^3 copy of the D3Q27 cumulant Taylor-Green workload (u0 = 0.05, the 512^3 rates),
    200 steps, against the FP64 oracle's velocity and density at 4096 sampled cells
    (tests/golden/tgv128_cumulant_oracle.npz, written by make_oracle_references.py from the
    oracle alone): FP32 relative L2 velocity error <= 1e-5, FP64 <= 1e-10."""
    import os
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "tgv128_cumulant_oracle.npz"))
    n, steps, u0 = int(ref["n"]), int(ref["steps"]), float(ref["u0"])
    om = O.regularized_rates("D3Q27", W.re_to_omega(u0, 512, 1600.0))
    rho, u = W.tgv3d_fields(n, u0=u0)
    zz, yy, xx = np.meshgrid(ref["z"], ref["y"], ref["x"], indexing="ij")
    for storage, bar in (("f32", 1e-5), ("f64", 1e-10)):
        lat = _lattice("D3Q27", "cumulant", om, (n, n, n), storage=storage)
        lat.lbm_init_equilibrium(rho, u)
        lat.lbm_step(steps)
        rg, ug = lat.lbm_macroscopic()
        lat.close()
        us = ug[:, zz, yy, xx]
        rel = np.linalg.norm(us - ref["u"]) / np.linalg.norm(ref["u"])
        drho = np.abs(rg[zz, yy, xx] - ref["rho"]).max()
        print("TGV 128^3 x %d %s: relative L2 velocity error %.3e, max |d rho| %.3e" % (steps, storage, rel, drho))
        assert rel <= bar
        assert drho <= (1e-6 if storage == "f32" else 1e-12)
