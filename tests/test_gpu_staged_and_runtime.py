"""The LDS-staged pull sweep and runtime paths, on the GPU, through the C ABI.

* The LDS-staged pull kernel (global-to-LDS loads of the gathered row segments) gives the
  register kernel's results bit for bit, and FP64 agrees with the oracle to 1e-13 after 5
  steps, for several tiles per row, one tile per row (both neighbours wrap into the same
  tile), ragged y and z, every stencil and storage type.  The same for the AA pattern with
  the LDS-shifted odd step.
* Time loops longer than one recorded graph (chunks of 256 steps) give the eager loop's
  results bit for bit, also for many distinct step counts (graph cache eviction).
* Autotuning a context that runs the MFMA ablation keeps the MFMA kernel and its results.
* Caller buffers that are not device memory are rejected; the D2Q9 velocity's z-component is
  zeroed by the host path of lbm_macroscopic.
"""
import numpy as np
import pytest

import lbm_workloads as W
import oracle as O
from paper_2211_02435_amd import lbm

pytestmark = pytest.mark.gpu


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


CASES = [("D3Q27", "cumulant", "reg"), ("D3Q27", "central", "gen"), ("D3Q27", "raw", "reg"),
         ("D3Q19", "raw", "reg"), ("D3Q19", "cumulant", "gen"), ("D3Q15", "central", "reg"),
         ("D2Q9", "central", "gen")]


@pytest.mark.parametrize("stencil,space,kind", CASES)
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("tw,nx", [(128, 384), (256, 256)])
def test_staged_sweep_matches_register_kernel_and_oracle(stencil, space, kind, storage, tw, nx):
    dims = (nx, 5, 3) if stencil != "D2Q9" else (nx, 7, 1)
    om = O.regularized_rates(stencil, 1.7, omega_bulk=1.2) if kind == "reg" else _general(stencil)
    m = O.Method(stencil, space, om)
    df0 = _state(m, dims)
    out = {}
    for staged in (False, True):
        lat = lbm.Lattice(stencil, space, om, dims, storage=storage)
        lat.lbm_set_launch(tw, 1, 1)
        if staged:
            lat.lbm_set_staged(True)
        assert lat.lbm_get_staged() == staged
        lat.lbm_set_populations(df0)
        lat.lbm_step(5)
        out[staged] = lat.lbm_get_populations()
        lat.close()
    assert np.array_equal(out[True], out[False]), np.abs(out[True] - out[False]).max()
    if storage == "f64":
        err = np.abs(out[True] - O.step(m, df0, 5)).max()
        print("%s %s %s staged tw %d: max|d df| vs oracle %.3e" % (stencil, space, kind, tw, err))
        assert err <= 1e-13


@pytest.mark.parametrize("stencil,space,kind", CASES)
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("bx,by,nx,ny", [(128, 1, 256, 5), (64, 4, 128, 7), (256, 1, 256, 3)])
def test_aa_shifted_odd_step_matches_per_cell_kernel_and_oracle(stencil, space, kind, storage, bx, by, nx, ny):
    """AA with the LDS-shifted odd step: bit-identical to the per-cell kernel over an odd and an
    even number of steps (both row ends wrap; ragged rows when ny % by != 0)."""
    dims = (nx, ny, 3) if stencil != "D2Q9" else (nx, ny, 1)
    om = O.regularized_rates(stencil, 1.7, omega_bulk=1.2) if kind == "reg" else _general(stencil)
    m = O.Method(stencil, space, om)
    df0 = _state(m, dims, seed=5)
    for steps in (3, 4):
        out = {}
        for staged in (False, True):
            lat = lbm.Lattice(stencil, space, om, dims, storage=storage, streaming="aa")
            lat.lbm_set_launch(bx, by, 1)
            lat.lbm_set_staged(staged)
            assert lat.lbm_get_staged() == staged
            lat.lbm_set_populations(df0)
            lat.lbm_step(steps)
            out[staged] = lat.lbm_get_populations()
            lat.close()
        assert np.array_equal(out[True], out[False]), np.abs(out[True] - out[False]).max()
        if storage == "f64":
            err = np.abs(out[True] - O.step(m, df0, steps)).max()
            assert err <= 1e-13, err


@pytest.mark.parametrize("stencil,space", [("D3Q27", "cumulant"), ("D2Q9", "central")])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("streaming", ["pull", "aa"])
def test_lds_variants_in_the_planes_layout(stencil, space, storage, streaming):
    """Both LDS variants with one population plane per population (padded plane stride)."""
    dims = (256, 6, 3) if stencil != "D2Q9" else (256, 9, 1)
    om = O.regularized_rates(stencil, 1.7, omega_bulk=1.2)
    m = O.Method(stencil, space, om)
    df0 = _state(m, dims, seed=8)
    out = {}
    for staged in (False, True):
        lat = lbm.Lattice(stencil, space, om, dims, storage=storage, streaming=streaming, layout="planes")
        assert lat.lbm_get_layout() == "planes"
        lat.lbm_set_launch(128, 1, 1)
        lat.lbm_set_staged(staged)
        lat.lbm_set_populations(df0)
        lat.lbm_step(5)
        out[staged] = lat.lbm_get_populations()
        lat.close()
    assert np.array_equal(out[True], out[False])
    if storage == "f64":
        assert np.abs(out[True] - O.step(m, df0, 5)).max() <= 1e-13


def test_staged_shallow_water_and_stream_only():
    om = O.regularized_rates("D2Q9", 0.695652)
    h, u = W.swe_bumps(256, seed=0)
    m = O.Method("D2Q9", "central", om, equilibrium="swe", gravity=0.1)
    for storage in ("f64", "f16"):
        res = []
        for staged in (False, True):
            lat = lbm.Lattice("D2Q9", "central", om, (256, 256, 1), storage=storage, equilibrium="swe", gravity=0.1)
            lat.lbm_set_launch(256, 1, 0)
            lat.lbm_set_staged(staged)
            lat.lbm_init_equilibrium(h, u)
            lat.lbm_step(7)
            res.append(lat.lbm_get_populations())
        assert np.array_equal(res[0], res[1])
        if storage == "f64":
            assert np.abs(res[1] - O.step(m, O.init_equilibrium(m, h, u), 7)).max() <= 1e-13
    # streaming only through the staged kernel: bit-exact index maps
    dims = (256, 3, 4)
    om = O.regularized_rates("D3Q27", 1.5)
    df0 = np.random.default_rng(9).standard_normal((27, 4, 3, 256))
    lat = lbm.Lattice("D3Q27", "cumulant", om, dims, storage="f64")
    lat.lbm_set_launch(256, 1, 1)
    lat.lbm_set_staged(True)
    lat.lbm_set_populations(df0)
    lat.lbm_debug_stream_only(3)
    want = df0
    mm = O.Method("D3Q27", "cumulant", om)
    for _ in range(3):
        want = O.stream(mm, want)
    assert np.array_equal(lat.lbm_get_populations(), want)


def test_aa_shifted_stream_only_bit_exact():
    dims = (128, 5, 3)
    om = O.regularized_rates("D3Q27", 1.5)
    df0 = np.random.default_rng(10).standard_normal((27, 3, 5, 128))
    lat = lbm.Lattice("D3Q27", "cumulant", om, dims, storage="f64", streaming="aa")
    lat.lbm_set_launch(64, 2, 1)
    lat.lbm_set_staged(True)
    lat.lbm_set_populations(df0)
    lat.lbm_debug_stream_only(3)
    mm = O.Method("D3Q27", "cumulant", om)
    want = df0
    for _ in range(3):
        want = O.stream(mm, want)
    assert np.array_equal(lat.lbm_get_populations(), want)


def test_staged_rejects_shapes_it_cannot_run():
    om = O.regularized_rates("D3Q27", 1.5)
    lat = lbm.Lattice("D3Q27", "cumulant", om, (200, 4, 4), storage="f32")
    lat.lbm_set_launch(128, 1, 0)
    with pytest.raises(lbm.LbmError) as e:
        lat.lbm_set_staged(True)  # nx not a multiple of the tile
    assert e.value.status == -2
    lat = lbm.Lattice("D3Q27", "cumulant", om, (256, 4, 4), storage="f32")
    lat.lbm_set_launch(128, 2, 0)
    with pytest.raises(lbm.LbmError):
        lat.lbm_set_staged(True)  # two rows per block
    lat.lbm_set_launch(256, 1, 0)
    lat.lbm_set_staged(True)
    lat.lbm_set_launch(128, 2, 0)  # another shape turns it off
    assert not lat.lbm_get_staged()
    for streaming in ("push", "esoteric", "twist"):  # no LDS variant for these patterns
        lat = lbm.Lattice("D3Q27", "cumulant", om, (256, 4, 4), storage="f32", streaming=streaming)
        lat.lbm_set_launch(256, 1, 0)
        with pytest.raises(lbm.LbmError):
            lat.lbm_set_staged(True)
    lat = lbm.Lattice("D3Q27", "cumulant", om, (256, 4, 4), storage="f32", streaming="aa")
    lat.lbm_set_launch(256, 2, 0)
    with pytest.raises(lbm.LbmError):
        lat.lbm_set_staged(True)  # more than 256 threads


@pytest.mark.parametrize("streaming", ["pull", "aa"])
def test_long_graph_loops_match_the_eager_loop(streaming):
    dims = (24, 6, 5)
    om = _general("D3Q27", seed=2)
    m = O.Method("D3Q27", "central", om)
    df0 = _state(m, dims, seed=7)
    res = []
    for graphs in (False, True):
        lat = lbm.Lattice("D3Q27", "central", om, dims, storage="f32", streaming=streaming)
        lat.lbm_set_graphs(graphs)
        lat.lbm_set_populations(df0)
        lat.lbm_graph_prepare(601)
        lat.lbm_step(601)           # two 256-step chunks, a remainder graph of 89 steps
        for n in range(2, 14):      # twelve more distinct lengths: the graph cache evicts
            lat.lbm_step(n)
        assert lat.lbm_time() == 601 + sum(range(2, 14))
        res.append(lat.lbm_get_populations())
    assert np.array_equal(res[0], res[1])


def test_batch_long_graph_loop_matches_the_eager_loop():
    boxes = [(16, 16, 16), (12, 12, 12)]
    rates = [O.regularized_rates("D3Q27", w) for w in (1.9, 1.3)]
    fields = [W.tgv3d_fields(d[0], u0=0.03) for d in boxes]
    rho = np.concatenate([f[0].ravel() for f in fields])
    u = np.concatenate([f[1].ravel() for f in fields])
    res = []
    for graphs in (False, True):
        bat = lbm.Batch("D3Q27", "central", boxes, rates, storage="f32")
        bat.lbm_batch_set_graphs(graphs)
        bat.lbm_batch_init_equilibrium(rho, u)
        bat.lbm_batch_step(300)
        for n in range(2, 12):
            bat.lbm_batch_step(n)
        res.append(bat.lbm_batch_get_populations())
    assert np.array_equal(res[0], res[1])


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_batch_persistent_grid_matches_one_block_per_tile(storage):
    """The persistent ensemble grid (resident blocks striding over the tile list) gives the
    one-block-per-tile results bit for bit, in both tile orders, for grids smaller and larger
    than the tile list, and FP64 agrees with the oracle."""
    boxes = [(16, 16, 16), (12, 12, 12), (20, 20, 20), (9, 7, 5)]
    rates = [O.regularized_rates("D3Q27", w) for w in (1.9, 1.3, 1.6, 1.75)]
    fields = [W.tgv3d_fields(d[0], d[1], d[2], u0=0.03 + 0.005 * k, phase=(0.1 * k, 0.2, 0.3))
              for k, d in enumerate(boxes)]
    rho = np.concatenate([f[0].ravel() for f in fields])
    u = np.concatenate([f[1].ravel() for f in fields])
    ref = None
    for threads, swz, lds, pers in [(256, 1, 0, 0), (256, 1, 0, 1), (64, 0, 65536, 1), (128, 1, 32768, 1),
                                    (512, 0, 0, 1)]:
        bat = lbm.Batch("D3Q27", "central", boxes, rates, storage=storage)
        bat.lbm_batch_set_launch(threads, swz, lds)
        bat.lbm_batch_set_persistent(pers)
        assert bat.lbm_batch_get_persistent() == bool(pers)
        bat.lbm_batch_init_equilibrium(rho, u)
        bat.lbm_batch_step(7)
        got = bat.lbm_batch_get_populations()
        if ref is None:
            ref = got
        else:
            assert np.array_equal(got, ref), (threads, swz, lds, pers)
    if storage == "f64":
        off = 0
        for d, om, (r, v) in zip(boxes, rates, fields):
            m = O.Method("D3Q27", "central", om)
            want = O.step(m, O.init_equilibrium(m, r, v), 7).ravel()
            assert np.abs(ref[off:off + want.size] - want).max() <= 1e-13
            off += want.size


def test_autotune_keeps_the_mfma_ablation():
    dims = (64, 8, 6)
    om = O.regularized_rates("D3Q27", 1.8)
    m = O.Method("D3Q27", "cumulant", om)
    df0 = _state(m, dims, seed=11)
    lat = lbm.Lattice("D3Q27", "cumulant", om, dims, storage="f64")
    lat.lbm_set_launch(64, 4, 0)
    lat.lbm_set_transform("dense_mfma")
    lat.lbm_set_populations(df0)
    lat.lbm_autotune()
    bx, by, _ = lat.lbm_get_launch()
    print("MFMA autotuned launch", bx, by)
    assert bx * by <= 256
    assert lat.lbm_get_transform() == "dense_mfma"
    assert lat.lbm_time() == 0
    lat.lbm_step(5)
    assert np.abs(lat.lbm_get_populations() - O.step(m, df0, 5)).max() <= 1e-13


def test_host_memory_is_rejected_as_a_caller_buffer():
    om = O.regularized_rates("D3Q27", 1.5)
    p = lbm.make_params("D3Q27", "cumulant", om, (8, 8, 8), "f32")
    need = lbm.lbm_required_bytes(p)
    host = np.zeros(need, dtype=np.uint8)
    p.buffers[0] = host.ctypes.data
    p.buffers[1] = host.ctypes.data
    p.buffer_bytes = need
    import ctypes
    ctx = ctypes.c_void_p()
    lib = lbm.load()
    st = lib.lbm_create(ctypes.byref(p), ctypes.byref(ctx))
    assert st == -1 and not ctx.value
    assert b"not device memory" in lib.lbm_last_error()


def test_d2q9_macroscopic_zeroes_the_z_velocity_on_the_host_path():
    rho, u = W.tgv2d_fields(32, 32, 1, u0=0.02)
    om = O.regularized_rates("D2Q9", 1.6)
    lat = lbm.Lattice("D2Q9", "central", om, (32, 32, 1), storage="f64")
    lat.lbm_init_equilibrium(rho, u)
    lat.lbm_step(3)
    r = np.empty((1, 32, 32))
    v = np.full((3, 1, 32, 32), np.nan)
    lbm.check(lat.lib.lbm_macroscopic(lat.ctx, lbm._dptr(r), lbm._dptr(v)))
    assert np.all(v[2] == 0.0)
    assert np.all(np.isfinite(v))


def test_contexts_stepped_from_two_host_threads_match_sequential_runs():
    """Two contexts (different stencils, spaces and streaming patterns, each on its own stream)
    stepped at the same time from two host threads, each capturing and replaying its own
    graphs, give bit for bit the states of the same runs made one after the other."""
    import threading
    specs = [("D3Q27", "cumulant", "pull", (70, 9, 5), 3), ("D3Q19", "raw", "aa", (40, 12, 10), 4)]

    def make(spec):
        stencil, space, streaming, dims, seed = spec
        om = _general(stencil, seed=seed)
        m = O.Method(stencil, space, om)
        lat = lbm.Lattice(stencil, space, om, dims, storage="f32", streaming=streaming)
        lat.lbm_set_populations(_state(m, dims, seed=seed))
        return lat

    ref = []
    for spec in specs:
        lat = make(spec)
        lat.lbm_step(300)
        ref.append(lat.lbm_get_populations())
        lat.close()
    lats = [make(spec) for spec in specs]
    errors = []

    def run(lat):
        try:
            for _ in range(6):
                lat.lbm_step(50)
            lat.lbm_synchronize()
        except Exception as e:  # reported in the main thread
            errors.append(e)

    threads = [threading.Thread(target=run, args=(lat,)) for lat in lats]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
    for lat, want in zip(lats, ref):
        assert lat.lbm_time() == 300
        np.testing.assert_array_equal(lat.lbm_get_populations(), want)
        lat.close()
