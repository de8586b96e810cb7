"""The allocation-free diagnostics entry point against lbm_diagnostics, through the C ABI.

lbm_diagnostics_noalloc keeps its partial sums in a static device array shared by every call
on the GPU.  Two calls in a row, the second on a smaller box (fewer reduction blocks), must
each give lbm_diagnostics' result for their own context, with a device and with a host
destination; FP64 states also agree with the oracle's diagnostics (1e-12 relative).
"""
import ctypes

import numpy as np
import pytest

import lbm_workloads as W
import oracle as O
from paper_2211_02435_amd import lbm

pytestmark = pytest.mark.gpu


def _ctx(stencil, space, dims, storage, seed):
    om = O.regularized_rates(stencil, 1.7)
    m = O.Method(stencil, space, om)
    nx, ny, nz = dims
    rho, u = W.random_near_equilibrium_fields((nz, ny, nx), seed=seed, drho=5e-3, umax=0.04)
    df = O.init_equilibrium(m, rho, u) + W.random_perturbation(m.st.q, (nz, ny, nx), seed=seed + 1, scale=2e-4)
    lat = lbm.Lattice(stencil, space, om, dims, storage=storage)
    lat.lbm_set_populations(df)
    lat.lbm_step(3)
    return lat, m


def _noalloc_device(lat):
    import torch
    out = torch.full((6,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    st = lat.lib.lbm_diagnostics_noalloc(lat.ctx, ctypes.c_void_p(out.data_ptr()))
    assert st == 0, lbm.last_error()
    lat.lbm_synchronize()
    return out.cpu().numpy()


def _noalloc_host(lat):
    out = np.full(6, np.nan)
    st = lat.lib.lbm_diagnostics_noalloc(lat.ctx, out.ctypes.data_as(ctypes.c_void_p))
    assert st == 0, lbm.last_error()
    return out


def _close(a, b):
    scale = np.maximum(np.abs(b), 1e-300)
    return np.all((np.abs(a - b) <= 1e-12 * scale) | (np.abs(a - b) <= 1e-15))


def test_noalloc_diagnostics_match_lbm_diagnostics_on_two_calls():
    big, m_big = _ctx("D3Q27", "cumulant", (300, 40, 30), "f64", seed=3)      # 1407 blocks
    small, m_small = _ctx("D3Q19", "raw", (40, 12, 10), "f32", seed=5)        # 19 blocks
    for lat, m in ((big, m_big), (small, m_small)):
        ref = lat.lbm_diagnostics()
        dev = _noalloc_device(lat)
        host = _noalloc_host(lat)
        print("ref", ref, "device", dev, "host", host)
        assert np.array_equal(dev, ref), (dev, ref)
        assert np.array_equal(host, ref), (host, ref)
        if lat is big:
            want = O.diagnostics(m, lat.lbm_get_populations())
            assert _close(dev, want), (dev, want)
    # and the big box once more after the small one (more blocks than the last call used)
    assert np.array_equal(_noalloc_device(big), big.lbm_diagnostics())


def test_noalloc_diagnostics_report_nonfinite_populations():
    lat, m = _ctx("D3Q27", "central", (64, 8, 6), "f64", seed=7)
    df = lat.lbm_get_populations()
    df[3, 2, 4, 10] = np.nan
    df[7, 5, 1, 63] = np.inf
    lat.lbm_set_populations(df)
    dev = _noalloc_device(lat)
    assert dev[5] == 2.0
    out = np.zeros(6)
    st = lat.lib.lbm_diagnostics_noalloc(lat.ctx, out.ctypes.data_as(ctypes.c_void_p))
    assert st == lbm.LBM_ENONFINITE and out[5] == 2.0
    st = lat.lib.lbm_diagnostics_noalloc(lat.ctx, None)
    assert st == -1


def test_noalloc_diagnostics_captured_in_a_caller_graph():
    """The caller this entry point is for: a HIP graph captured (here by torch) on the
    context's stream holds the two reduction kernels; every replay, with eager sweeps, another
    context's call on the same scratch array and synchronisations in between, gives
    lbm_diagnostics' result for the current state."""
    import torch
    lat, _ = _ctx("D3Q27", "cumulant", (70, 9, 5), "f32", seed=11)
    other, _ = _ctx("D3Q19", "raw", (40, 12, 10), "f64", seed=13)
    lat.lbm_set_graphs(False)
    out = torch.full((6,), float("nan"), dtype=torch.float64, device="cuda")
    _noalloc_device(lat)          # first call on this GPU looks up the scratch array's address
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=lat._torch_stream, capture_error_mode="thread_local"):
        st = lat.lib.lbm_diagnostics_noalloc(lat.ctx, ctypes.c_void_p(out.data_ptr()))
    assert st == 0, lbm.last_error()
    for k in range(4):
        lat.lbm_step(2)
        lat.lbm_synchronize()
        _noalloc_device(other)    # the shared array now holds another context's partial sums
        g.replay()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = lat.lbm_diagnostics()
        print("replay %d: %s" % (k, got))
        assert np.array_equal(got, ref), (k, got, ref)
