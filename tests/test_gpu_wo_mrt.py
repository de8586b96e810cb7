"""Raw-moment MRT in the weighted-orthogonal (WO-MRT) and the non-weighted orthogonal (O-MRT)
bases (sec. 2.3.1) on the GPU against the FP64 oracle, through the C ABI.

The orthogonal polynomials mix orders, so the relaxation carries the deviations of orders 2 and 3 into
orders 4, 5 and 6 (cross-order blocks applied beside the per-order ones).

Bars: FP64 max |df_gpu - df_oracle| <= 1e-13 after 4 steps from a non-equilibrium state (general
and regularized rates, pull / push / AA / Esoteric Pull / Esoteric Twist); with every rate 1 the WO and
graded runs agree bit for bit (same kernel, no cross term); the FP32 run stays within 1.5e-8 of
the oracle (two FP32 ulps per step at |df| ~ 0.02 over 4 steps).
"""
import numpy as np
import pytest

import lbm_workloads as W
import oracle as O
from paper_2211_02435_amd import lbm

pytestmark = pytest.mark.gpu

RAGGED3 = (70, 9, 5)
RAGGED2 = (70, 37, 1)


def _rates(stencil, kind):
    if kind == "reg":
        return O.regularized_rates(stencil, 1.7)
    rng = np.random.default_rng(3)
    om = rng.uniform(0.7, 1.9, O.stencil(stencil).q)
    om[O.stencil(stencil).conserved] = 0.0
    return om


def _noisy_state(m, dims, seed=11):
    nx, ny, nz = dims
    rho, u = W.random_near_equilibrium_fields((nz, ny, nx), seed=seed, drho=5e-3, umax=0.04)
    if m.st.d == 2:
        u[2] = 0.0
    df = O.init_equilibrium(m, rho, u)
    return df + W.random_perturbation(m.st.q, (nz, ny, nx), seed=seed + 1, scale=2e-4)


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19", "D3Q27"])
@pytest.mark.parametrize("kind", ["reg", "gen"])
@pytest.mark.parametrize("streaming", ["pull", "push", "aa", "esoteric", "twist"])
@pytest.mark.parametrize("basis", ["weighted_orthogonal", "orthogonal"])
def test_wo_mrt_fp64_matches_oracle(stencil, kind, streaming, basis):
    dims = RAGGED2 if stencil == "D2Q9" else RAGGED3
    om = _rates(stencil, kind)
    m = O.Method(stencil, "raw", om, basis=basis)
    df0 = _noisy_state(m, dims)
    lat = lbm.Lattice(stencil, "raw", om, dims, storage="f64", streaming=streaming, basis=basis)
    lat.lbm_set_populations(df0)
    lat.lbm_step(4)
    err = np.abs(lat.lbm_get_populations() - O.step(m, df0, 4)).max()
    print("%s %s %s %s max|d df| = %.3e" % (basis, stencil, kind, streaming, err))
    assert err <= 1e-13


def test_wo_mrt_differs_from_graded_where_the_oracle_says():
    """R-WO-MRT and R-MRT differ on D3Q27 (the deviatoric quartics carry shear parts) by what
    the oracle predicts, and agree on D2Q9."""
    for stencil, dims in (("D3Q27", RAGGED3), ("D2Q9", RAGGED2)):
        om = _rates(stencil, "reg")
        df0 = _noisy_state(O.Method(stencil, "raw", om), dims)
        got, want = {}, {}
        for basis in ("graded", "weighted_orthogonal"):
            lat = lbm.Lattice(stencil, "raw", om, dims, storage="f64", basis=basis)
            lat.lbm_set_populations(df0)
            lat.lbm_step(3)
            got[basis] = lat.lbm_get_populations()
            want[basis] = O.step(O.Method(stencil, "raw", om, basis=basis), df0, 3)
        d_gpu = got["weighted_orthogonal"] - got["graded"]
        d_orc = want["weighted_orthogonal"] - want["graded"]
        print("%s: max |WO - graded| gpu %.3e oracle %.3e" % (stencil, np.abs(d_gpu).max(), np.abs(d_orc).max()))
        assert np.abs(d_gpu - d_orc).max() <= 1e-13
        if stencil == "D3Q27":
            assert np.abs(d_orc).max() > 1e-8
        else:
            assert np.abs(d_orc).max() <= 1e-15


def test_wo_mrt_unit_rates_equal_graded_bit_for_bit():
    om = np.ones(27)
    rho, u = W.tgv3d_fields(*RAGGED3, u0=0.05, period=16)
    outs = []
    for basis in ("graded", "weighted_orthogonal"):
        lat = lbm.Lattice("D3Q27", "raw", om, RAGGED3, storage="f32", basis=basis)
        lat.lbm_init_equilibrium(rho, u)
        lat.lbm_step(5)
        outs.append(lat.lbm_get_populations())
    np.testing.assert_array_equal(outs[0], outs[1])


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q27"])
def test_wo_mrt_fp32_matches_oracle(stencil):
    dims = RAGGED2 if stencil == "D2Q9" else RAGGED3
    om = _rates(stencil, "gen")
    m = O.Method(stencil, "raw", om, basis="weighted_orthogonal")
    df0 = _noisy_state(m, dims, seed=21)
    lat = lbm.Lattice(stencil, "raw", om, dims, storage="f32", basis="weighted_orthogonal")
    lat.lbm_set_populations(df0)
    lat.lbm_step(4)
    err = np.abs(lat.lbm_get_populations() - O.step(m, df0, 4)).max()
    print("WO-MRT f32 %s max|d df| = %.3e" % (stencil, err))
    assert err <= 1.5e-8


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19", "D3Q27"])
@pytest.mark.parametrize("basis", ["weighted_orthogonal", "orthogonal"])
@pytest.mark.parametrize("model", ["guo", "he"])
@pytest.mark.parametrize("streaming", ["pull", "aa"])
def test_orthogonal_bases_with_a_body_force_match_the_oracle(stencil, basis, model, streaming):
    """With a force the first-order deviations are -F/2, so the blocks from order 1 into
    orders 3 and 5 act in the relaxation and in the weighting (I + B)/2 of the source."""
    dims = RAGGED2 if stencil == "D2Q9" else RAGGED3
    nx, ny, nz = dims
    om = _rates(stencil, "gen")
    m = O.Method(stencil, "raw", om, basis=basis, force_model=model)
    df0 = _noisy_state(m, dims, seed=31)
    field = np.random.default_rng(7).uniform(-1e-4, 1e-4, (3, nz, ny, nx))
    const = np.array([3e-5, -2e-5, 1e-5])
    if m.st.d == 2:
        field[2] = 0.0
        const[2] = 0.0
    lat = lbm.Lattice(stencil, "raw", om, dims, storage="f64", streaming=streaming, basis=basis, force=const,
                      force_model=model)
    lat.lbm_set_force_field(field)
    lat.lbm_set_populations(df0)
    lat.lbm_step(4)
    want = O.step(m, df0, 4, force=field + const[:, None, None, None])
    err = np.abs(lat.lbm_get_populations() - want).max()
    print("forced %s %s %s %s max|d df| = %.3e" % (basis, model, stencil, streaming, err))
    assert err <= 1e-13
