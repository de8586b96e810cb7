"""Edge cases of the sweep on the GPU against the FP64 oracle, through the C ABI.

* Degenerate periodic boxes: a single cell, two cells along one axis (x - 1 and x + 1 are the
  same cell), one-cell-thick slabs, for every streaming pattern.
* The limits of the rate range: omega = 0 on every non-conserved polynomial (the collision is
  the identity) and omega = 2 (the zero-viscosity limit of eq. MrtUpdateGeneral).
* lbm_step(0) changes nothing; lbm_step rejects a negative count.

Bars: FP64 max |df_gpu - df_oracle| <= 1e-13 after 5 steps from a non-equilibrium state.
"""
import numpy as np
import pytest

import lbm_workloads as W
import oracle as O
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
