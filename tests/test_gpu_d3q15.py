"""D3Q15 on the GPU (raw moments and SRT with the polynomial equilibrium, central moments and
cumulants with the Maxwellian) against the FP64 oracle, through the C ABI.

D3Q15 keeps the rest, face and corner velocities of D3Q27.  Its moment set has one monomial per
exponent-parity class of the mixed monomials (sec. 2.3); the set is closed under lowering
exponents, so the binomial shift maps it to itself, and the kernels collide on the 15
representatives and copy each representative into the rest of its class before the inverse
transform.

Bars: FP64 max |df_gpu - df_oracle| <= 1e-13 after 4 steps from a non-equilibrium state (pull,
AA, Esoteric Pull; planes and rows; with and without a body force); streaming bit-exact against
numpy.roll; FP32 within 1.5e-8 (two FP32 ulps per step at the largest deviation |df| ~ 0.02,
ulp 2^-29, over 4 steps); the Taylor-Green decay rate within 1 % of 2 nu k^2.
"""
import math

import numpy as np
import pytest

import lbm_workloads as W
import oracle as O
from paper_2211_02435_amd import lbm

pytestmark = pytest.mark.gpu

RAGGED3 = (70, 9, 5)


def _rates(space, kind):
    st = O.stencil("D3Q15")
    if space == "srt":
        om = np.full(st.q, 1.37)
        om[st.conserved] = 0.0
        return om
    if kind == "reg":
        return O.regularized_rates("D3Q15", 1.7, omega_bulk=1.2)
    rng = np.random.default_rng(3)
    om = rng.uniform(0.7, 1.9, st.q)
    om[st.conserved] = 0.0
    return om


def _noisy_state(m, dims=RAGGED3, seed=11):
    nx, ny, nz = dims
    rho, u = W.random_near_equilibrium_fields((nz, ny, nx), seed=seed, drho=5e-3, umax=0.04)
    df = O.init_equilibrium(m, rho, u)
    return df + W.random_perturbation(m.st.q, (nz, ny, nx), seed=seed + 1, scale=2e-4)


@pytest.mark.parametrize("space,kind", [("raw", "reg"), ("raw", "gen"), ("srt", "gen"), ("central", "reg"),
                                        ("central", "gen"), ("cumulant", "reg"), ("cumulant", "gen")])
@pytest.mark.parametrize("streaming", ["pull", "push", "aa", "esoteric", "twist"])
@pytest.mark.parametrize("layout", ["planes", "rows"])
def test_d3q15_sweep_fp64_matches_oracle(space, kind, streaming, layout):
    om = _rates(space, kind)
    m = O.Method("D3Q15", space, om)
    df0 = _noisy_state(m)
    lat = lbm.Lattice("D3Q15", space, om, RAGGED3, storage="f64", streaming=streaming, layout=layout)
    lat.lbm_set_populations(df0)
    lat.lbm_step(4)
    err = np.abs(lat.lbm_get_populations() - O.step(m, df0, 4)).max()
    print("D3Q15 %s %s %s %s max|d df| = %.3e" % (space, kind, streaming, layout, err))
    assert err <= 1e-13


@pytest.mark.parametrize("space", ["raw", "srt", "central", "cumulant"])
@pytest.mark.parametrize("streaming", ["pull", "esoteric", "twist"])
def test_d3q15_fp32_matches_oracle(space, streaming):
    om = _rates(space, "gen")
    m = O.Method("D3Q15", space, om)
    df0 = _noisy_state(m, seed=21)
    lat = lbm.Lattice("D3Q15", space, om, RAGGED3, storage="f32", streaming=streaming)
    lat.lbm_set_populations(df0)
    lat.lbm_step(4)
    err = np.abs(lat.lbm_get_populations() - O.step(m, df0, 4)).max()
    print("D3Q15 f32 %s %s max|d df| = %.3e" % (space, streaming, err))
    assert err <= 1.5e-8


@pytest.mark.parametrize("space", ["raw", "srt", "central", "cumulant"])
def test_d3q15_init_and_macroscopic_match_oracle(space):
    om = _rates(space, "reg")
    m = O.Method("D3Q15", space, om)
    rho, u = W.tgv3d_fields(*RAGGED3, u0=0.05, period=16)
    lat = lbm.Lattice("D3Q15", space, om, RAGGED3, storage="f64")
    lat.lbm_init_equilibrium(rho, u)
    want = O.init_equilibrium(m, rho, u)
    assert np.abs(lat.lbm_get_populations() - want).max() <= 4e-15
    rg, ug = lat.lbm_macroscopic()
    ro, uo = O.macroscopic(m, want)
    assert np.abs(rg - ro).max() <= 1e-15 and np.abs(ug - uo).max() <= 1e-15


@pytest.mark.parametrize("streaming", ["pull", "push", "aa", "esoteric", "twist"])
@pytest.mark.parametrize("n", [1, 2, 5])
@pytest.mark.parametrize("layout", ["planes", "rows"])
def test_d3q15_streaming_index_maps_bit_exact(streaming, n, layout):
    q = 15
    rng = np.random.default_rng(7)
    df = rng.integers(-1000, 1000, size=(q, RAGGED3[2], RAGGED3[1], RAGGED3[0])).astype(np.float64) / 1024.0
    lat = lbm.Lattice("D3Q15", "raw", _rates("raw", "reg"), RAGGED3, storage="f32", streaming=streaming,
                      layout=layout)
    lat.lbm_set_populations(df)
    lat.lbm_debug_stream_only(n)
    m = O.Method("D3Q15", "raw", np.zeros(q))
    want = df
    for _ in range(n):
        want = O.stream(m, want)
    np.testing.assert_array_equal(lat.lbm_get_populations(), want)


@pytest.mark.parametrize("space", ["raw", "srt", "central", "cumulant"])
@pytest.mark.parametrize("model", ["guo", "he"])
@pytest.mark.parametrize("streaming", ["pull", "aa"])
def test_d3q15_forced_fp64_matches_oracle(space, model, streaming):
    nx, ny, nz = RAGGED3
    om = _rates(space, "gen")
    m = O.Method("D3Q15", space, om, force_model=model)
    df0 = _noisy_state(m, seed=5)
    field = np.random.default_rng(7).uniform(-1e-4, 1e-4, (3, nz, ny, nx))
    const = np.array([3e-5, -2e-5, 1e-5])
    lat = lbm.Lattice("D3Q15", space, om, RAGGED3, storage="f64", streaming=streaming, force=const,
                      force_model=model)
    lat.lbm_set_force_field(field)
    lat.lbm_set_populations(df0)
    lat.lbm_step(4)
    want = O.step(m, df0, 4, force=field + const[:, None, None, None])
    err = np.abs(lat.lbm_get_populations() - want).max()
    print("D3Q15 forced (%s) %s %s max|d df| = %.3e" % (model, space, streaming, err))
    assert err <= 1e-13


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("space", ["raw", "cumulant"])
def test_d3q15_taylor_green_decay(storage, space):
    """z-invariant Taylor-Green vortex on 64 x 64 x 2 with regularized rates: the fitted decay
    rate of the velocity amplitude is 2 nu k^2 within 1 %."""
    omega = 1.1
    om = O.regularized_rates("D3Q15", omega)
    n, nz = 64, 2
    rho, u = W.tgv2d_fields(n, n, nz, u0=0.02)
    lat = lbm.Lattice("D3Q15", space, om, (n, n, nz), storage=storage)
    lat.lbm_init_equilibrium(rho, u)
    k = 2 * math.pi / n
    x = np.arange(n)
    ref = np.cos(k * x)[None, :] * np.sin(k * x)[:, None]
    amps, every = [], 100
    for i in range(9):
        if i:
            lat.lbm_step(every)
        _, uu = lat.lbm_macroscopic()
        amps.append((uu[0, 0] * ref).sum() / (ref * ref).sum())
    t = np.arange(9) * every
    rate = -np.polyfit(t[1:], np.log(amps[1:]), 1)[0]
    nu = O.omega_to_viscosity(omega)
    rel = abs(rate / (2 * nu * k * k) - 1)
    print("D3Q15 %s %s Taylor-Green decay-rate rel. error %.3e" % (space, storage, rel))
    assert rel < 1e-2
