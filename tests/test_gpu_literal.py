"""GPU parity of the SRT method and of the literal collision forms against the FP64 oracle.

SRT (population space, sec. 4.3 and 5.1) runs with the default deviation arithmetic on every
stencil.  The literal forms (LBM_ARITH_LITERAL) evaluate eq. MrtUpdateGeneral on absolute
storage, eq. MrtUpdateGeneralDeviationOnly and eq. MrtUpdateAbsoluteFromZeroCentered on
zero-centred storage as written (sec. 2.2); the oracle evaluates the same three forms.
Bar: FP64 max |df_gpu - df_oracle| <= 1e-13 after 4 steps from a non-equilibrium state.
"""
import numpy as np
import pytest

import lbm_workloads as W
import oracle as O
from paper_2211_02435_amd import lbm

pytestmark = pytest.mark.gpu

RAGGED3 = (70, 9, 5)
RAGGED2 = (70, 37, 1)


def _rates(stencil, space, kind):
    st = O.stencil(stencil)
    if space == "srt":
        om = np.full(st.q, 1.37 if kind == "gen" else 1.0)
        om[st.conserved] = 0.0
        return om
    if kind == "reg":
        return O.regularized_rates(stencil, 1.7, omega_bulk=1.2)
    rng = np.random.default_rng(3)
    om = rng.uniform(0.7, 1.9, st.q)
    om[st.conserved] = 0.0
    return om


def _noisy_state(m, dims, seed=11, noise=2e-4):
    nx, ny, nz = dims
    rho, u = W.random_near_equilibrium_fields((nz, ny, nx), seed=seed, drho=5e-3, umax=0.04)
    if m.st.d == 2:
        u[2] = 0.0
    df = O.init_equilibrium(m, rho, u)
    return df + W.random_perturbation(m.st.q, (nz, ny, nx), seed=seed + 1, scale=noise)


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19", "D3Q27"])
@pytest.mark.parametrize("streaming", ["pull", "push", "aa", "esoteric", "twist"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_srt_sweep_matches_oracle(stencil, streaming, storage):
    dims = RAGGED2 if stencil == "D2Q9" else RAGGED3
    om = _rates(stencil, "srt", "gen")
    m = O.Method(stencil, "srt", om)
    df0 = _noisy_state(m, dims)
    lat = lbm.Lattice(stencil, "srt", om, dims, storage=storage, streaming=streaming)
    lat.lbm_set_populations(df0)
    lat.lbm_step(4)
    got = lat.lbm_get_populations()
    want = O.step(m, df0, 4)
    err = np.abs(got - want).max()
    print("SRT %s %s %s max|d df| = %.3e" % (stencil, streaming, storage, err))
    assert err <= (1e-13 if storage == "f64" else 5e-9)


def test_srt_init_matches_oracle_on_d3q19():
    """D3Q19 has its own polynomial equilibrium (not M^-1 of truncated raw moments)."""
    om = _rates("D3Q19", "srt", "gen")
    rho, u = W.tgv3d_fields(*RAGGED3, u0=0.05, period=16)
    lat = lbm.Lattice("D3Q19", "srt", om, RAGGED3, storage="f64")
    lat.lbm_init_equilibrium(rho, u)
    want = O.init_equilibrium(O.Method("D3Q19", "srt", om), rho, u)
    assert np.abs(lat.lbm_get_populations() - want).max() <= 4e-15


FORMS = [(0, "default", "absolute"), (1, "delta", "delta"), (1, "absolute", "zc_absolute")]


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q27"])
@pytest.mark.parametrize("space", ["raw", "central", "cumulant", "srt"])
@pytest.mark.parametrize("zc,eq_form,oracle_form", FORMS)
@pytest.mark.parametrize("kind", ["reg", "gen"])
def test_literal_forms_fp64_match_oracle(stencil, space, zc, eq_form, oracle_form, kind):
    if space == "cumulant" and oracle_form == "delta":
        pytest.skip("no delta-equilibrium for cumulants (sec. 2.2)")
    dims = RAGGED2 if stencil == "D2Q9" else RAGGED3
    om = _rates(stencil, space, kind)
    m = O.Method(stencil, space, om)
    df0 = _noisy_state(m, dims)
    lat = lbm.Lattice(stencil, space, om, dims, storage="f64", zero_centered=bool(zc), eq_form=eq_form,
                      arithmetic="literal")
    lat.lbm_set_populations(df0)
    lat.lbm_step(4)
    got = lat.lbm_get_populations()
    if oracle_form == "absolute":
        want = O.step(m, df0 + m.f0[:, None, None, None], 4, form="absolute") - m.f0[:, None, None, None]
    else:
        want = O.step(m, df0, 4, form=oracle_form)
    err = np.abs(got - want).max()
    print("literal %s %s %s %s max|d df| = %.3e" % (stencil, space, oracle_form, kind, err))
    assert err <= 1e-13


@pytest.mark.parametrize("space,zc,eq_form", [("raw", 0, "default"), ("cumulant", 1, "absolute"),
                                              ("central", 1, "delta"), ("srt", 1, "delta")])
@pytest.mark.parametrize("storage,bar", [("f32", 1e-4), ("f16", 3e-2)])
def test_literal_low_precision_tracks_fp64(space, zc, eq_form, storage, bar):
    """FP32 and FP16-storage literal forms stay within their round-off of FP64 over 100
    Taylor-Green steps (FP16 keeps about 3 significant digits of |df| ~ 0.05)."""
    dims = (32, 32, 4)
    om = _rates("D3Q27", space, "reg") if space != "srt" else _rates("D3Q27", "srt", "gen")
    rho, u = W.tgv3d_fields(*dims, u0=0.05, period=32)
    out = {}
    for st in ("f64", storage):
        lat = lbm.Lattice("D3Q27", space, om, dims, storage=st, zero_centered=bool(zc), eq_form=eq_form,
                          arithmetic="literal")
        lat.lbm_init_equilibrium(rho, u)
        lat.lbm_step(100)
        out[st] = lat.lbm_macroscopic()[1]
    rel = np.linalg.norm(out[storage] - out["f64"]) / np.linalg.norm(out["f64"])
    print("literal %s vs FP64 %s zc=%d %s: velocity rel L2 %.2e" % (storage, space, zc, eq_form, rel))
    assert rel <= bar


def test_literal_and_deviation_agree_in_fp64():
    """Both arithmetic organisations compute the same collision; in FP64 they differ by
    round-off only."""
    dims = RAGGED3
    om = _rates("D3Q27", "cumulant", "gen")
    m = O.Method("D3Q27", "cumulant", om)
    df0 = _noisy_state(m, dims)
    outs = []
    for arith in ("deviation", "literal"):
        lat = lbm.Lattice("D3Q27", "cumulant", om, dims, storage="f64", arithmetic=arith)
        lat.lbm_set_populations(df0)
        lat.lbm_step(4)
        outs.append(lat.lbm_get_populations())
    assert np.abs(outs[0] - outs[1]).max() <= 1e-14


@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q27"])
@pytest.mark.parametrize("basis", ["weighted_orthogonal", "orthogonal"])
@pytest.mark.parametrize("zc,eq_form,oracle_form", FORMS)
def test_literal_forms_in_the_orthogonal_bases_match_oracle(stencil, basis, zc, eq_form, oracle_form):
    """The literal raw-moment forms with a weighted-orthogonal or orthogonal basis (cross-order
    relaxation blocks), general rates, FP64, against the oracle's forms."""
    dims = RAGGED2 if stencil == "D2Q9" else RAGGED3
    om = _rates(stencil, "raw", "gen")
    m = O.Method(stencil, "raw", om, basis=basis)
    df0 = _noisy_state(m, dims)
    lat = lbm.Lattice(stencil, "raw", om, dims, storage="f64", zero_centered=bool(zc), eq_form=eq_form,
                      arithmetic="literal", basis=basis)
    lat.lbm_set_populations(df0)
    lat.lbm_step(4)
    got = lat.lbm_get_populations()
    if oracle_form == "absolute":
        want = O.step(m, df0 + m.f0[:, None, None, None], 4, form="absolute") - m.f0[:, None, None, None]
    else:
        want = O.step(m, df0, 4, form=oracle_form)
    err = np.abs(got - want).max()
    print("literal %s %s %s max|d df| = %.3e" % (basis, stencil, oracle_form, err))
    assert err <= 1e-13
