"""Pins of the oracle's collision (sec. 2.2), equilibria (sec. 2.4, 5.2), streaming
(eq. LbUpdateScheme) and hydrodynamic behaviour (Taylor-Green decay, sec. 5.1)."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import lbm_workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")

CASES = [("D2Q9", "raw"), ("D2Q9", "central"), ("D2Q9", "cumulant"),
         ("D3Q19", "raw"), ("D3Q19", "central"), ("D3Q19", "cumulant"),
         ("D3Q27", "raw"), ("D3Q27", "central"), ("D3Q27", "cumulant"),
         ("D3Q15", "raw"), ("D3Q15", "central"), ("D3Q15", "cumulant")]


def _general_rates(name, seed):
    st = O.stencil(name)
    rng = np.random.default_rng(seed)
    om = rng.uniform(0.6, 1.9, st.q)
    om[st.conserved] = 0
    return om


def _state(method, n=24, seed=0, noise=1e-3):
    st = method.st
    rng = np.random.default_rng(seed)
    rho = 1 + 0.02 * rng.standard_normal(n)
    u = rng.uniform(-0.06, 0.06, (n, 3))
    if st.d == 2:
        u[:, 2] = 0
    feq = O.equilibrium_populations(method, rho, u)
    return feq - method.f0 + noise * rng.standard_normal(feq.shape)


def _forms(space):
    return ["absolute", "zc_absolute"] + (["delta"] if space != "cumulant" else [])


@pytest.mark.parametrize("name,space", CASES)
def test_three_collision_forms_agree(name, space):
    """eq. MrtUpdateGeneral, eq. MrtUpdateGeneralDeviationOnly and eq.
    MrtUpdateAbsoluteFromZeroCentered are algebraically identical (sec. 2.2)."""
    m = O.Method(name, space, _general_rates(name, 1))
    df = _state(m)
    outs = {}
    for form in _forms(space):
        if form == "absolute":
            outs[form] = O.collide_cells(m, df + m.f0, form) - m.f0
        else:
            outs[form] = O.collide_cells(m, df, form)
    ref = outs["zc_absolute"]
    for form, v in outs.items():
        np.testing.assert_allclose(v, ref, rtol=0, atol=1e-14, err_msg=form)


def test_delta_equilibrium_rejected_for_cumulants():
    m = O.Method("D3Q27", "cumulant", _general_rates("D3Q27", 2))
    with pytest.raises(ValueError):
        O.collide_cells(m, _state(m, n=2), "delta")


@pytest.mark.parametrize("name,space", CASES)
def test_equilibrium_is_fixed_point(name, space):
    m = O.Method(name, space, _general_rates(name, 3))
    df = _state(m, noise=0.0)
    out = O.collide_cells(m, df, O.default_form(m))
    np.testing.assert_allclose(out, df, rtol=0, atol=1e-15)


@pytest.mark.parametrize("name,space", CASES)
def test_per_cell_conservation(name, space):
    m = O.Method(name, space, _general_rates(name, 4))
    st = m.st
    df = _state(m)
    out = O.collide_cells(m, df, O.default_form(m))
    np.testing.assert_allclose(out.sum(axis=1), df.sum(axis=1), rtol=0, atol=1e-15)
    xi = st.xi.astype(float)
    np.testing.assert_allclose(out @ xi, df @ xi, rtol=0, atol=1e-15)


@pytest.mark.parametrize("name,space", CASES)
def test_zero_rates_identity_unit_rates_equilibrium(name, space):
    st = O.stencil(name)
    df = None
    m0 = O.Method(name, space, np.zeros(st.q))
    df = _state(m0)
    np.testing.assert_allclose(O.collide_cells(m0, df, O.default_form(m0)), df, rtol=0, atol=1e-15)
    om1 = np.ones(st.q)
    om1[st.conserved] = 0
    m1 = O.Method(name, space, om1)
    out = O.collide_cells(m1, df, O.default_form(m1))
    rho, u = O.macroscopic_from_delta(m1, df)
    want = O.equilibrium_populations(m1, rho, u) - m1.f0
    np.testing.assert_allclose(out, want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D3Q27"])
def test_raw_equal_rates_is_bgk(name):
    """Raw moments with one rate for every polynomial reduce to the single-relaxation-time
    (BGK) operator f* = f + omega (f^eq - f) (sec. 1, SRT)."""
    st = O.stencil(name)
    om = np.full(st.q, 1.37)
    m = O.Method(name, "raw", om)
    df = _state(m)
    out = O.collide_cells(m, df, "delta")
    rho, u = O.macroscopic_from_delta(m, df)
    feq = np.linalg.solve(st.M, O.raw_maxwellian_truncated(st, rho, u).T).T
    want = df + 1.37 * (feq - m.f0 - df)
    np.testing.assert_allclose(out, want, rtol=0, atol=4e-15)


def _srt(name, omega):
    st = O.stencil(name)
    om = np.full(st.q, omega)
    om[st.conserved] = 0
    return O.Method(name, "srt", om)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q15", "D3Q19", "D3Q27"])
def test_srt_equilibrium_moments(name):
    """The polynomial equilibrium carries the Maxwellian's moments up to second order:
    sum f = rho, sum f xi = rho u, sum f xi_a xi_b = rho (cs2 delta_ab + u_a u_b)."""
    st = O.stencil(name)
    rng = np.random.default_rng(7)
    rho = 1 + 0.1 * rng.standard_normal(5)
    u = rng.uniform(-0.1, 0.1, (5, 3))
    if st.d == 2:
        u[:, 2] = 0
    feq = O.srt_equilibrium(st, rho, u)
    for n in range(5):
        m0 = sum(feq[n, i] for i in range(st.q))
        assert abs(m0 - rho[n]) < 1e-15
        for a in range(st.d):
            m1 = sum(feq[n, i] * st.xi[i, a] for i in range(st.q))
            assert abs(m1 - rho[n] * u[n, a]) < 1e-15
            for b in range(st.d):
                m2 = sum(feq[n, i] * st.xi[i, a] * st.xi[i, b] for i in range(st.q))
                want = rho[n] * ((1 / 3 if a == b else 0.0) + u[n, a] * u[n, b])
                assert abs(m2 - want) < 1e-15


@pytest.mark.parametrize("name", ["D2Q9", "D3Q15", "D3Q19", "D3Q27"])
def test_srt_forms_agree_conserve_and_relax(name):
    m = _srt(name, 1.43)
    df = _state(m)
    a = O.collide_cells(m, df + m.f0, "absolute") - m.f0
    b = O.collide_cells(m, df, "delta")
    c = O.collide_cells(m, df, "zc_absolute")
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)
    np.testing.assert_allclose(c, b, rtol=0, atol=1e-15)
    xi = m.st.xi.astype(float)
    np.testing.assert_allclose(b.sum(axis=1), df.sum(axis=1), rtol=0, atol=1e-15)
    np.testing.assert_allclose(b @ xi, df @ xi, rtol=0, atol=1e-15)
    # unit rate: the post-collision state is the equilibrium of the pre-collision moments
    m1 = _srt(name, 1.0)
    rho, u = O.macroscopic_from_delta(m1, df)
    np.testing.assert_allclose(O.collide_cells(m1, df, "delta"),
                               O.srt_equilibrium(m1.st, rho, u) - m1.f0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
def test_srt_equals_raw_moment_bgk_on_tensor_product_stencils(name):
    """On D2Q9 and D3Q27 (products of the 1-D three-velocity set) the polynomial equilibrium is
    M^-1 of the raw Maxwellian moments truncated at second order, so one SRT collision equals
    the raw-moment collision with every rate omega."""
    st = O.stencil(name)
    m = _srt(name, 1.21)
    om = np.full(st.q, 1.21)
    om[st.conserved] = 0
    raw = O.Method(name, "raw", om)
    df = _state(m)
    np.testing.assert_allclose(O.collide_cells(m, df, "delta"), O.collide_cells(raw, df, "delta"),
                               rtol=0, atol=2e-15)


def test_srt_differs_from_raw_moment_bgk_on_d3q19():
    """D3Q19 lacks the corner velocities: its polynomial equilibrium has m_xxyy =
    rho (1/9 + (ux^2 + uy^2) / 3 - uz^2 / 6), not the truncated Maxwellian's
    rho (1/9 + (ux^2 + uy^2) / 3)."""
    st = O.stencil("D3Q19")
    rho = np.array([1.0])
    u = np.array([[0.03, -0.02, 0.05]])
    feq = O.srt_equilibrium(st, rho, u)[0]
    m220 = sum(feq[i] * st.xi[i, 0] ** 2 * st.xi[i, 1] ** 2 for i in range(st.q))
    want = 1 / 9 + (0.03 ** 2 + 0.02 ** 2) / 3 - 0.05 ** 2 / 6
    assert abs(m220 - want) < 1e-16


def test_d3q15_monomial_classes_by_brute_force():
    """D3Q15 (rest, faces, corners): every monomial x^a y^b z^c (a, b, c <= 2) with two or more
    nonzero exponents takes on each velocity the value of the basis monomial with the same
    exponent parities, and the monomials of the basis are the only independent ones."""
    st = O.stencil("D3Q15")
    xi = st.xi.astype(float)

    def row(e):
        return np.array([xi[i, 0] ** e[0] * xi[i, 1] ** e[1] * xi[i, 2] ** e[2] for i in range(st.q)])

    reps = [e for e in st.exps if sum(1 for k in e if k) >= 2]
    assert len(reps) == 8
    for a in range(3):
        for b in range(3):
            for c in range(3):
                e = (a, b, c)
                if sum(1 for k in e if k) < 2:
                    continue
                par = tuple(k % 2 for k in e)
                same = [r for r in reps if tuple(k % 2 for k in r) == par]
                assert len(same) == 1, e
                np.testing.assert_array_equal(row(e), row(same[0]))
    assert np.linalg.matrix_rank(st.M) == 15


def test_d3q15_polynomial_equilibrium_fourth_moment():
    """On D3Q15 only the corners carry x^2 y^2; summing the second-order polynomial equilibrium
    over them by hand gives m_xxyy = rho (1/9 + |u|^2 / 3), the same for xx zz and yy zz."""
    st = O.stencil("D3Q15")
    rho = np.array([1.02])
    u = np.array([[0.03, -0.02, 0.05]])
    feq = O.srt_equilibrium(st, rho, u)[0]
    want = 1.02 * (1 / 9 + (0.03 ** 2 + 0.02 ** 2 + 0.05 ** 2) / 3)
    for a, b in ((0, 1), (0, 2), (1, 2)):
        mom = sum(feq[i] * st.xi[i, a] ** 2 * st.xi[i, b] ** 2 for i in range(st.q))
        assert abs(mom - want) < 1e-16


def test_d3q15_central_equilibrium_carries_the_maxwellian_on_each_representative():
    """D3Q15 in central-moment space: the equilibrium populations have the Maxwellian's raw
    moments on the 15 representative monomials, e.g. sum f xi_x^2 xi_y^2 =
    rho (1/9 + (ux^2 + uy^2)/3 + ux^2 uy^2) and sum f xi_x^2 xi_z = rho uz (1/3 + ux^2)
    (moments of the continuous Maxwellian, worked out by hand); the other members of a class
    follow the representative, so x^2 z^2 takes the x^2 y^2 value."""
    st = O.stencil("D3Q15")
    m = O.Method("D3Q15", "central", O.regularized_rates("D3Q15", 1.3))
    rho = np.array([1.03])
    ux, uy, uz = 0.04, -0.03, 0.02
    feq = O.equilibrium_populations(m, rho, np.array([[ux, uy, uz]]))[0]
    xi = st.xi.astype(float)
    mom = lambda a, b, c: (feq * xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c).sum()
    want22 = 1.03 * (1 / 9 + (ux * ux + uy * uy) / 3 + ux * ux * uy * uy)
    assert abs(mom(2, 2, 0) - want22) < 4e-16
    assert abs(mom(2, 0, 2) - want22) < 4e-16
    assert abs(mom(2, 0, 1) - 1.03 * uz * (1 / 3 + ux * ux)) < 4e-16
    assert abs(mom(2, 0, 0) - 1.03 * (1 / 3 + ux * ux)) < 4e-16


def test_d3q15_raw_moment_bgk_equals_srt():
    """The raw-moment collision on D3Q15 with one rate on every non-conserved polynomial
    equals the population-space BGK collision with that rate."""
    st = O.stencil("D3Q15")
    om = np.full(st.q, 1.31)
    om[st.conserved] = 0
    raw = O.Method("D3Q15", "raw", om)
    m = _srt("D3Q15", 1.31)
    df = _state(m)
    for form in ("delta", "zc_absolute"):
        np.testing.assert_allclose(O.collide_cells(raw, df, form), O.collide_cells(m, df, "delta"),
                                   rtol=0, atol=2e-15)


def test_worked_propagation_example():
    """sec. 4.3: without a force the post-collision first-order raw moment is rho u_x."""
    m = O.Method("D3Q27", "central", _general_rates("D3Q27", 5))
    df = _state(m)
    rho, u = O.macroscopic_from_delta(m, df)
    out = O.collide_cells(m, df, "delta")
    mx = (out + m.f0) @ m.st.xi[:, 0].astype(float)
    np.testing.assert_allclose(mx, rho * u[:, 0], rtol=0, atol=1e-15)


def test_regularized_cumulant_higher_orders_at_equilibrium():
    """With every rate of order >= 3 equal to 1 the post-collision cumulants of order >= 3
    vanish (their Maxwellian values), sec. 4.3."""
    st = O.stencil("D3Q27")
    m = O.Method("D3Q27", "cumulant", O.regularized_rates("D3Q27", 1.8))
    df = _state(m)
    out = O.collide_cells(m, df, "zc_absolute") + m.f0
    rho = out.sum(axis=1)
    u = (out @ st.xi.astype(float)) / rho[:, None]
    kap = np.einsum("nji,ni->nj", O.central_matrix(st, u), out)
    C = O.cumulants_from_central(st, kap, rho, u)
    hi = [j for j, e in enumerate(st.exps) if sum(e) >= 3]
    np.testing.assert_allclose(C[:, hi], 0, atol=1e-15)


# ---------------------------------------------------------------- shallow water (sec. 5.2)
def test_swe_equilibrium_moments_and_typo_reading():
    st = O.stencil("D2Q9")
    rng = np.random.default_rng(7)
    n, g = 10, 0.1
    h = 1 + 0.2 * rng.random(n)
    u = np.zeros((n, 3))
    u[:, :2] = rng.uniform(-0.1, 0.1, (n, 2))
    f = O.swe_equilibrium(st, h, u, g)
    xi = st.xi.astype(float)
    np.testing.assert_allclose(f.sum(axis=1), h, atol=1e-15)
    np.testing.assert_allclose(f @ xi[:, :2], h[:, None] * u[:, :2], atol=1e-15)
    for a in range(2):
        for b in range(2):
            s = (f * xi[:, a] * xi[:, b]).sum(axis=1)
            want = g * h * h / 2 * (a == b) + h * u[:, a] * u[:, b]
            np.testing.assert_allclose(s, want, atol=1e-15)
    # the printed equation's -u.u/3 in f_i (i > 0) loses mass: sum f = h (1 - 5 u.u / 6)
    uu = (u * u).sum(axis=1)
    lam = np.where(np.abs(st.xi).sum(axis=1) == 1, 1.0, 0.25)
    f_typo = f.copy()
    f_typo[:, 1:] -= lam[None, 1:] * h[:, None] * uu[:, None] / 6
    np.testing.assert_allclose(f_typo.sum(axis=1), h * (1 - 5 * uu / 6), atol=1e-15)


def test_swe_lake_at_rest_is_fixed_point():
    om = O.regularized_rates("D2Q9", 0.7)
    m = O.Method("D2Q9", "central", om, equilibrium="swe", gravity=0.1)
    h = np.full((1, 6, 5), 1.3)
    u = np.zeros((3, 1, 6, 5))
    df = O.init_equilibrium(m, h, u)
    out = O.step(m, df, 3)
    np.testing.assert_allclose(out, df, rtol=0, atol=1e-15)


def _swek(space, omega=0.7, g=0.1):
    return O.Method("D2Q9", space, O.regularized_rates("D2Q9", omega), equilibrium="swe_maxwellian", gravity=g)


@pytest.mark.parametrize("space", ["central", "cumulant"])
def test_swe_maxwellian_equilibrium_moments(space):
    """Venturi's equilibrium (continuous Maxwellian, c^2 = g h / 2) carries the shallow-water
    fluxes: sum f = h, sum f xi = h u, sum f xi_a xi_b = g h^2 / 2 delta_ab + h u_a u_b, and
    factorises over the axes: h f(ix, iy) = fx(ix) fy(iy)."""
    g = 0.153
    m = _swek(space, g=g)
    st = m.st
    rng = np.random.default_rng(5)
    h = 0.5 + 2 * rng.random(6)
    u = np.zeros((6, 3))
    u[:, :2] = rng.uniform(-0.08, 0.08, (6, 2))
    f = O.equilibrium_populations(m, h, u)
    for n in range(6):
        assert abs(sum(f[n, i] for i in range(9)) - h[n]) < 1e-15
        for a in range(2):
            assert abs(sum(f[n, i] * st.xi[i, a] for i in range(9)) - h[n] * u[n, a]) < 1e-15
            for b in range(2):
                got = sum(f[n, i] * st.xi[i, a] * st.xi[i, b] for i in range(9))
                want = (0.5 * g * h[n] ** 2 if a == b else 0.0) + h[n] * u[n, a] * u[n, b]
                assert abs(got - want) < 1e-14
        tab = {(int(st.xi[i, 0]), int(st.xi[i, 1])): f[n, i] for i in range(9)}
        fx = {a: sum(tab[(a, b)] for b in (-1, 0, 1)) for a in (-1, 0, 1)}
        fy = {b: sum(tab[(a, b)] for a in (-1, 0, 1)) for b in (-1, 0, 1)}
        for (a, b), v in tab.items():
            assert abs(h[n] * v - fx[a] * fy[b]) < 1e-15


def test_swe_maxwellian_central_and_cumulant_equilibria_agree():
    m1, m2 = _swek("central"), _swek("cumulant")
    rng = np.random.default_rng(6)
    h = 1 + 0.3 * rng.random(4)
    u = np.zeros((4, 3))
    u[:, :2] = rng.uniform(-0.05, 0.05, (4, 2))
    np.testing.assert_allclose(O.equilibrium_populations(m1, h, u), O.equilibrium_populations(m2, h, u),
                               rtol=0, atol=1e-15)
    np.testing.assert_allclose(m1.f0, m2.f0, rtol=0, atol=1e-16)


@pytest.mark.parametrize("space", ["central", "cumulant"])
def test_swe_maxwellian_lake_at_rest_and_conservation(space):
    m = _swek(space)
    h = np.full((1, 6, 5), 1.3)
    df = O.init_equilibrium(m, h, np.zeros((3, 1, 6, 5)))
    np.testing.assert_allclose(O.step(m, df, 3), df, rtol=0, atol=1e-15)
    cells = _state(m)
    out = O.collide_cells(m, cells, "zc_absolute")
    xi = m.st.xi.astype(float)
    np.testing.assert_allclose(out.sum(axis=1), cells.sum(axis=1), rtol=0, atol=1e-15)
    np.testing.assert_allclose(out @ xi, cells @ xi, rtol=0, atol=1e-15)


def test_dam_break_rate_golden():
    g = json.load(open(GOLDEN))["dam_break_rate"]
    dx = g["domain_m"] / g["cells"]
    nu_lattice = g["nu_m2_per_s"] * g["dt_s"] / dx ** 2
    om = O.viscosity_to_omega(nu_lattice)
    assert round(om, g["printed_digits"]) == g["omega_s_approx"]
    v = json.load(open(GOLDEN))["viscosity_relation"]
    assert abs(O.viscosity_to_omega(v["nu"]) - v["omega"]) < 1e-15


# ---------------------------------------------------------------- streaming (eq. LbUpdateScheme)
@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
def test_streaming_moves_impulse_by_xi(name):
    m = O.Method(name, "raw", np.zeros(O.stencil(name).q))
    st = m.st
    shape = (5, 4, 3) if st.d == 3 else (1, 4, 3)
    for i in range(st.q):
        f = np.zeros((st.q,) + shape)
        f[i, 0, 1, 2] = 1.0
        g = O.stream(m, f)
        z = (0 + st.xi[i, 2]) % shape[0]
        y = (1 + st.xi[i, 1]) % shape[1]
        x = (2 + st.xi[i, 0]) % shape[2]
        assert g[i, z, y, x] == 1.0 and g.sum() == 1.0


def test_pure_streaming_returns_after_period():
    """All rates 0: the collision is the identity up to the round-off of T^-1 T, and N steps
    of periodic streaming on an N^3 box restore the initial state."""
    name = "D3Q27"
    m = O.Method(name, "central", np.zeros(27))
    rng = np.random.default_rng(8)
    df0 = 1e-3 * rng.standard_normal((27, 6, 6, 6))
    out = O.step(m, df0, 6)
    np.testing.assert_allclose(out, df0, rtol=0, atol=1e-15)


# ---------------------------------------------------------------- hydrodynamics (sec. 5.1)
def _tgv_amplitude(method, n, nz, u0, steps, every):
    rho, u = W.tgv2d_fields(n, n, nz, u0=u0)
    df = O.init_equilibrium(method, rho, u)
    k = 2 * math.pi / n
    x = np.arange(n)
    ref = np.cos(k * x)[None, :] * np.sin(k * x)[:, None]
    amps = []
    for t in range(0, steps + 1, every):
        _, uu = O.macroscopic(method, df)
        amps.append((uu[0, 0] * ref).sum() / (ref * ref).sum())
        if t < steps:
            df = O.step(method, df, every)
    return np.array(amps)


@pytest.mark.parametrize("space", ["raw", "central", "cumulant"])
def test_taylor_green_decay_rate_d2q9(space):
    """u(t) = u0 exp(-2 nu k^2 t) (eq. TGA_init) with nu = c_s^2 (1/omega - 1/2); the fitted
    rate on a 32^2 box at low Mach number is within 0.5 % of 2 nu k^2."""
    omega = 1.2
    om = O.regularized_rates("D2Q9", omega)
    m = O.Method("D2Q9", space, om)
    n, steps, every = 32, 200, 20
    amps = _tgv_amplitude(m, n, 1, 1e-3, steps, every)
    nu = O.omega_to_viscosity(omega)
    k = 2 * math.pi / n
    t = np.arange(0, steps + 1, every)
    rate = -np.polyfit(t[2:], np.log(amps[2:]), 1)[0]
    assert abs(rate / (2 * nu * k * k) - 1) < 5e-3


def test_taylor_green_second_order_convergence():
    """The relative decay-rate error falls about fourfold per doubling of the resolution."""
    omega = 1.2
    m = O.Method("D2Q9", "central", O.regularized_rates("D2Q9", omega))
    nu = O.omega_to_viscosity(omega)
    errs = []
    for n in (16, 32):
        steps = int(round(0.2 * n * n / (4 * math.pi ** 2 * nu)))  # same diffusive time
        every = max(1, steps // 10)
        amps = _tgv_amplitude(m, n, 1, 1e-3, every * 10, every)
        k = 2 * math.pi / n
        t = np.arange(0, every * 10 + 1, every)
        rate = -np.polyfit(t[2:], np.log(amps[2:]), 1)[0]
        errs.append(abs(rate / (2 * nu * k * k) - 1))
    ratio = errs[0] / errs[1]
    assert 3.0 < ratio < 5.5, (errs, ratio)


def test_taylor_green_energy_decay_d3q27_cumulant():
    """z-invariant Taylor-Green vortex on a D3Q27 cumulant box (32 x 32 x 1): the fitted
    decay rate of E follows 4 nu k^2 (E/E0 = exp(-4 nu k^2 t), sec. 5.1) within 1 %;
    mass and momentum stay at their initial values."""
    omega = 1.0
    m = O.Method("D3Q27", "cumulant", O.regularized_rates("D3Q27", omega))
    n = 32
    rho, u = W.tgv2d_fields(n, n, 1, u0=1e-3)
    df = O.init_equilibrium(m, rho, u)
    d0 = O.diagnostics(m, df)
    nu = O.omega_to_viscosity(omega)
    k = 2 * math.pi / n
    every = 2
    energies = [d0[4]]
    for _ in range(9):
        df = O.step(m, df, every)
        energies.append(O.diagnostics(m, df)[4])
    t = np.arange(10) * every
    rate = -np.polyfit(t[1:], np.log(energies[1:]), 1)[0]
    assert abs(rate / (4 * nu * k * k) - 1) < 1e-2
    d = O.diagnostics(m, df)
    assert abs(d[0] - d0[0]) < 1e-11 and np.abs(d[1:4] - d0[1:4]).max() < 1e-12


def test_taylor_green_decay_d3q15_raw():
    """z-invariant Taylor-Green vortex on D3Q15 with regularized raw-moment rates: the decay
    rate of the velocity amplitude is 2 nu k^2 within 1 %."""
    omega = 1.1
    m = O.Method("D3Q15", "raw", O.regularized_rates("D3Q15", omega))
    n = 32
    amps = _tgv_amplitude(m, n, 1, 1e-3, 160, 20)
    nu = O.omega_to_viscosity(omega)
    k = 2 * math.pi / n
    t = np.arange(0, 161, 20)
    rate = -np.polyfit(t[2:], np.log(amps[2:]), 1)[0]
    assert abs(rate / (2 * nu * k * k) - 1) < 1e-2


@pytest.mark.parametrize("space", ["central", "cumulant"])
def test_taylor_green_decay_d3q15_central_and_cumulant(space):
    """z-invariant Taylor-Green vortex on D3Q15 with regularized central-moment and cumulant
    rates: the decay rate is 2 nu k^2 within 1 %."""
    omega = 1.1
    m = O.Method("D3Q15", space, O.regularized_rates("D3Q15", omega))
    n = 32
    amps = _tgv_amplitude(m, n, 1, 1e-3, 160, 20)
    nu = O.omega_to_viscosity(omega)
    k = 2 * math.pi / n
    t = np.arange(0, 161, 20)
    rate = -np.polyfit(t[2:], np.log(amps[2:]), 1)[0]
    assert abs(rate / (2 * nu * k * k) - 1) < 1e-2


# ---------------------------------------------------------------- body force (Guo's model)
FORCE_CASES = [("D2Q9", "raw"), ("D2Q9", "cumulant"), ("D3Q19", "central"), ("D3Q27", "raw"),
               ("D3Q27", "central"), ("D3Q27", "cumulant"), ("D3Q27", "srt")]


@pytest.mark.parametrize("model", ["guo", "he"])
@pytest.mark.parametrize("name,space", FORCE_CASES)
def test_force_adds_exactly_F_of_momentum(name, space, model):
    st = O.stencil(name)
    if space == "srt":
        om = np.full(st.q, 1.3)
        om[st.conserved] = 0
    else:
        om = _general_rates(name, 9)
    m = O.Method(name, space, om, force_model=model)
    df = _state(m)
    rng = np.random.default_rng(4)
    F = rng.uniform(-1e-3, 1e-3, (df.shape[0], 3))
    if st.d == 2:
        F[:, 2] = 0
    xi = st.xi.astype(float)
    for form in _forms(space):
        fin = df + m.f0 if form == "absolute" else df
        out = O.collide_cells(m, fin, form, F)
        np.testing.assert_allclose(out.sum(axis=1), fin.sum(axis=1), rtol=0, atol=2e-15)
        np.testing.assert_allclose(out @ xi - fin @ xi, F, rtol=0, atol=2e-15)
        if form != "absolute":
            ref = O.collide_cells(m, df, O.default_form(m), F)
            np.testing.assert_allclose(out, ref, rtol=0, atol=1e-14, err_msg=form)


def test_uniform_force_accelerates_uniformly():
    """A uniform state under a uniform force: u (Guo's velocity) grows by F / rho per step."""
    m = O.Method("D3Q27", "cumulant", O.regularized_rates("D3Q27", 1.3))
    rho = np.full((2, 3, 4), 1.02)
    u = np.zeros((3, 2, 3, 4))
    u[0] = 0.01
    F = np.array([2e-4, -1e-4, 5e-5])
    df = O.init_equilibrium(m, rho, u)
    # the initial state has j = rho u, so Guo's velocity (j + F/2) / rho starts at u + F / (2 rho)
    for t in range(1, 6):
        df = O.step(m, df, 1, force=F)
        r, uu = O.macroscopic(m, df, force=F)
        want = np.array([0.01, 0.0, 0.0]) + F * t / 1.02 + 0.5 * F / 1.02
        np.testing.assert_allclose(uu.reshape(3, -1).T, np.broadcast_to(want, (24, 3)), rtol=0, atol=1e-15)


def test_he_source_moments():
    """He's source carries no mass and exactly F of momentum, and its second moment is
    u F + F u up to the lattice's O(u^2 F) defect of the equilibrium's third moments (the
    Hermite expansion of -F . grad_xi f_eq), on every stencil."""
    for name in ("D2Q9", "D3Q19", "D3Q27"):
        st = O.stencil(name)
        m = O.Method(name, "central", O.regularized_rates(name, 1.2), force_model="he")
        rng = np.random.default_rng(3)
        rho = 1 + 0.05 * rng.standard_normal(4)
        u = rng.uniform(-0.05, 0.05, (4, 3))
        F = rng.uniform(-1e-3, 1e-3, (4, 3))
        if st.d == 2:
            u[:, 2] = 0
            F[:, 2] = 0
        S = O.he_source(st, u, F, rho, O.equilibrium_populations(m, rho, u))
        xi = st.xi.astype(float)
        np.testing.assert_allclose(S.sum(axis=1), 0, atol=1e-18)
        np.testing.assert_allclose(S @ xi, F, rtol=0, atol=1e-17)
        for a in range(st.d):
            for b in range(st.d):
                got = (S * xi[None, :, a] * xi[None, :, b]).sum(axis=1)
                tol = 3 * np.abs(u).max() ** 2 * np.abs(F).max()
                np.testing.assert_allclose(got, u[:, a] * F[:, b] + F[:, a] * u[:, b], rtol=0, atol=tol)


@pytest.mark.parametrize("model", ["guo", "he"])
@pytest.mark.parametrize("space", ["raw", "central", "cumulant"])
def test_kolmogorov_flow_amplitude_second_order(space, model):
    """Steady shear flow under F_x = F0 sin(k y): nu u'' + F = 0 gives u_x = F0 / (nu k^2) sin(k y).
    Guo's model reproduces the amplitude with an error that falls as k^2 (sec. 2.1 source term)."""
    om = O.regularized_rates("D2Q9", 0.8)
    nu = O.omega_to_viscosity(0.8)
    F0 = 1e-5
    errs = []
    for n, steps in ((12, 250), (24, 900)):
        k = 2 * math.pi / n
        y = np.arange(n)
        F = np.zeros((3, 1, n, n))
        F[0] = F0 * np.sin(k * y)[None, :, None]
        m = O.Method("D2Q9", space, om, force_model=model)
        df = O.init_equilibrium(m, np.ones((1, n, n)), np.zeros((3, 1, n, n)))
        df = O.step(m, df, steps, force=F)
        _, u = O.macroscopic(m, df, force=F)
        amp = 2.0 / n * (u[0, 0, :, 0] * np.sin(k * y)).sum()  # projection on sin(k y)
        errs.append(abs(amp / (F0 / (nu * k * k)) - 1.0))
    assert errs[1] < 0.01
    assert 3.0 < errs[0] / errs[1] < 5.0


# ---------------------------------------------------------------- weighted-orthogonal raw basis
def _poly_values(st, P):
    """Values of the polynomials (rows of P over st.exps) at every velocity, by brute force."""
    xi = st.xi.astype(float)
    vals = np.zeros((P.shape[0], st.q))
    for r in range(P.shape[0]):
        for j, (a, b, c) in enumerate(st.exps):
            if P[r, j] != 0.0:
                vals[r] += P[r, j] * xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c
    return vals


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D3Q27"])
def test_wo_basis_orthogonal_and_triangular(name):
    """Every pair of WO polynomials is orthogonal under sum_i w_i a(xi_i) b(xi_i), and each is
    its graded polynomial plus a combination of the earlier graded ones."""
    st = O.stencil(name)
    Pw = O.weighted_orthogonal_matrix(st)
    v = _poly_values(st, Pw)
    G = (v * st.w[None, :]) @ v.T
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() < 1e-15
    T = np.linalg.solve(st.P.T, Pw.T).T  # Pw = T P
    np.testing.assert_allclose(np.diag(T), 1.0, rtol=0, atol=1e-14)
    assert np.abs(np.triu(T, 1)).max() < 1e-14


def _coeffs(st, terms):
    out = np.zeros(st.q)
    for c, e in terms:
        out[st.eidx[e]] += c
    return out


def test_wo_basis_d2q9_hermite_products():
    """On D2Q9 the weighted-orthogonal polynomials of orders 3 and 4 are the products of the
    one-dimensional ones 1, x, x^2 - 1/3 (textbook WO-MRT): x (y^2 - 1/3) and
    (x^2 - 1/3)(y^2 - 1/3); the trace becomes x^2 + y^2 - 2/3."""
    st = O.stencil("D2Q9")
    Pw = O.weighted_orthogonal_matrix(st)
    names = O.BASIS_NAMES["D2Q9"]
    want = {
        "x2+y2": [(1, (2, 0, 0)), (1, (0, 2, 0)), (-2 / 3, (0, 0, 0))],
        "xy2": [(1, (1, 2, 0)), (-1 / 3, (1, 0, 0))],
        "x2y": [(1, (2, 1, 0)), (-1 / 3, (0, 1, 0))],
        "x2y2": [(1, (2, 2, 0)), (-1 / 3, (2, 0, 0)), (-1 / 3, (0, 2, 0)), (1 / 9, (0, 0, 0))],
    }
    for nm, terms in want.items():
        np.testing.assert_allclose(Pw[names.index(nm)], _coeffs(st, terms), rtol=0, atol=1e-15, err_msg=nm)


def test_wo_basis_d3q27_top_polynomial_and_trace():
    """On D3Q27 (a product lattice) the last WO polynomial is (x^2-1/3)(y^2-1/3)(z^2-1/3) and
    the trace is x^2 + y^2 + z^2 - 1."""
    st = O.stencil("D3Q27")
    Pw = O.weighted_orthogonal_matrix(st)
    t = 1 / 3
    top = [(1, (2, 2, 2)), (-t, (2, 2, 0)), (-t, (2, 0, 2)), (-t, (0, 2, 2)),
           (t * t, (2, 0, 0)), (t * t, (0, 2, 0)), (t * t, (0, 0, 2)), (-t ** 3, (0, 0, 0))]
    np.testing.assert_allclose(Pw[-1], _coeffs(st, top), rtol=0, atol=1e-15)
    k = O.BASIS_NAMES["D3Q27"].index("x2+y2+z2")
    np.testing.assert_allclose(Pw[k], _coeffs(st, [(1, (2, 0, 0)), (1, (0, 2, 0)), (1, (0, 0, 2)),
                                                   (-1, (0, 0, 0))]), rtol=0, atol=1e-15)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D3Q27"])
def test_wo_mrt_unit_rates_basis_independent_and_shear_rate_not(name):
    """With every rate 1 the collision sets each non-conserved moment to equilibrium whatever
    the basis.  With the regularized rates (shear 1.7, the rest 1) the 3-D WO bases differ
    from the graded ones: their deviatoric fourth-order polynomials are not orthogonal to the
    shear polynomials before Gram-Schmidt (on D3Q27 <x2y2 - 2x2z2 + y2z2, x2 - y2>_w = -2/9),
    so they pick up shear parts and the shear deviation reaches the fourth-order moments.
    D2Q9's one fourth-order polynomial is isotropic and picks up only the trace, whose rate is
    1, so there R-WO-MRT equals R-MRT.  Mass, momentum and the equilibrium are kept."""
    st = O.stencil(name)
    ones = np.ones(st.q)
    g1, w1 = O.Method(name, "raw", ones), O.Method(name, "raw", ones, basis="weighted_orthogonal")
    df = _state(g1)
    np.testing.assert_allclose(O.collide_cells(w1, df, "delta"), O.collide_cells(g1, df, "delta"),
                               rtol=0, atol=1e-15)
    om = O.regularized_rates(name, 1.7)
    g, w = O.Method(name, "raw", om), O.Method(name, "raw", om, basis="weighted_orthogonal")
    a, b = O.collide_cells(g, df, "delta"), O.collide_cells(w, df, "delta")
    if name == "D2Q9":
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)
    else:
        assert np.abs(a - b).max() > 1e-7
    xi = st.xi.astype(float)
    np.testing.assert_allclose(b.sum(axis=1), df.sum(axis=1), rtol=0, atol=1e-15)
    np.testing.assert_allclose(b @ xi, df @ xi, rtol=0, atol=1e-15)
    for form in ("absolute", "zc_absolute"):
        c = O.collide_cells(w, df + w.f0, form) - w.f0 if form == "absolute" else O.collide_cells(w, df, form)
        np.testing.assert_allclose(c, b, rtol=0, atol=1e-14)
    eq = _state(w, noise=0.0)
    np.testing.assert_allclose(O.collide_cells(w, eq, "delta"), eq, rtol=0, atol=4e-15)


def test_taylor_green_decay_rate_wo_mrt():
    """R-WO-MRT keeps the shear viscosity: the D2Q9 decay rate is 2 nu k^2 within 0.5 %."""
    omega = 1.2
    m = O.Method("D2Q9", "raw", O.regularized_rates("D2Q9", omega), basis="weighted_orthogonal")
    n, steps, every = 32, 200, 20
    amps = _tgv_amplitude(m, n, 1, 1e-3, steps, every)
    nu = O.omega_to_viscosity(omega)
    k = 2 * math.pi / n
    t = np.arange(0, steps + 1, every)
    rate = -np.polyfit(t[2:], np.log(amps[2:]), 1)[0]
    assert abs(rate / (2 * nu * k * k) - 1) < 5e-3


def test_o_mrt_basis_is_lallemand_luo_on_d2q9():
    """Without weights (O-MRT) the Gram-Schmidt of the graded D2Q9 basis gives the classical
    polynomials of Lallemand and Luo: energy 3(x^2 + y^2) - 4, energy flux 3 x y^2 - 2 x and
    3 x^2 y - 2 y, and 9 x^2 y^2 - 6 (x^2 + y^2) + 4 (each divided by its leading coefficient),
    mutually orthogonal under the plain sum over the nine velocities."""
    st = O.stencil("D2Q9")
    Po = O.weighted_orthogonal_matrix(st, weighted=False)
    names = O.BASIS_NAMES["D2Q9"]
    want = {
        "x2+y2": [(1, (2, 0, 0)), (1, (0, 2, 0)), (-4 / 3, (0, 0, 0))],
        "xy2": [(1, (1, 2, 0)), (-2 / 3, (1, 0, 0))],
        "x2y": [(1, (2, 1, 0)), (-2 / 3, (0, 1, 0))],
        "x2y2": [(1, (2, 2, 0)), (-2 / 3, (2, 0, 0)), (-2 / 3, (0, 2, 0)), (4 / 9, (0, 0, 0))],
    }
    for nm, terms in want.items():
        np.testing.assert_allclose(Po[names.index(nm)], _coeffs(st, terms), rtol=0, atol=1e-15, err_msg=nm)
    v = _poly_values(st, Po)
    off = v @ v.T - np.diag(np.diag(v @ v.T))
    assert np.abs(off).max() < 1e-14


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D3Q27"])
def test_o_mrt_collision_invariants(name):
    """O-MRT: unit rates give the graded result, regularized rates keep mass, momentum and the
    equilibrium, and the three forms agree."""
    st = O.stencil(name)
    ones = np.ones(st.q)
    g1, o1 = O.Method(name, "raw", ones), O.Method(name, "raw", ones, basis="orthogonal")
    df = _state(g1)
    np.testing.assert_allclose(O.collide_cells(o1, df, "delta"), O.collide_cells(g1, df, "delta"),
                               rtol=0, atol=1e-15)
    o = O.Method(name, "raw", O.regularized_rates(name, 1.7, omega_bulk=1.3), basis="orthogonal")
    b = O.collide_cells(o, df, "delta")
    xi = st.xi.astype(float)
    np.testing.assert_allclose(b.sum(axis=1), df.sum(axis=1), rtol=0, atol=1e-15)
    np.testing.assert_allclose(b @ xi, df @ xi, rtol=0, atol=1e-15)
    np.testing.assert_allclose(O.collide_cells(o, df + o.f0, "absolute") - o.f0, b, rtol=0, atol=1e-14)
    eq = _state(o, noise=0.0)
    np.testing.assert_allclose(O.collide_cells(o, eq, "delta"), eq, rtol=0, atol=4e-15)
