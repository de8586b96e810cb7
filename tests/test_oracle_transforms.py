"""Pins of the oracle's lattice, moment, central-moment and cumulant definitions.

Each test checks the oracle against something other than itself: textbook closed forms,
the binomial relation of sec. 4.2 evaluated independently, SymPy differentiation of the
cumulant-generating function of sec. 2.3.3, exact arithmetic on dyadic inputs.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")
STENCILS = ["D2Q9", "D3Q15", "D3Q19", "D3Q27"]


@pytest.mark.parametrize("name", STENCILS)
def test_stencil_structure(name):
    st = O.stencil(name)
    assert st.q == int(name[-2:] if name != "D2Q9" else 9)
    assert tuple(st.xi[0]) == (0, 0, 0)  # xi_0 = 0 (sec. 2.1)
    assert len({tuple(v) for v in st.xi}) == st.q
    np.testing.assert_array_equal(st.xi[st.opp], -st.xi)
    if name == "D3Q19":
        assert (np.abs(st.xi).sum(axis=1) <= 2).all()
    if name == "D3Q15":  # rest, the six faces and the eight corners
        assert sorted(np.abs(st.xi).sum(axis=1).tolist()) == [0] + [1] * 6 + [3] * 8


@pytest.mark.parametrize("name", STENCILS)
def test_weights_isotropy(name):
    """Textbook lattice isotropy: sum w = 1, sum w xi_a xi_b = c_s^2 delta_ab,
    sum w xi_a^2 xi_b^2 = c_s^4 (a != b), sum w xi_a^4 = 3 c_s^4, odd moments vanish."""
    st = O.stencil(name)
    w, xi = st.w, st.xi.astype(float)
    d = st.d
    assert abs(w.sum() - 1) < 1e-15
    for a in range(d):
        assert abs((w * xi[:, a]).sum()) < 1e-16
        assert abs((w * xi[:, a] ** 4).sum() - 3 * O.CS2 ** 2) < 1e-15
        for b in range(d):
            s2 = (w * xi[:, a] * xi[:, b]).sum()
            assert abs(s2 - (O.CS2 if a == b else 0.0)) < 1e-15
            if a != b:
                assert abs((w * xi[:, a] ** 2 * xi[:, b] ** 2).sum() - O.CS2 ** 2) < 1e-15


@pytest.mark.parametrize("name", STENCILS)
def test_background_is_weights(name):
    """sec. 2.4: f0 = M^-1 m0 reduces to the lattice weights for the hydrodynamic equilibrium."""
    st = O.stencil(name)
    f0 = np.linalg.solve(st.M, O.background_moments(st))
    np.testing.assert_allclose(f0, st.w, rtol=0, atol=1e-15)


def test_moment_matrix_tensor_factorisation():
    """D3Q27: M is the threefold Kronecker product of the 1-D matrix rows
    (1, 1, 1), (-1, 0, 1), (1, 0, 1) acting on velocities (-1, 0, 1)."""
    st = O.stencil("D3Q27")
    one_d = {0: {-1: 1, 0: 1, 1: 1}, 1: {-1: -1, 0: 0, 1: 1}, 2: {-1: 1, 0: 0, 1: 1}}
    for j, e in enumerate(st.exps):
        for i in range(st.q):
            v = one_d[e[0]][st.xi[i, 0]] * one_d[e[1]][st.xi[i, 1]] * one_d[e[2]][st.xi[i, 2]]
            assert st.M[j, i] == v


@pytest.mark.parametrize("name", STENCILS)
def test_basis_invertible_and_graded(name):
    st = O.stencil(name)
    assert abs(np.linalg.det(st.P)) > 1e-6
    for p, poly in enumerate(st.basis):
        orders = {sum(e) for e in poly}
        assert len(orders) == 1, "every basis polynomial is homogeneous in one order"
    assert len(O.BASIS_NAMES[name]) == st.q


def test_d2q9_basis_matches_listing():
    """The D2Q9 basis is the one of the shallow-water listing (sec. 5.2)."""
    import sympy as sp
    g = json.load(open(GOLDEN))["swe_listing_basis"]
    x, y = sp.symbols("x y")
    st = O.stencil("D2Q9")
    for text, poly in zip(g["polys"], st.basis):
        expr = sp.expand(sp.sympify(text, locals={"x": x, "y": y}))
        mine = sum(c * x ** e[0] * y ** e[1] for e, c in poly.items())
        assert sp.simplify(expr - mine) == 0
    om = O.regularized_rates("D2Q9", omega_shear=0.7)
    want = [0, 0, 0, 0.7, 0.7, 1, 1, 1, 1]
    np.testing.assert_array_equal(om, want)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
def test_truncated_raw_equilibrium_is_textbook(name):
    """On D2Q9 and D3Q27, M^-1 of the second-order truncated Maxwellian moments is the
    textbook polynomial equilibrium w rho (1 + 3 xi.u + 9/2 (xi.u)^2 - 3/2 u.u)."""
    st = O.stencil(name)
    rng = np.random.default_rng(1)
    n = 16
    rho = 1 + 0.05 * rng.standard_normal(n)
    u = rng.uniform(-0.1, 0.1, size=(n, 3))
    if st.d == 2:
        u[:, 2] = 0
    m = O.raw_maxwellian_truncated(st, rho, u)
    f = np.linalg.solve(st.M, m.T).T
    xu = u @ st.xi.T.astype(float)
    uu = (u * u).sum(axis=1)[:, None]
    want = st.w[None, :] * rho[:, None] * (1 + 3 * xu + 4.5 * xu ** 2 - 1.5 * uu)
    np.testing.assert_allclose(f, want, rtol=0, atol=1e-15)


def test_d3q19_truncated_equilibrium_reading():
    """Reading: on D3Q19 the truncated Maxwellian moments are used as stated in sec. 4.3;
    they differ from the standard polynomial D3Q19 equilibrium only in the three fourth-order
    moments, by terms of second order in u (the standard equilibrium is not what the
    paper's default equilibrium produces)."""
    st = O.stencil("D3Q19")
    rho = np.array([1.02])
    u = np.array([[0.03, -0.02, 0.05]])
    m = O.raw_maxwellian_truncated(st, rho, u)
    xu = u @ st.xi.T.astype(float)
    uu = (u * u).sum(axis=1)[:, None]
    poly = st.w[None, :] * rho[:, None] * (1 + 3 * xu + 4.5 * xu ** 2 - 1.5 * uu)
    diff = (poly @ st.M.T - m)[0]
    for j, e in enumerate(st.exps):
        if sum(e) < 4:
            assert abs(diff[j]) < 1e-16, e
    d4 = {st.exps[j]: diff[j] for j in range(st.q) if sum(st.exps[j]) == 4}
    # m_{x^2 y^2} of the polynomial equilibrium lacks the u_z^2 contribution: -rho u_z^2 / 6
    assert abs(d4[(2, 2, 0)] - (-rho[0] * u[0, 2] ** 2 / 6)) < 1e-16
    assert abs(d4[(2, 0, 2)] - (-rho[0] * u[0, 1] ** 2 / 6)) < 1e-16
    assert abs(d4[(0, 2, 2)] - (-rho[0] * u[0, 0] ** 2 / 6)) < 1e-16


@pytest.mark.parametrize("name", STENCILS)
def test_central_matrix_matches_binomial_relation_exactly(name):
    """eq. RawToCentralMomentsBinomial, evaluated with explicit binomial coefficients on the
    raw moments, equals the oracle's K(u) f bit for bit on dyadic inputs (all products and
    sums are exact in FP64), and K(0) = M."""
    st = O.stencil(name)
    rng = np.random.default_rng(2)
    n = 8
    f = rng.integers(-8, 9, size=(n, st.q)).astype(float)
    u = rng.integers(-4, 5, size=(n, 3)) / 16.0
    if st.d == 2:
        u[:, 2] = 0
    kappa = np.einsum("nji,ni->nj", O.central_matrix(st, u), f)
    m = f @ st.M.T
    for j, (al, be, ga) in enumerate(st.exps):
        acc = np.zeros(n)
        for a in range(al + 1):
            for b in range(be + 1):
                for c in range(ga + 1):
                    coef = math.comb(al, a) * math.comb(be, b) * math.comb(ga, c)
                    acc = acc + coef * (-u[:, 0]) ** (al - a) * (-u[:, 1]) ** (be - b) \
                        * (-u[:, 2]) ** (ga - c) * m[:, st.eidx[(a, b, c)]]
        np.testing.assert_array_equal(kappa[:, j], acc)
    np.testing.assert_array_equal(O.central_matrix(st, np.zeros((1, 3)))[0], st.M)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19"])
def test_cumulants_match_sympy_log_mgf(name):
    """The set-partition cumulants equal SymPy's derivatives of log M at zero (sec. 2.3.3)."""
    import sympy as sp
    st = O.stencil(name)
    rng = np.random.default_rng(3)
    f_rat = [Fraction(int(v), 64) for v in rng.integers(1, 40, size=st.q)]
    # make sure every needed lower-order derivative is cached by walking orders upward
    X = sp.symbols("X0 X1 X2")
    Mgf = sum(sp.Rational(fi.numerator, fi.denominator)
              * sp.exp(sum(X[d] * int(st.xi[i, d]) for d in range(3))) for i, fi in enumerate(f_rat))
    logM = sp.log(Mgf)
    rho_r = sum(f_rat)
    f = np.array([float(v) for v in f_rat])[None, :]
    rho = f.sum(axis=1)
    u = (f @ st.xi.astype(float)) / rho[:, None]
    kappa = np.einsum("nji,ni->nj", O.central_matrix(st, u), f)
    C = O.cumulants_from_central(st, kappa, rho, u)[0]
    zero = {X[0]: 0, X[1]: 0, X[2]: 0}
    for j, e in enumerate(st.exps):
        if sum(e) < 2:
            continue
        dexpr = sp.diff(logM, *[a for d in range(3) for a in [X[d]] * e[d]])
        want = float(sp.Rational(rho_r.numerator, rho_r.denominator) * dexpr.subs(zero))
        assert abs(C[j] - want) <= 1e-13 * max(1.0, abs(want)), (e, C[j], want)


def test_cumulants_match_sympy_log_mgf_d3q27_selected():
    """D3Q27: the nonlinear fourth-, fifth- and sixth-order cumulants (the expensive ones of
    sec. 4.3) equal SymPy's derivatives of log M."""
    import sympy as sp
    st = O.stencil("D3Q27")
    rng = np.random.default_rng(4)
    f_rat = [Fraction(int(v), 128) for v in rng.integers(1, 50, size=st.q)]
    X = sp.symbols("X0 X1 X2")
    Mgf = sum(sp.Rational(fi.numerator, fi.denominator)
              * sp.exp(sum(X[d] * int(st.xi[i, d]) for d in range(3))) for i, fi in enumerate(f_rat))
    logM = sp.log(Mgf)
    rho_r = sum(f_rat)
    f = np.array([float(v) for v in f_rat])[None, :]
    rho = f.sum(axis=1)
    u = (f @ st.xi.astype(float)) / rho[:, None]
    kappa = np.einsum("nji,ni->nj", O.central_matrix(st, u), f)
    C = O.cumulants_from_central(st, kappa, rho, u)[0]
    zero = {X[0]: 0, X[1]: 0, X[2]: 0}
    for e in [(2, 0, 0), (1, 1, 0), (1, 1, 1), (2, 2, 0), (2, 1, 1), (1, 2, 2), (2, 2, 2)]:
        dexpr = sp.diff(logM, *[a for d in range(3) for a in [X[d]] * e[d]])
        want = float(sp.Rational(rho_r.numerator, rho_r.denominator) * dexpr.subs(zero))
        got = C[st.eidx[e]]
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want)), (e, got, want)


def test_cumulant_independence_property():
    """sec. 2.3.3: cumulants express statistical independence -- for a product-form
    distribution f_xyz = a_x b_y c_z every mixed cumulant vanishes."""
    st = O.stencil("D3Q27")
    rng = np.random.default_rng(5)
    a, b, c = (rng.uniform(0.1, 1.0, 3) for _ in range(3))
    f = np.array([a[x + 1] * b[y + 1] * c[z + 1] for x, y, z in st.xi])[None, :]
    rho = f.sum(axis=1)
    u = (f @ st.xi.astype(float)) / rho[:, None]
    kappa = np.einsum("nji,ni->nj", O.central_matrix(st, u), f)
    C = O.cumulants_from_central(st, kappa, rho, u)[0]
    for j, e in enumerate(st.exps):
        if sum(e) >= 2 and sum(1 for v in e if v > 0) >= 2:
            assert abs(C[j]) < 1e-15, e
    # pure cumulants are those of the 1-D marginals: C_200 = rho var_x
    px = a / a.sum()
    var = (px * np.array([1, 0, 1])).sum() - ((px * np.array([-1, 0, 1])).sum()) ** 2
    assert abs(C[st.eidx[(2, 0, 0)]] - rho[0] * var) < 1e-15


def test_cumulant_roundtrip_and_textbook_low_orders():
    st = O.stencil("D3Q27")
    rng = np.random.default_rng(6)
    n = 32
    rho = 1 + 0.05 * rng.standard_normal(n)
    u = rng.uniform(-0.1, 0.1, (n, 3))
    f = np.linalg.solve(O.central_matrix(st, u), O.central_maxwellian(st, rho)[:, :, None])[:, :, 0]
    f = f + 1e-3 * rng.standard_normal(f.shape)
    rho = f.sum(axis=1)
    u = (f @ st.xi.astype(float)) / rho[:, None]
    kappa = np.einsum("nji,ni->nj", O.central_matrix(st, u), f)
    C = O.cumulants_from_central(st, kappa, rho, u)
    back = O.central_from_cumulants(st, C, rho)
    hi = [j for j, e in enumerate(st.exps) if sum(e) >= 2]
    np.testing.assert_allclose(back[:, hi], kappa[:, hi], rtol=0, atol=1e-15)
    k = lambda e: kappa[:, st.eidx[e]]
    np.testing.assert_allclose(C[:, st.eidx[(1, 1, 0)]], k((1, 1, 0)), atol=1e-17)
    np.testing.assert_allclose(C[:, st.eidx[(2, 1, 0)]], k((2, 1, 0)), atol=1e-17)
    want220 = k((2, 2, 0)) - (k((2, 0, 0)) * k((0, 2, 0)) + 2 * k((1, 1, 0)) ** 2) / rho
    np.testing.assert_allclose(C[:, st.eidx[(2, 2, 0)]], want220, atol=1e-17)


def test_gaussian_cumulants_isserlis():
    """Cumulants of the Maxwellian are c_s^2 on the diagonal and zero elsewhere; mapping them
    back gives the Gaussian central moments (Isserlis): kappa_220 = rho c_s^4,
    kappa_222 = rho c_s^6, kappa_211 = 0."""
    st = O.stencil("D3Q27")
    rho = np.array([1.1, 0.9])
    u = np.array([[0.01, 0.02, 0.03], [0.0, 0.0, 0.0]])
    Ceq = O.cumulant_maxwellian(st, rho, u)
    kap = O.central_from_cumulants(st, Ceq, rho)
    np.testing.assert_allclose(kap, O.central_maxwellian(st, rho), atol=1e-16)
