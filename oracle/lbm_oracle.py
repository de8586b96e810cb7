"""FP64 CPU oracle: dense definitions of the zero-centred MRT-LBM collision and streaming.

TEST INFRASTRUCTURE ONLY -- imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py; never by the product path.

Paper: Hennig, Holzer, Ruede, "Advanced Automatic Code Generation for Multiple
Relaxation-Time Lattice Boltzmann Methods", arXiv 2211.02435.

Every function states the passage it follows and what pins it (the tests in
tests/test_oracle_*.py check it against something other than itself):

  Stencil / weights          sec. 2.1 (D2Q9/D3Q15/D3Q19/D3Q27, xi_0 = 0)
        pin: w == M^-1 m0 (sec. 2.4, background equals the weights), isotropy sums
  D3Q15 moment set           one monomial per exponent-parity class of the mixed monomials
        pin: the classes by brute force over the velocities; the raw (polynomial) and
             central (Maxwellian) equilibria's fourth moments worked out by hand
  weighted_orthogonal_matrix WO-MRT / O-MRT bases (sec. 2.3.1): Gram-Schmidt under the weights
        or the plain sum
        pin: orthogonality by brute force, D2Q9 / D3Q27 Hermite product forms (WO), the
        Lallemand-Luo D2Q9 polynomials (O), unit-rate basis independence, Taylor-Green
        viscosity
  moment_matrix              eq. DiscreteRawMomentsDef (sec. 2.3.1)
        pin: closed-form 1-D factorisation, w == M^-1 m0, textbook 2nd-order equilibrium
  central_matrix             eq. DiscreteRawMomentsDef for central moments (sec. 2.3.2)
        pin: binomial relation eq. RawToCentralMomentsBinomial evaluated independently,
             K(0) == M
  cumulants_from_central /   eq. CumulantGeneratingFunction (sec. 2.3.3) written through
  central_from_cumulants     set partitions (multivariate Faa di Bruno for log / exp)
        pin: symbolic derivatives of log M(Xi) with SymPy on exact rational populations,
             independence of product-form distributions, round trip
  equilibrium_mono           sec. 2.4 (continuous Maxwellian, raw moments truncated at
                             second order in u as stated in sec. 4.3), sec. 5.2 (Zhou)
        pin: textbook D2Q9/D3Q27 polynomial equilibrium, SWE moments h, hu, gh^2/2 + huu
  swe_maxwellian_mono        sec. 5.2, Venturi's cumulant shallow-water method: the continuous
                             Maxwellian with c_s^2 = g h / 2
        pin: population moments h, hu, g h^2 / 2 + h u u (the shallow-water flux, the same as
             Zhou's discrete equilibrium); product form over the axes; the central-moment and
             cumulant spaces give the same equilibrium populations
  collide                    eq. MrtUpdateGeneral, eq. MrtUpdateGeneralDeviationOnly,
                             eq. MrtUpdateAbsoluteFromZeroCentered (sec. 2.2)
        pin: the three forms agree, equilibrium is a fixed point, per-cell conservation,
             all rates 0 -> identity, all rates 1 -> equilibrium, raw space with equal
             rates -> BGK, Taylor-Green decay exp(-2 nu k^2 t) (sec. 5.1)
  srt_equilibrium / 'srt'    single relaxation time (eq. MrtUpdateGeneral with the identity
                             transform and S = omega I; the SRT method of sec. 4.3 and 5.1)
                             with the second-order polynomial equilibrium
        pin: moments of orders 0..2 are rho, rho u, rho (cs2 delta + u u) on every stencil;
             on the tensor-product stencils D2Q9 / D3Q27 one SRT collision equals the
             raw-moment collision with all rates omega (moment-space BGK)
  guo_source / he_source     source term f^F of eq. LbUpdateScheme and q^F of
                             eq. MrtUpdateGeneral (sec. 2.1, 2.2) with Guo's force model: the
                             equilibrium velocity u = (j + F/2) / rho, q^F the source's moments
                             in the collision space at u, weighted by (I - S/2); He's model
                             weights (xi - u) . F by the equilibrium populations instead
        pin: every cell gains exactly F of momentum and no mass; a uniform force accelerates a
             uniform state by F / rho per step; the steady Kolmogorov flow under
             F_x = F0 sin(k y) has the analytic amplitude F0 / (nu k^2) to second order
  stream                     eq. LbUpdateScheme (sec. 2.1), periodic
        pin: impulse moves by xi_i; N steps of pure streaming on an N-periodic box return
             the initial state
  full 3-D run parity        parity unpinned beyond the pins above: the paper prints no
                             worked numeric example of a complete 3-D update.

Conventions the paper leaves open (velocity order, 3-D polynomial bases, truncation of
the raw equilibrium, the shallow-water equilibrium typo) are fixed as documented at the
definitions below.
"""
import itertools
import math
from collections import Counter
from functools import lru_cache

import numpy as np

CS2 = 1.0 / 3.0  # squared lattice speed of sound; background density rho0 = 1 (sec. 2.4)

# --------------------------------------------------------------------------------------
# Stencils (sec. 2.1).  The paper fixes only xi_0 = 0; opposite pairs are adjacent here:
# opp(i) = i+1 for odd i, i-1 for even i > 0.
# --------------------------------------------------------------------------------------
_D2Q9 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
         (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0)]
_D3Q27 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
          (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
          (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
          (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
          (1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1),
          (1, -1, 1), (-1, 1, -1), (-1, 1, 1), (1, -1, -1)]
_D3Q19 = _D3Q27[:19]
_D3Q15 = _D3Q27[:7] + _D3Q27[19:]  # rest, faces, corners (no edges)


def _mono(a, b, c=0):
    return {(a, b, c): 1.0}


def _poly(*terms):
    out = {}
    for coef, e in terms:
        out[e] = out.get(e, 0.0) + coef
    return out


# Polynomial bases (sec. 2.3: an ordered sequence of q linearly independent polynomials).
# D2Q9 is the basis of the shallow-water listing in sec. 5.2.  The paper prints no 3-D
# basis; a graded basis is used (each polynomial homogeneous in one order): conserved
# 1, x, y, z; shear xy, xz, yz, x^2-y^2, x^2-z^2; bulk x^2+y^2+z^2; third order as
# +/- pairs plus xyz; fourth order as two deviatoric combinations, the trace and the
# three x^2yz-type monomials; fifth and sixth order monomials.
_BASIS_2D = [
    _mono(0, 0), _mono(1, 0), _mono(0, 1),
    _mono(1, 1), _poly((1, (2, 0, 0)), (-1, (0, 2, 0))), _poly((1, (2, 0, 0)), (1, (0, 2, 0))),
    _mono(1, 2), _mono(2, 1), _mono(2, 2),
]
_B3_LOW = [
    _mono(0, 0, 0), _mono(1, 0, 0), _mono(0, 1, 0), _mono(0, 0, 1),
    _mono(1, 1, 0), _mono(1, 0, 1), _mono(0, 1, 1),
    _poly((1, (2, 0, 0)), (-1, (0, 2, 0))), _poly((1, (2, 0, 0)), (-1, (0, 0, 2))),
    _poly((1, (2, 0, 0)), (1, (0, 2, 0)), (1, (0, 0, 2))),
    _poly((1, (1, 2, 0)), (1, (1, 0, 2))), _poly((1, (1, 2, 0)), (-1, (1, 0, 2))),
    _poly((1, (2, 1, 0)), (1, (0, 1, 2))), _poly((1, (2, 1, 0)), (-1, (0, 1, 2))),
    _poly((1, (2, 0, 1)), (1, (0, 2, 1))), _poly((1, (2, 0, 1)), (-1, (0, 2, 1))),
]
_B3_XYZ = [_mono(1, 1, 1)]
_B3_O4 = [
    _poly((1, (2, 2, 0)), (-2, (2, 0, 2)), (1, (0, 2, 2))),
    _poly((1, (2, 2, 0)), (1, (2, 0, 2)), (-2, (0, 2, 2))),
    _poly((1, (2, 2, 0)), (1, (2, 0, 2)), (1, (0, 2, 2))),
]
_B3_HIGH = [_mono(2, 1, 1), _mono(1, 2, 1), _mono(1, 1, 2),
            _mono(1, 2, 2), _mono(2, 1, 2), _mono(2, 2, 1), _mono(2, 2, 2)]

# D3Q15 lacks the edges, so on its velocities every monomial with two or more nonzero
# exponents equals another one of the same exponent parities (x y^2 = x z^2 = x y^2 z^2,
# x^2 y^2 = x^2 z^2 = y^2 z^2 = x^2 y^2 z^2, ...); one monomial stands for each such class.
_B3_15 = _B3_LOW[:10] + [_mono(1, 1, 1), _mono(1, 2, 0), _mono(2, 1, 0), _mono(2, 0, 1), _mono(2, 2, 0)]

_BASES = {
    "D2Q9": _BASIS_2D,
    "D3Q19": _B3_LOW + _B3_O4,
    "D3Q27": _B3_LOW + _B3_XYZ + _B3_O4 + _B3_HIGH,
    "D3Q15": _B3_15,
}

BASIS_NAMES = {
    "D2Q9": ["1", "x", "y", "xy", "x2-y2", "x2+y2", "xy2", "x2y", "x2y2"],
    "D3Q19": ["1", "x", "y", "z", "xy", "xz", "yz", "x2-y2", "x2-z2", "x2+y2+z2",
              "xy2+xz2", "xy2-xz2", "x2y+yz2", "x2y-yz2", "x2z+y2z", "x2z-y2z",
              "x2y2-2x2z2+y2z2", "x2y2+x2z2-2y2z2", "x2y2+x2z2+y2z2"],
}
BASIS_NAMES["D3Q27"] = (BASIS_NAMES["D3Q19"][:16] + ["xyz"] + BASIS_NAMES["D3Q19"][16:]
                        + ["x2yz", "xy2z", "xyz2", "xy2z2", "x2yz2", "x2y2z", "x2y2z2"])
BASIS_NAMES["D3Q15"] = BASIS_NAMES["D3Q19"][:10] + ["xyz", "xy2", "x2y", "x2z", "x2y2"]


class Stencil:
    """Velocity set, lattice weights, monomial set and polynomial basis (sec. 2.1, 2.3)."""

    def __init__(self, name):
        vel = {"D2Q9": _D2Q9, "D3Q19": _D3Q19, "D3Q27": _D3Q27, "D3Q15": _D3Q15}[name]
        self.name = name
        self.d = 2 if name == "D2Q9" else 3
        self.q = len(vel)
        self.xi = np.array(vel, dtype=np.int64)
        norm2 = (self.xi ** 2).sum(axis=1)
        wtab = {"D2Q9": {0: 4 / 9, 1: 1 / 9, 2: 1 / 36},
                "D3Q19": {0: 1 / 3, 1: 1 / 18, 2: 1 / 36},
                "D3Q27": {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216},
                "D3Q15": {0: 2 / 9, 1: 1 / 9, 3: 1 / 72}}[name]
        self.w = np.array([wtab[int(n)] for n in norm2])
        self.opp = np.array([0] + [i + 1 if i % 2 == 1 else i - 1 for i in range(1, self.q)])
        self.basis = _BASES[name]
        # monomial set E: every monomial that occurs in the basis, in graded order
        exps = sorted({e for p in self.basis for e in p}, key=lambda e: (sum(e), e))
        self.exps = exps
        self.eidx = {e: j for j, e in enumerate(exps)}
        assert len(exps) == self.q
        self.conserved = list(range(self.d + 1))  # basis rows 1, x, y(, z)
        self.M = moment_matrix(self)
        self.P = np.zeros((self.q, self.q))
        for p, poly in enumerate(self.basis):
            for e, c in poly.items():
                self.P[p, self.eidx[e]] = c

    def order(self, j):
        return sum(self.exps[j])


@lru_cache(maxsize=None)
def weighted_orthogonal_matrix(st, weighted=True):
    """Orthogonal raw-moment bases (sec. 2.3.1 and the operation-count discussion): WO-MRT,
    the Gram-Schmidt of the graded basis, in its order, under
    <a, b> = sum_i w_i a(xi_i) b(xi_i); with weighted=False the plain sum over the velocities
    (O-MRT).  Rows of the returned matrix are the new polynomials' monomial coefficients
    (columns as st.exps); each is its graded counterpart minus a combination of the earlier
    ones."""
    wts = st.w if weighted else np.ones(st.q)
    G = (st.M * wts[None, :]) @ st.M.T  # <monomial_j, monomial_l>
    rows = []
    for k in range(st.q):
        p = st.P[k].copy()
        for r in rows:
            p = p - (p @ G @ r) / (r @ G @ r) * r
        rows.append(p)
    return np.array(rows)


def stencil(name):
    return Stencil(name)


def moment_matrix(st):
    """Monomial raw-moment matrix, eq. DiscreteRawMomentsDef: M[j, i] = prod_d xi_{i,d}^{E_j,d}."""
    M = np.ones((st.q, st.q))
    for j, e in enumerate(st.exps):
        for i in range(st.q):
            v = 1.0
            for d in range(3):
                v *= float(st.xi[i, d]) ** e[d]
            M[j, i] = v
    return M


def background_moments(st):
    """Raw moments m0 of the rest-state Maxwellian Psi(rho0=1, u=0) (sec. 2.4).

    Gaussian moments per axis: <1> = 1, <xi> = 0, <xi^2> = c_s^2, and the axes are
    independent, so m0_{abc} = prod_d nu(E_d) with nu = (1, 0, c_s^2)."""
    nu = (1.0, 0.0, CS2)
    return np.array([nu[e[0]] * nu[e[1]] * nu[e[2]] for e in st.exps])


def central_matrix(st, u):
    """Central-moment matrix K(u) per cell, sec. 2.3.2:
    K[n, j, i] = prod_d (xi_{i,d} - u_{n,d})^{E_j,d}.  u: (n, 3) -> (n, q, q)."""
    u = np.asarray(u, dtype=np.float64)
    diff = st.xi[None, :, :].astype(np.float64) - u[:, None, :]  # (n, q, 3)
    pw = np.stack([np.ones_like(diff), diff, diff * diff], axis=-1)  # (n, q, 3, 3)
    K = np.empty((u.shape[0], st.q, st.q))
    for j, e in enumerate(st.exps):
        K[:, j, :] = pw[:, :, 0, e[0]] * pw[:, :, 1, e[1]] * pw[:, :, 2, e[2]]
    return K


# --------------------------------------------------------------------------------------
# Cumulants (sec. 2.3.3, sec. 4.2.1).  C(Xi) = log M(Xi); c_abc are its derivatives at 0
# and C_abc = rho c_abc.  The derivatives of log of a generating function are written
# through set partitions of the multiset of axis letters of the monomial:
#   c(B) = sum_pi (|pi|-1)! (-1)^(|pi|-1) prod_{b in pi} k(b)      (moments -> cumulants)
#   k(B) = sum_pi prod_{b in pi} c(b)                              (cumulants -> moments)
# with k the normalised moments.  Cumulants of order >= 2 do not depend on the frame, so
# they are taken from central moments k = kappa / rho (eq. CumulantAndCentralMomentGenFuncs).
# Orders 0 and 1 are the conserved density and momentum and are passed through; the
# logarithm of C_000 therefore never appears.
# --------------------------------------------------------------------------------------
def _set_partitions(items):
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for part in _set_partitions(rest):
        yield [[first]] + part
        for k in range(len(part)):
            yield part[:k] + [[first] + part[k]] + part[k + 1:]


@lru_cache(maxsize=None)
def partition_terms(e):
    """Counter {(n_blocks, sorted tuple of block exponents): multiplicity} over all set
    partitions of the labelled letters of x^a y^b z^c."""
    letters = [0] * e[0] + [1] * e[1] + [2] * e[2]
    terms = Counter()
    for part in _set_partitions(list(range(len(letters)))):
        blocks = tuple(sorted(tuple(sum(1 for k in blk if letters[k] == ax) for ax in range(3))
                              for blk in part))
        terms[(len(part), blocks)] += 1
    return terms


def cumulants_from_central(st, kappa, rho, u):
    """Rescaled monomial cumulants C (n, q) from monomial central moments kappa (n, q).
    Orders 0 and 1 hold the conserved (rho, rho*u); orders >= 2 are taken in the co-moving
    frame, where the first-order central moments vanish (their blocks are dropped)."""
    k = kappa / rho[:, None]
    out = np.empty_like(kappa)
    for j, e in enumerate(st.exps):
        n = sum(e)
        if n == 0:
            out[:, j] = rho
        elif n == 1:
            out[:, j] = rho * u[:, e.index(1)]
        else:
            c = np.zeros_like(rho)
            for (nb, blocks), mult in partition_terms(e).items():
                if any(sum(b) == 1 for b in blocks):
                    continue  # a first-order factor: zero in the co-moving frame
                term = np.full_like(rho, mult * math.factorial(nb - 1) * (-1.0) ** (nb - 1))
                for b in blocks:
                    term = term * k[:, st.eidx[b]]
                c = c + term
            out[:, j] = rho * c
    return out


def central_from_cumulants(st, C, rho):
    """Monomial central moments kappa (n, q) from rescaled cumulants C (n, q).
    In the co-moving frame the first-order cumulants vanish; kappa_000 = rho."""
    c = C / rho[:, None]
    kappa = np.empty_like(C)
    for j, e in enumerate(st.exps):
        n = sum(e)
        if n == 0:
            kappa[:, j] = rho
        elif n == 1:
            kappa[:, j] = 0.0
        else:
            s = np.zeros_like(rho)
            for (nb, blocks), mult in partition_terms(e).items():
                if any(sum(b) == 1 for b in blocks):
                    continue  # a first-order cumulant factor, zero in the co-moving frame
                term = np.full_like(rho, float(mult))
                for b in blocks:
                    term = term * c[:, st.eidx[b]]
                s = s + term
            kappa[:, j] = rho * s
    return kappa


# --------------------------------------------------------------------------------------
# Equilibria (sec. 2.4, sec. 5.2)
# --------------------------------------------------------------------------------------
def raw_maxwellian_truncated(st, rho, u):
    """Raw moments of the continuous Maxwellian, m_abc = rho prod_d mu(E_d, u_d) with
    mu = (1, u, c_s^2 + u^2), expanded and truncated at second order in u (the default
    equilibrium of sec. 4.3: 'moments truncated at the second order in velocity')."""
    factors = {0: [(0, 1.0, 0)], 1: [(1, 1.0, 1)], 2: [(0, CS2, 0), (2, 1.0, 2)]}
    # each factor term: (u-degree, coefficient, power of u_d)
    out = np.zeros((rho.shape[0], st.q))
    for j, e in enumerate(st.exps):
        acc = np.zeros_like(rho)
        for combo in itertools.product(*(factors[e[d]] for d in range(3))):
            deg = sum(t[0] for t in combo)
            if deg > 2:
                continue
            v = np.ones_like(rho)
            for d, t in enumerate(combo):
                v = v * t[1] * u[:, d] ** t[2]
            acc = acc + v
        out[:, j] = rho * acc
    return out


def central_maxwellian(st, rho):
    """Central moments of the continuous Maxwellian: rho prod_d nu(E_d), nu = (1, 0, c_s^2).
    They do not depend on u, so the second-order truncation changes nothing."""
    nu = (1.0, 0.0, CS2)
    g = np.array([nu[e[0]] * nu[e[1]] * nu[e[2]] for e in st.exps])
    return rho[:, None] * g[None, :]


def cumulant_maxwellian(st, rho, u):
    """Rescaled cumulants of the continuous Maxwellian: C_200 = C_020 = C_002 = rho c_s^2,
    every other cumulant of order >= 2 is zero; orders 0, 1 carry (rho, rho u)."""
    out = np.zeros((rho.shape[0], st.q))
    for j, e in enumerate(st.exps):
        n = sum(e)
        if n == 0:
            out[:, j] = rho
        elif n == 1:
            out[:, j] = rho * u[:, e.index(1)]
        elif n == 2 and max(e) == 2:
            out[:, j] = rho * CS2
    return out


def srt_equilibrium(st, rho, u):
    """Second-order polynomial equilibrium of the SRT method (sec. 2.4 expanded to second order
    in u): f_eq_i = w_i rho (1 + xi.u / cs2 + (xi.u)^2 / (2 cs2^2) - u.u / (2 cs2))."""
    xu = u @ st.xi.T.astype(np.float64)  # (n, q)
    uu = (u * u).sum(axis=1)[:, None]
    return st.w[None, :] * rho[:, None] * (1.0 + xu / CS2 + xu * xu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2))


def swe_maxwellian_mono(st, space, h, u, g):
    """Equilibrium of Venturi's shallow-water method (sec. 5.2): the continuous Maxwellian of
    sec. 2.4 with density h and squared speed of sound c^2 = g h / 2, as monomial central
    moments h prod_d nu(E_d), nu = (1, 0, c^2), or as rescaled cumulants (C_000 = h,
    C_100 = h u_x, C_010 = h u_y, C_200 = C_020 = h c^2, every other one zero)."""
    c2 = 0.5 * g * h
    out = np.zeros((h.shape[0], st.q))
    for j, e in enumerate(st.exps):
        n = sum(e)
        if space == "central":
            v = h.copy()
            for d in range(3):
                v = v * (1.0 if e[d] == 0 else (0.0 if e[d] == 1 else c2))
            out[:, j] = v
        else:
            if n == 0:
                out[:, j] = h
            elif n == 1:
                out[:, j] = h * u[:, e.index(1)]
            elif n == 2 and max(e) == 2:
                out[:, j] = h * c2
    return out


def swe_equilibrium(st, h, u, g):
    """Discrete shallow-water equilibrium of Zhou on D2Q9 (sec. 5.2, eq.
    DiscreteShallowWaterEquilibrium and the listing).  Reading: the last term of f_i,
    i > 0, is -u.u/6 as in the listing; the printed equation's -u.u/3 would make
    sum_i f_i = h (1 - 5 u.u / 6) and violate mass conservation.
    lambda_i = 1 for |xi|_1 = 1 and 1/4 otherwise."""
    assert st.name == "D2Q9"
    xu = u[:, None, 0] * st.xi[None, :, 0] + u[:, None, 1] * st.xi[None, :, 1]
    uu = (u[:, 0] ** 2 + u[:, 1] ** 2)[:, None]
    l1 = np.abs(st.xi).sum(axis=1)
    lam = np.where(l1 == 1, 1.0, 0.25)[None, :]
    hh = h[:, None]
    f = lam * hh * (g * hh / 6 + xu / 3 + xu * xu / 2 - uu / 6)
    f[:, 0] = h * (1 - 5 * g * h / 6 - 2 * uu[:, 0] / 3)
    return f


# --------------------------------------------------------------------------------------
# Method definition and collision (sec. 2.2)
# --------------------------------------------------------------------------------------
class Method:
    """stencil, collision space, one relaxation rate per basis polynomial, equilibrium.

    space: 'raw' | 'central' | 'cumulant' | 'srt';
    equilibrium: 'maxwellian' | 'swe' (Zhou's discrete equilibrium) | 'swe_maxwellian'
    (Venturi's continuous Maxwellian with c^2 = g h / 2; central or cumulant space).
    Rates of the conserved polynomials (1, x, y, z) are ignored (pass-through).  'srt' works
    on the populations themselves with one rate, the common value of the non-conserved rates."""

    def __init__(self, stencil_name, space, omegas, equilibrium="maxwellian", gravity=None, force_model="guo",
                 basis="graded"):
        self.st = stencil(stencil_name)
        # polynomial basis of the raw-moment relaxation: the graded one, or its
        # weighted-orthogonal counterpart (WO-MRT)
        assert basis in ("graded", "weighted_orthogonal", "orthogonal")
        self.basis = basis
        if basis != "graded":
            assert space == "raw" and stencil_name != "D3Q15"
            self.P = weighted_orthogonal_matrix(self.st, weighted=basis == "weighted_orthogonal")
        else:
            self.P = self.st.P
        self.space = space
        self.omegas = np.asarray(omegas, dtype=np.float64)
        assert self.omegas.shape == (self.st.q,)
        self.equilibrium = equilibrium
        self.gravity = gravity
        assert force_model in ("guo", "he")
        self.force_model = force_model
        if stencil_name == "D3Q15":
            assert equilibrium == "maxwellian"
        if space == "srt":
            assert equilibrium == "maxwellian"
            rest = self.omegas[self.st.d + 1:]
            assert np.all(rest == rest[0]), "SRT needs one rate"
        if equilibrium == "swe":
            assert stencil_name == "D2Q9" and space in ("raw", "central")
            # background: the rest state h = 1, u = 0 of the discrete equilibrium
            self.f0 = swe_equilibrium(self.st, np.ones(1), np.zeros((1, 3)), gravity)[0]
        elif equilibrium == "swe_maxwellian":
            assert stencil_name == "D2Q9" and space in ("central", "cumulant")
            one, zero = np.ones(1), np.zeros((1, 3))
            self.f0 = self.backward(swe_maxwellian_mono(self.st, space, one, zero, gravity), one, zero)[0]
        else:
            self.f0 = self.st.w.copy()

    # --- transforms T and T^-1 in monomial form ---------------------------------------
    def forward(self, f, rho, u):
        st = self.st
        if self.space == "srt":
            return np.array(f, dtype=np.float64)
        if self.space == "raw":
            return f @ st.M.T
        kappa = np.einsum("nji,ni->nj", central_matrix(st, u), f)
        if self.space == "central":
            return kappa
        return cumulants_from_central(st, kappa, rho, u)

    def backward(self, qm, rho, u):
        st = self.st
        if self.space == "srt":
            return qm
        if self.space == "raw":
            return np.linalg.solve(st.M, qm.T).T
        if self.space == "cumulant":
            qm = central_from_cumulants(st, qm, rho)
        return np.linalg.solve(central_matrix(st, u), qm[:, :, None])[:, :, 0]

    def equilibrium_mono(self, rho, u):
        st = self.st
        if self.equilibrium == "swe":
            feq = swe_equilibrium(st, rho, u, self.gravity)
            return self.forward(feq, rho, u)
        if self.equilibrium == "swe_maxwellian":
            return swe_maxwellian_mono(st, self.space, rho, u, self.gravity)
        if self.space == "srt":
            return srt_equilibrium(st, rho, u)
        if self.space == "raw" and st.name == "D3Q15":
            # its monomials coincide in classes, so it cannot carry the Maxwellian's moments:
            # the equilibrium is the second-order polynomial one, in moments
            return srt_equilibrium(st, rho, u) @ st.M.T
        if self.space == "raw":
            return raw_maxwellian_truncated(st, rho, u)
        if self.space == "central":
            return central_maxwellian(st, rho)
        return cumulant_maxwellian(st, rho, u)

    def force_moments(self, S, u):
        """q^F: the source populations S in the collision space at velocity u (monomial form);
        for cumulants the source enters in central-moment space."""
        st = self.st
        if self.space == "srt":
            return S
        if self.space == "raw":
            return S @ st.M.T
        return np.einsum("nji,ni->nj", central_matrix(st, u), S)

    def weighted_force(self, qF):
        """(I - S/2) q^F in the polynomial basis; the conserved rows (rate 0) take all of q^F."""
        st = self.st
        if self.space == "srt":
            return (1.0 - 0.5 * self.omegas[st.d + 1]) * qF
        om = self.omegas.copy()
        om[st.conserved] = 0.0
        q = qF @ self.P.T
        return np.linalg.solve(self.P, ((1.0 - 0.5 * om)[None, :] * q).T).T

    def relax(self, q_mono, q_eq_mono):
        """q = P q_mono; q* = q + S (q_eq - q) on non-conserved rows; back to monomials.
        SRT: q are the populations, q* = q + omega (q_eq - q) on every one of them."""
        st = self.st
        if self.space == "srt":
            om = self.omegas[st.d + 1]
            return q_mono + om * (q_eq_mono - q_mono)
        q = q_mono @ self.P.T
        qe = q_eq_mono @ self.P.T
        om = self.omegas.copy()
        om[st.conserved] = 0.0
        qs = q + om[None, :] * (qe - q)
        return np.linalg.solve(self.P, qs.T).T


def guo_source(st, u, F):
    """Guo's forcing populations (n, q): S_i = w_i [(xi_i - u) / cs2 + (xi_i . u) xi_i / cs2^2] . F
    (the momentum source of sec. 2.1 in the model of Guo, Zheng and Shi)."""
    xi = st.xi.astype(np.float64)
    xu = u @ xi.T
    xF = F @ xi.T
    uF = (u * F).sum(axis=1)[:, None]
    return st.w[None, :] * ((xF - uF) / CS2 + xu * xF / (CS2 * CS2))


def he_source(st, u, F, rho, feq):
    """He's forcing populations (n, q): S_i = (xi_i - u) . F f_eq_i / (rho cs2), with feq the
    method's absolute equilibrium populations (the source term of sec. 2.1 in the model of He,
    Shan and Doolen)."""
    xi = st.xi.astype(np.float64)
    xF = F @ xi.T
    uF = (u * F).sum(axis=1)[:, None]
    return (xF - uF) * feq / (CS2 * rho[:, None])


def macroscopic_from_delta(method, df_cells):
    """eq. DensityAndVelocityFromDeviation: rho = rho0 + sum df, u = sum df xi / rho."""
    st = method.st
    rho = 1.0 + df_cells.sum(axis=1)
    u = (df_cells @ st.xi.astype(np.float64)) / rho[:, None]
    return rho, u


def _collide_forced(m, f_cells, form, F):
    """The three forms with Guo's source term: u = (j + F/2) / rho, q* = q + S(q_eq - q) +
    (I - S/2) q^F.  For cumulants the relaxed cumulants return to central moments, whose
    first-order entries keep their pre-collision value -F/2 (conserved), and (I - S/2) kappa^F
    is added there."""
    st = m.st
    xi = st.xi.astype(np.float64)
    f0 = m.f0[None, :]
    if form == "absolute":
        f_abs = f_cells
        rho = f_cells.sum(axis=1)
        j = f_cells @ xi
    else:
        f_abs = f_cells + f0
        rho = 1.0 + f_cells.sum(axis=1)
        j = f_cells @ xi
    u = (j + 0.5 * F) / rho[:, None]
    if m.force_model == "he":
        S = he_source(st, u, F, rho, equilibrium_populations(m, rho, u))
    else:
        S = guo_source(st, u, F)
    qFw = m.weighted_force(m.force_moments(S, u))
    if m.space == "cumulant":
        if form == "delta":
            raise ValueError("the cumulant transform is nonlinear: no delta-equilibrium (sec. 3)")
        kappa = np.einsum("nji,ni->nj", central_matrix(st, u), f_abs)
        C = cumulants_from_central(st, kappa, rho, u)
        Cs = m.relax(C, m.equilibrium_mono(rho, u))
        ks = central_from_cumulants(st, Cs, rho)
        first = [k for k, e in enumerate(st.exps) if sum(e) == 1]
        ks[:, first] = kappa[:, first]
        ks = ks + qFw
        out = np.linalg.solve(central_matrix(st, u), ks[:, :, None])[:, :, 0]
        return out if form == "absolute" else out - f0
    if form == "delta":
        dq = m.forward(f_cells, rho, u)
        dq_eq = m.equilibrium_mono(rho, u) - m.forward(np.broadcast_to(m.f0, f_cells.shape), rho, u)
        return m.backward(m.relax(dq, dq_eq) + qFw, rho, u)
    qs = m.relax(m.forward(f_abs, rho, u), m.equilibrium_mono(rho, u)) + qFw
    out = m.backward(qs, rho, u)
    return out if form == "absolute" else out - f0


def collide_cells(method, f_cells, form, F=None):
    """Collision of every cell; f_cells is (n, q); F (n, 3) an optional body force per cell
    (Guo's model, see _collide_forced).

    form 'absolute'    : eq. MrtUpdateGeneral on absolute populations (input/output f).
    form 'delta'       : eq. MrtUpdateGeneralDeviationOnly (linear T only; input/output df).
    form 'zc_absolute' : eq. MrtUpdateAbsoluteFromZeroCentered (input/output df)."""
    m = method
    st = m.st
    if F is not None:
        return _collide_forced(m, f_cells, form, np.asarray(F, dtype=np.float64))
    if form == "absolute":
        rho = f_cells.sum(axis=1)
        u = (f_cells @ st.xi.astype(np.float64)) / rho[:, None]
        qm = m.forward(f_cells, rho, u)
        return m.backward(m.relax(qm, m.equilibrium_mono(rho, u)), rho, u)
    rho, u = macroscopic_from_delta(m, f_cells)
    if form == "delta":
        if m.space == "cumulant":
            raise ValueError("the cumulant transform is nonlinear: no delta-equilibrium (sec. 3)")
        dq = m.forward(f_cells, rho, u)  # linear T applied to df
        q0 = m.forward(np.broadcast_to(m.f0, f_cells.shape), rho, u)
        dq_eq = m.equilibrium_mono(rho, u) - q0
        return m.backward(m.relax(dq, dq_eq), rho, u)
    if form == "zc_absolute":
        f = f_cells + m.f0[None, :]
        qm = m.forward(f, rho, u)
        return m.backward(m.relax(qm, m.equilibrium_mono(rho, u)), rho, u) - m.f0[None, :]
    raise ValueError(form)


def default_form(method):
    """Form evaluated by default: delta-equilibrium for raw and central moments with the
    Maxwellian, absolute equilibrium on zero-centred storage for cumulants and for the
    shallow-water equilibrium."""
    if method.space == "cumulant" or method.equilibrium in ("swe", "swe_maxwellian"):
        return "zc_absolute"
    return "delta"


# --------------------------------------------------------------------------------------
# Fields: natural SoA layout df[i, z, y, x]  (q, nz, ny, nx)
# --------------------------------------------------------------------------------------
def collide(method, df, form=None, chunk=4096, force=None):
    """force: None, a constant (3,) body force, or a field (3, nz, ny, nx)."""
    form = form or default_form(method)
    q = method.st.q
    cells = df.reshape(q, -1).T
    Fc = None
    if force is not None:
        force = np.asarray(force, dtype=np.float64)
        Fc = (np.broadcast_to(force[:, None], (3, cells.shape[0])) if force.ndim == 1
              else force.reshape(3, -1)).T
    out = np.empty_like(cells)
    for s in range(0, cells.shape[0], chunk):
        out[s:s + chunk] = collide_cells(method, np.ascontiguousarray(cells[s:s + chunk]), form,
                                         None if Fc is None else np.ascontiguousarray(Fc[s:s + chunk]))
    return out.T.reshape(df.shape)


def stream(method, f):
    """eq. LbUpdateScheme (streaming): f_i(x + xi_i) <- f*_i(x), periodic in every axis."""
    st = method.st
    out = np.empty_like(f)
    for i in range(st.q):
        out[i] = np.roll(f[i], shift=(int(st.xi[i, 2]), int(st.xi[i, 1]), int(st.xi[i, 0])),
                         axis=(0, 1, 2))
    return out


def step(method, df, n=1, form=None, force=None):
    """n time steps: collide (with the optional body force), then stream (eq. LbUpdateScheme)."""
    for _ in range(n):
        df = stream(method, collide(method, df, form, force=force))
    return df


def equilibrium_populations(method, rho, u):
    """Equilibrium populations f^eq = T^-1(q^eq) of the method's space and equilibrium;
    for the shallow-water equilibrium the discrete populations themselves (sec. 2.4)."""
    if method.equilibrium == "swe":
        return swe_equilibrium(method.st, rho, u, method.gravity)
    return method.backward(method.equilibrium_mono(rho, u), rho, u)


def init_equilibrium(method, rho, u, chunk=4096):
    """Zero-centred initial state df(0) = f^eq(rho, u) - f0.  rho: (nz, ny, nx); u: (3, nz, ny, nx)."""
    shape = rho.shape
    r = rho.reshape(-1)
    uu = u.reshape(3, -1).T
    out = np.empty((r.shape[0], method.st.q))
    for s in range(0, r.shape[0], chunk):
        out[s:s + chunk] = equilibrium_populations(method, r[s:s + chunk], uu[s:s + chunk]) - method.f0
    return out.T.reshape((method.st.q,) + shape)


def macroscopic(method, df, force=None):
    """rho (nz, ny, nx) and u (3, nz, ny, nx) of the canonical state df; with a body force the
    velocity is Guo's u = (j + F/2) / rho."""
    q = method.st.q
    cells = df.reshape(q, -1).T
    rho, u = macroscopic_from_delta(method, cells)
    if force is not None:
        force = np.asarray(force, dtype=np.float64)
        Fc = (np.broadcast_to(force[:, None], (3, cells.shape[0])) if force.ndim == 1 else force.reshape(3, -1)).T
        u = u + 0.5 * Fc / rho[:, None]
    return rho.reshape(df.shape[1:]), u.T.reshape((3,) + df.shape[1:])


def diagnostics(method, df):
    """[sum drho, sum jx, sum jy, sum jz, sum rho |u|^2 / 2, #non-finite] over the box, with
    drho = sum_i df_i and j = sum_i df_i xi_i summed directly (eq.
    DensityAndVelocityFromDeviation), so no background value is subtracted."""
    st = method.st
    cells = df.reshape(st.q, -1).T
    drho = cells.sum(axis=1)
    j = cells @ st.xi.astype(np.float64)
    ke = 0.5 * ((j * j).sum(axis=1) / (1.0 + drho)).sum()
    return np.array([drho.sum(), j[:, 0].sum(), j[:, 1].sum(), j[:, 2].sum(), ke,
                     float((~np.isfinite(df)).sum())])


def viscosity_to_omega(nu):
    """Shear viscosity nu = c_s^2 (1/omega - 1/2)  (sec. 5.1: nu = 1/6 <-> omega = 1)."""
    return 1.0 / (nu / CS2 + 0.5)


def omega_to_viscosity(omega):
    return CS2 * (1.0 / omega - 0.5)


def regularized_rates(stencil_name, omega_shear, omega_bulk=1.0):
    """'R-' rates (sec. 4.3): shear rate on xy, xz, yz and the deviatoric diagonals, the bulk
    rate on the trace, 1 for every higher-order polynomial, 0 for the conserved ones."""
    names = BASIS_NAMES[stencil_name]
    st = stencil(stencil_name)
    om = np.ones(st.q)
    om[st.conserved] = 0.0
    shear = {"xy", "xz", "yz", "x2-y2", "x2-z2"}
    for k, nm in enumerate(names):
        if nm in shear:
            om[k] = omega_shear
        elif nm in ("x2+y2", "x2+y2+z2"):
            om[k] = omega_bulk
    return om
