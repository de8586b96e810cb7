// Host-only part of the library: parameter validation and the relaxation matrix.
//
// Pure host code (no HIP runtime calls), so the CPU test suite can exercise it without a GPU.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_method.hpp"

namespace lbm {

thread_local std::string g_last_error;

lbm_status fail(lbm_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

int stencil_q(int s) { return s == LBM_D2Q9 ? 9 : (s == LBM_D3Q19 ? 19 : (s == LBM_D3Q15 ? 15 : 27)); }
int stencil_d(int s) { return s == LBM_D2Q9 ? 2 : 3; }
size_t storage_bytes(int st) { return st == LBM_STORE_F64 ? 8 : (st == LBM_STORE_F32 ? 4 : 2); }

// Population plane stride in elements for the PLANES layout: ncells rounded up to 256 bytes
// plus a padding that staggers the start of the q planes across HBM channels (a power-of-two
// plane size puts the q streams of a cell at the same channel offset).  LBM_PLANE_PAD_BYTES
// overrides the default padding.
size_t plane_elems(const lbm_params *p) {
  const size_t ncells = size_t(p->nx) * size_t(p->ny) * size_t(p->nz);
  const size_t eb = storage_bytes(p->storage);
  size_t pad_bytes = kDefaultPlanePadBytes;
  if (const char *env = std::getenv("LBM_PLANE_PAD_BYTES")) pad_bytes = size_t(std::strtoull(env, nullptr, 10));
  const size_t align = 256 / eb;
  const size_t base = (ncells + align - 1) / align * align;
  return base + (pad_bytes / 256) * align;
}

int resolve_layout(const lbm_params *p) {
  if (p->layout == LBM_LAYOUT_PLANES || p->layout == LBM_LAYOUT_ROWS) return p->layout;
  // measured: rows for every storage and streaming pattern under the autotuned launch; planes
  // only where a rows z-plane (q padded rows per y) would not fit 32-bit lane offsets
  const double align = 256.0 / double(storage_bytes(p->storage));
  const double nxp = std::ceil(double(p->nx) / align) * align;
  const double rows_plane = double(p->ny) * double(stencil_q(p->stencil)) * nxp * double(storage_bytes(p->storage));
  return rows_plane >= 4294967295.0 ? LBM_LAYOUT_PLANES : LBM_LAYOUT_ROWS;
}

// element strides of population i, z and y (x has stride 1) and elements per buffer
void storage_strides(const lbm_params *p, uint64_t *ps, uint64_t *zs, uint64_t *ys, uint64_t *elems) {
  const uint64_t nx = uint64_t(p->nx), ny = uint64_t(p->ny), nz = uint64_t(p->nz);
  const uint64_t q = uint64_t(stencil_q(p->stencil));
  if (resolve_layout(p) == LBM_LAYOUT_PLANES) {
    *ps = plane_elems(p);
    *ys = nx;
    *zs = ny * nx;
    *elems = q * *ps;
  } else {
    const uint64_t align = 256 / storage_bytes(p->storage);
    const uint64_t nxp = (nx + align - 1) / align * align;
    *ps = nxp;
    *ys = q * nxp;
    *zs = ny * *ys;
    *elems = nz * *zs;
  }
}

int internal_space(int public_space) { return public_space == LBM_SPACE_SRT ? kSpaceSrt : public_space; }

int literal_form(const lbm_params *p) {
  if (!p->zero_centered) return kLitA;
  return resolve_eq_form(p) == LBM_EQFORM_DELTA ? kLitB : kLitC;
}

int resolve_eq_form(const lbm_params *p) {
  if (p->eq_form != LBM_EQFORM_DEFAULT) return p->eq_form;
  if (p->space == LBM_SPACE_CUMULANT || p->equilibrium != LBM_EQ_MAXWELLIAN) return LBM_EQFORM_ABSOLUTE;
  return LBM_EQFORM_DELTA;
}

// ---------------------------------------------------------------------------------------
// polynomial bases (documented in lbm.h): each polynomial is a list of (coef, a, b, c)
// ---------------------------------------------------------------------------------------
struct Term {
  double c;
  int a, b, z;
};
using Poly = std::vector<Term>;

static std::vector<Poly> basis_of(int s) {
  std::vector<Poly> B;
  if (s == LBM_D2Q9) {
    B = {{{1, 0, 0, 0}}, {{1, 1, 0, 0}}, {{1, 0, 1, 0}}, {{1, 1, 1, 0}},
         {{1, 2, 0, 0}, {-1, 0, 2, 0}}, {{1, 2, 0, 0}, {1, 0, 2, 0}},
         {{1, 1, 2, 0}}, {{1, 2, 1, 0}}, {{1, 2, 2, 0}}};
    return B;
  }
  if (s == LBM_D3Q15) {
    // graded; the cubic and quartic entries name the representative monomial of their class
    B = {{{1, 0, 0, 0}}, {{1, 1, 0, 0}}, {{1, 0, 1, 0}}, {{1, 0, 0, 1}},
         {{1, 1, 1, 0}}, {{1, 1, 0, 1}}, {{1, 0, 1, 1}},
         {{1, 2, 0, 0}, {-1, 0, 2, 0}}, {{1, 2, 0, 0}, {-1, 0, 0, 2}},
         {{1, 2, 0, 0}, {1, 0, 2, 0}, {1, 0, 0, 2}},
         {{1, 1, 1, 1}}, {{1, 1, 2, 0}}, {{1, 2, 1, 0}}, {{1, 2, 0, 1}}, {{1, 2, 2, 0}}};
    return B;
  }
  B = {{{1, 0, 0, 0}}, {{1, 1, 0, 0}}, {{1, 0, 1, 0}}, {{1, 0, 0, 1}},
       {{1, 1, 1, 0}}, {{1, 1, 0, 1}}, {{1, 0, 1, 1}},
       {{1, 2, 0, 0}, {-1, 0, 2, 0}}, {{1, 2, 0, 0}, {-1, 0, 0, 2}},
       {{1, 2, 0, 0}, {1, 0, 2, 0}, {1, 0, 0, 2}},
       {{1, 1, 2, 0}, {1, 1, 0, 2}}, {{1, 1, 2, 0}, {-1, 1, 0, 2}},
       {{1, 2, 1, 0}, {1, 0, 1, 2}}, {{1, 2, 1, 0}, {-1, 0, 1, 2}},
       {{1, 2, 0, 1}, {1, 0, 2, 1}}, {{1, 2, 0, 1}, {-1, 0, 2, 1}}};
  if (s == LBM_D3Q27) B.push_back({{1, 1, 1, 1}});
  B.push_back({{1, 2, 2, 0}, {-2, 2, 0, 2}, {1, 0, 2, 2}});
  B.push_back({{1, 2, 2, 0}, {1, 2, 0, 2}, {-2, 0, 2, 2}});
  B.push_back({{1, 2, 2, 0}, {1, 2, 0, 2}, {1, 0, 2, 2}});
  if (s == LBM_D3Q27) {
    B.push_back({{1, 2, 1, 1}});
    B.push_back({{1, 1, 2, 1}});
    B.push_back({{1, 1, 1, 2}});
    B.push_back({{1, 1, 2, 2}});
    B.push_back({{1, 2, 1, 2}});
    B.push_back({{1, 2, 2, 1}});
    B.push_back({{1, 2, 2, 2}});
  }
  return B;
}

static bool mono_present(int s, int e) {
  const int a = e % 3, b = (e / 3) % 3, c = e / 9;
  if (s == LBM_D2Q9) return c == 0;
  if (s == LBM_D3Q19) return a == 0 || b == 0 || c == 0;
  if (s == LBM_D3Q15) {
    // 1 and the pure powers, and one representative per exponent-parity class of the mixed
    // monomials: xy, xz, yz, xyz, x2y2, xy2, x2y, x2z
    if ((a != 0) + (b != 0) + (c != 0) < 2) return true;
    return e == 4 || e == 10 || e == 12 || e == 13 || e == 8 || e == 7 || e == 5 || e == 11;
  }
  return true;
}

// Gauss-Jordan inverse with partial pivoting (n <= 27)
static bool invert(std::vector<double> &A, int n) {
  std::vector<double> I(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) I[size_t(i) * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[size_t(r) * n + c]) > std::fabs(A[size_t(piv) * n + c])) piv = r;
    if (std::fabs(A[size_t(piv) * n + c]) < 1e-12) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(A[size_t(c) * n + k], A[size_t(piv) * n + k]);
        std::swap(I[size_t(c) * n + k], I[size_t(piv) * n + k]);
      }
    const double d = A[size_t(c) * n + c];
    for (int k = 0; k < n; ++k) {
      A[size_t(c) * n + k] /= d;
      I[size_t(c) * n + k] /= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = A[size_t(r) * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        A[size_t(r) * n + k] -= f * A[size_t(c) * n + k];
        I[size_t(r) * n + k] -= f * I[size_t(c) * n + k];
      }
    }
  }
  A.swap(I);
  return true;
}

static const int kO2_3[6] = {2, 6, 18, 4, 10, 12};
static const int kO3_3[7] = {7, 19, 5, 21, 11, 15, 13};
static const int kO4_3[6] = {8, 20, 24, 14, 16, 22};
static const int kO5_3[3] = {25, 23, 17};
static const int kO2_2[3] = {2, 6, 4};
static const int kO3_2[2] = {7, 5};

// velocities and weights of a stencil (host copy for the weighted inner product)
static void host_lattice(int s, std::vector<std::array<int, 3>> *xi, std::vector<double> *w) {
  const int d = stencil_d(s);
  for (int z = (d == 3 ? -1 : 0); z <= (d == 3 ? 1 : 0); ++z)
    for (int y = -1; y <= 1; ++y)
      for (int x = -1; x <= 1; ++x) {
        const int n2 = x * x + y * y + z * z;
        double wt;
        if (s == LBM_D2Q9) wt = n2 == 0 ? 4.0 / 9 : (n2 == 1 ? 1.0 / 9 : 1.0 / 36);
        else if (s == LBM_D3Q19) wt = n2 == 0 ? 1.0 / 3 : (n2 == 1 ? 1.0 / 18 : (n2 == 2 ? 1.0 / 36 : 0.0));
        else if (s == LBM_D3Q15) wt = n2 == 0 ? 2.0 / 9 : (n2 == 1 ? 1.0 / 9 : (n2 == 3 ? 1.0 / 72 : 0.0));
        else wt = n2 == 0 ? 8.0 / 27 : (n2 == 1 ? 2.0 / 27 : (n2 == 2 ? 1.0 / 54 : 1.0 / 216));
        if (wt == 0.0) continue;
        xi->push_back({x, y, z});
        w->push_back(wt);
      }
}

// v^e for a velocity component v in {-1, 0, 1}: 1, v or v^2 by the parity of e
static double ipow(int v, int e) { return e == 0 ? 1.0 : (e % 2 ? double(v) : double(v * v)); }

// rows of P (monomial coefficients over the present monomials `cols`) orthogonalised in order
// under <a, b> = sum_i w_i a(xi_i) b(xi_i), or the plain sum over the velocities (weighted false)
static void weighted_gram_schmidt(int s, const std::vector<int> &cols, std::vector<double> &P, bool weighted) {
  const int q = int(cols.size());
  std::vector<std::array<int, 3>> xi;
  std::vector<double> w;
  host_lattice(s, &xi, &w);
  if (!weighted) std::fill(w.begin(), w.end(), 1.0);
  // G[j][l] = <monomial_j, monomial_l>
  std::vector<double> G(size_t(q) * q, 0.0);
  for (int j = 0; j < q; ++j)
    for (int l = 0; l < q; ++l) {
      const int ej = cols[j], el = cols[l];
      double acc = 0.0;
      for (size_t i = 0; i < xi.size(); ++i)
        acc += w[i] * ipow(xi[i][0], ej % 3 + el % 3) * ipow(xi[i][1], (ej / 3) % 3 + (el / 3) % 3) *
               ipow(xi[i][2], ej / 9 + el / 9);
      G[size_t(j) * q + l] = acc;
    }
  auto dot = [&](const double *a, const double *b) {
    double acc = 0.0;
    for (int j = 0; j < q; ++j)
      for (int l = 0; l < q; ++l) acc += a[j] * G[size_t(j) * q + l] * b[l];
    return acc;
  };
  for (int k = 0; k < q; ++k) {
    double *pk = &P[size_t(k) * q];
    for (int r = 0; r < k; ++r) {
      const double *pr = &P[size_t(r) * q];
      const double c = dot(pk, pr) / dot(pr, pr);
      for (int j = 0; j < q; ++j) pk[j] -= c * pr[j];
    }
  }
}

lbm_status relaxation_blocks(int s, int basis, const double *omegas, RelaxHost *out) {
  const int q = stencil_q(s), d = stencil_d(s);
  const std::vector<Poly> B = basis_of(s);
  if (int(B.size()) != q) return fail(LBM_EINVAL, "internal: basis size mismatch");
  // monomial columns: present grid indices in increasing order
  std::vector<int> cols;
  int colof[27];
  for (int e = 0; e < 27; ++e) {
    colof[e] = -1;
    if (mono_present(s, e)) {
      colof[e] = int(cols.size());
      cols.push_back(e);
    }
  }
  if (int(cols.size()) != q) return fail(LBM_EINVAL, "internal: monomial count mismatch");
  std::vector<double> P(size_t(q) * q, 0.0);
  for (int r = 0; r < q; ++r)
    for (const Term &t : B[r]) P[size_t(r) * q + colof[t.a + 3 * t.b + 9 * t.z]] += t.c;
  if (basis == LBM_BASIS_WEIGHTED_ORTHOGONAL || basis == LBM_BASIS_ORTHOGONAL)
    weighted_gram_schmidt(s, cols, P, basis == LBM_BASIS_WEIGHTED_ORTHOGONAL);
  std::vector<double> Pinv = P;
  if (!invert(Pinv, q)) return fail(LBM_EINVAL, "internal: singular basis");
  // A = P^-1 S P with the conserved rows (1, x, y, z) at rate 0
  std::vector<double> SP(size_t(q) * q);
  for (int r = 0; r < q; ++r) {
    const double w = (r <= d) ? 0.0 : omegas[r];
    for (int k = 0; k < q; ++k) SP[size_t(r) * q + k] = w * P[size_t(r) * q + k];
  }
  std::vector<double> A(size_t(q) * q, 0.0);
  for (int i = 0; i < q; ++i)
    for (int k = 0; k < q; ++k) {
      double acc = 0.0;
      for (int r = 0; r < q; ++r) acc += Pinv[size_t(i) * q + r] * SP[size_t(r) * q + k];
      A[size_t(i) * q + k] = acc;
    }
  auto ord = [&](int e) { return e % 3 + (e / 3) % 3 + e / 9; };
  // order couplings the kernels apply: within an order, and (orthogonal bases) from orders
  // 1 -> 3, 1 -> 5, 2 -> 4, 2 -> 6, 4 -> 6, 3 -> 5; order 0 meets zero deviations, and order 1
  // nonzero ones only with a body force
  auto coupled = [](int oi, int ok) {
    return oi == ok || ok == 0 || oi <= 1 || (oi == 3 && ok == 1) || (oi == 5 && (ok == 1 || ok == 3)) ||
           (oi == 4 && ok == 2) || (oi == 6 && (ok == 2 || ok == 4));
  };
  for (int i = 0; i < q; ++i)
    for (int k = 0; k < q; ++k)
      if (!coupled(ord(cols[i]), ord(cols[k])) && std::fabs(A[size_t(i) * q + k]) > 1e-13)
        return fail(LBM_EINVAL, "internal: relaxation matrix couples orders the kernels do not");
  auto bval = [&](int ei, int ek) -> double {
    if (colof[ei] < 0 || colof[ek] < 0) return 0.0;
    const double a = A[size_t(colof[ei]) * q + colof[ek]];
    const double b = (ei == ek ? 1.0 : 0.0) - a;
    // entries below 1e-14 are the round-off of exact zeros (a rate of 1, an orthogonal pair):
    // kept exactly zero, as the regularized-kernel test below treats them
    return std::fabs(b) < 1e-14 ? 0.0 : b;
  };
  std::memset(out, 0, sizeof(*out));
  if (d == 3) {
    for (int j = 0; j < 6; ++j)
      for (int k = 0; k < 6; ++k) out->b2[j][k] = bval(kO2_3[j], kO2_3[k]);
    for (int j = 0; j < 7; ++j)
      for (int k = 0; k < 7; ++k) out->b3[j][k] = bval(kO3_3[j], kO3_3[k]);
    for (int j = 0; j < 6; ++j)
      for (int k = 0; k < 6; ++k) out->b4[j][k] = bval(kO4_3[j], kO4_3[k]);
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) out->b5[j][k] = bval(kO5_3[j], kO5_3[k]);
    out->b6 = bval(26, 26);
    const int o1[3] = {1, 3, 9};
    for (int j = 0; j < 7; ++j)
      for (int k = 0; k < 3; ++k) out->c31[j][k] = bval(kO3_3[j], o1[k]);
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) out->c51[j][k] = bval(kO5_3[j], o1[k]);
    for (int j = 0; j < 6; ++j)
      for (int k = 0; k < 6; ++k) out->c42[j][k] = bval(kO4_3[j], kO2_3[k]);
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 7; ++k) out->c53[j][k] = bval(kO5_3[j], kO3_3[k]);
    for (int k = 0; k < 6; ++k) {
      out->c62[k] = bval(26, kO2_3[k]);
      out->c64[k] = bval(26, kO4_3[k]);
    }
  } else {
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) out->b2[j][k] = bval(kO2_2[j], kO2_2[k]);
    for (int j = 0; j < 2; ++j)
      for (int k = 0; k < 2; ++k) out->b3[j][k] = bval(kO3_2[j], kO3_2[k]);
    out->b4[0][0] = bval(8, 8);
    for (int k = 0; k < 3; ++k) out->c42[0][k] = bval(8, kO2_2[k]);
    for (int j = 0; j < 2; ++j)
      for (int k = 0; k < 2; ++k) out->c31[j][k] = bval(kO3_2[j], k == 0 ? 1 : 3);
  }
  double cmax = 0.0;
  for (int j = 0; j < 6; ++j)
    for (int k = 0; k < 6; ++k) cmax = std::fmax(cmax, std::fabs(out->c42[j][k]));
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 7; ++k) cmax = std::fmax(cmax, std::fabs(out->c53[j][k]));
  for (int k = 0; k < 6; ++k) cmax = std::fmax(cmax, std::fmax(std::fabs(out->c62[k]), std::fabs(out->c64[k])));
  out->cross = cmax > 1e-14;
  double c1 = 0.0;
  for (int j = 0; j < 7; ++j)
    for (int k = 0; k < 3; ++k) c1 = std::fmax(c1, std::fabs(out->c31[j][k]));
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) c1 = std::fmax(c1, std::fabs(out->c51[j][k]));
  out->cross1 = c1 > 1e-14;
  // regularized: every block into an order >= 3 (from the orders >= 2 the kernels use) is zero
  double hi = 0.0;
  for (int i = 0; i < q; ++i)
    for (int k = 0; k < q; ++k)
      if (ord(cols[i]) >= 3 && ord(cols[k]) >= 2) hi = std::fmax(hi, std::fabs(bval(cols[i], cols[k])));
  out->regularized = hi < 1e-14;
  return LBM_OK;
}

lbm_status validate(const lbm_params *p) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  if (p->stencil < LBM_D2Q9 || p->stencil > LBM_D3Q15) return fail(LBM_EINVAL, "stencil out of range");
  if (p->space < LBM_SPACE_RAW || p->space > LBM_SPACE_SRT) return fail(LBM_EINVAL, "space out of range");
  if (p->arithmetic < LBM_ARITH_DEVIATION || p->arithmetic > LBM_ARITH_LITERAL)
    return fail(LBM_EINVAL, "arithmetic out of range");
  if (p->equilibrium < LBM_EQ_MAXWELLIAN || p->equilibrium > LBM_EQ_SHALLOW_WATER_CONTINUOUS)
    return fail(LBM_EINVAL, "equilibrium out of range");
  if (p->eq_form < LBM_EQFORM_DEFAULT || p->eq_form > LBM_EQFORM_DELTA) return fail(LBM_EINVAL, "eq_form out of range");
  if (p->storage < LBM_STORE_F64 || p->storage > LBM_STORE_F16) return fail(LBM_EINVAL, "storage out of range");
  if (p->streaming < LBM_STREAM_PULL || p->streaming > LBM_STREAM_PUSH)
    return fail(LBM_EINVAL, "streaming out of range");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(LBM_EINVAL, "dims must be >= 1");
  const int q = stencil_q(p->stencil);
  if (!p->omegas) return fail(LBM_EINVAL, "omegas is NULL");
  if (p->n_omegas != q) return fail(LBM_EINVAL, "n_omegas must equal q = " + std::to_string(q));
  for (int i = 0; i < q; ++i) {
    const double w = p->omegas[i];
    if (!std::isfinite(w)) return fail(LBM_EINVAL, "relaxation rate " + std::to_string(i) + " is not finite");
    if (i > stencil_d(p->stencil) && (w < 0.0 || w > 2.0))
      return fail(LBM_EINVAL, "relaxation rate " + std::to_string(i) + " outside [0, 2]");
  }
  if (p->equilibrium != LBM_EQ_MAXWELLIAN && !(p->gravity > 0.0 && std::isfinite(p->gravity)))
    return fail(LBM_EINVAL, "shallow-water equilibrium needs gravity > 0");
  // admissibility (sec. 3)
  if (!p->zero_centered) {
    if (p->eq_form == LBM_EQFORM_DELTA)
      return fail(LBM_EUNSUPPORTED, "the delta-equilibrium requires zero-centred storage");
    if (p->equilibrium != LBM_EQ_MAXWELLIAN)
      return fail(LBM_EUNSUPPORTED, "absolute population storage is implemented for the Maxwellian equilibrium");
  }
  if (p->space == LBM_SPACE_CUMULANT && p->eq_form == LBM_EQFORM_DELTA)
    return fail(LBM_EUNSUPPORTED, "the cumulant transform is nonlinear: no delta-equilibrium in cumulant space");
  if (p->stencil == LBM_D2Q9 && p->nz != 1) return fail(LBM_EUNSUPPORTED, "D2Q9 requires nz == 1");
  if (p->basis < LBM_BASIS_GRADED || p->basis > LBM_BASIS_ORTHOGONAL) return fail(LBM_EINVAL, "basis out of range");
  if (p->basis != LBM_BASIS_GRADED) {
    if (p->space != LBM_SPACE_RAW) return fail(LBM_EUNSUPPORTED, "the orthogonal bases are raw-moment bases");
    if (p->equilibrium != LBM_EQ_MAXWELLIAN)
      return fail(LBM_EUNSUPPORTED, "the orthogonal bases run with the Maxwellian equilibrium");
    if (p->stencil == LBM_D3Q15) return fail(LBM_EUNSUPPORTED, "no orthogonal basis for D3Q15");
  }
  if (p->stencil == LBM_D3Q15) {
    if (p->equilibrium != LBM_EQ_MAXWELLIAN)
      return fail(LBM_EUNSUPPORTED, "D3Q15 takes the Maxwellian equilibrium");
    if (p->arithmetic != LBM_ARITH_DEVIATION)
      return fail(LBM_EUNSUPPORTED, "D3Q15 runs with the deviation arithmetic");
  }
  if (p->space == LBM_SPACE_SRT) {
    if (p->equilibrium != LBM_EQ_MAXWELLIAN)
      return fail(LBM_EUNSUPPORTED, "SRT is implemented with the Maxwellian (polynomial) equilibrium");
    for (int i = stencil_d(p->stencil) + 2; i < q; ++i)
      if (p->omegas[i] != p->omegas[stencil_d(p->stencil) + 1])
        return fail(LBM_EINVAL, "SRT needs one rate: every non-conserved rate must be equal");
  }
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(p->force[d])) return fail(LBM_EINVAL, "force must be finite");
  if (p->force_model < LBM_FORCE_GUO || p->force_model > LBM_FORCE_HE) return fail(LBM_EINVAL, "force_model out of range");
  const bool forced = p->force[0] != 0.0 || p->force[1] != 0.0 || p->force[2] != 0.0;
  if (forced && p->equilibrium != LBM_EQ_MAXWELLIAN)
    return fail(LBM_EUNSUPPORTED, "the body force is implemented with the Maxwellian equilibrium");
  if (forced && p->arithmetic == LBM_ARITH_LITERAL)
    return fail(LBM_EUNSUPPORTED, "the body force runs with the deviation arithmetic");
  if (p->arithmetic == LBM_ARITH_LITERAL) {
    if (p->stencil != LBM_D2Q9 && p->stencil != LBM_D3Q27)
      return fail(LBM_EUNSUPPORTED, "LITERAL arithmetic is implemented for D2Q9 and D3Q27");
    if (p->streaming != LBM_STREAM_PULL) return fail(LBM_EUNSUPPORTED, "LITERAL arithmetic runs with pull streaming");
    if (p->equilibrium != LBM_EQ_MAXWELLIAN)
      return fail(LBM_EUNSUPPORTED, "LITERAL arithmetic is implemented for the Maxwellian equilibrium");
  }
  if (p->equilibrium == LBM_EQ_SHALLOW_WATER_CONTINUOUS) {
    if (p->stencil != LBM_D2Q9) return fail(LBM_EUNSUPPORTED, "the shallow-water equilibria are two-dimensional (D2Q9)");
    if (p->space != LBM_SPACE_CENTRAL && p->space != LBM_SPACE_CUMULANT)
      return fail(LBM_EUNSUPPORTED, "the continuous shallow-water equilibrium is used in central-moment or cumulant space");
    if (p->eq_form == LBM_EQFORM_DELTA)
      return fail(LBM_EUNSUPPORTED, "the shallow-water equilibrium is relaxed in absolute form");
  }
  if (p->equilibrium == LBM_EQ_SHALLOW_WATER) {
    if (p->stencil != LBM_D2Q9) return fail(LBM_EUNSUPPORTED, "the shallow-water equilibrium is two-dimensional (D2Q9)");
    if (p->space == LBM_SPACE_CUMULANT)
      return fail(LBM_EUNSUPPORTED, "shallow water in cumulant space is not implemented");
    if (p->eq_form == LBM_EQFORM_DELTA)
      return fail(LBM_EUNSUPPORTED, "the shallow-water equilibrium is relaxed in absolute form");
  }
  if (!p->periodic[0] || !p->periodic[1] || !p->periodic[2])
    return fail(LBM_EUNSUPPORTED, "only periodic boundaries are implemented");
  // cell indices in natural order (readers, force fields, diagnostics) are 32-bit
  const double ncells = double(p->nx) * double(p->ny) * double(p->nz);
  if (ncells >= 4294967296.0) return fail(LBM_EUNSUPPORTED, "a box must have fewer than 2^32 cells");
  if (p->layout < LBM_LAYOUT_AUTO || p->layout > LBM_LAYOUT_ROWS) return fail(LBM_EINVAL, "layout out of range");
  {
    uint64_t ps, zs, ys, elems;
    storage_strides(p, &ps, &zs, &ys, &elems);
    if (double(zs) * double(storage_bytes(p->storage)) >= 4294967295.0)
      return fail(LBM_EUNSUPPORTED, "one z-plane of the population storage must stay below 4 GiB (32-bit lane offsets)");
  }
  if (p->nx > 2147483647 || p->ny > 2147483647 || p->nz > 2147483647) return fail(LBM_EINVAL, "dims too large");
  return LBM_OK;
}

}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_params_default(lbm_params *p) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->stencil = LBM_D3Q27;
  p->space = LBM_SPACE_CUMULANT;
  p->equilibrium = LBM_EQ_MAXWELLIAN;
  p->eq_form = LBM_EQFORM_DEFAULT;
  p->arithmetic = LBM_ARITH_DEVIATION;
  p->zero_centered = 1;
  p->nx = p->ny = p->nz = 1;
  p->periodic[0] = p->periodic[1] = p->periodic[2] = 1;
  p->storage = LBM_STORE_F32;
  p->streaming = LBM_STREAM_PULL;
  return LBM_OK;
}

extern "C" lbm_status lbm_validate(const lbm_params *p) {
  const lbm_status s = validate(p);
  if (s != LBM_OK) return s;
  RelaxHost r;
  return relaxation_blocks(p->stencil, p->basis, p->omegas, &r);
}

extern "C" lbm_status lbm_required_bytes(const lbm_params *p, size_t *bytes) {
  const lbm_status s = validate(p);
  if (s != LBM_OK) return s;
  if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
  const size_t nbuf = (p->streaming == LBM_STREAM_PULL || p->streaming == LBM_STREAM_PUSH) ? 2 : 1;
  uint64_t ps, zs, ys, elems;
  storage_strides(p, &ps, &zs, &ys, &elems);
  *bytes = nbuf * size_t(elems) * storage_bytes(p->storage);
  return LBM_OK;
}

extern "C" const char *lbm_last_error(void) { return g_last_error.c_str(); }
extern "C" const char *lbm_version(void) { return "lbm-mi355x 0.1 (gfx950)"; }
