// Device building blocks of the zero-centred MRT lattice Boltzmann sweep for gfx950.
//
// One thread owns one cell.  Its populations live in registers as a 3x3x3 grid (3x3 in
// 2-D) indexed by velocity, g[(cx+1) + 3 (cy+1) + 9 (cz+1)]; the Chimera passes of
// eq. RawMomentChimeraTransform (sec. 4.1.1) turn the same grid, axis by axis, into
// monomial raw moments indexed by exponents, m[a + 3 b + 9 c].  Velocities missing from
// the stencil enter as zero (D3Q19 corners), as the paper prescribes; moments missing from
// the D3Q19 monomial set are zeroed before the backward pass, which then reproduces the
// structured D3Q19 inverse with zero corner populations.
//
// Precision organisation.  All intermediate quantities are deviations:
//   dm      = M df                  raw moments of the stored deviations
//   dm_eq   = m_eq(rho, u) - m0     equilibrium moments minus background moments
//   Dm      = dm - dm_eq            non-equilibrium raw moments (zero at orders 0, 1)
//   Dk      = K(u) M^-1 Dm          non-equilibrium central moments (binomial Chimera)
//   DC      = F(Dk)                 non-equilibrium cumulants (equilibrium cumulants are
//                                   Gaussian, so every DC vanishes at equilibrium)
// relaxation acts on these with the per-order blocks of (I - P^-1 S P), and the backward
// path rebuilds dm* = dm_eq + binom(+u)(Dk*) before the inverse Chimera.  In exact
// arithmetic this is eq. MrtUpdateGeneralDeviationOnly (raw, central) and
// eq. MrtUpdateAbsoluteFromZeroCentered (cumulants), sec. 2.2; no large background value
// is ever subtracted from another, so FP32 keeps the accuracy of the deviations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#define LBM_HD __host__ __device__ __forceinline__

namespace lbm {

enum StencilId { D2Q9 = 0, D3Q19 = 1, D3Q27 = 2, D3Q15 = 3 };
// SRT: single relaxation time in population space (eq. MrtUpdateGeneral with T = identity
// and S = omega I); IDENTITY: streaming only (no collision)
enum SpaceId { RAW = 0, CENTRAL = 1, CUMULANT = 2, IDENTITY = 3, SRT = 4 };
// MAXWELL: continuous Maxwellian (sec. 2.4); SWE: Zhou's discrete shallow-water equilibrium;
// SWEK: Venturi's shallow-water equilibrium, the continuous Maxwellian with c^2 = g h / 2 (sec. 5.2)
enum EqId { MAXWELL = 0, SWE = 1, SWEK = 2 };
// PULL: gather from x - xi.  AA_EVEN: own slots, write to the opposite slot.
// AA_ODD: read opposite slot at x - xi, write own slot at x + xi.
// ESO_EVEN / ESO_ODD: the Esoteric-Pull in-place pattern (see lbm_kernels.hpp).
enum PatternId { PULL = 0, AA_EVEN = 1, AA_ODD = 2, ESO_EVEN = 3, ESO_ODD = 4, TW_EVEN = 5, TW_ODD = 6, PUSH = 7 };
// Layout of the canonical state df(t) in a buffer, for readers and writers.
enum GatherId { G_SHIFTED = 0, G_NATURAL = 1, G_AA_ODD = 2, G_ESO_EVEN = 3, G_ESO_ODD = 4, G_TW_EVEN = 5, G_TW_ODD = 6 };

// ---------------------------------------------------------------------------------------
// compile-time loop
// ---------------------------------------------------------------------------------------
template <class F, int... I>
LBM_HD void sfor_impl(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
LBM_HD void sfor(F &&f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------------------------------
// lattices (velocity order documented in lbm.h)
// ---------------------------------------------------------------------------------------
__host__ __device__ constexpr int vel27(int i, int d) {
  constexpr signed char t[27][3] = {
      {0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},
      {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},
      {-1, 0, 1},  {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1},  {1, 1, 1},   {-1, -1, -1},
      {1, 1, -1},  {-1, -1, 1}, {1, -1, 1},  {-1, 1, -1}, {-1, 1, 1},  {1, -1, -1}};
  return t[i][d];
}
__host__ __device__ constexpr int vel9(int i, int d) {
  constexpr signed char t[9][2] = {{0, 0}, {1, 0},   {-1, 0}, {0, 1}, {0, -1},
                                   {1, 1}, {-1, -1}, {1, -1}, {-1, 1}};
  return d < 2 ? t[i][d] : 0;
}

// D3Q15: the rest, the six faces and the eight corners of D3Q27, in D3Q27's order
__host__ __device__ constexpr int vel15(int i, int d) { return vel27(i < 7 ? i : i + 12, d); }

template <int S>
struct Lat {
  static constexpr int D = (S == D2Q9) ? 2 : 3;
  static constexpr int Q = (S == D2Q9) ? 9 : (S == D3Q19 ? 19 : (S == D3Q15 ? 15 : 27));
  static constexpr int G = (D == 2) ? 9 : 27;  // register grid size
  __host__ __device__ static constexpr int c(int i, int d) {
    return S == D2Q9 ? vel9(i, d) : (S == D3Q15 ? vel15(i, d) : vel27(i, d));
  }
  __host__ __device__ static constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
  // grid index of velocity i
  __host__ __device__ static constexpr int gidx(int i) {
    return (c(i, 0) + 1) + 3 * (c(i, 1) + 1) + (D == 3 ? 9 * (c(i, 2) + 1) : 0);
  }
  // lattice weight of velocity i (background f0 = w of the Maxwellian equilibrium, sec. 2.4)
  __host__ __device__ static constexpr double w(int i) {
    const int n = (c(i, 0) != 0) + (c(i, 1) != 0) + (c(i, 2) != 0);
    if (S == D2Q9) return n == 0 ? 4.0 / 9.0 : (n == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
    if (S == D3Q19) return n == 0 ? 1.0 / 3.0 : (n == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    if (S == D3Q15) return n == 0 ? 2.0 / 9.0 : (n == 1 ? 1.0 / 9.0 : 1.0 / 72.0);
    return n == 0 ? 8.0 / 27.0 : (n == 1 ? 2.0 / 27.0 : (n == 2 ? 1.0 / 54.0 : 1.0 / 216.0));
  }
  // is the monomial x^a y^b z^c part of the stencil's moment set?  D3Q15 (no edge velocities):
  // a monomial with two or more nonzero exponents takes on the lattice the values of the
  // lowest-index one of its exponent-parity class, which represents the class
  __host__ __device__ static constexpr bool has_mono(int a, int b, int cc) {
    if (S == D2Q9) return cc == 0;
    if (S == D3Q19) return a == 0 || b == 0 || cc == 0;
    if (S == D3Q15) return rep(a + 3 * b + 9 * cc) == a + 3 * b + 9 * cc;
    return true;
  }
  __host__ __device__ static constexpr bool has_mono_e(int e) {
    return has_mono(e % 3, (e / 3) % 3, e / 9);
  }
  // D3Q15: the class representative of monomial e (e itself on the other stencils)
  __host__ __device__ static constexpr int rep(int e) {
    if (S != D3Q15) return e;
    const int a = e % 3, b = (e / 3) % 3, cc = e / 9;
    if ((a != 0) + (b != 0) + (cc != 0) < 2) return e;  // 1 and the pure powers
    const int par = (a & 1) + 2 * (b & 1) + 4 * (cc & 1);
    // parity (x, y, z odd) -> representative: xy 4, xz 10, yz 12, xyz 13, x2y2 8, xy2 7,
    // x2y 5, x2z 11
    constexpr int t[8] = {8, 7, 5, 4, 11, 10, 12, 13};
    return t[par];
  }
  __host__ __device__ static constexpr int ord(int e) { return e % 3 + (e / 3) % 3 + e / 9; }
};

template <class T>
struct Cs {
  static constexpr T cs2 = T(1) / T(3);
  static constexpr T cs4 = T(1) / T(9);
};

// ---------------------------------------------------------------------------------------
// Chimera passes on the register grid
// ---------------------------------------------------------------------------------------
// raw Chimera along one axis: (f_-1, f_0, f_+1) -> (m_0, m_1, m_2)
template <class T>
LBM_HD void fwd_line(T &a, T &b, T &c) {
  T s = c + a;
  T d = c - a;
  a = s + b;
  b = d;
  c = s;
}
// its inverse: (m_0, m_1, m_2) -> (f_-1, f_0, f_+1)
template <class T>
LBM_HD void inv_line(T &a, T &b, T &c) {
  T m0 = a, m1 = b, m2 = c;
  a = T(0.5) * (m2 - m1);
  b = m0 - m2;
  c = T(0.5) * (m2 + m1);
}
// binomial Chimera along one axis with shift s (s = -u forward, +u backward), sec. 4.2:
// (k0, k1, k2) -> (k0, k1 + s k0, k2 + 2 s k1 + s^2 k0)
template <class T>
LBM_HD void shift_line(T &a, T &b, T &c, T s) {
  T n1 = fma(s, a, b);
  T n2 = fma(s, b + n1, c);
  b = n1;
  c = n2;
}

// apply `op(line entries)` along axis AX for every line of the grid
template <int D, int AX, class Op>
LBM_HD void for_lines(Op &&op) {
  constexpr int stride = AX == 0 ? 1 : (AX == 1 ? 3 : 9);
  constexpr int nlines = (D == 3) ? 9 : 3;
  sfor<nlines>([&](auto L) {
    constexpr int l = decltype(L)::value;
    int base;
    if constexpr (AX == 0) base = 3 * l;                         // (b, c) = (l % 3, l / 3)
    else if constexpr (AX == 1) base = (l % 3) + 9 * (l / 3);     // (a, c)
    else base = l;                                                // (a, b)
    op(base, stride);
  });
}

template <int S, class T>
LBM_HD void chimera_forward(T *g) {
  constexpr int D = Lat<S>::D;
  if constexpr (D == 3) for_lines<D, 2>([&](int b, int s) { fwd_line(g[b], g[b + s], g[b + 2 * s]); });
  for_lines<D, 1>([&](int b, int s) { fwd_line(g[b], g[b + s], g[b + 2 * s]); });
  for_lines<D, 0>([&](int b, int s) { fwd_line(g[b], g[b + s], g[b + 2 * s]); });
}
template <int S, class T>
LBM_HD void chimera_inverse(T *g) {
  constexpr int D = Lat<S>::D;
  for_lines<D, 0>([&](int b, int s) { inv_line(g[b], g[b + s], g[b + 2 * s]); });
  for_lines<D, 1>([&](int b, int s) { inv_line(g[b], g[b + s], g[b + 2 * s]); });
  if constexpr (D == 3) for_lines<D, 2>([&](int b, int s) { inv_line(g[b], g[b + s], g[b + 2 * s]); });
}
// central <- raw with shift (-u), or raw <- central with (+u); passes z, y, x
template <int S, class T>
LBM_HD void binomial(T *g, T sx, T sy, T sz) {
  constexpr int D = Lat<S>::D;
  if constexpr (D == 3) for_lines<D, 2>([&](int b, int s) { shift_line(g[b], g[b + s], g[b + 2 * s], sz); });
  for_lines<D, 1>([&](int b, int s) { shift_line(g[b], g[b + s], g[b + 2 * s], sy); });
  for_lines<D, 0>([&](int b, int s) { shift_line(g[b], g[b + s], g[b + 2 * s], sx); });
}

// ---------------------------------------------------------------------------------------
// Maxwellian equilibrium moments in deviation form (sec. 2.4)
//   mu(0) = 1, mu(1) = u, mu(2) = c_s^2 + u^2;  background mu0 = (1, 0, c_s^2)
//   dm_eq = drho * prod mu0 + rho * (prod mu - prod mu0)
// prod mu - prod mu0 is expanded over the axes with exponent 2 that take their u^2 part;
// every axis with exponent 1 contributes u_d.  TRUNC drops terms of u-degree > 2 (the raw
// equilibrium truncated at second order, sec. 4.3).
// ---------------------------------------------------------------------------------------
template <int E, bool TRUNC, class T>
LBM_HD T meq_dev(T drho, T rho, const T *u, const T *uu) {
  constexpr int a = E % 3, b = (E / 3) % 3, c = E / 9;
  constexpr int ex[3] = {a, b, c};
  constexpr int n1 = (a == 1) + (b == 1) + (c == 1);
  T t = T(0);
  bool any = false;
  // subsets of the exponent-2 axes taking u^2 (bit d set)
  sfor<8>([&](auto Sb) {
    constexpr int sb = decltype(Sb)::value;
    constexpr bool valid = ((sb & 1) == 0 || ex[0] == 2) && ((sb & 2) == 0 || ex[1] == 2) &&
                           ((sb & 4) == 0 || ex[2] == 2);
    constexpr int nsq = ((sb & 1) != 0) + ((sb & 2) != 0) + ((sb & 4) != 0);
    constexpr int deg = n1 + 2 * nsq;
    constexpr bool nonempty = deg > 0;  // excludes the background term itself
    constexpr bool keep = valid && nonempty && (!TRUNC || deg <= 2);
    if constexpr (keep) {
      T term = T(1);
      bool first = true;
      sfor<3>([&](auto Dd) {
        constexpr int d = decltype(Dd)::value;
        if constexpr (ex[d] == 1) {
          term = first ? u[d] : term * u[d];
          first = false;
        } else if constexpr (ex[d] == 2) {
          if constexpr ((sb >> d) & 1) {
            term = first ? uu[d] : term * uu[d];
          } else {
            term = first ? Cs<T>::cs2 : term * Cs<T>::cs2;
          }
          first = false;
        }
      });
      t = any ? t + term : term;
      any = true;
    }
  });
  constexpr T m0 = (a == 1 || b == 1 || c == 1)
                       ? T(0)
                       : ((a == 2 ? Cs<T>::cs2 : T(1)) * (b == 2 ? Cs<T>::cs2 : T(1)) *
                          (c == 2 ? Cs<T>::cs2 : T(1)));
  if constexpr (E == 0) {
    return drho;
  } else if constexpr (m0 == T(0)) {
    return rho * t;
  } else {
    return fma(drho, m0, rho * t);
  }
}

// ---------------------------------------------------------------------------------------
// relaxation blocks: B = I - P^-1 S P per order, rows/cols in the order lists below
// ---------------------------------------------------------------------------------------
template <class T>
struct Relax {
  T b2[6][6];
  T b3[7][7];
  T b4[6][6];
  T b5[3][3];
  T b6;
  // cross-order blocks (orthogonal raw bases), applied to the pre-relaxation deviations by
  // the CROSS kernels: orders 1 -> 3, 2 -> 4, 1 -> 5, 3 -> 5, 2 -> 6 and 4 -> 6 (order 1 is
  // nonzero only with a body force)
  T c31[7][3];
  T c42[6][6];
  T c51[3][3];
  T c53[3][7];
  T c62[6];
  T c64[6];
};

// exponent grid indices of each order (3-D); 2-D uses the c = 0 entries
__host__ __device__ constexpr int o2_3d(int k) { constexpr int t[6] = {2, 6, 18, 4, 10, 12}; return t[k]; }
__host__ __device__ constexpr int o3_3d(int k) { constexpr int t[7] = {7, 19, 5, 21, 11, 15, 13}; return t[k]; }
__host__ __device__ constexpr int o4_3d(int k) { constexpr int t[6] = {8, 20, 24, 14, 16, 22}; return t[k]; }
__host__ __device__ constexpr int o5_3d(int k) { constexpr int t[3] = {25, 23, 17}; return t[k]; }
__host__ __device__ constexpr int o2_2d(int k) { constexpr int t[3] = {2, 6, 4}; return t[k]; }
__host__ __device__ constexpr int o3_2d(int k) { constexpr int t[2] = {7, 5}; return t[k]; }

template <int S, int N, class IDX, class T, class M>
LBM_HD void relax_block(T *v, const M &B, IDX idx) {
  T in[N];
  sfor<N>([&](auto K) { in[K] = v[idx(K)]; });
  sfor<N>([&](auto J) {
    constexpr int j = decltype(J)::value;
    if constexpr (Lat<S>::has_mono_e(idx(j))) {
      T acc = T(0);
      sfor<N>([&](auto K) {
        constexpr int k = decltype(K)::value;
        if constexpr (Lat<S>::has_mono_e(idx(k))) acc = fma(B[j][k], in[k], acc);
      });
      v[idx(j)] = acc;
    }
  });
}

// v <- B v on the orders present; orders >= 3 set to zero when REG (their rate is 1).
template <int S, bool REG, class T>
LBM_HD void relax(T *v, const Relax<T> &R) {
  if constexpr (Lat<S>::D == 3) {
    relax_block<S, 6>(v, R.b2, [](int k) { return o2_3d(k); });
    if constexpr (REG) {
      sfor<27>([&](auto E) {
        constexpr int e = decltype(E)::value;
        if constexpr (Lat<S>::ord(e) >= 3) v[e] = T(0);
      });
    } else {
      relax_block<S, 7>(v, R.b3, [](int k) { return o3_3d(k); });
      relax_block<S, 6>(v, R.b4, [](int k) { return o4_3d(k); });
      if constexpr (S == D3Q27) {
        relax_block<S, 3>(v, R.b5, [](int k) { return o5_3d(k); });
        v[26] = R.b6 * v[26];
      }
    }
  } else {
    relax_block<S, 3>(v, R.b2, [](int k) { return o2_2d(k); });
    if constexpr (REG) {
      v[5] = T(0);
      v[7] = T(0);
      v[8] = T(0);
    } else {
      relax_block<S, 2>(v, R.b3, [](int k) { return o3_2d(k); });
      v[8] = R.b4[0][0] * v[8];
    }
  }
}

// ---------------------------------------------------------------------------------------
// cumulants in non-equilibrium form (sec. 2.3.3, 4.2.1)
// The Maxwellian has Gaussian cumulants: C_aa = rho c_s^2, all others zero.  Writing every
// central moment as Gaussian part + D and every cumulant as equilibrium part + DC, the
// moment/cumulant relations (set partitions of the monomial's letters; blocks of one letter
// vanish in the co-moving frame) become the expressions below; every term is a deviation.
// ---------------------------------------------------------------------------------------
__host__ __device__ constexpr int mono(int a, int b, int c) { return a + 3 * b + 9 * c; }

// axis-generic index: exponent e_x along axis X etc.
template <int X, int Y, int Z>
__host__ __device__ constexpr int mi(int ex, int ey, int ez) {
  int e[3] = {0, 0, 0};
  e[X] = ex;
  e[Y] = ey;
  e[Z] = ez;
  return mono(e[0], e[1], e[2]);
}

// forward (central -> cumulant), SIGN = -1; backward (cumulant -> central), SIGN = +1.
// Fourth order x^2 y^2 type (axes A, B):
//   DC = Dk -/+ cs2 (D_aa + D_bb) -/+ (D_aa D_bb + 2 D_ab^2) / rho    [forward: inputs Dk]
template <int A, int B, int C, int SIGN, class T>
LBM_HD T cum_aabb(const T *in, T rinv) {
  constexpr int aabb = mi<A, B, C>(2, 2, 0), aa = mi<A, B, C>(2, 0, 0), bb = mi<A, B, C>(0, 2, 0),
                ab = mi<A, B, C>(1, 1, 0);
  T lin = Cs<T>::cs2 * (in[aa] + in[bb]);
  T quad = (in[aa] * in[bb] + T(2) * in[ab] * in[ab]) * rinv;
  return SIGN < 0 ? in[aabb] - lin - quad : in[aabb] + lin + quad;
}
// x^2 y z type: DC = Dk -/+ cs2 D_bc -/+ (D_aa D_bc + 2 D_ab D_ac) / rho
template <int A, int B, int C, int SIGN, class T>
LBM_HD T cum_aabc(const T *in, T rinv) {
  constexpr int aabc = mi<A, B, C>(2, 1, 1), aa = mi<A, B, C>(2, 0, 0), bc = mi<A, B, C>(0, 1, 1),
                ab = mi<A, B, C>(1, 1, 0), ac = mi<A, B, C>(1, 0, 1);
  T lin = Cs<T>::cs2 * in[bc];
  T quad = (in[aa] * in[bc] + T(2) * in[ab] * in[ac]) * rinv;
  return SIGN < 0 ? in[aabc] - lin - quad : in[aabc] + lin + quad;
}
// x^2 y^2 z type: DC = Dk -/+ cs2 (D_bbc + D_aac)
//   -/+ (D_aa D_bbc + D_bb D_aac + 4 D_ab D_abc + 2 D_ac D_abb + 2 D_bc D_aab) / rho
template <int A, int B, int C, int SIGN, class T>
LBM_HD T cum_aabbc(const T *in, T rinv) {
  constexpr int aabbc = mi<A, B, C>(2, 2, 1), aa = mi<A, B, C>(2, 0, 0), bb = mi<A, B, C>(0, 2, 0),
                ab = mi<A, B, C>(1, 1, 0), ac = mi<A, B, C>(1, 0, 1), bc = mi<A, B, C>(0, 1, 1),
                bbc = mi<A, B, C>(0, 2, 1), aac = mi<A, B, C>(2, 0, 1), abc = mi<A, B, C>(1, 1, 1),
                abb = mi<A, B, C>(1, 2, 0), aab = mi<A, B, C>(2, 1, 0);
  T lin = Cs<T>::cs2 * (in[bbc] + in[aac]);
  T quad = (in[aa] * in[bbc] + in[bb] * in[aac] + T(4) * in[ab] * in[abc] + T(2) * in[ac] * in[abb] +
            T(2) * in[bc] * in[aab]) *
           rinv;
  return SIGN < 0 ? in[aabbc] - lin - quad : in[aabbc] + lin + quad;
}
// x^2 y^2 z^2
template <int SIGN, class T>
LBM_HD T cum_222(const T *in, T rinv) {
  const T d200 = in[mono(2, 0, 0)], d020 = in[mono(0, 2, 0)], d002 = in[mono(0, 0, 2)];
  const T d110 = in[mono(1, 1, 0)], d101 = in[mono(1, 0, 1)], d011 = in[mono(0, 1, 1)];
  const T lin4 = in[mono(0, 2, 2)] + in[mono(2, 0, 2)] + in[mono(2, 2, 0)];
  const T lin2 = d200 + d020 + d002;
  const T q24 = d200 * in[mono(0, 2, 2)] + d020 * in[mono(2, 0, 2)] + d002 * in[mono(2, 2, 0)] +
                T(4) * (d110 * in[mono(1, 1, 2)] + d101 * in[mono(1, 2, 1)] + d011 * in[mono(2, 1, 1)]) +
                T(2) * (in[mono(2, 1, 0)] * in[mono(0, 1, 2)] + in[mono(2, 0, 1)] * in[mono(0, 2, 1)] +
                        in[mono(1, 2, 0)] * in[mono(1, 0, 2)]) +
                T(4) * in[mono(1, 1, 1)] * in[mono(1, 1, 1)];
  const T q22 = d200 * d020 + d200 * d002 + d020 * d002 + T(2) * (d011 * d011 + d101 * d101 + d110 * d110);
  const T c222 = d200 * d020 * d002 + T(2) * (d200 * d011 * d011 + d020 * d101 * d101 + d002 * d110 * d110) +
                 T(8) * d110 * d101 * d011;
  if constexpr (SIGN < 0) {
    return in[mono(2, 2, 2)] - Cs<T>::cs2 * lin4 + Cs<T>::cs4 * lin2 - q24 * rinv +
           T(2) * Cs<T>::cs2 * q22 * rinv + T(2) * c222 * rinv * rinv;
  } else {
    return in[mono(2, 2, 2)] + Cs<T>::cs2 * lin4 + Cs<T>::cs4 * lin2 + q24 * rinv + Cs<T>::cs2 * q22 * rinv +
           c222 * rinv * rinv;
  }
}

// in-place map of orders >= 4 (orders 2, 3 are unchanged); REG: inputs of order >= 3 are 0
// c2 is the equilibrium's squared speed of sound (1/3 for the Maxwellian, g h / 2 for SWEK;
// the 3-D maps use 1/3)
template <int S, int SIGN, bool REG, class T>
LBM_HD void cumulant_map(T *v, T rinv, T c2 = Cs<T>::cs2) {
  if constexpr (Lat<S>::D == 2) {
    constexpr int e22 = mono(2, 2, 0), e20 = mono(2, 0, 0), e02 = mono(0, 2, 0), e11 = mono(1, 1, 0);
    T lin = c2 * (v[e20] + v[e02]);
    T quad = (v[e20] * v[e02] + T(2) * v[e11] * v[e11]) * rinv;
    v[e22] = SIGN < 0 ? v[e22] - lin - quad : v[e22] + lin + quad;
  } else {
    T in[27];
    sfor<27>([&](auto E) { in[E] = v[E]; });
    v[mono(2, 2, 0)] = cum_aabb<0, 1, 2, SIGN>(in, rinv);
    v[mono(2, 0, 2)] = cum_aabb<0, 2, 1, SIGN>(in, rinv);
    v[mono(0, 2, 2)] = cum_aabb<1, 2, 0, SIGN>(in, rinv);
    if constexpr (S == D3Q27) {
      v[mono(2, 1, 1)] = cum_aabc<0, 1, 2, SIGN>(in, rinv);
      v[mono(1, 2, 1)] = cum_aabc<1, 0, 2, SIGN>(in, rinv);
      v[mono(1, 1, 2)] = cum_aabc<2, 0, 1, SIGN>(in, rinv);
      if constexpr (!REG) {
        v[mono(2, 2, 1)] = cum_aabbc<0, 1, 2, SIGN>(in, rinv);
        v[mono(2, 1, 2)] = cum_aabbc<0, 2, 1, SIGN>(in, rinv);
        v[mono(1, 2, 2)] = cum_aabbc<1, 2, 0, SIGN>(in, rinv);
      } else {
        v[mono(2, 2, 1)] = T(0);
        v[mono(2, 1, 2)] = T(0);
        v[mono(1, 2, 2)] = T(0);
      }
      v[mono(2, 2, 2)] = cum_222<SIGN>(in, rinv);
    }
  }
}

// ---------------------------------------------------------------------------------------
// Shallow-water equilibrium of Zhou (sec. 5.2) in deviation form about f0 = f^eq(1, 0):
//   f_0 - f0_0 = dh - 5 g (h^2 - 1) / 6 - 2 h u.u / 3
//   f_i - f0_i = lambda_i [ g (h^2 - 1) / 6 + h (xi.u / 3 + (xi.u)^2 / 2 - u.u / 6) ]
// ---------------------------------------------------------------------------------------
template <class T>
LBM_HD void swe_feq_dev(T *g9, T dh, T h, T ux, T uy, T grav) {
  const T h2m1 = dh * (T(2) + dh);
  const T uu = ux * ux + uy * uy;
  const T a = grav * h2m1 * T(1.0 / 6.0);  // g (h^2 - 1) / 6
  const T d = a - h * uu * T(1.0 / 6.0);   // ... - h u.u / 6
  const T b = h * T(1.0 / 3.0), c = T(0.5) * h;
  sfor<9>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = vel9(i, 0), cy = vel9(i, 1);
    constexpr int gi = (cx + 1) + 3 * (cy + 1);
    if constexpr (i == 0) {
      g9[gi] = dh - T(5) * a - T(2.0 / 3.0) * h * uu;
    } else {
      constexpr T lam = (cx != 0 && cy != 0) ? T(0.25) : T(1);
      T xu = T(0);
      if constexpr (cx != 0) xu = cx > 0 ? xu + ux : xu - ux;
      if constexpr (cy != 0) xu = cy > 0 ? xu + uy : xu - uy;
      g9[gi] = lam * (d + xu * (b + c * xu));
    }
  });
}

// Raw moments of Zhou's equilibrium as deviations about its rest state (h = 1, u = 0), in
// closed form: h, h u, g (h^2 - 1) / 2 + h u_a^2, h ux uy, h u_b / 3 (x^2 y and x y^2),
// g (h^2 - 1) / 6 + h u.u / 3 (x^2 y^2); the same as M applied to swe_feq_dev.
template <class T>
LBM_HD void swe_meq_dev(T *m, T dh, T h, const T *u, T grav) {
  const T ux = u[0], uy = u[1];
  const T h2m1 = dh * (T(2) + dh);
  const T h3 = h * T(1.0 / 3.0);
  m[mono(0, 0, 0)] = dh;
  m[mono(1, 0, 0)] = h * ux;
  m[mono(0, 1, 0)] = h * uy;
  m[mono(2, 0, 0)] = T(0.5) * grav * h2m1 + h * ux * ux;
  m[mono(0, 2, 0)] = T(0.5) * grav * h2m1 + h * uy * uy;
  m[mono(1, 1, 0)] = h * ux * uy;
  m[mono(2, 1, 0)] = h3 * uy;
  m[mono(1, 2, 0)] = h3 * ux;
  m[mono(2, 2, 0)] = grav * h2m1 * T(1.0 / 6.0) + h3 * (ux * ux + uy * uy);
}

// ---------------------------------------------------------------------------------------
// Venturi's shallow-water equilibrium (D2Q9) as raw-moment deviations about the rest state
// h = 1, u = 0 (whose squared speed of sound is c0 = g / 2):
//   m_eq(a, b) = h prod_d mu(E_d),  mu = (1, u_d, c^2 + u_d^2),  c^2 = g h / 2.
// The u-free part of a moment with k exponent-2 axes is c0^k (h^(k+1) - 1), written with
// dh = h - 1 as dh, dh (2 + dh), dh (3 + dh (3 + dh)); every other term carries u.
// ---------------------------------------------------------------------------------------
template <class T>
LBM_HD void swek_meq_dev(T *m, T dh, T h, const T *u, T grav) {
  const T c0 = T(0.5) * grav;
  const T c2 = c0 * h;
  const T ux = u[0], uy = u[1];
  const T uxx = ux * ux, uyy = uy * uy;
  const T k1 = c0 * (dh * (T(2) + dh));
  m[mono(0, 0, 0)] = dh;
  m[mono(1, 0, 0)] = h * ux;
  m[mono(0, 1, 0)] = h * uy;
  m[mono(2, 0, 0)] = k1 + h * uxx;
  m[mono(0, 2, 0)] = k1 + h * uyy;
  m[mono(1, 1, 0)] = h * ux * uy;
  m[mono(2, 1, 0)] = h * (c2 + uxx) * uy;
  m[mono(1, 2, 0)] = h * ux * (c2 + uyy);
  m[mono(2, 2, 0)] = c0 * c0 * (dh * (T(3) + dh * (T(3) + dh))) + h * (c2 * (uxx + uyy) + uxx * uyy);
}

// ---------------------------------------------------------------------------------------
// Single relaxation time in population space.  The second-order polynomial equilibrium
//   f_eq_i = w_i rho (1 + xi.u / cs2 + (xi.u)^2 / (2 cs4) - u.u / (2 cs2))
// in deviation form about f0 = w:
//   df_eq_i = w_i (drho + rho (3 xi.u + 9/2 (xi.u)^2 - 3/2 u.u)),
// relaxed as df* = df_eq + (1 - omega)(df - df_eq); 1 - omega arrives as R.b2[0][0].
// ---------------------------------------------------------------------------------------
template <int S, class T>
LBM_HD void srt_feq_dev(T *feq, T drho, T rho, const T *u) {
  using L = Lat<S>;
  const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::c(i, 0), cy = L::c(i, 1), cz = L::c(i, 2);
    T xu = T(0);
    if constexpr (cx != 0) xu = cx > 0 ? xu + u[0] : xu - u[0];
    if constexpr (cy != 0) xu = cy > 0 ? xu + u[1] : xu - u[1];
    if constexpr (cz != 0) xu = cz > 0 ? xu + u[2] : xu - u[2];
    const T poly = T(3) * xu + T(4.5) * xu * xu - T(1.5) * uu;
    feq[L::gidx(i)] = T(L::w(i)) * (drho + rho * poly);
  });
}

// ---------------------------------------------------------------------------------------
// Guo's forcing populations (the source term of eq. LbUpdateScheme, sec. 2.1):
//   S_i = w_i [ (xi_i - u) / cs2 + (xi_i . u) xi_i / cs4 ] . F,  in grid order
// ---------------------------------------------------------------------------------------
template <int S, class T>
LBM_HD void guo_source(T *src, const T *u, const T *F) {
  using L = Lat<S>;
  sfor<L::G>([&](auto E) { src[E] = T(0); });
  const T uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    T xF = T(0), xu = T(0);
    sfor<3>([&](auto Dd) {
      constexpr int d = decltype(Dd)::value;
      if constexpr (L::c(i, d) > 0) {
        xF += F[d];
        xu += u[d];
      } else if constexpr (L::c(i, d) < 0) {
        xF -= F[d];
        xu -= u[d];
      }
    });
    src[L::gidx(i)] = T(L::w(i)) * (T(3) * (xF - uF) + T(9) * xu * xF);
  });
}

// He's forcing populations (He, Shan and Doolen): S_i = (xi_i - u) . F f_eq_i / (rho cs2),
// with f_eq the method's equilibrium populations, here w_i + fe_i (fe: their deviations)
template <int S, class T>
LBM_HD void he_source(T *src, const T *fe, const T *u, const T *F, T rinv) {
  using L = Lat<S>;
  sfor<L::G>([&](auto E) { src[E] = T(0); });
  const T uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int gi = L::gidx(i);
    T xF = T(0);
    sfor<3>([&](auto Dd) {
      constexpr int d = decltype(Dd)::value;
      if constexpr (L::c(i, d) > 0) xF += F[d];
      else if constexpr (L::c(i, d) < 0) xF -= F[d];
    });
    src[gi] = T(3) * (xF - uF) * (T(L::w(i)) + fe[gi]) * rinv;
  });
}

enum ForceModel { FORCE_GUO = 0, FORCE_HE = 1 };

// Cross-order part of the relaxation for a basis whose polynomials mix orders (the orthogonal
// bases): x holds c31 v1 at the order-3 entries, c42 v2 at order 4, c53 v3 + c51 v1 at order 5
// and c62 v2 + c64 v4 at order 6, from the pre-relaxation deviations v (other entries
// untouched).  v1 is -F/2 with a body force, else zero.
template <int S, class T, bool FORCE>
LBM_HD void cross_orders(T *x, const T *v, const Relax<T> &R) {
  constexpr int e1[3] = {1, 3, 9};  // x, y, z
  if constexpr (Lat<S>::D == 3) {
    sfor<7>([&](auto J) {
      constexpr int j = decltype(J)::value;
      T acc = T(0);
      if constexpr (FORCE) sfor<3>([&](auto K) { acc += R.c31[j][K] * v[e1[K]]; });
      x[o3_3d(j)] = acc;
    });
    sfor<6>([&](auto J) {
      constexpr int j = decltype(J)::value;
      T acc = T(0);
      sfor<6>([&](auto K) { acc += R.c42[j][K] * v[o2_3d(K)]; });
      x[o4_3d(j)] = acc;
    });
    if constexpr (S == D3Q27) {
      sfor<3>([&](auto J) {
        constexpr int j = decltype(J)::value;
        T acc = T(0);
        sfor<7>([&](auto K) { acc += R.c53[j][K] * v[o3_3d(K)]; });
        if constexpr (FORCE) sfor<3>([&](auto K) { acc += R.c51[j][K] * v[e1[K]]; });
        x[o5_3d(j)] = acc;
      });
      T acc = T(0);
      sfor<6>([&](auto K) { acc += R.c62[K] * v[o2_3d(K)] + R.c64[K] * v[o4_3d(K)]; });
      x[26] = acc;
    }
  } else {
    sfor<2>([&](auto J) {
      constexpr int j = decltype(J)::value;
      x[o3_2d(j)] = FORCE ? R.c31[j][0] * v[1] + R.c31[j][1] * v[3] : T(0);
    });
    x[8] = R.c42[0][0] * v[o2_2d(0)] + R.c42[0][1] * v[o2_2d(1)] + R.c42[0][2] * v[o2_2d(2)];
  }
}

// ---------------------------------------------------------------------------------------
// the collision in moment space: m holds dm = M df (exponent-grid order) on entry and the
// post-collision dm* on exit.  Missing monomials (D3Q19) leave as zero.
// ---------------------------------------------------------------------------------------
// With FORCE, F is the body force of the cell (Guo's model): the equilibrium velocity is
// u = (j + F/2) / rho, the first-order non-equilibrium moments are -F/2, and the source
// moments weighted by (I - P^-1 S P / 2) = (I + B) / 2 are added in the collision space
// (raw moments, or central moments for the central and cumulant spaces); momentum grows by F.
// With CROSS the raw-moment relaxation adds the cross-order blocks of an orthogonal basis
// (a separate instantiation, so the graded kernels carry none of that arithmetic).
template <int S, int SP, int EQ, bool REG, class T, bool FORCE = false, bool CROSS = false>
LBM_HD void collide_moments(T *m, const Relax<T> &R, T grav, const T *F = nullptr, int fmodel = FORCE_GUO) {
  static_assert(!(FORCE && REG), "the forced collision uses the general kernel");
  static_assert(!CROSS || (SP == RAW && !REG && S != D3Q15),
                "the cross-order blocks belong to the general raw-moment kernel");
  constexpr int D = Lat<S>::D;
  constexpr int G = Lat<S>::G;
  constexpr int EX = 1, EY = 3, EZ = 9;
  const T drho = m[0];
  T jx = m[EX], jy = m[EY];
  T jz = (D == 3) ? m[EZ] : T(0);
  if constexpr (FORCE) {
    jx += T(0.5) * F[0];
    jy += T(0.5) * F[1];
    if constexpr (D == 3) jz += T(0.5) * F[2];
  }
  const T rho = T(1) + drho;
  const T rinv = T(1) / rho;
  T u[3] = {jx * rinv, jy * rinv, jz * rinv};
  T uu[3] = {u[0] * u[0], u[1] * u[1], u[2] * u[2]};

  // equilibrium moments (deviation form)
  T meq[G];
  if constexpr (EQ == SWE) {
    static_assert(S == D2Q9, "the shallow-water equilibria are two-dimensional");
    swe_meq_dev(meq, drho, rho, u, grav);
  } else if constexpr (EQ == SWEK) {
    static_assert(S == D2Q9, "the shallow-water equilibria are two-dimensional");
    swek_meq_dev(meq, drho, rho, u, grav);
  } else if constexpr (S == D3Q15 && SP == RAW) {
    // D3Q15's raw monomial classes cannot carry the Maxwellian's raw moments: its raw
    // equilibrium is the second-order polynomial one, taken to moments by the Chimera
    // (consistent within every class)
    sfor<G>([&](auto E) { meq[E] = T(0); });
    srt_feq_dev<S>(meq, drho, rho, u);
    chimera_forward<S>(meq);
  } else {
    // the Maxwellian's value on each monomial of the set; on D3Q15 (central moments and
    // cumulants) every other member of a class takes its representative's value, which
    // keeps the grid consistent for the inverse Chimera (rep(e) < e is already set)
    sfor<G>([&](auto E) {
      constexpr int e = decltype(E)::value;
      if constexpr (Lat<S>::has_mono_e(e)) meq[e] = meq_dev<e, SP == RAW>(drho, rho, u, uu);
      else meq[e] = S == D3Q15 ? meq[Lat<S>::rep(e)] : T(0);
    });
    meq[EX] = jx;
    meq[EY] = jy;
    if constexpr (D == 3) meq[EZ] = jz;
  }

  // non-equilibrium raw moments (orders >= 2; with a force also order 1, where it is -F/2)
  T v[G];
  sfor<G>([&](auto E) {
    constexpr int e = decltype(E)::value;
    if constexpr (Lat<S>::ord(e) == 0) v[e] = T(0);
    else if constexpr (Lat<S>::ord(e) == 1) v[e] = FORCE ? m[e] - meq[e] : T(0);
    else if constexpr (REG && Lat<S>::ord(e) > 2) v[e] = T(0);
    else v[e] = m[e] - meq[e];
  });

  // the source's moments (raw, shifted to central for the central and cumulant spaces),
  // weighted by (I + B) / 2 on orders >= 2 and taken whole on the conserved orders
  auto add_force = [&](T *vv, bool central) {
    if constexpr (FORCE) {
      T fs[G];
      if (fmodel == FORCE_HE) {
        T fe[G];  // equilibrium populations (deviations) of the method at the shifted u
        sfor<G>([&](auto E) { fe[E] = meq[E]; });
        chimera_inverse<S>(fe);
        he_source<S>(fs, fe, u, F, rinv);
      } else {
        guo_source<S>(fs, u, F);
      }
      chimera_forward<S>(fs);
      if (central) binomial<S>(fs, -u[0], -u[1], -u[2]);
      T wfs[G];
      sfor<G>([&](auto E) { wfs[E] = fs[E]; });
      if constexpr (CROSS) {
        T xf[G];
        cross_orders<S, T, true>(xf, fs, R);
        relax<S, false>(wfs, R);
        sfor<G>([&](auto E) {
          constexpr int e = decltype(E)::value;
          if constexpr (Lat<S>::has_mono_e(e) && Lat<S>::ord(e) >= 3) wfs[e] += xf[e];
        });
      } else {
        relax<S, false>(wfs, R);
      }
      sfor<G>([&](auto E) {
        constexpr int e = decltype(E)::value;
        if constexpr (Lat<S>::has_mono_e(e) && Lat<S>::ord(e) >= 2) vv[e] += T(0.5) * (fs[e] + wfs[e]);
        else if constexpr (Lat<S>::ord(e) == 1) vv[e] += fs[e];
      });
    }
  };

  if constexpr (SP == RAW) {
    if constexpr (CROSS) {
      T x[G];
      cross_orders<S, T, FORCE>(x, v, R);
      relax<S, false>(v, R);
      sfor<G>([&](auto E) {
        constexpr int e = decltype(E)::value;
        if constexpr (Lat<S>::has_mono_e(e) && Lat<S>::ord(e) >= 3) v[e] += x[e];
      });
    } else {
      relax<S, REG>(v, R);
    }
    add_force(v, false);
  } else {
    // to central moments; with zero orders 0, 1 the order-2 entries are unchanged
    if constexpr (!REG) binomial<S>(v, -u[0], -u[1], -u[2]);
    if constexpr (SP == CENTRAL) {
      relax<S, REG>(v, R);
    } else {
      const T c2 = EQ == SWEK ? T(0.5) * grav * rho : Cs<T>::cs2;
      if constexpr (!REG) cumulant_map<S, -1, false>(v, rinv, c2);
      relax<S, REG>(v, R);
      cumulant_map<S, +1, REG>(v, rinv, c2);
    }
    add_force(v, true);
    binomial<S>(v, u[0], u[1], u[2]);
  }
  // dm* = dm_eq + non-equilibrium part; conserved moments exactly (plus F with a force)
  sfor<G>([&](auto E) {
    constexpr int e = decltype(E)::value;
    if constexpr (!Lat<S>::has_mono_e(e)) m[e] = S == D3Q15 ? m[Lat<S>::rep(e)] : T(0);  // rep(e) < e: final
    else if constexpr (Lat<S>::ord(e) >= 2 || (FORCE && Lat<S>::ord(e) == 1)) m[e] = meq[e] + v[e];
  });
}

// ---------------------------------------------------------------------------------------
// Single relaxation time: see srt_feq_dev above.
// ---------------------------------------------------------------------------------------
template <int S, class T, bool FORCE = false>
LBM_HD void collide_srt(T *g, const Relax<T> &R, const T *F = nullptr, int fmodel = FORCE_GUO) {
  using L = Lat<S>;
  T drho = T(0), j[3] = {T(0), T(0), T(0)};
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    const T v = g[L::gidx(i)];
    drho += v;
    sfor<3>([&](auto Dd) {
      constexpr int d = decltype(Dd)::value;
      if constexpr (L::c(i, d) > 0) j[d] += v;
      else if constexpr (L::c(i, d) < 0) j[d] -= v;
    });
  });
  if constexpr (FORCE) {
    sfor<3>([&](auto Dd) { j[decltype(Dd)::value] += T(0.5) * F[decltype(Dd)::value]; });
  }
  const T rho = T(1) + drho;
  const T rinv = T(1) / rho;
  const T u[3] = {j[0] * rinv, j[1] * rinv, j[2] * rinv};
  T feq[Lat<S>::G];
  srt_feq_dev<S>(feq, drho, rho, u);
  const T b = R.b2[0][0];
  sfor<L::Q>([&](auto I) {
    constexpr int gi = L::gidx(decltype(I)::value);
    g[gi] = fma(b, g[gi] - feq[gi], feq[gi]);
  });
  if constexpr (FORCE) {
    T src[Lat<S>::G];
    if (fmodel == FORCE_HE) he_source<S>(src, feq, u, F, rinv);
    else guo_source<S>(src, u, F);
    const T wf = T(0.5) * (T(1) + b);  // 1 - omega / 2
    sfor<L::Q>([&](auto I) {
      constexpr int gi = L::gidx(decltype(I)::value);
      g[gi] = fma(wf, src[gi], g[gi]);
    });
  }
}

// ---------------------------------------------------------------------------------------
// the collision: g holds df (grid order, missing velocities zero) and receives df*
// ---------------------------------------------------------------------------------------
template <int S, int SP, int EQ, bool REG, class T, bool FORCE = false, bool CROSS = false>
LBM_HD void collide(T *g, const Relax<T> &R, T grav, const T *F = nullptr, int fmodel = FORCE_GUO) {
  if constexpr (SP == SRT) {
    collide_srt<S, T, FORCE>(g, R, F, fmodel);
  } else if constexpr (SP != IDENTITY) {
    chimera_forward<S>(g);
    collide_moments<S, SP, EQ, REG, T, FORCE, CROSS>(g, R, grav, F, fmodel);
    chimera_inverse<S>(g);
  }
}

// equilibrium populations df_eq(rho, u) in grid order (initialisation), sec. 2.4
template <int S, int SP, int EQ, class T>
LBM_HD void equilibrium_dev(T *g, T drho, const T *u, T grav) {
  constexpr int G = Lat<S>::G;
  const T rho = T(1) + drho;
  if constexpr (EQ == SWE) {
    swe_feq_dev(g, drho, rho, u[0], u[1], grav);
  } else if constexpr (EQ == SWEK) {
    swek_meq_dev(g, drho, rho, u, grav);
    chimera_inverse<S>(g);
  } else if constexpr (SP == SRT || (S == D3Q15 && SP == RAW)) {
    sfor<G>([&](auto E) { g[E] = T(0); });
    srt_feq_dev<S>(g, drho, rho, u);
  } else {
    T uu[3] = {u[0] * u[0], u[1] * u[1], u[2] * u[2]};
    sfor<G>([&](auto E) {
      constexpr int e = decltype(E)::value;
      if constexpr (Lat<S>::has_mono_e(e)) g[e] = meq_dev<e, SP == RAW>(drho, rho, u, uu);
      else g[e] = S == D3Q15 ? g[Lat<S>::rep(e)] : T(0);
    });
    chimera_inverse<S>(g);
  }
}

}  // namespace lbm
