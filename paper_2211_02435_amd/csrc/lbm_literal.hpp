// Literal evaluation of the three collision forms of sec. 2.2, for the round-off study of
// sec. 5.1 (the energy plateau of the decaying Taylor-Green vortex).
//
// The default sweep evaluates every form with one deviation-organised arithmetic in which no
// background value is ever subtracted from another.  Here each form is evaluated the way it is
// written, so that their different round-off can be measured:
//   LIT_A  absolute storage, eq. MrtUpdateGeneral:  q = T(f), f* = T^-1(q*), with q, q_eq and
//          every intermediate absolute (rho near 1, moments near their background values);
//   LIT_B  zero-centred storage, eq. MrtUpdateGeneralDeviationOnly:  dq = T(df), the
//          equilibrium deviation formed by subtraction, dq_eq = q_eq(rho, u) - T(f0)
//          (raw and central moments and SRT only: the transform must be linear in f);
//   LIT_C  zero-centred storage, eq. MrtUpdateAbsoluteFromZeroCentered:  q = T(df + f0),
//          df* = T^-1(q*) - f0.  The raw-moment stage of T is linear, so the background
//          enters as its raw moments, m = M df + m0, and leaves as dm* = m* - m0 before the
//          inverse (where a generated kernel folds the constants f0); the nonlinear stages
//          (central moments, cumulants, relaxation against the absolute equilibrium) run on
//          the absolute moments.  SRT has T = identity: f = df + f0 per population.
// Relaxation is q* = q_eq + (I - P^-1 S P)(q - q_eq) on the orders >= 2 in every form (the
// conserved rows are carried), the same blocks as the default sweep.
// Cumulants are absolute here: C = rho c with c the derivatives of the logarithm of the
// normalised moment-generating function (sec. 2.3.3, sec. 4.2.1), written through the set
// partitions of each monomial's letters into blocks of at least two letters (first-order
// central moments vanish in the co-moving frame).
#pragma once

#include "lbm_kernels.hpp"

namespace lbm {

enum LiteralForm { LIT_A = 0, LIT_B = 1, LIT_C = 2 };

// background raw moment of exponent index e: prod over axes of (1, 0, cs2)
template <int E, class T>
__host__ __device__ constexpr T background_moment() {
  constexpr int a = E % 3, b = (E / 3) % 3, c = E / 9;
  return (a == 1 || b == 1 || c == 1)
             ? T(0)
             : (a == 2 ? Cs<T>::cs2 : T(1)) * (b == 2 ? Cs<T>::cs2 : T(1)) * (c == 2 ? Cs<T>::cs2 : T(1));
}

// absolute cumulants from absolute central moments (orders 4..6; orders 2, 3 coincide)
template <int A, int B, int C, class T>
LBM_HD T lit_aabb(const T *k, T rinv, int sign) {
  constexpr int aabb = mi<A, B, C>(2, 2, 0), aa = mi<A, B, C>(2, 0, 0), bb = mi<A, B, C>(0, 2, 0),
                ab = mi<A, B, C>(1, 1, 0);
  const T p = (k[aa] * k[bb] + T(2) * k[ab] * k[ab]) * rinv;
  return sign < 0 ? k[aabb] - p : k[aabb] + p;
}
template <int A, int B, int C, class T>
LBM_HD T lit_aabc(const T *k, T rinv, int sign) {
  constexpr int aabc = mi<A, B, C>(2, 1, 1), aa = mi<A, B, C>(2, 0, 0), bc = mi<A, B, C>(0, 1, 1),
                ab = mi<A, B, C>(1, 1, 0), ac = mi<A, B, C>(1, 0, 1);
  const T p = (k[aa] * k[bc] + T(2) * k[ab] * k[ac]) * rinv;
  return sign < 0 ? k[aabc] - p : k[aabc] + p;
}
template <int A, int B, int C, class T>
LBM_HD T lit_aabbc(const T *k, T rinv, int sign) {
  constexpr int aabbc = mi<A, B, C>(2, 2, 1), aa = mi<A, B, C>(2, 0, 0), bb = mi<A, B, C>(0, 2, 0),
                ab = mi<A, B, C>(1, 1, 0), ac = mi<A, B, C>(1, 0, 1), bc = mi<A, B, C>(0, 1, 1),
                bbc = mi<A, B, C>(0, 2, 1), aac = mi<A, B, C>(2, 0, 1), abc = mi<A, B, C>(1, 1, 1),
                abb = mi<A, B, C>(1, 2, 0), aab = mi<A, B, C>(2, 1, 0);
  const T p = (k[aa] * k[bbc] + k[bb] * k[aac] + T(4) * k[ab] * k[abc] + T(2) * k[ac] * k[abb] +
               T(2) * k[bc] * k[aab]) *
              rinv;
  return sign < 0 ? k[aabbc] - p : k[aabbc] + p;
}
// x^2 y^2 z^2.  Partitions into blocks of >= 2 letters: (2,4) 15, (3,3) 10, (2,2,2) 15.
// forward:  C = k6 - (S24 + S33) / rho + 2 S222 / rho^2   (S over central moments)
// backward: k6 = C + (S24 + S33) / rho + S222 / rho^2     (S over cumulants)
template <class T>
LBM_HD T lit_222(const T *k, T rinv, int sign) {
  const T k200 = k[mono(2, 0, 0)], k020 = k[mono(0, 2, 0)], k002 = k[mono(0, 0, 2)];
  const T k110 = k[mono(1, 1, 0)], k101 = k[mono(1, 0, 1)], k011 = k[mono(0, 1, 1)];
  const T s24 = k200 * k[mono(0, 2, 2)] + k020 * k[mono(2, 0, 2)] + k002 * k[mono(2, 2, 0)] +
                T(4) * (k110 * k[mono(1, 1, 2)] + k101 * k[mono(1, 2, 1)] + k011 * k[mono(2, 1, 1)]);
  const T s33 = T(2) * (k[mono(2, 1, 0)] * k[mono(0, 1, 2)] + k[mono(2, 0, 1)] * k[mono(0, 2, 1)] +
                        k[mono(1, 2, 0)] * k[mono(1, 0, 2)]) +
                T(4) * k[mono(1, 1, 1)] * k[mono(1, 1, 1)];
  const T s222 = k200 * k020 * k002 + T(2) * (k200 * k011 * k011 + k020 * k101 * k101 + k002 * k110 * k110) +
                 T(8) * k110 * k101 * k011;
  if (sign < 0) return k[mono(2, 2, 2)] - (s24 + s33) * rinv + T(2) * s222 * rinv * rinv;
  return k[mono(2, 2, 2)] + (s24 + s33) * rinv + s222 * rinv * rinv;
}

// in place: central moments -> cumulants (SIGN -1) or back (SIGN +1), orders 4..6
template <int S, int SIGN, class T>
LBM_HD void lit_cumulant_map(T *v, T rinv) {
  T in[Lat<S>::G];
  sfor<Lat<S>::G>([&](auto E) { in[E] = v[E]; });
  if constexpr (Lat<S>::D == 2) {
    v[mono(2, 2, 0)] = lit_aabb<0, 1, 2>(in, rinv, SIGN);
  } else {
    v[mono(2, 2, 0)] = lit_aabb<0, 1, 2>(in, rinv, SIGN);
    v[mono(2, 0, 2)] = lit_aabb<0, 2, 1>(in, rinv, SIGN);
    v[mono(0, 2, 2)] = lit_aabb<1, 2, 0>(in, rinv, SIGN);
    if constexpr (S == D3Q27) {
      v[mono(2, 1, 1)] = lit_aabc<0, 1, 2>(in, rinv, SIGN);
      v[mono(1, 2, 1)] = lit_aabc<1, 0, 2>(in, rinv, SIGN);
      v[mono(1, 1, 2)] = lit_aabc<2, 0, 1>(in, rinv, SIGN);
      v[mono(2, 2, 1)] = lit_aabbc<0, 1, 2>(in, rinv, SIGN);
      v[mono(2, 1, 2)] = lit_aabbc<0, 2, 1>(in, rinv, SIGN);
      v[mono(1, 2, 2)] = lit_aabbc<1, 2, 0>(in, rinv, SIGN);
      v[mono(2, 2, 2)] = lit_222(in, rinv, SIGN);
    }
  }
}

// SRT in the three literal forms; g holds f (LIT_A) or df (LIT_B, LIT_C)
template <int S, int FORM, class T>
LBM_HD void lit_srt(T *g, const Relax<T> &R) {
  using L = Lat<S>;
  if constexpr (FORM == LIT_C) sfor<L::Q>([&](auto I) { g[L::gidx(I)] += T(L::w(I)); });
  T s0 = T(0), j[3] = {T(0), T(0), T(0)};
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    const T v = g[L::gidx(i)];
    s0 += v;
    sfor<3>([&](auto Dd) {
      constexpr int d = decltype(Dd)::value;
      if constexpr (L::c(i, d) > 0) j[d] += v;
      else if constexpr (L::c(i, d) < 0) j[d] -= v;
    });
  });
  const T rho = FORM == LIT_B ? T(1) + s0 : s0;
  const T rinv = T(1) / rho;
  const T u[3] = {j[0] * rinv, j[1] * rinv, j[2] * rinv};
  const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const T b = R.b2[0][0];
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int gi = L::gidx(i);
    const T xu = T(L::c(i, 0)) * u[0] + T(L::c(i, 1)) * u[1] + T(L::c(i, 2)) * u[2];
    T feq = T(L::w(i)) * rho * (T(1) + T(3) * xu + T(4.5) * xu * xu - T(1.5) * uu);
    if constexpr (FORM == LIT_B) feq = feq - T(L::w(i));
    g[gi] = feq + b * (g[gi] - feq);
  });
  if constexpr (FORM == LIT_C) sfor<L::Q>([&](auto I) { g[L::gidx(I)] -= T(L::w(I)); });
}

// the literal collision; g holds f (LIT_A) or df (LIT_B, LIT_C) in grid order
template <int S, int SP, int FORM, class T, bool CROSS = false>
LBM_HD void collide_literal(T *g, const Relax<T> &R) {
  static_assert(!(SP == CUMULANT && FORM == LIT_B), "no delta-equilibrium for the nonlinear cumulant transform");
  static_assert(!CROSS || SP == RAW, "the cross-order blocks belong to the orthogonal raw-moment bases");
  if constexpr (SP == SRT) {
    lit_srt<S, FORM>(g, R);
    return;
  } else {
    using L = Lat<S>;
    constexpr int D = L::D, G = L::G;
    constexpr int EX = 1, EY = 3, EZ = 9;
    chimera_forward<S>(g);  // m = M f (LIT_A), or dm = M df
    if constexpr (FORM == LIT_C) {
      sfor<G>([&](auto E) {
        constexpr int e = decltype(E)::value;
        if constexpr (L::has_mono_e(e) && background_moment<e, T>() != T(0)) g[e] = g[e] + background_moment<e, T>();
      });
    }
    const T rho = FORM == LIT_B ? T(1) + g[0] : g[0];
    const T rinv = T(1) / rho;
    T u[3] = {g[EX] * rinv, g[EY] * rinv, D == 3 ? g[EZ] * rinv : T(0)};
    T uu[3] = {u[0] * u[0], u[1] * u[1], u[2] * u[2]};

    // equilibrium in collision space (absolute), then minus the background for LIT_B
    T qeq[G];
    if constexpr (SP == RAW) {
      sfor<G>([&](auto E) {
        constexpr int e = decltype(E)::value;
        // rho prod mu truncated at second order in u: meq_dev with drho = rho is rho (m0 + t)
        qeq[e] = meq_dev<e, true>(rho, rho, u, uu);
        if constexpr (FORM == LIT_B) qeq[e] = qeq[e] - background_moment<e, T>();
      });
    } else {
      T q0[G];
      if constexpr (FORM == LIT_B) {
        sfor<G>([&](auto E) { q0[E] = background_moment<decltype(E)::value, T>(); });
        binomial<S>(q0, -u[0], -u[1], -u[2]);  // central moments of f0 about u
      }
      sfor<G>([&](auto E) {
        constexpr int e = decltype(E)::value;
        constexpr int a = e % 3, b = (e / 3) % 3, c = e / 9;
        if constexpr (SP == CENTRAL) {
          qeq[e] = rho * background_moment<e, T>();  // rho prod (1, 0, cs2)
          if constexpr (FORM == LIT_B) qeq[e] = qeq[e] - q0[e];
        } else {
          // cumulants of the Maxwellian: C_000 = rho, C_aa = rho cs2, all others zero
          constexpr bool second = (a + b + c == 2) && (a == 2 || b == 2 || c == 2);
          qeq[e] = e == 0 ? rho : (second ? rho * Cs<T>::cs2 : T(0));
        }
      });
      binomial<S>(g, -u[0], -u[1], -u[2]);  // central moments (or their deviations)
      if constexpr (SP == CUMULANT) lit_cumulant_map<S, -1>(g, rinv);
    }

    // relax the orders >= 2 toward equilibrium
    T v[G];
    sfor<G>([&](auto E) {
      constexpr int e = decltype(E)::value;
      v[e] = L::ord(e) < 2 ? T(0) : g[e] - qeq[e];
    });
    if constexpr (CROSS) {
      // orthogonal raw basis: the blocks between orders (orders 0 and 1 carry no deviation)
      T x[G];
      cross_orders<S, T, false>(x, v, R);
      relax<S, false>(v, R);
      sfor<G>([&](auto E) {
        constexpr int e = decltype(E)::value;
        if constexpr (L::has_mono_e(e) && L::ord(e) >= 3) v[e] += x[e];
      });
    } else {
      relax<S, false>(v, R);
    }
    sfor<G>([&](auto E) {
      constexpr int e = decltype(E)::value;
      if constexpr (!L::has_mono_e(e)) g[e] = T(0);
      else if constexpr (L::ord(e) >= 2) g[e] = qeq[e] + v[e];
    });

    if constexpr (SP == CUMULANT) lit_cumulant_map<S, +1>(g, rinv);
    if constexpr (SP != RAW) binomial<S>(g, u[0], u[1], u[2]);
    if constexpr (FORM == LIT_C) {
      sfor<G>([&](auto E) {
        constexpr int e = decltype(E)::value;
        if constexpr (L::has_mono_e(e) && background_moment<e, T>() != T(0)) g[e] = g[e] - background_moment<e, T>();
      });
    }
    chimera_inverse<S>(g);
  }
}

// the literal sweep: pull streaming, one cell per thread, the buffers hold f (LIT_A) or df
template <int S, int SP, int FORM, class ST, class CT, bool CROSS = false>
__global__ void __launch_bounds__(512) sweep_literal_kernel(SweepArgs<ST, CT> a) {
  using L = Lat<S>;
  const CellPos p = tile_cell_args(a, 1);
  if (!p.valid) return;
  const Nbr<L::D> nb(p.x, p.y, p.z, a.nx, a.ny, a.nz, a.L);
  CT g[L::G];
  sfor<L::G>([&](auto E) { g[E] = CT(0); });
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::c(i, 0), cy = L::c(i, 1), cz = L::c(i, 2);
    g[L::gidx(i)] = CT(ldp(a.src, uint64_t(i) * a.L.ps + nb.zpart(cz, -1), nb.lane(cx, cy, -1)));
  });
  collide_literal<S, SP, FORM, CT, CROSS>(g, a.R);
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    stp(a.dst, uint64_t(i) * a.L.ps + nb.zpart(0, 1), nb.lane(0, 0, 1), ST(g[L::gidx(i)]));
  });
}

}  // namespace lbm
