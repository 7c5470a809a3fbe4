// Per-node arithmetic of the forced lattice-Boltzmann step (device code, gfx950).
//
// Li, Duan & Shan, "Second-order force scheme for lattice Boltzmann method"
// (arXiv 2212.07494).  Lattice units; c_s^2 = 1/3 on D2Q9, D3Q19, D3Q27 and 2/3 on the
// high-order lattice D3Q39 (L::CS2N / L::CS2D); Hermite polynomials written in lattice
// units (H_m(e) = prod_a h_{m_a}(e_a), h_0 = 1, h_1 = e, h_2 = e^2 - c_s^2, ...).
//
// Everything here is templated on the lattice L (constants from lbm_tables.h) and the
// arithmetic type T (double or float), and every loop runs over compile-time indices
// (static_for), so the coefficient tables fold into immediates and zero coefficients
// disappear.  The operation order is fixed and identical in both precisions:
//   * each sum starts from -0.0 (the additive identity) and adds its non-zero terms
//     in index order;
//   * products of velocity components are formed left to right over x, y, z;
//   * constants are exact rationals rounded once;
//   * the MRT moment transforms (projection, shifts, reconstruction) add each term
//     with one explicit fused multiply-add (fmadd); nothing else is fused (the
//     library is compiled with -ffp-contract=off).
// With T = double this reproduces an FP64 implementation written in that order
// bit for bit.
//
// Populations are handled as deviations d_i = f-bar_i - w_i s from a constant shift
// s (s = 0 for plain storage): the mass moment carries d-rho = sum_i d_i and
// rho = s + d-rho, every other moment of d equals that of f-bar (sum_i w_i H_m = 0
// for m != 0), the step changes no mass, and where a full state is reconstructed
// (the initial state) the rest coefficient multiplies d-rho.  The same code thus
// serves plain and shifted storage and keeps the full relative precision of the
// small deviations in binary32.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "lbm_tables.h"

namespace lbm {

template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  [&]<int... I>(std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
  }(std::make_integer_sequence<int, N>{});
}

// Constant tables in the arithmetic precision.
template <class L, class T>
struct Tab;
template <class L>
struct Tab<L, double> {
  static constexpr double w(int i) { return L::W[i]; }
  static constexpr double h(int k, int i) { return L::H[k][i]; }
  static constexpr double minv(int i, int k) { return L::MINV[i][k]; }
};
template <class L>
struct Tab<L, float> {
  static constexpr float w(int i) { return L::Wf[i]; }
  static constexpr float h(int k, int i) { return L::Hf[k][i]; }
  static constexpr float minv(int i, int k) { return L::MINVf[i][k]; }
};

template <class T>
struct Macro {
  T drho, rho;
  T j[3];  // sum_i f-bar_i e_i = rho u-bar
  T u[3], F[3];
};

// Density, physical velocity and force density (Sec. II.B, eq:half_F and after):
// rho-bar = rho, rho u-bar = rho u - F/2 with F = rho g, so u = j/rho + g/2.
template <class L, class T>
__device__ __forceinline__ Macro<T> macroscopic(const T (&d)[L::Q], T shift, const T (&g)[3]) {
  Macro<T> M;
  T s = T(-0.0);
  static_for<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    s = s + d[i];
  });
  M.drho = s;
  M.rho = shift + s;
  static_for<L::D>([&](auto A) {
    constexpr int a = decltype(A)::value;
    T j = T(-0.0);
    static_for<L::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int ea = L::E[i][a];
      if constexpr (ea == 1) j = j + d[i];
      if constexpr (ea == -1) j = j + (-d[i]);
      if constexpr (ea > 1 || ea < -1) j = j + T(ea) * d[i];
    });
    M.j[a] = j;
    M.u[a] = j / M.rho + T(0.5) * g[a];
    M.F[a] = M.rho * g[a];
  });
  if constexpr (L::D == 2) {
    M.j[2] = T(0);
    M.u[2] = T(0);
    M.F[2] = T(0);
  }
  return M;
}

// u^m = prod_a u_a^{m_a}, left to right over x, y, z starting from 1.
template <class L, int K, class T>
__device__ __forceinline__ T upow(const T (&u)[3]) {
  T p = T(1);
  static_for<3>([&](auto A) {
    constexpr int a = decltype(A)::value;
    static_for<L::MI[K][a]>([&](auto) { p = p * u[a]; });
  });
  return p;
}

template <class T>
struct BGKCoef {
  T omega, hforce;  // 1/tau-hat, 1 - omega/2
};
template <class T>
struct SMRTCoef {
  T q2, q3;  // 1 - omega_n for orders 2 and 3
  // Factor 1 - omega_3/2 of the third-order force content (read only by the collisions
  // that carry it, see collide_smrt).
  T fq3;
  // Bulk rate: (q_bulk - q2) / D for the trace of the second-order moment (0 = one
  // rate for the whole order).
  T dqb;
  // Third-order trace rate: (q_31 - q3) / 2 for the pairs D_abb + D_acc (0 = one rate).
  T dq31;
};

// a * b + c rounded once (fused multiply-add).  The MRT collisions accumulate their moment
// transforms with it, in the same places as the oracle.
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Whether c is +-2^n: then c u^l is exact, and c u^l N rounds once inside an fma.  The
// shift coefficients C(m,l) are products of binomials C(m_a, l_a): powers of two where
// m_a <= 2 (D2Q9, D3Q19, D3Q27); D3Q39's orders 3 and 4 along one axis bring 3 and 6,
// for which the product c u^l is rounded first (the same expression in the oracle).
constexpr bool pow2_coef(int c) {
  const int a = c < 0 ? -c : c;
  return a > 0 && (a & (a - 1)) == 0;
}

// Whether MI[k] is a diagonal second-order index (2 e_a).
template <class L>
constexpr bool is_diag2(int k) {
  return L::ORD[k] == 2 && (L::MI[k][0] == 2 || L::MI[k][1] == 2 || L::MI[k][2] == 2);
}

// Central moment D_m = sum_{l <= m} C(m,l) (-u)^l N_{m-l} from the non-equilibrium raw
// moments N (the shift to the frame moving with u).
template <class L, int K, class T>
__device__ __forceinline__ T central(const T (&U)[L::NM], const T (&N)[L::NM]) {
  T Dm = N[K];
  static_for<L::NT[K]>([&](auto Tt) {
    constexpr int t = decltype(Tt)::value;
    constexpr int kl = L::TL[K][t], km = L::TM[K][t];
    static_assert(L::NM < L::Q || pow2_coef(L::CDN[K][t]));
    Dm = fmadd(T(L::CDN[K][t]) * U[kl], N[km], Dm);
  });
  return Dm;
}

// For a third-order index a + 2b (one axis with exponent 1, another with 2), the index of
// its trace partner a + 2c (c the third axis), which carries with it the axis-a component
// of the third-order trace; -1 otherwise or if the lattice lacks the partner.
template <class L>
constexpr int trace_partner3(int k) {
  if (L::ORD[k] != 3) return -1;
  int a = -1, b = -1;
  for (int t = 0; t < 3; ++t) {
    if (L::MI[k][t] == 1) a = t;
    if (L::MI[k][t] == 2) b = t;
  }
  if (a < 0 || b < 0) return -1;
  const int c = 3 - a - b;
  int m[3] = {0, 0, 0};
  m[a] = 1;
  m[c] = 2;
  for (int j = 0; j < L::NM; ++j)
    if (L::MI[j][0] == m[0] && L::MI[j][1] == m[1] && L::MI[j][2] == m[2]) return j;
  return -1;
}

// The population order pairs each velocity with its opposite, (e, -e) at i = 2p-1, 2p
// after the rest population, and H_m(-e) = (-1)^|m| H_m(e): an even-order moment is a sum
// over the pair sums, an odd-order one over the pair differences (the rest population
// enters only even moments), and the rows of the inverse transform split the same way.
// Whether L's tables in type T obey this exactly (required by the folded transforms).
template <class L, class T>
constexpr bool pair_symmetric() {
  for (int k = 0; k < L::NM; ++k) {
    const T sg = (L::ORD[k] % 2) ? T(-1) : T(1);
    if (sg < T(0) && (Tab<L, T>::h(k, 0) != T(0) || Tab<L, T>::minv(0, k) != T(0)))
      return false;
    for (int i = 1; i + 1 < L::Q; i += 2)
      if (Tab<L, T>::h(k, i + 1) != sg * Tab<L, T>::h(k, i) ||
          Tab<L, T>::minv(i + 1, k) != sg * Tab<L, T>::minv(i, k))
        return false;
  }
  return true;
}

// The populations folded over their pairs, p = 1..NP (index 0 unused): sums s_p =
// d_{2p-1} + d_{2p} and differences a_p = d_{2p-1} - d_{2p}.
template <class L, class T>
struct PairFold {
  static constexpr int NP = (L::Q - 1) / 2;
  T s[NP + 1], a[NP + 1];
  __device__ __forceinline__ explicit PairFold(const T (&d)[L::Q]) {
    static_assert(pair_symmetric<L, T>());
    static_for<NP>([&](auto Pp) {
      constexpr int p = decltype(Pp)::value + 1;
      s[p] = d[2 * p - 1] + d[2 * p];
      a[p] = d[2 * p - 1] - d[2 * p];
    });
  }
  // Raw moment k (order >= 1): from -0.0, the rest population, then each pair's sum (even
  // order) or difference (odd order), one fma a nonzero term.
  template <int k>
  __device__ __forceinline__ T project(const T (&d)[L::Q]) const {
    constexpr bool odd = L::ORD[k] % 2;
    T acc = T(-0.0);
    constexpr T h0 = Tab<L, T>::h(k, 0);
    if constexpr (h0 != T(0)) acc = fmadd(h0, d[0], acc);
    static_for<NP>([&](auto Pp) {
      constexpr int p = decltype(Pp)::value + 1;
      constexpr T h = Tab<L, T>::h(k, 2 * p - 1);
      if constexpr (h != T(0)) acc = fmadd(h, odd ? a[p] : s[p], acc);
    });
    return acc;
  }
};

// d += M^-1 dA folded over the pairs: the rest population sums its row over k >= 1; each
// pair sums its first member's row over the even- and the odd-order moments apart (E, O,
// each from -0.0 in k order, one fma a nonzero term) and takes d_{2p-1} + (E + O),
// d_{2p} + (E - O).
template <class L, class T>
__device__ __forceinline__ void reconstruct_folded(T (&d)[L::Q], const T (&dA)[L::NM]) {
  static_assert(pair_symmetric<L, T>());
  T acc = T(-0.0);
  static_for<L::NM>([&](auto K) {
    constexpr int k = decltype(K)::value;
    constexpr T cf = Tab<L, T>::minv(0, k);
    if constexpr (k > 0 && cf != T(0)) acc = fmadd(cf, dA[k], acc);
  });
  d[0] = d[0] + acc;
  static_for<(L::Q - 1) / 2>([&](auto Pp) {
    constexpr int i = 2 * decltype(Pp)::value + 1;
    T ev = T(-0.0), od = T(-0.0);
    static_for<L::NM>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr T cf = Tab<L, T>::minv(i, k);
      if constexpr (k > 0 && cf != T(0)) {
        if constexpr (L::ORD[k] % 2)
          od = fmadd(cf, dA[k], od);
        else
          ev = fmadd(cf, dA[k], ev);
      }
    });
    d[i] = d[i] + (ev + od);
    d[i + 1] = d[i + 1] + (ev - od);
  });
}

// The reconstruction applied to the post-collision moments themselves, d*_i = sum_k
// MINV[i][k] a*_k, for a lattice whose index set is smaller than Q (D3Q39: MINV is the
// paper's Hermite sum to order 4).  There the increment form d + MINV dA would keep the
// part of d that no carried moment sees, which the paper's reconstruction drops; the
// moments of orders 0 to 3 of the result are exactly a* (the quadrature is exact to
// degree 7; a*_0 is the deviation mass, MINV[i][0] = w_i).  Folded over the pairs as in
// reconstruct_folded: the rest population sums its row over every k from k = 0; each pair
// sums its first member's row over the even- and the odd-order moments apart and takes
// (E + O), (E - O).
template <class L, class T>
__device__ __forceinline__ void reconstruct_full_folded(T (&d)[L::Q], const T (&as)[L::NM]) {
  static_assert(pair_symmetric<L, T>());
  T acc = T(-0.0);
  static_for<L::NM>([&](auto K) {
    constexpr int k = decltype(K)::value;
    constexpr T cf = Tab<L, T>::minv(0, k);
    if constexpr (cf != T(0)) acc = fmadd(cf, as[k], acc);
  });
  d[0] = acc;
  static_for<(L::Q - 1) / 2>([&](auto Pp) {
    constexpr int i = 2 * decltype(Pp)::value + 1;
    T ev = T(-0.0), od = T(-0.0);
    static_for<L::NM>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr T cf = Tab<L, T>::minv(i, k);
      if constexpr (cf != T(0)) {
        if constexpr (L::ORD[k] % 2)
          od = fmadd(cf, as[k], od);
        else
          ev = fmadd(cf, as[k], ev);
      }
    });
    d[i] = ev + od;
    d[i + 1] = ev - od;
  });
}

// Index of the multi-index MI[k] - e_a in L's canonical list (-1 if absent).
template <class L>
constexpr int sub_index(int k, int a) {
  int m[3] = {L::MI[k][0], L::MI[k][1], L::MI[k][2]};
  if (m[a] == 0) return -1;
  m[a] -= 1;
  for (int j = 0; j < L::NM; ++j)
    if (L::MI[j][0] == m[0] && L::MI[j][1] == m[1] && L::MI[j][2] == m[2]) return j;
  return -1;
}

// BGK with the second-order force term (Sec. II.B, eq:explict_eq), formed as
// eq:evolution writes it, f-bar plus the change:
//   f*_i = f_i + [(1 - omega/2) F_i - omega (f_i - f_eq_i)] + (conserved-moment fix-up)
//   f_eq_i = w_i (rho + rho P_i),  P_i = (k e.u + (k^2/2) (e.u)^2) - (k/2) u.u
//   F_i   = w_i (k (e.F - u.F) + k^2 (e.F)(e.u))
// with k = 1/c_s^2 (3, 4.5, 1.5 and 9 at c_s^2 = 1/3): the truncated Hermite equilibrium
// and the second-order force.  In deviation form the leading rho of f_eq becomes d-rho.
template <class L, class T>
struct BGKConst {
  static constexpr T k1 = T(L::ICS2);                    // 1 / c_s^2
  static constexpr T k2h = T(0.5 * L::ICS2 * L::ICS2);   // 1 / (2 c_s^4)
  static constexpr T k1h = T(0.5 * L::ICS2);             // 1 / (2 c_s^2)
  static constexpr T k2 = T(L::ICS2 * L::ICS2);          // 1 / c_s^4
};

// e_i . v, summed over the non-zero components in x, y, z order (multiples of v_a for
// |e_ia| > 1).
template <class L, int i, class T>
__device__ __forceinline__ T edot(const T (&v)[3]) {
  T s = T(-0.0);
  static_for<3>([&](auto A) {
    constexpr int a = decltype(A)::value;
    constexpr int ea = L::E[i][a];
    if constexpr (ea == 1) s = s + v[a];
    if constexpr (ea == -1) s = s + (-v[a]);
    if constexpr (ea > 1 || ea < -1) s = s + T(ea) * v[a];
  });
  return s;
}
template <class L, class T>
__device__ __forceinline__ void collide_bgk(T (&d)[L::Q], T shift, const T (&g)[3],
                                            const BGKCoef<T> &c) {
  const Macro<T> M = macroscopic<L>(d, shift, g);
  T ch[L::Q];  // the change Omega_i + F_i of each population
  T usq = T(-0.0), uF = T(-0.0);
  static_for<L::D>([&](auto A) {
    constexpr int a = decltype(A)::value;
    usq = usq + M.u[a] * M.u[a];
  });
  static_for<L::D>([&](auto A) {
    constexpr int a = decltype(A)::value;
    uF = uF + M.u[a] * M.F[a];
  });
  using K = BGKConst<L, T>;
  static_for<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    const T eu = edot<L, i>(M.u), eF = edot<L, i>(M.F);
    constexpr T wi = Tab<L, T>::w(i);
    const T P = (K::k1 * eu + K::k2h * (eu * eu)) - K::k1h * usq;
    const T feq = wi * (M.drho + M.rho * P);
    const T G = K::k1 * (eF - uF) + K::k2 * (eF * eu);
    const T Fi = wi * G;
    ch[i] = c.hforce * Fi - c.omega * (d[i] - feq);
  });
  // The change's moments of orders 0 and 1 set to their exact values, 0 and F, through
  // the inverse transform's columns k = 0 (mass) and k = 1..D (momentum, the canonical
  // order puts e_x, e_y, e_z there): without this, binary32 weights bias the momentum
  // by about omega rho u per step (sum_i 3 fl(w_i) e_ix^2 != 1).  Zero in exact
  // arithmetic.
  T r[1 + L::D];
  {
    T s = T(-0.0);
    static_for<L::Q>([&](auto I) { s = s + ch[decltype(I)::value]; });
    r[0] = -s;
  }
  static_for<L::D>([&](auto A) {
    constexpr int a = decltype(A)::value;
    static_assert(L::ORD[1 + a] == 1 && L::MI[1 + a][a] == 1);
    T s = T(-0.0);
    static_for<L::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int ea = L::E[i][a];
      if constexpr (ea == 1) s = s + ch[i];
      if constexpr (ea == -1) s = s + (-ch[i]);
      if constexpr (ea > 1 || ea < -1) s = s + T(ea) * ch[i];
    });
    r[1 + a] = M.F[a] - s;
  });
  static_for<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    T corr = T(-0.0);
    static_for<1 + L::D>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr T cf = Tab<L, T>::minv(i, k);
      if constexpr (cf != T(0)) corr = corr + cf * r[k];
    });
    d[i] = d[i] + (ch[i] + corr);
  });
}

// Reconstruction f_i = sum_k MINV[i][k] a_k over the moments of order <= 4
// (reconstruction after eq:bbd1; orders 5 and 6 of D3Q27 are zero).
template <class L, class T>
__device__ __forceinline__ void reconstruct(const T (&a)[L::NM], T (&out)[L::Q]) {
  static_for<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    T acc = T(-0.0);
    static_for<L::NM>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr T c = Tab<L, T>::minv(i, k);
      if constexpr (c != T(0) && L::ORD[k] <= 4) acc = acc + c * a[k];
    });
    out[i] = acc;
  });
}

// SMRT with the force in the first central moment (Sec. II.C, eq:domg, eq:RHS, eq:bbd1):
//   A_m = sum_i d_i H_m(e_i)                         (eq:dft)
//   N_m = A_m - rho u^m,  N_{e_a} = -F_a/2             (non-equilibrium raw moments)
//   D_m = sum_{l <= m} C(m,l) (-u)^l N_{m-l}           (shift to the frame moving with u)
//   P_m = (1 - omega_|m|) D_m (|m| = 2, 3), P_{e_a} = F_a/2, order 4 trimmed
//   R_m = sum_{l <= m} C(m,l) u^l P_{m-l}              (back to raw moments, |m| <= 4)
//   a*_m = rho u^m + R_m (|m| <= 4), 0 above order 4
// applied as eq:evolution writes the step, f-bar + (Omega + F): the increment is
// MINV (a* - a), whose moment changes are 0 for the mass, F for the momentum,
// R_m - N_m for orders 2..4 and -A_m above.  Equal to MINV a* in real arithmetic; in
// floating point the conserved moments never pass through the rounded coefficients,
// so they carry no per-step bias.
// HI56: carry the orders above 4 (D3Q27's 5 and 6) as rho u^m + R_m, their central parts
// trimmed like order 4, instead of dropping them.
// On a lattice whose index set is smaller than Q (D3Q39) the state is rebuilt from the
// post-collision moments a*_0 = d-rho, a*_e = j + F, a*_m = rho u^m + R_m (|m| = 2..4)
// by reconstruct_full_folded, and the order-4 moments are not projected (a* of order 4
// does not depend on them).
// FC: the non-equilibrium force content carried, 0 (none: d_F^(n) = 0 for n >= 2, the
// paper's runs), 3 (d_F^(3)) or 4 (d_F^(3) and d_F^(4)).  SPLIT: whether the traces at
// orders 2 and 3 may relax at rates of their own (dqb, dq31); without it one rate per
// order.  Both are compile-time choices, so the step without them carries none of their
// code.
template <class L, bool HI56, class T, int FC = 0, bool SPLIT = true>
__device__ __forceinline__ void collide_smrt(T (&d)[L::Q], T shift, const T (&g)[3],
                                             const SMRTCoef<T> &c) {
  constexpr int NM = L::NM;
  constexpr bool FULL = L::NM < L::Q;
  constexpr bool FO4 = FC == 4;
  static_assert(FC == 0 || FC == 3 || FC == 4);
  static_assert(!FO4 || (!HI56 && !FULL));
  const Macro<T> M = macroscopic<L>(d, shift, g);
  T U[NM], E[NM], N[NM], P[NM], dA[NM], C2[NM], C3[NM];
  static_for<NM>([&](auto K) {
    constexpr int k = decltype(K)::value;
    U[k] = upow<L, k>(M.u);
    E[k] = M.rho * U[k];
  });
  const PairFold<L, T> pf(d);
  static_for<NM>([&](auto K) {
    constexpr int k = decltype(K)::value;
    constexpr int n = L::ORD[k];
    if constexpr (n == 1) {
      constexpr int a = L::MI[k][0] ? 0 : (L::MI[k][1] ? 1 : 2);
      N[k] = T(-0.5) * M.F[a];
    } else if constexpr (n >= 2) {
      if constexpr (FULL && n == 4) {
        N[k] = T(0);  // not needed: a* of order 4 is rho u^m + R_m
      } else {
        const T acc = pf.template project<k>(d);
        // orders 2..4: non-equilibrium part; above 4: the raw moment itself
        if constexpr (n <= 4)
          N[k] = acc - E[k];
        else
          N[k] = acc;
      }
    } else {
      N[k] = T(0);
    }
  });
  // eq:domg per irreducible component at order 2: the trace S^(2,0) (bulk part) may relax
  // at its own rate, P_aa += (q_bulk - q2)/D tr(D), the traceless part keeps q2 (a zero
  // coefficient leaves every P unchanged).
  T tb = T(-0.0);
  if constexpr (SPLIT) {
    static_for<NM>([&](auto K) {
      constexpr int k = decltype(K)::value;
      if constexpr (is_diag2<L>(k)) tb = tb + central<L, k>(U, N);
    });
    tb = c.dqb * tb;
  }
  // The same at order 3: the trace S^(3,1), carried per axis a by D_abb + D_acc, may relax
  // at its own rate, P_abb += (q_31 - q3)/2 (D_abb + D_acc) and likewise P_acc; the
  // differences D_abb - D_acc and D_xyz keep q3.
  T t3[NM];
  if constexpr (SPLIT) {
    static_for<NM>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr int p = trace_partner3<L>(k);
      if constexpr (p > k) {
        t3[k] = c.dq31 * (central<L, k>(U, N) + central<L, p>(U, N));
        t3[p] = t3[k];
      }
    });
  }
  static_for<NM>([&](auto K) {
    constexpr int k = decltype(K)::value;
    constexpr int n = L::ORD[k];
    if constexpr (n == 1) {
      constexpr int a = L::MI[k][0] ? 0 : (L::MI[k][1] ? 1 : 2);
      P[k] = T(0.5) * M.F[a];
    } else if constexpr (n == 2 || n == 3) {
      const T Dm = central<L, k>(U, N);
      if constexpr (n == 2) C2[k] = Dm;
      if constexpr (n == 3 && FO4) C3[k] = Dm;
      P[k] = (n == 2 ? c.q2 : c.q3) * Dm;
      if constexpr (SPLIT && is_diag2<L>(k)) P[k] = P[k] + tb;
      if constexpr (SPLIT && trace_partner3<L>(k) >= 0) P[k] = P[k] + t3[k];
      if constexpr (n == 3) {
        // Third-order force content (eq:Frc at theta = 1, d_F^(3) = 3 g d^(2)): the
        // symmetric product sum_a m_a g_a d_{m - e_a} of the acceleration with the central
        // non-equilibrium second moment of f itself, which eq:newf and eq:evolution make
        // the mean (D + P)/2 of the moment before and after the collision (P final here:
        // order 2 precedes order 3), relaxed as a force term by 1 - omega_3/2.
        if constexpr (FC >= 3) {
          T sF = T(-0.0);
          static_for<3>([&](auto A) {
            constexpr int a = decltype(A)::value;
            constexpr int j = sub_index<L>(k, a);
            if constexpr (j >= 0) sF = sF + (T(L::MI[k][a]) * g[a]) * (T(0.5) * (C2[j] + P[j]));
          });
          P[k] = P[k] + c.fq3 * sF;
        }
      }
    } else if constexpr (FO4 && n == 4) {
      // Fourth-order force content (eq:Frc, d_F^(4) = 4 g d^(3)), the same product with the
      // central third moment of f, (D + P)/2 of order 3, entering the trimmed order 4
      // (omega_4 = 1) with 1 - omega_4/2 = 1/2.
      T s4 = T(-0.0);
      static_for<3>([&](auto A) {
        constexpr int a = decltype(A)::value;
        constexpr int j = sub_index<L>(k, a);
        if constexpr (j >= 0) s4 = s4 + (T(L::MI[k][a]) * g[a]) * (T(0.5) * (C3[j] + P[j]));
      });
      P[k] = T(0.5) * s4;
    } else {
      P[k] = T(0);
    }
  });
  static_for<NM>([&](auto K) {
    constexpr int k = decltype(K)::value;
    constexpr int n = L::ORD[k];
    if constexpr (n == 0) {
      if constexpr (FULL)
        dA[k] = M.drho;
      else
        dA[k] = T(0);
    } else if constexpr (n == 1) {
      constexpr int a = L::MI[k][0] ? 0 : (L::MI[k][1] ? 1 : 2);
      if constexpr (FULL)
        dA[k] = M.j[a] + M.F[a];
      else
        dA[k] = M.F[a];
    } else if constexpr (n > 4) {
      if constexpr (HI56) {
        // a*_m = rho u^m + R_m with the central parts of orders >= 4 trimmed
        T R = T(-0.0);
        static_for<L::NT[k]>([&](auto Tt) {
          constexpr int t = decltype(Tt)::value;
          constexpr int kl = L::TL[k][t], km = L::TM[k][t];
          static_assert(pow2_coef(L::CUP[k][t]));
          if constexpr (L::ORD[km] <= 3) R = fmadd(T(L::CUP[k][t]) * U[kl], P[km], R);
        });
        dA[k] = R - (N[k] - E[k]);
      } else if constexpr (FULL) {
        dA[k] = T(0);
      } else {
        dA[k] = -N[k];
      }
    } else {
      T R = (n <= 3 || (FO4 && n == 4)) ? P[k] : T(-0.0);
      static_for<L::NT[k]>([&](auto Tt) {
        constexpr int t = decltype(Tt)::value;
        constexpr int kl = L::TL[k][t], km = L::TM[k][t];
        static_assert(FULL || pow2_coef(L::CUP[k][t]));
        if constexpr (L::ORD[km] <= 3) R = fmadd(T(L::CUP[k][t]) * U[kl], P[km], R);
      });
      if constexpr (FULL)
        dA[k] = E[k] + R;
      else
        dA[k] = R - N[k];
    }
  });
  if constexpr (FULL)
    reconstruct_full_folded<L>(d, dA);
  else
    reconstruct_folded<L>(d, dA);
}

// Raw-moment MRT with force (the paper's appendix, eq:RHS_a in its explicit form): every
// raw Hermite moment of order n relaxes as a*_m = rho u^m + (1 - omega_n) N_m +
// (1 - omega_n/2) a_F,m with the raw force moments a_F,m = sum_a m_a u^{m - e_a} F_a
// (non-equilibrium force content neglected, theta = 1).  Momentum gains F (a*_e =
// rho u + F/2 whatever omega_1); order 4 is trimmed (omega_4 = 1: a* = rho u^m + a_F/2);
// orders above 4 are dropped.  The state is advanced by the reconstruction of the moment
// changes, as in collide_smrt.
template <class T>
struct RMRTCoef {
  T q2, q3;  // 1 - omega_n
  T h2, h3;  // 1 - omega_n / 2
};

template <class L, class T>
__device__ __forceinline__ void collide_rmrt(T (&d)[L::Q], T shift, const T (&g)[3],
                                             const RMRTCoef<T> &c) {
  constexpr int NM = L::NM;
  constexpr bool FULL = L::NM < L::Q;  // rebuild from a* (see collide_smrt)
  const Macro<T> M = macroscopic<L>(d, shift, g);
  T U[NM], dA[NM];
  static_for<NM>([&](auto K) {
    constexpr int k = decltype(K)::value;
    U[k] = upow<L, k>(M.u);
  });
  const PairFold<L, T> pf(d);
  static_for<NM>([&](auto K) {
    constexpr int k = decltype(K)::value;
    constexpr int n = L::ORD[k];
    if constexpr (n == 0) {
      if constexpr (FULL)
        dA[k] = M.drho;
      else
        dA[k] = T(0);
    } else if constexpr (n == 1) {
      constexpr int a = L::MI[k][0] ? 0 : (L::MI[k][1] ? 1 : 2);
      if constexpr (FULL)
        dA[k] = M.j[a] + M.F[a];
      else
        dA[k] = M.F[a];
    } else {
      T acc = T(0);  // a* of order 4 does not depend on the pre-collision moment
      if constexpr (!(FULL && n == 4)) acc = pf.template project<k>(d);
      if constexpr (n > 4) {
        if constexpr (FULL)
          dA[k] = T(0);
        else
          dA[k] = -acc;
      } else {
        const T Ek = M.rho * U[k];
        const T Nk = acc - Ek;
        T aF = T(-0.0);
        static_for<3>([&](auto A) {
          constexpr int a = decltype(A)::value;
          constexpr int j = sub_index<L>(k, a);
          if constexpr (j >= 0) aF = aF + (T(L::MI[k][a]) * U[j]) * M.F[a];
        });
        T t;
        if constexpr (n == 2) {
          t = c.q2 * Nk;
          t = t + c.h2 * aF;
        } else if constexpr (n == 3) {
          t = c.q3 * Nk;
          t = t + c.h3 * aF;
        } else {
          t = T(0.5) * aF;
        }
        if constexpr (FULL)
          dA[k] = Ek + t;
        else
          dA[k] = t - Nk;
      }
    }
  });
  if constexpr (FULL)
    reconstruct_full_folded<L>(d, dA);
  else
    reconstruct_folded<L>(d, dA);
}

// Initial stored state f-bar = f_eq - F_i/2 (eq:newf with Omega = 0): density and
// physical velocity are then exactly rho and u.  BGK: its second-order equilibrium
// and force term.  SMRT: equilibrium moments rho u^m and raw force moments
// a_F,m = sum_a m_a u^{m-e_a} F_a (the appendix's a_F^(1..4) at theta = 1), |m| <= 4.
template <class L, class T, int COLL>
__device__ __forceinline__ void init_node(T rho, const T (&u)[3], const T (&g)[3], T shift,
                                          T (&out)[L::Q]) {
  T F[3];
  static_for<3>([&](auto A) {
    constexpr int a = decltype(A)::value;
    F[a] = rho * g[a];
  });
  const T drho = rho - shift;
  if constexpr (COLL == 0) {
    T usq = T(-0.0), uF = T(-0.0);
    static_for<L::D>([&](auto A) {
      constexpr int a = decltype(A)::value;
      usq = usq + u[a] * u[a];
    });
    static_for<L::D>([&](auto A) {
      constexpr int a = decltype(A)::value;
      uF = uF + u[a] * F[a];
    });
    using K = BGKConst<L, T>;
    static_for<L::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      const T eu = edot<L, i>(u), eF = edot<L, i>(F);
      constexpr T wi = Tab<L, T>::w(i);
      const T P = (K::k1 * eu + K::k2h * (eu * eu)) - K::k1h * usq;
      const T feq = wi * (drho + rho * P);
      const T G = K::k1 * (eF - uF) + K::k2 * (eF * eu);
      out[i] = feq - T(0.5) * (wi * G);
    });
  } else {
    constexpr int NM = L::NM;
    T a[NM];
    static_for<NM>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr int n = L::ORD[k];
      if constexpr (n == 0) {
        a[k] = drho;
      } else if constexpr (n > 4) {
        a[k] = T(0);
      } else {
        T aF = T(-0.0);
        static_for<3>([&](auto A) {
          constexpr int al = decltype(A)::value;
          constexpr int ma = L::MI[k][al];
          if constexpr (ma > 0) {
            // u^{m - e_al}
            T p = T(1);
            static_for<3>([&](auto B) {
              constexpr int b = decltype(B)::value;
              constexpr int mb = L::MI[k][b] - (b == al ? 1 : 0);
              static_for<mb>([&](auto) { p = p * u[b]; });
            });
            aF = aF + T(ma) * (p * F[al]);
          }
        });
        a[k] = rho * upow<L, k>(u) - T(0.5) * aF;
      }
    });
    reconstruct<L>(a, out);
  }
}

}  // namespace lbm
