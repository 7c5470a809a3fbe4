/*
 * Plain CPU oracle of the forced lattice-Boltzmann time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call this
 * file; only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header or table generator with the HIP
 * library: its lattice tables are produced by oracle/lattice.py in exact
 * rational arithmetic and passed in already rounded.
 *
 * Built three times: with REAL = double (FP64), with REAL = float (an emulation of
 * the library's reduced-precision modes: FP32 arithmetic in the same order, stores
 * rounded to binary32 or binary16), and with REAL = double and PLAIN defined.
 *
 * Two operation orders.  The default build ("operation-order twin") fixes the rounding
 * order described below, which the HIP library follows too, so the two can be compared
 * bit for bit.  The PLAIN build is the textbook form of the same step: every moment a
 * sum over all populations in index order, sum_i f_i H_m(e_i) (eq:dft); the Hermite
 * shifts as plain sums of C(m,l) u^l N_{m-l}; the increment of each population as a
 * plain row of the inverse transform, sum_m Minv_im (a*_m - a_m); no fused multiply-add
 * and no folding over opposite velocities.  In real arithmetic both builds compute the
 * same map; in floating point they differ by rounding only, which bounds how far any
 * implementation of this fixed order may sit from the plain definition.
 *
 * Paper: X. Li, W. Duan, X. Shan, "Second-order force scheme for lattice
 * Boltzmann method" (arXiv 2212.07494).  Each function cites the passage it
 * follows.  Lattice units; c_s^2 = 1/3 on D2Q9, D3Q19 and D3Q27, 2/3 on the
 * high-order lattice D3Q39 (passed in as 1/c_s^2); Hermite polynomials in lattice
 * units (H_m(e) = c_s^|m| times the paper's tensor Hermite polynomial of e/c_s).
 *
 * State.  The oracle holds the paper's stored variable f-bar(x, t) (the
 * pre-collision population after the change of variable eq:newf) and advances
 * it with the explicit evolution eq:evolution: collide at x, then stream the
 * post-collision value to x + e_i.  To allow reduced-precision storage the
 * array holds deviations d_i = f-bar_i - w_i s from a constant shift s (s = 0
 * gives the plain populations; the arithmetic below then is literally the
 * paper's).
 *
 * Fixed operation order.  Every sum starts from -0.0 (the additive identity,
 * so an empty sum is -0 and a one-term sum is that term exactly), adds its
 * terms in the stated index order, and skips terms whose constant coefficient
 * is exactly zero.  Products of velocity components are formed left to right
 * over x, y, z.  Constants are exact rationals rounded once.  The SMRT and RMRT
 * projection, central shift, back-shift and reconstruction accumulate each term
 * with one fused multiply-add (fmar); in the shifts the binomial coefficient scales
 * u^l first (exactly where it is a power of two, as on D2Q9, D3Q19 and D3Q27).  The SMRT and RMRT
 * projections and reconstructions are folded over the opposite-velocity pairs of the
 * population order (project_folded, reconstruct_folded).  Nothing else is fused.
 * Compiled with
 * -ffp-contract=off, no fast-math.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef REAL
#define REAL double
#endif
typedef REAL real;

/* a * b + c rounded once (fused multiply-add), in the precision of real.  The SMRT
 * collision accumulates its moment transforms with it (the paper fixes no rounding
 * order; one rounding per term is the more accurate choice). */
static inline real fmar(real a, real b, real c) {
#ifdef PLAIN
  return a * b + c; /* two roundings (the build never contracts) */
#else
  return sizeof(real) == sizeof(float) ? (real)fmaf((float)a, (float)b, (float)c)
                                       : (real)fma((double)a, (double)b, (double)c);
#endif
}

#define MAXQ 39

typedef struct {
  int32_t D, Q, NM;
  const int32_t *e;    /* Q x 3 velocity components */
  const int32_t *opp;  /* Q: index of -e_i */
  const int32_t *mi;   /* NM x 3 multi-indices, canonical order */
  const real *w;       /* Q weights */
  const real *H;       /* NM x Q: H_m(e_i) */
  const real *Minv;    /* Q x NM: the reconstruction, f = Minv a (exact inverse of H when
                          NM == Q; the Hermite sum w_i H_m(e_i) / (m! c_s^(2|m|)) of
                          the orders up to 4 when NM < Q) */
  double ics2;         /* 1 / c_s^2 (3 or 3/2, exact in either precision) */
} oracle_lattice;

typedef struct {
  int32_t collision;   /* 0 = BGK, 1 = SMRT, 2 = RMRT */
  int32_t nx, ny, nz;
  int32_t wall[3];     /* per axis: 1 = halfway bounce-back walls on both faces, 0 = periodic */
  int32_t store16;     /* 1: round every stored value to binary16 (emulation only) */
  real shift;          /* s: stored value is f-bar_i - w_i s */
  real omega;          /* BGK: 1 / tau-hat */
  real hforce;         /* BGK: 1 - omega / 2 */
  real q2, q3;         /* SMRT: 1 - omega_n, omega_n = 1 / tau-hat_n */
  real fq3;            /* SMRT: 1 - omega_3/2, the factor of the third-order force
                          content, 0 when the non-equilibrium force content is neglected */
  real h2, h3;         /* RMRT: 1 - omega_n / 2 */
  real dqb;            /* SMRT: (q_bulk - q2)/D for the trace of order 2 (0 = one rate) */
  real dq31;           /* SMRT: (q_31 - q3)/2 for the trace of order 3 (0 = one rate) */
  int32_t max_order;   /* SMRT: highest Hermite order carried after the collision, 4 or 6 */
  int32_t fo4;         /* SMRT: 1 adds the fourth-order force content (with fq3 != 0) */
  const uint8_t *solid; /* N flags, nonzero = solid node (no fluid); NULL = none */
} oracle_params;

/* ---- binary16 rounding (IEEE 754 round to nearest, ties to even) ------------------ */
static float round_to_half(float x) {
  union { float f; uint32_t u; } v = {x};
  uint32_t sign = v.u & 0x80000000u;
  uint32_t ax = v.u & 0x7fffffffu;
  float a;
  memcpy(&a, &ax, 4);
  float r;
  if (ax >= 0x7f800000u) {
    r = a; /* inf / nan stay */
  } else if (a >= 65520.0f) {
    r = INFINITY; /* beyond the largest half after rounding */
  } else if (a < 6.103515625e-05f) {
    /* subnormal half: quantum 2^-24 */
    float q = 5.9604644775390625e-08f;
    float n = a / q; /* exact: power-of-two scaling */
    float fl = floorf(n);
    float rem = n - fl;
    if (rem > 0.5f || (rem == 0.5f && fmodf(fl, 2.0f) != 0.0f)) fl += 1.0f;
    r = fl * q;
  } else {
    int ex;
    frexpf(a, &ex); /* a = m 2^ex, m in [0.5, 1) */
    float q = ldexpf(1.0f, ex - 11); /* 10 fraction bits + hidden bit */
    float n = a / q;
    float fl = floorf(n);
    float rem = n - fl;
    if (rem > 0.5f || (rem == 0.5f && fmodf(fl, 2.0f) != 0.0f)) fl += 1.0f;
    r = fl * q;
  }
  union { float f; uint32_t u; } o = {r};
  o.u |= sign;
  return o.f;
}

float oracle_round_half(float x) { return round_to_half(x); }

static real store_value(const oracle_params *P, real x) {
  if (P->store16) return (real)round_to_half((float)x);
  return x;
}

/* ---- multi-index helpers --------------------------------------------------------- */
static int mabs(const int32_t *m) { return m[0] + m[1] + m[2]; }

static int find_index(const oracle_lattice *L, int a, int b, int c) {
  for (int k = 0; k < L->NM; ++k) {
    const int32_t *m = L->mi + 3 * k;
    if (m[0] == a && m[1] == b && m[2] == c) return k;
  }
  return -1;
}

static int binom(int n, int k) {
  int c = 1;
  for (int j = 1; j <= k; ++j) c = c * (n - k + j) / j;
  return c;
}

/* u^m = prod_a u_a^{m_a}, multiplied left to right over x, y, z starting from 1. */
static real upow(const int32_t *m, const real u[3]) {
  real p = (real)1;
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < m[a]; ++k) p = p * u[a];
  return p;
}

/* ---- macroscopic quantities (Sec. II.B, eq:half_F and the relations after it) ----- */
/* rho-bar = rho; rho u-bar = rho u - F/2, so u = j/rho + g/2 with F = rho g. */
typedef struct {
  real drho, rho, j[3], u[3], F[3];
} macro_t;

static void macroscopic(const oracle_lattice *L, const oracle_params *P, const real *f,
                        const real g[3], macro_t *M) {
  real s = -0.0;
  for (int i = 0; i < L->Q; ++i) s = s + f[i];
  M->drho = s;
  M->rho = P->shift + s;
  for (int a = 0; a < 3; ++a) {
    real ja = -0.0;
    for (int i = 0; i < L->Q; ++i) {
      int ea = L->e[3 * i + a];
      if (ea != 0) ja = ja + (real)ea * f[i];
    }
    M->j[a] = ja;
  }
  for (int a = 0; a < 3; ++a) {
    M->u[a] = M->j[a] / M->rho + (real)0.5 * g[a];
    M->F[a] = M->rho * g[a];
  }
}

/* ---- BGK (Sec. II.B, eq:explict_eq) ------------------------------------------------ */
/* Second-order truncated equilibrium evaluated at e_i (expansion after
 * eq:collision_BGK): w_i rho [1 + e.u/c_s^2 + ((e.u)^2 - c_s^2 u^2)/(2 c_s^4)], written
 * as w_i (rho + rho P_i) with P_i = (k e.u + (k^2/2) (e.u)^2) - (k/2) u.u, k = 1/c_s^2
 * (3, 4.5, 1.5 for c_s^2 = 1/3); in deviation form the leading rho becomes drho
 * (sum_i w_i s = s). */
static real bgk_P(const oracle_lattice *L, int i, const real u[3], real *eu_out) {
  real eu = -0.0;
  for (int a = 0; a < 3; ++a) {
    int ea = L->e[3 * i + a];
    if (ea != 0) eu = eu + (real)ea * u[a];
  }
  real usq = -0.0;
  for (int a = 0; a < L->D; ++a) usq = usq + u[a] * u[a];
  *eu_out = eu;
  const real k = (real)L->ics2;
  return (k * eu + (real)(0.5 * L->ics2 * L->ics2) * (eu * eu)) - (real)(0.5 * L->ics2) * usq;
}

/* Force term truncated to second order (the familiar form below eq:Fr, evaluated at
 * e_i): F_i = w_i [ (e_i - u).F / c_s^2 + (e_i.F)(e_i.u) / c_s^4 ], F = rho g (the
 * factors 3 and 9 for c_s^2 = 1/3). */
static real bgk_force(const oracle_lattice *L, int i, const real u[3], const real F[3],
                      real eu) {
  real eF = -0.0;
  for (int a = 0; a < 3; ++a) {
    int ea = L->e[3 * i + a];
    if (ea != 0) eF = eF + (real)ea * F[a];
  }
  real uF = -0.0;
  for (int a = 0; a < L->D; ++a) uF = uF + u[a] * F[a];
  real G = (real)L->ics2 * (eF - uF) + (real)(L->ics2 * L->ics2) * (eF * eu);
  return L->w[i] * G;
}

/* The change of the populations over a BGK collision, Omega_i + F_i =
 * (1 - omega/2) F_i - omega (f_i - f_eq_i), has mass 0 and momentum F in exact
 * arithmetic (the equilibrium carries rho and rho u, the force term 0 and F).  Formed
 * population by population in floating point, those two moments pass through the
 * rounded weights (in binary32, sum_i 3 fl(w_i) e_ix^2 != 1), which biases the momentum
 * by about omega rho u times the weights' rounding at every step.  As for the MRT
 * collisions, the post-collision state is formed as eq:evolution writes it, f-bar plus
 * the change, and the change's conserved moments are set to their exact values through
 * the inverse transform's columns of orders 0 and 1: each population gains
 * Minv_i0 (0 - sum_j c_j) + sum_a Minv_i,e_a (F_a - sum_j c_j e_ja).  In exact arithmetic
 * the correction is zero. */
static void collide_bgk(const oracle_lattice *L, const oracle_params *P, const real *f,
                        const real g[3], real *out) {
  macro_t M;
  macroscopic(L, P, f, g, &M);
  const int Q = L->Q, NM = L->NM;
  real c[MAXQ];
  for (int i = 0; i < Q; ++i) {
    real eu;
    real Pi = bgk_P(L, i, M.u, &eu);
    real feq = L->w[i] * (M.drho + M.rho * Pi);
    real Fi = bgk_force(L, i, M.u, M.F, eu);
    c[i] = P->hforce * Fi - P->omega * (f[i] - feq);
  }
  /* the change's moments of orders 0 and 1 against their exact values: r[k] per
   * multi-index k of order <= 1 (canonical order puts them first) */
  real r[4];
  int nk = 0;
  for (int k = 0; k < NM && mabs(L->mi + 3 * k) <= 1; ++k, ++nk) {
    const int32_t *m = L->mi + 3 * k;
    real s = -0.0;
    if (mabs(m) == 0) {
      for (int i = 0; i < Q; ++i) s = s + c[i];
      r[k] = -s;
    } else {
      const int a = m[0] ? 0 : (m[1] ? 1 : 2);
      for (int i = 0; i < Q; ++i) {
        const int ea = L->e[3 * i + a];
        if (ea == 1) s = s + c[i];
        if (ea == -1) s = s + (-c[i]);
        if (ea > 1 || ea < -1) s = s + (real)ea * c[i];
      }
      r[k] = M.F[a] - s;
    }
  }
  for (int i = 0; i < Q; ++i) {
    real corr = -0.0;
    for (int k = 0; k < nk; ++k) {
      const real cf = L->Minv[i * NM + k];
      if (cf != 0) corr = corr + cf * r[k];
    }
    out[i] = f[i] + (c[i] + corr);
  }
}

/* ---- SMRT (Sec. II.C, eq:domg, eq:RHS, eq:bbd1 and the reconstruction after it) --- */
/*
 * Raw moments A_m = sum_i f_i H_m(e_i) (eq:dft).  Non-equilibrium raw moments
 * N_m = A_m - rho u^m (isothermal equilibrium a_0 = rho u^n), with N_0 = 0 and
 * N_{e_a} = -F_a/2 (the first-order relation rho u-bar = rho u - F/2).
 * Central non-equilibrium moments by the Hermite shift to the frame moving with u:
 *   D_m = sum_{l <= m} C(m,l) (-u)^l N_{m-l}.
 * Relaxation (eq:RHS with d_0 = 0 for n >= 1 and d_F^(n) = 0 for n >= 2 when the
 * non-equilibrium part of the force is neglected): P_m = (1 - omega_|m|) D_m for
 * |m| = 2, 3; P_{e_a} = F_a/2; order 4 trimmed (P_m = 0).
 * Back to raw moments: R_m = sum_{l <= m} C(m,l) u^l P_{m-l} for 1 <= |m| <= 4
 * (this is eq:bbd1 written per multi-index), post-collision a*_m = rho u^m + R_m for
 * |m| <= 4 and 0 above order 4 (reconstruction after eq:bbd1).
 * The post-collision state is formed as eq:evolution writes it, f-bar + (Omega + F):
 * the increment is the reconstruction Minv (a* - a) of the moment changes, which are 0
 * for the mass, F for the momentum, R_m - N_m for orders 2..4 and -a_m above.  In real
 * arithmetic this equals Minv a*; in floating point it keeps the conserved moments
 * away from the rounded reconstruction coefficients, so mass and momentum carry no
 * per-step bias (with Minv a* they would be scaled by sum_i e_i^2 fl(Minv) != 1).
 */
/* Index bookkeeping of the two Hermite shifts, built once per call: for each m the
 * sub-multi-indices l (canonical order, l != 0, l != m), the index of m - l and the
 * integer coefficient (C(m,l) (-1)^|l| for the shift to the moving frame, C(m,l) back). */
typedef struct {
  int n[MAXQ];
  int kl[MAXQ][MAXQ], km[MAXQ][MAXQ], cdown[MAXQ][MAXQ], cup[MAXQ][MAXQ];
} smrt_plan;

static void make_plan(const oracle_lattice *L, smrt_plan *S) {
  for (int k = 0; k < L->NM; ++k) {
    const int32_t *m = L->mi + 3 * k;
    S->n[k] = 0;
    for (int kl = 1; kl < L->NM; ++kl) {
      const int32_t *l = L->mi + 3 * kl;
      if (l[0] > m[0] || l[1] > m[1] || l[2] > m[2] || kl == k) continue;
      int c = binom(m[0], l[0]) * binom(m[1], l[1]) * binom(m[2], l[2]);
      int t = S->n[k]++;
      S->kl[k][t] = kl;
      S->km[k][t] = find_index(L, m[0] - l[0], m[1] - l[1], m[2] - l[2]);
      S->cup[k][t] = c;
      S->cdown[k][t] = (mabs(l) % 2) ? -c : c;
    }
  }
}

/* The population order pairs each velocity with its opposite, (e, -e) at i = 2p-1, 2p
 * after the rest population i = 0, and H_m(-e) = (-1)^|m| H_m(e).  So a raw moment of
 * even order is a sum over the pair sums f_{2p-1} + f_{2p} and one of odd order over the
 * pair differences (the rest population enters only even moments), and the same split
 * holds for the rows of the inverse transform.  The collisions that use it check the
 * tables once: both relations must hold exactly. */
static void check_pair_symmetry(const oracle_lattice *L) {
#ifdef PLAIN
  (void)L; /* the plain transforms do not fold */
  return;
#endif
  const int NM = L->NM, Q = L->Q;
  for (int k = 0; k < NM; ++k) {
    const real sg = (mabs(L->mi + 3 * k) % 2) ? (real)-1 : (real)1;
    if (sg < 0 && (L->H[k * Q] != 0 || L->Minv[k] != 0)) abort();
    for (int i = 1; i + 1 < Q; i += 2)
      if (L->H[k * Q + i + 1] != sg * L->H[k * Q + i] ||
          L->Minv[(i + 1) * NM + k] != sg * L->Minv[i * NM + k])
        abort();
  }
}

/* Raw moment k of f folded over the pairs: the rest population, then pair p = 1, 2, ...
 * with its sum s_p (even order) or difference a_p (odd order), each term one fma from
 * -0.0, zero coefficients skipped. */
static real project_folded(const oracle_lattice *L, int k, const real *f, const real *s,
                           const real *a) {
  const int Q = L->Q;
#ifdef PLAIN
  /* eq:dft as written: sum over every population in index order */
  (void)s;
  (void)a;
  real P = -0.0;
  for (int i = 0; i < Q; ++i) P = P + L->H[k * Q + i] * f[i];
  return P;
#endif
  const int odd = mabs(L->mi + 3 * k) % 2;
  real A = -0.0;
  if (L->H[k * Q] != 0) A = fmar(L->H[k * Q], f[0], A);
  for (int p = 1; 2 * p < Q; ++p) {
    real h = L->H[k * Q + 2 * p - 1];
    if (h != 0) A = fmar(h, odd ? a[p] : s[p], A);
  }
  return A;
}

/* f + Minv dA folded over the pairs: the rest population sums its row over k = 1..NM-1;
 * each pair sums its first member's row separately over the even-order and the odd-order
 * moments (E, O, each from -0.0 in k order, one fma a term, zeros skipped) and takes
 * f_{2p-1} + (E + O), f_{2p} + (E - O). */
static void reconstruct_folded(const oracle_lattice *L, const real *f, const real *dA,
                               real *out) {
  const int Q = L->Q, NM = L->NM;
#ifdef PLAIN
  /* each population plus its row of the inverse transform applied to the changes */
  for (int i = 0; i < Q; ++i) {
    real r = -0.0;
    for (int k = 0; k < NM; ++k) r = r + L->Minv[i * NM + k] * dA[k];
    out[i] = f[i] + r;
  }
  return;
#endif
  real acc = -0.0;
  for (int k = 1; k < NM; ++k) {
    real c = L->Minv[k];
    if (c != 0) acc = fmar(c, dA[k], acc);
  }
  out[0] = f[0] + acc;
  for (int p = 1; 2 * p < Q; ++p) {
    const int i = 2 * p - 1;
    real ev = -0.0, od = -0.0;
    for (int k = 1; k < NM; ++k) {
      real c = L->Minv[i * NM + k];
      if (c == 0) continue;
      if (mabs(L->mi + 3 * k) % 2)
        od = fmar(c, dA[k], od);
      else
        ev = fmar(c, dA[k], ev);
    }
    out[i] = f[i] + (ev + od);
    out[i + 1] = f[i + 1] + (ev - od);
  }
}

/* The paper's reconstruction applied to the post-collision moments themselves (after
 * eq:bbd1), f*_i = sum_m Minv_im a*_m, on a lattice whose index set is smaller than Q
 * (D3Q39: the Hermite sum to order 4).  There the increment form f + Minv (a* - a) would
 * keep whatever part of f the NM moments do not describe, which the paper's formula
 * drops, so the state is rebuilt from a*; the quadrature being exact to degree 7, the
 * moments of orders 0 to 3 of the result are exactly a* (mass a*_0 = d-rho in deviation
 * form, Minv_i0 = w_i).  Folded over the pairs like reconstruct_folded: the rest
 * population sums its row over every k from k = 0; each pair sums its first member's row
 * over the even-order and the odd-order moments apart (from -0.0 in k order, one fma a
 * nonzero term) and takes (E + O), (E - O). */
static void reconstruct_full_folded(const oracle_lattice *L, const real *as, real *out) {
  const int Q = L->Q, NM = L->NM;
#ifdef PLAIN
  /* each population as its plain row of the reconstruction */
  for (int i = 0; i < Q; ++i) {
    real r = -0.0;
    for (int k = 0; k < NM; ++k) r = r + L->Minv[i * NM + k] * as[k];
    out[i] = r;
  }
  return;
#endif
  real acc = -0.0;
  for (int k = 0; k < NM; ++k) {
    real c = L->Minv[k];
    if (c != 0) acc = fmar(c, as[k], acc);
  }
  out[0] = acc;
  for (int p = 1; 2 * p < Q; ++p) {
    const int i = 2 * p - 1;
    real ev = -0.0, od = -0.0;
    for (int k = 0; k < NM; ++k) {
      real c = L->Minv[i * NM + k];
      if (c == 0) continue;
      if (mabs(L->mi + 3 * k) % 2)
        od = fmar(c, as[k], od);
      else
        ev = fmar(c, as[k], ev);
    }
    out[i] = ev + od;
    out[i + 1] = ev - od;
  }
}

static void collide_smrt(const oracle_lattice *L, const oracle_params *P, const smrt_plan *S,
                         const real *f, const real g[3], real *out) {
  macro_t M;
  macroscopic(L, P, f, g, &M);
  const int NM = L->NM;
  real U[MAXQ], E[MAXQ], N[MAXQ], Pc[MAXQ], D2[MAXQ], D3[MAXQ], ps[MAXQ], pa[MAXQ];
  for (int k = 0; k < NM; ++k) {
    U[k] = upow(L->mi + 3 * k, M.u);
    E[k] = M.rho * U[k];
  }
  for (int p = 1; 2 * p < L->Q; ++p) {
    ps[p] = f[2 * p - 1] + f[2 * p];
    pa[p] = f[2 * p - 1] - f[2 * p];
  }
  /* non-equilibrium raw moments */
  for (int k = 0; k < NM; ++k) {
    const int32_t *m = L->mi + 3 * k;
    int n = mabs(m);
    N[k] = 0;
    if (n == 1) {
      int a = m[0] ? 0 : (m[1] ? 1 : 2);
      N[k] = (real)-0.5 * M.F[a];
    } else if (n == 2 || n == 3) {
      N[k] = project_folded(L, k, f, ps, pa) - E[k];
    }
  }
  /* shift to the moving frame, relax */
  for (int k = 0; k < NM; ++k) {
    const int32_t *m = L->mi + 3 * k;
    int n = mabs(m);
    Pc[k] = 0;
    if (n == 1) {
      int a = m[0] ? 0 : (m[1] ? 1 : 2);
      Pc[k] = (real)0.5 * M.F[a];
    } else if (n == 2 || n == 3) {
      real D = N[k]; /* l = 0 term; l = m multiplies N_0 = 0 */
      for (int t = 0; t < S->n[k]; ++t)
        D = fmar((real)S->cdown[k][t] * U[S->kl[k][t]], N[S->km[k][t]], D);
      if (n == 2) D2[k] = D;
      if (n == 3) D3[k] = D;
      Pc[k] = (n == 2 ? P->q2 : P->q3) * D;
    }
  }
  if (P->dqb != 0) {
    /* eq:domg per irreducible component at order 2: the trace (bulk part) relaxes with
     * its own rate, P_aa += (q_bulk - q2)/D tr(D) (dqb holds (q_bulk - q2)/D), the
     * traceless part keeps q2 */
    real tr = -0.0;
    for (int k = 0; k < NM; ++k) {
      const int32_t *m = L->mi + 3 * k;
      if (mabs(m) == 2 && (m[0] == 2 || m[1] == 2 || m[2] == 2)) tr = tr + D2[k];
    }
    for (int k = 0; k < NM; ++k) {
      const int32_t *m = L->mi + 3 * k;
      if (mabs(m) == 2 && (m[0] == 2 || m[1] == 2 || m[2] == 2)) Pc[k] = Pc[k] + P->dqb * tr;
    }
  }
  if (P->dq31 != 0) {
    /* eq:domg at order 3: the trace S^(3,1), sum_b D_abb, relaxes with its own rate.  The
     * lattice carries its axis-a component as D_abb + D_acc (D_aaa has no Hermite moment
     * on it), so each such pair gains (q_31 - q3)/2 (D_abb + D_acc) (dq31 holds the half
     * difference); the pair's difference and D_xyz keep q3 */
    for (int a = 0; a < 3; ++a) {
      const int b = (a + 1) % 3, c = (a + 2) % 3;
      int mb[3] = {0, 0, 0}, mc[3] = {0, 0, 0};
      mb[a] = 1;
      mb[b] = 2;
      mc[a] = 1;
      mc[c] = 2;
      int jb = find_index(L, mb[0], mb[1], mb[2]), jc = find_index(L, mc[0], mc[1], mc[2]);
      if (jb < 0 || jc < 0) continue;
      if (jb > jc) {
        const int t = jb;
        jb = jc;
        jc = t;
      }
      const real s = D3[jb] + D3[jc];
      Pc[jb] = Pc[jb] + P->dq31 * s;
      Pc[jc] = Pc[jc] + P->dq31 * s;
    }
  }
  /* Non-equilibrium force content (eq:Frc at theta = 1): d_F^(n) = n g d^(n-1), the
   * symmetric product, per multi-index sum_a m_a g_a d^(n-1)_{m - e_a}, where d^(n-1) is
   * the central non-equilibrium moment of f itself.  By eq:newf and eq:evolution f is the
   * mean of the populations before and after the collision, so d^(n-1) = (D + P)/2 with D
   * and P the pre- and post-collision central moments of order n - 1 (P with its own
   * rates, the bulk rate included).  The content enters order n with (1 - omega_n/2)
   * (eq:RHS): order 3 with fq3; order 4, trimmed (omega_4 = 1), with 1/2.  Canonical order
   * puts every order before the next, so each order's P is final before it is used. */
  if (P->fq3 != 0) {
    for (int k = 0; k < NM; ++k) {
      const int32_t *m = L->mi + 3 * k;
      if (mabs(m) != 3) continue;
      real s = -0.0;
      for (int a = 0; a < 3; ++a) {
        if (m[a] == 0) continue;
        int j = find_index(L, m[0] - (a == 0), m[1] - (a == 1), m[2] - (a == 2));
        if (j < 0) continue;
        s = s + ((real)m[a] * g[a]) * ((real)0.5 * (D2[j] + Pc[j]));
      }
      Pc[k] = Pc[k] + P->fq3 * s;
    }
  }
  if (P->fo4) {
    for (int k = 0; k < NM; ++k) {
      const int32_t *m = L->mi + 3 * k;
      if (mabs(m) != 4) continue;
      real s = -0.0;
      for (int a = 0; a < 3; ++a) {
        if (m[a] == 0) continue;
        int j = find_index(L, m[0] - (a == 0), m[1] - (a == 1), m[2] - (a == 2));
        if (j < 0) continue;
        s = s + ((real)m[a] * g[a]) * ((real)0.5 * (D3[j] + Pc[j]));
      }
      Pc[k] = (real)0.5 * s;
    }
  }
  /* back to raw moments; the change of every moment over the collision, or (full: the
   * index set is smaller than Q) the post-collision moments a* themselves */
  const int full = L->NM < L->Q;
  real dA[MAXQ];
  for (int k = 0; k < NM; ++k) {
    const int32_t *m = L->mi + 3 * k;
    int n = mabs(m);
    if (n == 0) { /* mass is unchanged */
      dA[k] = full ? M.drho : 0;
      continue;
    }
    if (n == 1) { /* momentum gains F (a*^(1) = rho u + F/2 = j + F) */
      int a = m[0] ? 0 : (m[1] ? 1 : 2);
      dA[k] = full ? M.j[a] + M.F[a] : M.F[a];
      continue;
    }
    /* pre-collision raw moment of order >= 4 (orders 2, 3 are already in N); a* of
     * order 4 does not depend on it */
    real Nk = N[k];
    if (n >= 4 && !(full && n == 4)) {
      real A = project_folded(L, k, f, ps, pa);
      if (n > 4 && P->max_order < n) { /* orders above 4 are not carried: a*_m = 0 */
        dA[k] = full ? (real)0 : -A;
        continue;
      }
      /* carried orders: equilibrium plus the back-shift of the relaxed central moments,
       * whose own parts at orders 4 and above are trimmed to zero */
      Nk = A - E[k];
    }
    /* l = 0 term; at order 4 P_m is 0 (trimmed) or the fourth-order force content */
    real R = (n <= 3 || (n == 4 && P->fo4)) ? Pc[k] : (real)-0.0;
    for (int t = 0; t < S->n[k]; ++t) {
      int km = S->km[k][t];
      if (mabs(L->mi + 3 * km) > 3) continue; /* P = 0 at order 4 */
      R = fmar((real)S->cup[k][t] * U[S->kl[k][t]], Pc[km], R);
    }
    /* a*_m - a_m = (rho u^m + R_m) - (rho u^m + N_m); full: a*_m = rho u^m + R_m */
    dA[k] = full ? E[k] + R : R - Nk;
  }
  /* eq:evolution: f-bar + Omega + F, the increment reconstructed from dA; full: the
   * post-collision state rebuilt from a* */
  if (full)
    reconstruct_full_folded(L, dA, out);
  else
    reconstruct_folded(L, f, dA, out);
}

/* ---- raw-moment MRT (the appendix: eq:RHS_a in its explicit form, eq:bbd1) ------- */
/*
 * Every raw Hermite moment relaxes in the rest frame:
 *   a*_m = a0_m + (1 - omega_n) abar1_m + (1 - omega_n/2) aF_m,   n = |m| >= 1,
 * with a0_m = rho u^m, abar1_m = A_m - rho u^m the non-equilibrium raw moment of f-bar
 * (abar1_{e_a} = -F_a/2), and the raw force moments of eq:bbd1 at theta = 1,
 * aF_m = sum_a m_a u^{m - e_a} F_a (aF_{e_a} = F_a: the momentum gains F for any omega_1).
 * Order 4 is trimmed (omega_4 = 1, so a*_m = rho u^m + aF_m/2); orders above 4 are set
 * to 0 (the reconstruction sums to order 4).  As in collide_smrt the state is advanced by
 * the reconstruction of the changes a*_m - A_m.
 */
static void collide_rmrt(const oracle_lattice *L, const oracle_params *P, const real *f,
                         const real g[3], real *out) {
  macro_t M;
  macroscopic(L, P, f, g, &M);
  const int NM = L->NM;
  const int full = L->NM < L->Q; /* rebuild from a* (see reconstruct_full_folded) */
  real U[MAXQ], dA[MAXQ], ps[MAXQ], pa[MAXQ];
  for (int k = 0; k < NM; ++k) U[k] = upow(L->mi + 3 * k, M.u);
  for (int p = 1; 2 * p < L->Q; ++p) {
    ps[p] = f[2 * p - 1] + f[2 * p];
    pa[p] = f[2 * p - 1] - f[2 * p];
  }
  for (int k = 0; k < NM; ++k) {
    const int32_t *m = L->mi + 3 * k;
    int n = mabs(m);
    if (n == 0) {
      dA[k] = full ? M.drho : 0;
      continue;
    }
    if (n == 1) {
      int a = m[0] ? 0 : (m[1] ? 1 : 2);
      dA[k] = full ? M.j[a] + M.F[a] : M.F[a];
      continue;
    }
    /* the pre-collision moment (a* of order 4 does not depend on it) */
    real A = (full && n == 4) ? (real)0 : project_folded(L, k, f, ps, pa);
    if (n > 4) {
      dA[k] = full ? (real)0 : -A;
      continue;
    }
    const real E = M.rho * U[k];
    real N = A - E;
    real aF = -0.0;
    for (int a = 0; a < 3; ++a) {
      if (m[a] == 0) continue;
      int j = find_index(L, m[0] - (a == 0), m[1] - (a == 1), m[2] - (a == 2));
      if (j < 0) continue;
      aF = aF + ((real)m[a] * U[j]) * M.F[a];
    }
    real t;
    if (n == 2) {
      t = P->q2 * N;
      t = t + P->h2 * aF;
    } else if (n == 3) {
      t = P->q3 * N;
      t = t + P->h3 * aF;
    } else {
      t = (real)0.5 * aF;
    }
    dA[k] = full ? E + t : t - N;
  }
  if (full)
    reconstruct_full_folded(L, dA, out);
  else
    reconstruct_folded(L, f, dA, out);
}

static void collide(const oracle_lattice *L, const oracle_params *P, const smrt_plan *S,
                    const real *f, const real *g, real *out) {
  if (P->collision == 0)
    collide_bgk(L, P, f, g, out);
  else if (P->collision == 2)
    collide_rmrt(L, P, f, g, out);
  else
    collide_smrt(L, P, S, f, g, out);
}

void oracle_collide_node(const oracle_lattice *L, const oracle_params *P, const real *f,
                         const real *g, real *out) {
  smrt_plan S;
  make_plan(L, &S);
  check_pair_symmetry(L);
  collide(L, P, &S, f, g, out);
}

/* ---- equilibrium minus half force: the initial stored state ------------------------- */
/* eq:newf with Omega = 0 at t = 0: f-bar = f_eq - F_i / 2, so that rho-bar = rho and
 * u = u-bar + F/(2 rho) return the prescribed (rho, u).  BGK uses its second-order
 * equilibrium and force term; SMRT uses the equilibrium moments rho u^m and the raw
 * force moments a_F,m = sum_a m_a u^{m - e_a} F_a (appendix, a_F^(1..4) at theta = 1),
 * both up to order 4, reconstructed with Minv. */
void oracle_init_node(const oracle_lattice *L, const oracle_params *P, real rho,
                      const real *u, const real *g, real *out) {
  real F[3];
  for (int a = 0; a < 3; ++a) F[a] = rho * g[a];
  real drho = rho - P->shift;
  if (P->collision == 0) {
    for (int i = 0; i < L->Q; ++i) {
      real eu;
      real Pi = bgk_P(L, i, u, &eu);
      real feq = L->w[i] * (drho + rho * Pi);
      real Fi = bgk_force(L, i, u, F, eu);
      out[i] = feq - (real)0.5 * Fi;
    }
    return;
  }
  const int NM = L->NM;
  real a[MAXQ];
  for (int k = 0; k < NM; ++k) {
    const int32_t *m = L->mi + 3 * k;
    int n = mabs(m);
    if (n == 0) {
      a[k] = drho;
      continue;
    }
    if (n > 4) {
      a[k] = 0;
      continue;
    }
    real aF = -0.0;
    for (int al = 0; al < 3; ++al) {
      if (m[al] == 0) continue;
      int32_t r[3] = {m[0], m[1], m[2]};
      r[al] -= 1;
      aF = aF + (real)m[al] * (upow(r, u) * F[al]);
    }
    a[k] = rho * upow(m, u) - (real)0.5 * aF;
  }
  for (int i = 0; i < L->Q; ++i) {
    real acc = -0.0;
    for (int k = 0; k < NM; ++k) {
      real c = L->Minv[i * NM + k];
      if (c != 0 && mabs(L->mi + 3 * k) <= 4) acc = acc + c * a[k];
    }
    out[i] = acc;
  }
}

/* ---- whole-lattice operations -------------------------------------------------------- */
static int64_t node_count(const oracle_params *P) {
  return (int64_t)P->nx * P->ny * P->nz;
}

/* Initial state from per-node rho (N) and u (3 x N, component planes) and g (3 x N). */
void oracle_init(const oracle_lattice *L, const oracle_params *P, const real *rho,
                 const real *u, const real *g, real *f) {
  const int64_t N = node_count(P);
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    real un[3] = {u[n], u[N + n], u[2 * N + n]};
    real gn[3] = {g[n], g[N + n], g[2 * N + n]};
    real out[MAXQ];
    oracle_init_node(L, P, rho[n], un, gn, out);
    for (int i = 0; i < L->Q; ++i) f[i * N + n] = store_value(P, out[i]);
  }
}

/* One explicit step (eq:evolution): collide at every node, then stream the
 * post-collision value to x + e_i (the streaming after the SMRT reconstruction).
 * Periodic axes wrap; across a wall face the value returns to the same node in the
 * opposite direction (halfway bounce-back, a stationary no-slip wall midway between
 * the last fluid node and the next).  g is the acceleration field (3 x N) and gscale
 * the time factor s(t) applied to it. */
void oracle_step(const oracle_lattice *L, const oracle_params *P, const real *f,
                 real *fnew, const real *g, real gscale) {
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  const int64_t N = node_count(P);
  const int dims[3] = {nx, ny, nz};
  smrt_plan S;
  make_plan(L, &S);
  check_pair_symmetry(L);
#pragma omp parallel for schedule(static)
  for (int z = 0; z < nz; ++z) {
    for (int y = 0; y < ny; ++y) {
      for (int x = 0; x < nx; ++x) {
        const int64_t n = ((int64_t)z * ny + y) * nx + x;
        if (P->solid && P->solid[n]) { /* no fluid: nothing streams in or out */
          for (int i = 0; i < L->Q; ++i) fnew[i * N + n] = f[i * N + n];
          continue;
        }
        real fi[MAXQ], out[MAXQ];
        for (int i = 0; i < L->Q; ++i) fi[i] = f[i * N + n];
        real gn[3];
        for (int a = 0; a < 3; ++a) gn[a] = g[a * N + n] * gscale;
        collide(L, P, &S, fi, gn, out);
        const int c[3] = {x, y, z};
        for (int i = 0; i < L->Q; ++i) {
          int d[3];
          int wall_hit = 0;
          for (int a = 0; a < 3; ++a) {
            d[a] = c[a] + L->e[3 * i + a];
            if (d[a] < 0 || d[a] >= dims[a]) {
              if (P->wall[a])
                wall_hit = 1;
              else
                d[a] = ((d[a] % dims[a]) + dims[a]) % dims[a];
            }
          }
          real v = store_value(P, out[i]);
          const int64_t dn = ((int64_t)d[2] * ny + d[1]) * nx + d[0];
          /* halfway bounce-back at a wall face or against a solid node: the population
           * returns to its own node in the opposite direction */
          if (wall_hit || (P->solid && P->solid[dn]))
            fnew[(int64_t)L->opp[i] * N + n] = v;
          else
            fnew[(int64_t)i * N + dn] = v;
        }
      }
    }
  }
}

void oracle_run(const oracle_lattice *L, const oracle_params *P, real *f, real *tmp,
                const real *g, const real *gscale, int64_t nsteps) {
  const int64_t N = node_count(P);
  for (int64_t t = 0; t < nsteps; ++t) {
    oracle_step(L, P, f, tmp, g, gscale ? gscale[t] : (real)1);
    memcpy(f, tmp, sizeof(real) * (size_t)N * (size_t)L->Q);
  }
}

/* Physical density and velocity of the stored state (eq:half_F: u = u-bar + F/(2 rho)). */
void oracle_moments(const oracle_lattice *L, const oracle_params *P, const real *f,
                    const real *g, real gscale, real *rho, real *u) {
  const int64_t N = node_count(P);
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n) {
    if (P->solid && P->solid[n]) { /* no fluid */
      if (rho) rho[n] = 0;
      if (u)
        for (int a = 0; a < 3; ++a) u[a * N + n] = 0;
      continue;
    }
    real fi[MAXQ];
    for (int i = 0; i < L->Q; ++i) fi[i] = f[i * N + n];
    real gn[3];
    for (int a = 0; a < 3; ++a) gn[a] = g[a * N + n] * gscale;
    macro_t M;
    macroscopic(L, P, fi, gn, &M);
    if (rho) rho[n] = M.rho;
    if (u)
      for (int a = 0; a < 3; ++a) u[a * N + n] = M.u[a];
  }
}

/* The BGK pieces on their own, for the force-moment pins. */
void oracle_bgk_terms(const oracle_lattice *L, real rho, const real *u, const real *g,
                      real *feq, real *Fi) {
  real F[3];
  for (int a = 0; a < 3; ++a) F[a] = rho * g[a];
  for (int i = 0; i < L->Q; ++i) {
    real eu;
    real Pi = bgk_P(L, i, u, &eu);
    feq[i] = L->w[i] * (rho + rho * Pi);
    Fi[i] = bgk_force(L, i, u, F, eu);
  }
}

int oracle_real_size(void) { return (int)sizeof(real); }

/* Threads of the whole-lattice loops (the results do not depend on it); returns the
 * count in effect. */
int oracle_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
}

/* 1 for the PLAIN build (textbook operation order), 0 for the operation-order twin. */
int oracle_is_plain(void) {
#ifdef PLAIN
  return 1;
#else
  return 0;
#endif
}
