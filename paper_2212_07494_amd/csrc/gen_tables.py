"""Generate lbm_tables.h: compile-time lattice constants of the HIP library.

Run at build time.  Every constant is an exact rational (``fractions.Fraction``)
rounded once, to nearest-even, to binary64 and to binary32, and printed as a
hexadecimal floating literal so the compiler reads back the identical bits.

Contents per lattice (lattice units; D2Q9, D3Q19, D3Q27 with c_s^2 = 1/3 and the
high-order D3Q39 with c_s^2 = 2/3):
  CS2N / CS2D    c_s^2 = CS2N / CS2D;  ICS2 = 1 / c_s^2 (3 or 1.5, exact)
  E[i][3]        discrete velocities in the library's population order
  OPP[i]         index of -e_i
  W / Wf[i]      Gauss-Hermite weights
  MI[k][3]       multi-indices m of the Hermite moments the lattice carries,
                 ordered by |m|, then m descending lexicographically (x first)
  ORD[k]         |m|
  H / Hf[k][i]   lattice Hermite polynomial H_m(e_i) = prod_a h_{m_a}(e_a), h_0 = 1,
                 h_1 = e, h_2 = e^2 - c2, h_3 = e^3 - 3 c2 e, h_4 = e^4 - 6 c2 e^2 + 3 c2^2
                 (c2 = c_s^2; Sec. II.A, eq:dft)
  MINV / MINVf[i][k]  reconstruction f_i = sum_k MINV[i][k] a_k
  shift plan     for each m: the sub-multi-indices l (0 < l < m) with the index of
                 m - l and the binomial weights of the Hermite shift between the rest
                 frame and the frame moving with u (down: C(m,l)(-1)^|l|, up: C(m,l)).

Derivation of MINV.  Where the lattice carries Q moments (D2Q9, D3Q19, D3Q27) it inverts
a_k = sum_i H[k][i] f_i: weighted least squares is exact for an invertible M, so
MINV = W M^T (M W M^T)^-1.  On D2Q9 and D3Q27 the Gram matrix M W M^T is diagonal
(m! c_s^(2|m|)), which gives the paper's reconstruction w_i H_m(e_i)/(m! c_s^(2|m|));
on D3Q19 it has nine off-diagonal pairs and is inverted exactly.  D3Q39 carries the 35
moments of orders <= 4 (NM < Q) and MINV is the paper's reconstruction itself, the
Hermite sum w_i H_m(e_i)/(m! c_s^(2|m|)); being exact to degree 7, it returns every
moment of order <= 3 unchanged.
"""
from __future__ import annotations

import os
import sys
from fractions import Fraction as Fr
from itertools import product
from math import comb, factorial

LATTICE_NAMES = ("D2Q9", "D3Q19", "D3Q27", "D3Q39")


def sound_speed2(name):
    return Fr(2, 3) if name == "D3Q39" else Fr(1, 3)


def lattice(name):
    if name == "D3Q39":
        # rest, then shells |e|^2 = 1, 3, 4, 8, 9, each velocity before its opposite
        fams = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1), (1, 1, -1), (1, -1, 1),
                (1, -1, -1), (2, 0, 0), (0, 2, 0), (0, 0, 2), (2, 2, 0), (2, -2, 0),
                (2, 0, 2), (2, 0, -2), (0, 2, 2), (0, 2, -2), (3, 0, 0), (0, 3, 0), (0, 0, 3)]
        vel = [(0, 0, 0)]
        for v in fams:
            vel += [v, tuple(-c for c in v)]
        shell = {0: Fr(1, 12), 1: Fr(1, 12), 3: Fr(1, 27), 4: Fr(2, 135), 8: Fr(1, 432),
                 9: Fr(1, 1620)}
        w = [shell[sum(c * c for c in v)] for v in vel]
        ms = [m for m in product(range(5), repeat=3) if sum(m) <= 4]
        ms.sort(key=lambda m: (sum(m), [-c for c in m]))
        return vel, w, ms
    if name == "D2Q9":
        vel = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
               (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0)]
    else:
        axes = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
        diag = [(1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)]
        corner = [(1, 1, 1), (1, 1, -1), (1, -1, 1), (1, -1, -1)]
        groups = axes + diag + (corner if name == "D3Q27" else [])
        vel = [(0, 0, 0)]
        for v in groups:
            vel += [v, tuple(-c for c in v)]
    # weights: D2Q9 and D3Q27 are tensor products of the 1-D rule (2/3, 1/6, 1/6)
    one_d = {0: Fr(2, 3), 1: Fr(1, 6), -1: Fr(1, 6)}
    if name == "D3Q19":
        wsh = {0: Fr(1, 3), 1: Fr(1, 18), 2: Fr(1, 36)}
        w = [wsh[sum(c * c for c in v)] for v in vel]
    else:
        dim = 2 if name == "D2Q9" else 3
        w = []
        for v in vel:
            p = Fr(1)
            for a in range(dim):
                p *= one_d[v[a]]
            w.append(p)
    if name == "D2Q9":
        ms = [(a, b, 0) for a in range(3) for b in range(3)]
    elif name == "D3Q27":
        ms = list(product(range(3), repeat=3))
    else:
        ms = [m for m in product(range(3), repeat=3) if sum(1 for c in m if c) <= 2]
    ms.sort(key=lambda m: (sum(m), [-c for c in m]))
    return vel, w, ms


def herm(m, e, c2):
    p = Fr(1)
    for k, c in zip(m, e):
        p *= {0: Fr(1), 1: Fr(c), 2: Fr(c * c) - c2, 3: Fr(c ** 3) - 3 * c2 * c,
              4: Fr(c ** 4) - 6 * c2 * c * c + 3 * c2 * c2}[k]
    return p


def solve_inverse(G):
    """Exact inverse of a small symmetric positive-definite rational matrix
    (Cholesky-free: Gauss elimination on the augmented matrix, pivoting on the diagonal)."""
    n = len(G)
    A = [[Fr(x) for x in row] + [Fr(1 if i == j else 0) for j in range(n)]
         for i, row in enumerate(G)]
    for c in range(n):
        piv = A[c][c]
        assert piv != 0
        A[c] = [v / piv for v in A[c]]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c]
                A[r] = [a - f * b for a, b in zip(A[r], A[c])]
    return [row[n:] for row in A]


def reconstruction(vel, w, ms, c2):
    Q = len(vel)
    M = [[herm(m, e, c2) for e in vel] for m in ms]
    if len(ms) < Q:  # the Hermite sum over the carried orders
        R = [[w[i] * M[k][i] / (factorial(m[0]) * factorial(m[1]) * factorial(m[2])
                                * c2 ** sum(m)) for k, m in enumerate(ms)] for i in range(Q)]
        return M, R
    G = [[sum(M[a][i] * w[i] * M[b][i] for i in range(Q)) for b in range(Q)] for a in range(Q)]
    Gi = solve_inverse(G)
    # MINV[i][k] = w_i sum_b M[b][i] Gi[b][k]
    return M, [[w[i] * sum(M[b][i] * Gi[b][k] for b in range(Q)) for k in range(Q)]
               for i in range(Q)]


# ---- one-time rounding, verified exactly -------------------------------------------------

def f64(x: Fr) -> float:
    return x.numerator / x.denominator  # correctly rounded int/int division


def f32_hex(x: Fr) -> str:
    import numpy as np
    v = np.float32(f64(x))
    # verify nearest-even against the exact rational (guards against double rounding)
    if x != 0:
        lo = np.nextafter(v, np.float32(-np.inf))
        hi = np.nextafter(v, np.float32(np.inf))
        d = abs(Fr(float(v)) - x)
        for nb in (lo, hi):
            dn = abs(Fr(float(nb)) - x)
            assert d < dn or (d == dn and (int(np.float32(v).view(np.uint32)) & 1) == 0), x
    return float(v).hex()


def c_hex(v: float) -> str:
    if v == 0:
        return "0.0"
    return v.hex()


def emit(name, out):
    vel, w, ms = lattice(name)
    Q, NM = len(vel), len(ms)
    c2 = sound_speed2(name)
    M, Minv = reconstruction(vel, w, ms, c2)
    if NM == Q:  # exactness check: Minv * M = I
        for i in range(Q):
            for j in range(Q):
                s = sum(Minv[i][k] * M[k][j] for k in range(Q))
                assert s == (1 if i == j else 0)
    else:  # moments of orders <= 3 come back unchanged: (M Minv)_ab = delta_ab there
        for a in range(NM):
            for b in range(NM):
                if sum(ms[a]) <= 3 or sum(ms[b]) <= 3:
                    s = sum(M[a][i] * Minv[i][b] for i in range(Q))
                    assert s == (1 if a == b else 0)
    dim = 2 if name == "D2Q9" else 3
    # shift plan
    index = {m: k for k, m in enumerate(ms)}
    plan = []
    for m in ms:
        terms = []
        for kl, l in enumerate(ms):
            if kl == 0 or l == m or any(a > b for a, b in zip(l, m)):
                continue
            r = tuple(b - a for a, b in zip(l, m))
            c = 1
            for a, b in zip(l, m):
                c *= comb(b, a)
            down = -c if sum(l) % 2 else c
            terms.append((kl, index[r], down, c))
        plan.append(terms)
    maxt = max(1, max(len(t) for t in plan))

    def arr2(rows, fmt):
        return "{" + ", ".join("{" + ", ".join(fmt(v) for v in r) + "}" for r in rows) + "}"

    p = out.append
    p(f"struct {name} {{")
    p(f"  static constexpr int D = {dim}, Q = {Q}, NM = {NM}, MAXT = {maxt};")
    p(f"  static constexpr int CS2N = {c2.numerator}, CS2D = {c2.denominator};")
    p(f"  static constexpr double ICS2 = {c_hex(f64(1 / c2))};")
    p(f"  static constexpr int E[{Q}][3] = {arr2(vel, str)};")
    p(f"  static constexpr int OPP[{Q}] = {{{', '.join(str(vel.index(tuple(-c for c in e))) for e in vel)}}};")
    p(f"  static constexpr int MI[{NM}][3] = {arr2(ms, str)};")
    p(f"  static constexpr int ORD[{NM}] = {{{', '.join(str(sum(m)) for m in ms)}}};")
    p(f"  static constexpr double W[{Q}] = {{{', '.join(c_hex(f64(x)) for x in w)}}};")
    p(f"  static constexpr float Wf[{Q}] = {{{', '.join(f32_hex(x) + 'f' for x in w)}}};")
    p(f"  static constexpr double H[{NM}][{Q}] = {arr2(M, lambda x: c_hex(f64(x)))};")
    p(f"  static constexpr float Hf[{NM}][{Q}] = {arr2(M, lambda x: (f32_hex(x) + 'f') if x else '0.0f')};")
    p(f"  static constexpr double MINV[{Q}][{NM}] = {arr2(Minv, lambda x: c_hex(f64(x)))};")
    p(f"  static constexpr float MINVf[{Q}][{NM}] = {arr2(Minv, lambda x: (f32_hex(x) + 'f') if x else '0.0f')};")
    pad = [t + [(0, 0, 0, 0)] * (maxt - len(t)) for t in plan]
    p(f"  static constexpr int NT[{NM}] = {{{', '.join(str(len(t)) for t in plan)}}};")
    p(f"  static constexpr int TL[{NM}][{maxt}] = {arr2([[t[0] for t in r] for r in pad], str)};")
    p(f"  static constexpr int TM[{NM}][{maxt}] = {arr2([[t[1] for t in r] for r in pad], str)};")
    p(f"  static constexpr int CDN[{NM}][{maxt}] = {arr2([[t[2] for t in r] for r in pad], str)};")
    p(f"  static constexpr int CUP[{NM}][{maxt}] = {arr2([[t[3] for t in r] for r in pad], str)};")
    p("};")
    p("")


def generate(path):
    out = ["// Generated by gen_tables.py -- lattice constants, exact rationals rounded once.",
           "// Do not edit by hand.", "#pragma once", "", "namespace lbm {", ""]
    for name in LATTICE_NAMES:
        emit(name, out)
    out.append("}  // namespace lbm")
    text = "\n".join(out) + "\n"
    old = open(path).read() if os.path.exists(path) else None
    if old != text:
        with open(path, "w") as fh:
            fh.write(text)
    return path


if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    print(generate(sys.argv[1] if len(sys.argv) > 1 else os.path.join(here, "lbm_tables.h")))
