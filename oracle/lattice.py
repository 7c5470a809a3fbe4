"""Exact-rational lattice tables for the CPU oracle (test infrastructure only).

This module belongs to the oracle: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code
with the HIP path, which derives its own copy of the same tables.

What it defines (paper Sec. II.A, discrete Hermite transform, eq:dft):

* the discrete velocities e_i of D2Q9, D3Q19 and D3Q27 (c_s^2 = 1/3) and of the
  high-order lattice D3Q39 (c_s^2 = 2/3, exact to degree 7) in lattice units
  (Delta x = Delta t = 1), with their Gauss-Hermite weights w_i;
* the lattice Hermite polynomials, written in lattice units so that no square root
  appears: per axis H0(e) = 1, H1(e) = e, H2(e) = e^2 - c_s^2, H3(e) = e^3 - 3 c_s^2 e,
  H4(e) = e^4 - 6 c_s^2 e^2 + 3 c_s^4, and for a multi-index m = (mx, my, mz) the
  product H_m(e) = prod_a H_{m_a}(e_a).  This is the paper's tensor Hermite
  polynomial of xi = e / c_s scaled by c_s^|m| (one component of H^(n), n = |m|);
* the index set I of multi-indices each lattice represents, in a fixed
  canonical order (|m| ascending, then m descending lexicographically with x
  most significant);
* the projection matrix M[m][i] = H_m(e_i) (the forward transform of eq:dft)
  and the reconstruction.  On D2Q9, D3Q19 and D3Q27 the index set has Q members and
  the reconstruction is the exact inverse of M; on D2Q9 and D3Q27 it equals the
  paper's reconstruction w_i sum_m a_m H_m(e_i) / (m! c_s^(2|m|)) (second half of
  eq:dft); on D3Q19 the basis is not orthogonal and the exact inverse is used
  (reading documented with the oracle).  On D3Q39 the index set is every m with
  |m| <= 4 (35 < Q = 39 moments) and the reconstruction is the paper's Hermite sum to
  order 4 itself, which is not an inverse: the populations it builds carry exactly the
  moments of orders 0 to 3 given to it (the quadrature is exact to degree 7), and
  nothing that the 35 moments do not describe.

Everything is computed in exact rational arithmetic (``fractions.Fraction``)
and rounded once to the target float format when a table is handed to C.
"""
from __future__ import annotations

import struct
from fractions import Fraction
from functools import lru_cache
from itertools import product
from math import factorial

import numpy as np

CS2 = Fraction(1, 3)  # lattice speed of sound squared of D2Q9, D3Q19, D3Q27

LATTICES = ("D2Q9", "D3Q19", "D3Q27")
HIGH_ORDER = ("D3Q39",)  # multi-speed lattices: periodic boxes only
ALL_LATTICES = LATTICES + HIGH_ORDER

# Population order shared with the library's storage layout: rest particle
# first, then pairs (e, -e) so that the opposite of i is i+1 (i odd) or i-1.
_VEL = {
    "D2Q9": [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
             (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0)],
}
_D3Q19 = [(0, 0, 0),
          (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
          (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
          (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
          (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
_VEL["D3Q19"] = _D3Q19
_VEL["D3Q27"] = _D3Q19 + [(1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1),
                          (1, -1, 1), (-1, 1, -1), (1, -1, -1), (-1, 1, 1)]
# D3Q39: the rest particle, then per speed shell |e|^2 = 1, 3, 4, 8, 9 each velocity
# followed by its opposite.
_VEL["D3Q39"] = [(0, 0, 0)] + [
    v for e in [(1, 0, 0), (0, 1, 0), (0, 0, 1),
                (1, 1, 1), (1, 1, -1), (1, -1, 1), (1, -1, -1),
                (2, 0, 0), (0, 2, 0), (0, 0, 2),
                (2, 2, 0), (2, -2, 0), (2, 0, 2), (2, 0, -2), (0, 2, 2), (0, 2, -2),
                (3, 0, 0), (0, 3, 0), (0, 0, 3)]
    for v in (e, tuple(-c for c in e))]


def dim(lat: str) -> int:
    return 2 if lat == "D2Q9" else 3


def cs2(lat: str) -> Fraction:
    """Lattice speed of sound squared: sum_i w_i e_ix^2."""
    return Fraction(2, 3) if lat == "D3Q39" else CS2


def velocities(lat: str) -> list[tuple[int, int, int]]:
    return list(_VEL[lat])


def opposite(lat: str) -> list[int]:
    v = _VEL[lat]
    return [v.index(tuple(-c for c in e)) for e in v]


def weights(lat: str) -> list[Fraction]:
    """Gauss-Hermite weights; they depend only on |e|^2 (the speed shell)."""
    shell = {
        "D2Q9": {0: Fraction(4, 9), 1: Fraction(1, 9), 2: Fraction(1, 36)},
        "D3Q19": {0: Fraction(1, 3), 1: Fraction(1, 18), 2: Fraction(1, 36)},
        "D3Q27": {0: Fraction(8, 27), 1: Fraction(2, 27), 2: Fraction(1, 54),
                  3: Fraction(1, 216)},
        "D3Q39": {0: Fraction(1, 12), 1: Fraction(1, 12), 3: Fraction(1, 27),
                  4: Fraction(2, 135), 8: Fraction(1, 432), 9: Fraction(1, 1620)},
    }[lat]
    return [shell[sum(c * c for c in e)] for e in _VEL[lat]]


def _canonical(ms):
    return sorted(ms, key=lambda m: (sum(m), tuple(-c for c in m)))


def index_set(lat: str) -> list[tuple[int, int, int]]:
    """Multi-indices of the Hermite polynomials the lattice carries."""
    if lat == "D2Q9":
        ms = [(a, b, 0) for a, b in product(range(3), repeat=2)]
    elif lat == "D3Q27":
        ms = list(product(range(3), repeat=3))
    elif lat == "D3Q39":  # every order up to 4
        ms = [m for m in product(range(5), repeat=3) if sum(m) <= 4]
    else:  # D3Q19: at most two non-zero components
        ms = [m for m in product(range(3), repeat=3) if sum(c > 0 for c in m) <= 2]
    return _canonical(ms)


def hermite_1d(k: int, e: int, c2: Fraction = CS2) -> Fraction:
    """c^k He_k(e / c), c^2 = c2: the probabilists' Hermite polynomial in lattice units."""
    if k == 0:
        return Fraction(1)
    if k == 1:
        return Fraction(e)
    if k == 2:
        return Fraction(e * e) - c2
    if k == 3:
        return Fraction(e ** 3) - 3 * c2 * e
    if k == 4:
        return Fraction(e ** 4) - 6 * c2 * e * e + 3 * c2 * c2
    raise ValueError(k)


def hermite(m, e, c2: Fraction = CS2) -> Fraction:
    p = Fraction(1)
    for ma, ea in zip(m, e):
        p *= hermite_1d(ma, ea, c2)
    return p


def mfact(m) -> int:
    p = 1
    for c in m:
        p *= factorial(c)
    return p


@lru_cache(maxsize=None)
def projection(lat: str) -> tuple[tuple[Fraction, ...], ...]:
    """M[m][i] = H_m(e_i): raw Hermite moments a_m = sum_i f_i H_m(e_i)."""
    return tuple(tuple(hermite(m, e, cs2(lat)) for e in _VEL[lat]) for m in index_set(lat))


def _inverse(A):
    n = len(A)
    a = [list(r) + [Fraction(int(i == j)) for j in range(n)] for i, r in enumerate(A)]
    for c in range(n):
        p = next(r for r in range(c, n) if a[r][c] != 0)
        a[c], a[p] = a[p], a[c]
        pv = a[c][c]
        a[c] = [x / pv for x in a[c]]
        for r in range(n):
            if r != c and a[r][c] != 0:
                fac = a[r][c]
                a[r] = [x - fac * y for x, y in zip(a[r], a[c])]
    return [row[n:] for row in a]


@lru_cache(maxsize=None)
def reconstruction(lat: str) -> tuple[tuple[Fraction, ...], ...]:
    """Reconstruction Minv[i][m], f = Minv a: the exact inverse of the projection where
    the index set has Q members, the paper's Hermite sum (reconstruction_orthogonal)
    on D3Q39."""
    if lat in HIGH_ORDER:
        return reconstruction_orthogonal(lat)
    return tuple(tuple(r) for r in _inverse([list(r) for r in projection(lat)]))


@lru_cache(maxsize=None)
def reconstruction_orthogonal(lat: str):
    """The paper's reconstruction coefficient w_i H_m(e_i) / (m! c_s^(2|m|))."""
    w = weights(lat)
    c2 = cs2(lat)
    return tuple(tuple(w[i] * hermite(m, e, c2) / (mfact(m) * c2 ** sum(m))
                       for m in index_set(lat))
                 for i, e in enumerate(_VEL[lat]))


# --- one-time rounding of exact rationals -------------------------------------------

def to_f64(x: Fraction) -> float:
    # int / int true division in Python is correctly rounded (IEEE RNE).
    return x.numerator / x.denominator


def to_f32(x: Fraction) -> np.float32:
    """Round an exact rational once to binary32 (round to nearest, ties to even)."""
    if x == 0:
        return np.float32(0.0)
    sign = -1 if x < 0 else 1
    a = abs(x)
    # find exponent E with 2^E <= a < 2^(E+1)
    E = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** E > a:
        E -= 1
    elif Fraction(2) ** (E + 1) <= a:
        E += 1
    E = max(E, -126)  # subnormal range keeps the same quantum
    q = Fraction(2) ** (E - 23)
    n = a / q
    fl = n.numerator // n.denominator
    rem = n - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    val = float(fl) * float(q)  # exact: fl < 2^25, q a power of two
    return np.float32(sign * val)


def tables(lat: str, real=np.float64) -> dict:
    """Numeric tables for the C oracle, each entry rounded once from its rational."""
    rnd = to_f64 if real == np.float64 else to_f32
    Q = len(_VEL[lat])
    ms = index_set(lat)
    return {
        "D": dim(lat),
        "Q": Q,
        "NM": len(ms),
        "e": np.array(_VEL[lat], dtype=np.int32),
        "opp": np.array(opposite(lat), dtype=np.int32),
        "mi": np.array(ms, dtype=np.int32),
        "w": np.array([rnd(x) for x in weights(lat)], dtype=real),
        "H": np.array([[rnd(x) for x in row] for row in projection(lat)], dtype=real),
        "Minv": np.array([[rnd(x) for x in row] for row in reconstruction(lat)], dtype=real),
        "ics2": real(rnd(1 / cs2(lat))),  # 3 or 3/2, exact in binary
    }


def f32_bits(x: np.float32) -> int:
    return struct.unpack("<I", struct.pack("<f", float(x)))[0]
