"""Pins of the oracle's lattice tables against the quadrature and Hermite facts they
must satisfy (paper Sec. II.A: Gauss-Hermite quadrature and eq:dft)."""
import json
import os
from fractions import Fraction
from itertools import product

import numpy as np
import pytest

from oracle import lattice as lat

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("L", lat.LATTICES)
def test_weights_golden(L):
    """Textbook weights of the three quadratures (tests/golden/lattice_weights.json)."""
    with open(os.path.join(GOLDEN, "lattice_weights.json")) as fh:
        gold = json.load(fh)["weights"][L]
    w = lat.weights(L)
    for e, wi in zip(lat.velocities(L), w):
        shell = str(sum(c * c for c in e))
        assert wi == Fraction(gold[shell])


@pytest.mark.parametrize("L", lat.LATTICES)
def test_quadrature_isotropy(L):
    """Degree-5 quadrature: weighted velocity moments equal the Gaussian's (c_s^2 = 1/3)
    up to fourth order and vanish at odd orders up to five."""
    E = lat.velocities(L)
    w = lat.weights(L)
    D = lat.dim(L)
    axes = range(D)
    assert sum(w) == 1
    for a in axes:
        assert sum(wi * e[a] for wi, e in zip(w, E)) == 0
    for a, b in product(axes, repeat=2):
        assert sum(wi * e[a] * e[b] for wi, e in zip(w, E)) == (Fraction(1, 3) if a == b else 0)
    for idx in product(axes, repeat=3):
        assert sum(wi * e[idx[0]] * e[idx[1]] * e[idx[2]] for wi, e in zip(w, E)) == 0
    for a, b, c, d in product(axes, repeat=4):
        m4 = sum(wi * e[a] * e[b] * e[c] * e[d] for wi, e in zip(w, E))
        iso = Fraction(1, 9) * ((a == b) * (c == d) + (a == c) * (b == d) + (a == d) * (b == c))
        assert m4 == iso
    for idx in product(axes, repeat=5):
        assert sum(wi * np.prod([e[i] for i in idx]) for wi, e in zip(w, E)) == 0


@pytest.mark.parametrize("L", lat.LATTICES)
def test_hermite_norms_and_orthogonality(L):
    """sum_i w_i H_m(e_i)^2 = m! c_s^(2|m|); D2Q9 and D3Q27 fully orthogonal; D3Q19 has
    exactly nine non-orthogonal pairs (its basis drops the components with three
    non-zero indices, so a few fourth-order polynomials alias lower ones)."""
    w = lat.weights(L)
    M = lat.projection(L)
    ms = lat.index_set(L)
    Q = len(w)
    assert len(ms) == Q
    for k, m in enumerate(ms):
        assert sum(w[i] * M[k][i] ** 2 for i in range(Q)) == lat.mfact(m) * lat.CS2 ** sum(m)
    bad = []
    for a in range(Q):
        for b in range(a + 1, Q):
            if sum(w[i] * M[a][i] * M[b][i] for i in range(Q)) != 0:
                bad.append((ms[a], ms[b]))
    if L == "D3Q19":
        assert len(bad) == 9
        assert ((2, 0, 0), (0, 2, 2)) in bad and ((2, 1, 0), (0, 1, 2)) in bad
    else:
        assert bad == []


@pytest.mark.parametrize("L", lat.LATTICES)
def test_reconstruction_is_inverse(L):
    M = lat.projection(L)
    Mi = lat.reconstruction(L)
    Q = len(M)
    for i in range(Q):
        for j in range(Q):
            assert sum(Mi[i][k] * M[k][j] for k in range(Q)) == (1 if i == j else 0)
    # rest column is the weights: Minv applied to (1, 0, ...) gives w
    assert [r[0] for r in Mi] == lat.weights(L)
    if L != "D3Q19":
        # orthogonal lattices: the inverse is the paper's w_i H_m / (m! c_s^(2|m|))
        assert tuple(map(tuple, lat.reconstruction_orthogonal(L))) == Mi


@pytest.mark.parametrize("L", lat.LATTICES)
def test_opposites(L):
    E = lat.velocities(L)
    opp = lat.opposite(L)
    for i, e in enumerate(E):
        assert E[opp[i]] == tuple(-c for c in e)
        assert opp[opp[i]] == i


def test_one_time_rounding():
    """Rationals are rounded once, to nearest-even, in both formats."""
    assert lat.to_f64(Fraction(1, 3)) == 1 / 3
    assert lat.f32_bits(lat.to_f32(Fraction(1, 3))) == 0x3EAAAAAB
    assert lat.f32_bits(lat.to_f32(Fraction(2, 3))) == 0x3F2AAAAB
    assert lat.f32_bits(lat.to_f32(Fraction(-1, 36))) == np.float32(-1 / 36).view(np.uint32)
    # an exact tie between two binary32 neighbours rounds to the even one
    tie = Fraction(2 ** 24 + 1, 2 ** 24)
    assert lat.to_f32(tie) == np.float32(1.0)
    rng = np.random.default_rng(1)
    for _ in range(200):
        f = Fraction(int(rng.integers(1, 10 ** 6)), int(rng.integers(1, 10 ** 6)))
        # binary32 from binary64 rounding agrees except at (here absent) double-rounding ties
        assert lat.to_f32(f) == np.float32(float(f))
