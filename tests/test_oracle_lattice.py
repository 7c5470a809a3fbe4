"""Pins of the oracle's lattice tables against the quadrature and Hermite facts they
must satisfy (paper Sec. II.A: Gauss-Hermite quadrature and eq:dft), for the three
degree-5 lattices and the degree-7 lattice D3Q39."""
import json
import os
from fractions import Fraction
from itertools import product

import numpy as np
import pytest

from oracle import lattice as lat

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("L", lat.ALL_LATTICES)
def test_weights_golden(L):
    """Textbook weights of the quadratures (tests/golden/lattice_weights.json)."""
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


def _gauss_moment(m, c2):
    """E[x^m] of the isotropic Gaussian of variance c2 per axis: prod_a (m_a - 1)!! c2^(m_a/2)
    for even m_a, 0 if any m_a is odd."""
    p = Fraction(1)
    for k in m:
        if k % 2:
            return Fraction(0)
        for j in range(k - 1, 0, -2):
            p *= j
        p *= c2 ** (k // 2)
    return p


DEGREE = {"D2Q9": 5, "D3Q19": 5, "D3Q27": 5, "D3Q39": 7}


@pytest.mark.parametrize("L", lat.ALL_LATTICES)
def test_quadrature_degree(L):
    """Every weighted velocity moment sum_i w_i e^m equals the Gaussian's with variance
    c_s^2 (1/3, or 2/3 on D3Q39) up to the lattice's degree (5, or 7 on D3Q39), and some
    moment of the next even degree does not: the weights and c_s^2 are the unique solution
    of these conditions on the velocity set."""
    E = lat.velocities(L)
    w = lat.weights(L)
    D = lat.dim(L)
    c2 = lat.cs2(L)
    assert c2 == sum(wi * e[0] ** 2 for wi, e in zip(w, E))
    for deg in range(DEGREE[L] + 2):
        for m in product(range(deg + 1), repeat=D):
            if sum(m) != deg:
                continue
            got = sum(wi * np.prod([e[a] ** m[a] for a in range(D)]) for wi, e in zip(w, E))
            if deg <= DEGREE[L]:
                assert got == _gauss_moment(m, c2), (m, got)
    deg = DEGREE[L] + 1
    assert any(sum(wi * e[0] ** deg for wi, e in zip(w, E)) != _gauss_moment((deg,), c2)
               for _ in [0])


@pytest.mark.parametrize("L", lat.ALL_LATTICES)
def test_hermite_tables_against_numpy(L):
    """H_m(e_i) = c_s^|m| prod_a He_{m_a}(e_ia / c_s) with numpy's probabilists' Hermite
    series (numpy.polynomial.hermite_e), to rounding."""
    from numpy.polynomial import hermite_e as He
    c = float(lat.cs2(L)) ** 0.5
    M = np.array([[float(x) for x in row] for row in lat.projection(L)])
    E = np.array(lat.velocities(L), float)
    for k, m in enumerate(lat.index_set(L)):
        want = np.ones(len(E))
        for a in range(3):
            want *= He.hermeval(E[:, a] / c, [0] * m[a] + [1]) * c ** m[a]
        assert np.max(np.abs(M[k] - want)) <= 1e-12 * max(1.0, np.max(np.abs(want))), m


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


def test_d3q39_hermite_orthogonality_to_degree_seven():
    """D3Q39 carries every multi-index with |m| <= 4 (35 of them); sum_i w_i H_m H_m' =
    delta m! c_s^(2|m|) whenever |m| + |m'| <= 7 (the quadrature's degree), and the
    order-4 block is not orthogonal."""
    L = "D3Q39"
    w = lat.weights(L)
    M = lat.projection(L)
    ms = lat.index_set(L)
    assert len(ms) == 35 and all(sum(m) <= 4 for m in ms) and len(set(ms)) == 35
    c2 = lat.cs2(L)
    off4 = 0
    for a, ma in enumerate(ms):
        for b, mb in enumerate(ms):
            g = sum(w[i] * M[a][i] * M[b][i] for i in range(len(w)))
            if sum(ma) + sum(mb) <= 7:
                assert g == (lat.mfact(ma) * c2 ** sum(ma) if a == b else 0), (ma, mb)
            elif g != (lat.mfact(ma) * c2 ** sum(ma) if a == b else 0):
                off4 += 1
    assert off4 > 0


def test_d3q39_reconstruction_keeps_orders_to_three():
    """The D3Q39 reconstruction is the paper's Hermite sum w_i H_m(e_i) / (m! c_s^(2|m|))
    over |m| <= 4: projecting what it builds returns every moment of order <= 3 exactly
    (the rows and the columns of M R of those orders are the identity), the order-4 block
    is not the identity (degree 8 exceeds the quadrature), the rest column is w_i, and
    nothing in the null space of M survives (R M kills it).  On the 39 velocities the 35
    polynomials span 29 dimensions: the 20 of orders <= 3 and 9 of order 4 (six
    fourth-order monomials alias lower ones, e.g. e_x^3 e_y = e_x e_y^3 on every
    velocity), so the null space of M has dimension 10."""
    L = "D3Q39"
    M = lat.projection(L)
    R = lat.reconstruction(L)
    ms = lat.index_set(L)
    assert R == lat.reconstruction_orthogonal(L)
    Q, NM = len(lat.velocities(L)), len(ms)
    MR = [[sum(M[a][i] * R[i][b] for i in range(Q)) for b in range(NM)] for a in range(NM)]
    for a in range(NM):
        for b in range(NM):
            if sum(ms[a]) <= 3 or sum(ms[b]) <= 3:
                assert MR[a][b] == (1 if a == b else 0), (ms[a], ms[b])
    assert any(MR[a][b] != (1 if a == b else 0) for a in range(NM) for b in range(NM))
    assert [r[0] for r in R] == lat.weights(L)
    Mf = np.array([[float(x) for x in r] for r in M])
    Rf = np.array([[float(x) for x in r] for r in R])
    _, sv, vt = np.linalg.svd(Mf)
    rank = int(np.sum(sv > 1e-10))
    assert rank == 29
    assert np.linalg.matrix_rank(Mf[[k for k, m in enumerate(ms) if sum(m) <= 3]]) == 20
    null = vt[rank:]
    assert null.shape == (Q - rank, Q) == (10, 39)
    assert np.max(np.abs(Rf @ (Mf @ null.T))) < 1e-13


@pytest.mark.parametrize("L", lat.ALL_LATTICES)
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
