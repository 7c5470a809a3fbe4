"""Pins of the oracle's per-node arithmetic against identities the paper states.

* P-F1: the BGK force term has zero mass, first moment rho g and second moment
  rho (g u + u g) (paper Sec. I and eq:af: a_F^(0) = 0, a_F^(1) = rho g; the
  second-order truncation below eq:Fr).
* P-M: the initial state returns the prescribed rho and u (eq:half_F).
* SMRT post-collision moments equal eq:bbd1 evaluated literally in tensor form
  (orders 0..4, theta = 1, order 4 by the recursion), a formulation independent of
  the oracle's multi-index Hermite shifts.
* BGK post-collision moments equal those of eq:explict_eq in moment form.

The high-order lattice D3Q39 (c_s^2 = 2/3) takes part wherever the statement holds on it;
its post-collision state is the paper's Hermite sum to order 4, whose fourth-order
moments on the 39 velocities are those of the sum (the product M R of the tables
applied to the post-collision moments), not the moments themselves.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import Oracle
from oracle import lattice as lat

CS2 = 1.0 / 3.0


def _cs2(L):
    return float(lat.cs2(L))


def _as_lattice_moments(o, want):
    """Moments the lattice returns for post-collision moments `want` (one per index):
    themselves where the reconstruction inverts the projection, M R want on D3Q39."""
    if o.L["NM"] == o.Q:
        return np.asarray(want)
    return (o.L["H"] @ o.L["Minv"]) @ np.asarray(want)


def _setup(L, seed):
    rng = np.random.default_rng(seed)
    D = lat.dim(L)
    rho = 1.0 + 0.1 * rng.uniform(-1, 1)
    u = np.zeros(3)
    g = np.zeros(3)
    u[:D] = rng.uniform(-0.08, 0.08, D)
    g[:D] = rng.uniform(-1e-3, 1e-3, D)
    return rho, u, g


def _tol(terms):
    return 16 * np.finfo(np.float64).eps * np.sum(np.abs(terms))


@pytest.mark.parametrize("L", lat.ALL_LATTICES)
@pytest.mark.parametrize("seed", range(5))
def test_bgk_force_moments(L, seed):
    rho, u, g = _setup(L, seed)
    o = Oracle(L, "bgk", (2, 2, 2 if lat.dim(L) == 3 else 1))
    feq, Fi = o.bgk_terms(rho, u, g)
    e = o.L["e"].astype(np.float64)
    assert abs(Fi.sum()) <= _tol(Fi)
    m1 = (Fi[:, None] * e).sum(0)
    for a in range(3):
        assert abs(m1[a] - rho * g[a]) <= _tol(Fi * e[:, a]) + 1e-30
    m2 = np.einsum("i,ia,ib->ab", Fi, e, e)
    want = rho * (np.outer(g, u) + np.outer(u, g))
    assert np.all(np.abs(m2 - want) <= _tol(Fi) + 1e-30)
    # equilibrium: mass rho, momentum rho u, second moment rho (uu + c_s^2 I)
    assert abs(feq.sum() - rho) <= _tol(feq)
    assert np.allclose((feq[:, None] * e).sum(0), rho * u, rtol=0, atol=1e-15)
    D = lat.dim(L)
    want2 = rho * (np.outer(u, u) + _cs2(L) * np.diag([1.0] * D + [0.0] * (3 - D)))
    assert np.allclose(np.einsum("i,ia,ib->ab", feq, e, e), want2, rtol=0, atol=1e-15)


@pytest.mark.parametrize("L", lat.ALL_LATTICES)
@pytest.mark.parametrize("coll", ["bgk", "smrt"])
@pytest.mark.parametrize("shift", [0.0, 1.0])
def test_init_recovers_rho_u(L, coll, shift):
    rng = np.random.default_rng(3)
    D = lat.dim(L)
    shape = (3, 4, 2 if D == 3 else 1)
    N = int(np.prod(shape))
    rho = 1.0 + 0.05 * rng.uniform(-1, 1, N)
    u = np.zeros((3, N))
    g = np.zeros((3, N))
    u[:D] = rng.uniform(-0.05, 0.05, (D, N))
    g[:D] = rng.uniform(-1e-3, 1e-3, (D, N))
    o = Oracle(L, coll, shape, tau=(0.7, 0.9 if coll == "smrt" else 0.7, 1.0), shift=shift)
    f = o.init(rho, u, g)
    r2, u2 = o.moments(f, g)
    assert np.max(np.abs(r2 - rho)) <= 8 * np.finfo(float).eps * 2
    assert np.max(np.abs(u2 - u)) <= 1e-15


# --- eq:bbd1 in tensor form ---------------------------------------------------------

def _sym_outer(*parts):
    """Sum over all distinct placements of index groups: sym product as written in the
    paper (e.g. 3 u a2 -> u_a a_bc + u_b a_ac + u_c a_ab)."""
    order = sum(p.ndim for p in parts)
    out = np.zeros((3,) * order)
    sizes = [p.ndim for p in parts]
    seen = set()
    for perm in itertools.permutations(range(order)):
        # assign positions to parts in order; identical placements counted once
        key = []
        pos = 0
        for s in sizes:
            key.append(tuple(sorted(perm[pos:pos + s])))
            pos += s
        key = tuple(key)
        if key in seen:
            continue
        seen.add(key)
        letters = "abcdefgh"[:order]
        subs = []
        for grp in key:
            subs.append("".join(letters[i] for i in grp))
        out += np.einsum(",".join(subs) + "->" + letters, *parts)
    return out


def _lattice_hermite_tensors(e, c2):
    I = np.eye(3)
    H2 = np.einsum("a,b->ab", e, e) - c2 * I
    H3 = np.einsum("a,b,c->abc", e, e, e) - c2 * (
        np.einsum("a,bc->abc", e, I) + np.einsum("b,ac->abc", e, I) + np.einsum("c,ab->abc", e, I))
    return H2, H3


def _component(T, m):
    idx = (0,) * m[0] + (1,) * m[1] + (2,) * m[2]
    return T[idx] if idx else T


@pytest.mark.parametrize("L", lat.ALL_LATTICES)
@pytest.mark.parametrize("seed", range(4))
def test_smrt_matches_bbd1_tensor_form(L, seed):
    rho0, u0, g = _setup(L, seed)
    D = lat.dim(L)
    o = Oracle(L, "smrt", (1, 1, 1), tau=(0.62, 0.83, 1.0))
    E = o.L["e"].astype(np.float64)
    # a pre-collision state: equilibrium plus a seeded non-equilibrium perturbation
    f = o.init_node(rho0, u0, g)
    rng = np.random.default_rng(100 + seed)
    f = f * (1 + 0.02 * rng.uniform(-1, 1, f.size))
    out = o.collide_node(f, g)
    # macroscopic (eq:half_F)
    rho = f.sum()
    j = (f[:, None] * E).sum(0)
    u = j / rho + g / 2
    F = rho * g
    w2, w3 = 1 / 0.62, 1 / 0.83
    c2 = _cs2(L)
    a2 = sum(fi * _lattice_hermite_tensors(e, c2)[0] for fi, e in zip(f, E))
    a3 = sum(fi * _lattice_hermite_tensors(e, c2)[1] for fi, e in zip(f, E))
    # non-equilibrium parts (a_0^(n) = rho u^n at theta = 1)
    a2_1 = a2 - rho * _sym_outer(u, u) / 2  # sym_outer(u,u) = 2 uu
    a3_1 = a3 - rho * np.einsum("a,b,c->abc", u, u, u)
    a1_p = F / 2
    aF2 = _sym_outer(F, u)             # 2 F u   (appendix a_F^(2))
    aF3 = _sym_outer(F, np.einsum("a,b->ab", u, u))  # 3 F u u  (appendix a_F^(3))
    a2_p = (1 - w2) * a2_1 + (1 - w2 / 2) * aF2
    a3_p = ((1 - w3) * a3_1 + (w3 - w2) * _sym_outer(u, a2_1)
            + (1 - w3 / 2) * aF3 + (w3 / 2 - w2 / 2) * _sym_outer(u, aF2))
    uu = np.einsum("a,b->ab", u, u)
    a4_p = (_sym_outer(u, a3_p) - _sym_outer(uu, a2_p)
            + _sym_outer(np.einsum("a,b,c->abc", u, u, u), a1_p))
    # post-collision lattice moments of the oracle's output
    M = o.L["H"]
    mom = M @ out
    ms = [tuple(m) for m in o.L["mi"]]
    wants = []
    for k, m in enumerate(ms):
        n = sum(m)
        if n == 0:
            want = rho
        elif n == 1:
            want = _component(rho * u + a1_p, m)
        elif n == 2:
            want = _component(rho * uu + a2_p, m)
        elif n == 3:
            want = _component(rho * np.einsum("a,b,c->abc", u, u, u) + a3_p, m)
        elif n == 4:
            want = _component(rho * np.einsum("a,b,c,d->abcd", u, u, u, u) + a4_p, m)
        else:
            want = 0.0
        wants.append(want)
    wants = _as_lattice_moments(o, wants)
    for k, m in enumerate(ms):
        assert abs(mom[k] - wants[k]) <= 1e-14 * max(1.0, abs(wants[k])), (m, mom[k], wants[k])
    assert D in (2, 3)


@pytest.mark.parametrize("L", lat.ALL_LATTICES)
def test_bgk_post_collision_moments(L):
    """Moments of eq:explict_eq: mass kept, momentum j + F, second Hermite moment
    (1 - omega)(a2 - rho uu) + rho uu + (1 - omega/2)(F u + u F)."""
    rho0, u0, g = _setup(L, 7)
    tau = 0.71
    o = Oracle(L, "bgk", (1, 1, 1), tau=(tau, tau, 1.0))
    E = o.L["e"].astype(np.float64)
    f = o.init_node(rho0, u0, g)
    f = f * (1 + 0.02 * np.random.default_rng(5).uniform(-1, 1, f.size))
    out = o.collide_node(f, g)
    rho = f.sum()
    j = (f[:, None] * E).sum(0)
    u = j / rho + g / 2
    F = rho * g
    om = 1 / tau
    assert abs(out.sum() - rho) < 1e-15
    assert np.allclose((out[:, None] * E).sum(0), j + F, rtol=0, atol=1e-16)
    D = lat.dim(L)
    I = np.diag([1.0] * D + [0.0] * (3 - D))
    a2 = np.einsum("i,ia,ib->ab", f, E, E) - _cs2(L) * rho * I
    a2o = np.einsum("i,ia,ib->ab", out, E, E) - _cs2(L) * rho * I
    uu = np.outer(u, u)
    want = (1 - om) * (a2 - rho * uu) + rho * uu + (1 - om / 2) * (np.outer(F, u) + np.outer(u, F))
    assert np.allclose(a2o, want, rtol=0, atol=2e-15)


@pytest.mark.parametrize("L", lat.ALL_LATTICES)
@pytest.mark.parametrize("coll", ["bgk", "smrt", "rmrt"])
@pytest.mark.parametrize("plain", [False, True])
def test_shifted_storage_is_a_change_of_variables(L, coll, plain):
    """Storing d_i = f_i - w_i s is a change of variables, not a different scheme: since
    sum_i w_i = 1 and sum_i w_i H_m(e_i) = 0 for m != 0, the deviations carry every
    moment but the mass, so the collision of d with shift s is the collision of f,
    less w_i s (to round-off), for any s, force and rates."""
    rng = np.random.default_rng(41)
    w = np.array([float(x) for x in lat.weights(L)])
    D = lat.dim(L)
    tau = (0.63, 0.63 if coll == "bgk" else 0.91, 1.0)
    for s in (1.0, 0.97, 2.5):
        f = w * (s + 0.05 * rng.uniform(-1, 1, w.size))
        g = np.zeros(3)
        g[:D] = rng.uniform(-1e-3, 1e-3, D)
        o0 = Oracle(L, coll, (1, 1, 1), tau=tau, plain=plain)
        os_ = Oracle(L, coll, (1, 1, 1), tau=tau, shift=s, plain=plain)
        want = o0.collide_node(f, g) - w * s
        got = os_.collide_node(f - w * s, g)
        assert np.max(np.abs(got - want)) <= 1e-14 * s, (s, np.max(np.abs(got - want)))


@pytest.mark.parametrize("L", lat.ALL_LATTICES)
def test_smrt_equal_rates_one_is_half_force(L):
    """SMRT with omega_2 = omega_3 = 1: every non-equilibrium moment is replaced by half
    the raw force moment, a*^(n) = rho u^n + a_F^(n)/2 for n = 1..4 (appendix, theta = 1)."""
    rho, u, g = _setup(L, 11)
    o = Oracle(L, "smrt", (1, 1, 1), tau=(1.0, 1.0, 1.0))
    f = o.init_node(rho, u, g)
    f = f * (1 + 0.03 * np.random.default_rng(9).uniform(-1, 1, f.size))
    out = o.collide_node(f, g)
    E = o.L["e"].astype(np.float64)
    r = f.sum()
    uu = (f[:, None] * E).sum(0) / r + g / 2
    F = r * g
    mom = o.L["H"] @ out
    wants = []
    for k, m in enumerate(o.L["mi"]):
        m = tuple(m)
        n = sum(m)
        if n == 0:
            wants.append(r)
            continue
        if n > 4:
            wants.append(0.0)
            continue
        up = np.prod([uu[a] ** m[a] for a in range(3)])
        aF = 0.0
        for a in range(3):
            if m[a]:
                r_ = list(m)
                r_[a] -= 1
                aF += m[a] * np.prod([uu[b] ** r_[b] for b in range(3)]) * F[a]
        wants.append(r * up + aF / 2)
    wants = _as_lattice_moments(o, wants)
    for k, m in enumerate(o.L["mi"]):
        if 0 < sum(m) <= 4:
            assert math.isclose(mom[k], wants[k], rel_tol=0, abs_tol=1e-15), (m, mom[k], wants[k])


# Number of independent Hermite moments of order 3 each velocity set resolves: D2Q9 has
# xxy, xyy; D3Q19 the six with one repeated index; D3Q27 those and xyz.
# D3Q39 carries all ten.
ORDER3 = {"D2Q9": 2, "D3Q19": 6, "D3Q27": 7, "D3Q39": 10}


@pytest.mark.parametrize("L", lat.ALL_LATTICES)
@pytest.mark.parametrize("coll,tau2,tau3", [("bgk", 0.8, 1.0), ("smrt", 0.8, 1.0),
                                            ("smrt", 0.62, 0.7), ("smrt", 1.3, 2.5)])
def test_linearised_collision_spectrum(L, coll, tau2, tau3):
    """About rest and unforced, the collision relaxes each Hermite order n by 1 - 1/tau_n
    (eq:domg with a_F = 0): eigenvalue 1 for mass and momentum; for SMRT 1 - 1/tau2 on
    the D(D+1)/2 second-order moments, 1 - 1/tau3 on the third-order ones and 0 above
    (order 4 trimmed, higher orders dropped); for BGK 1 - 1/tau on all non-conserved
    ones.  Central differences of the oracle's collision are exact here up to rounding
    because the linearisation is taken at a point where the map is a polynomial."""
    o = Oracle(L, coll, (1, 1, 1), tau=(tau2, tau3, 1.0))
    Q, D = o.Q, o.D
    f0 = o.init_node(1.0, [0, 0, 0], [0, 0, 0])
    h = 1e-5
    J = np.empty((Q, Q))
    for q in range(Q):
        d = np.zeros(Q)
        d[q] = h
        J[:, q] = (o.collide_node(f0 + d, [0, 0, 0]) - o.collide_node(f0 - d, [0, 0, 0])) / (2 * h)
    lam = np.sort(np.linalg.eigvals(J).real)
    if coll == "bgk":
        want = [1.0] * (1 + D) + [1 - 1 / tau2] * (Q - 1 - D)
    else:
        n2 = D * (D + 1) // 2
        n3 = ORDER3[L]
        want = ([1.0] * (1 + D) + [1 - 1 / tau2] * n2 + [1 - 1 / tau3] * n3
                + [0.0] * (Q - 1 - D - n2 - n3))
    assert np.max(np.abs(lam - np.sort(want))) < 1e-8, (lam, sorted(want))


def _collision_jacobian(o):
    """Central differences of the collision about rest, unforced (exact up to rounding:
    the map is a polynomial there)."""
    Q = o.Q
    f0 = o.init_node(1.0, [0, 0, 0], [0, 0, 0])
    h = 1e-5
    J = np.empty((Q, Q))
    for q in range(Q):
        d = np.zeros(Q)
        d[q] = h
        J[:, q] = (o.collide_node(f0 + d, [0, 0, 0]) - o.collide_node(f0 - d, [0, 0, 0])) / (2 * h)
    return J


@pytest.mark.parametrize("L", lat.ALL_LATTICES)
@pytest.mark.parametrize("tau_b", [0.55, 0.9, 1.7])
def test_bulk_rate_collision_spectrum(L, tau_b):
    """eq:domg per irreducible component at order 2: with its own rate for the trace,
    exactly one second-order eigenvalue moves to 1 - 1/tau_bulk, the D(D+1)/2 - 1
    traceless ones keep 1 - 1/tau2."""
    tau2, tau3 = 0.8, 1.0
    o = Oracle(L, "smrt", (1, 1, 1), tau=(tau2, tau3, 1.0), tau_bulk=tau_b)
    Q, D = o.Q, o.D
    lam = np.sort(np.linalg.eigvals(_collision_jacobian(o)).real)
    n2 = D * (D + 1) // 2
    n3 = ORDER3[L]
    want = ([1.0] * (1 + D) + [1 - 1 / tau_b] + [1 - 1 / tau2] * (n2 - 1)
            + [1 - 1 / tau3] * n3 + [0.0] * (Q - 1 - D - n2 - n3))
    assert np.max(np.abs(lam - np.sort(want))) < 1e-8, (lam, sorted(want))


def _hermite3(E):
    """The lattice's third-order Hermite polynomials at c_s^2 = 1/3, written out:
    H_abb(e) = e_a (e_b^2 - 1/3) for a != b, H_xyz(e) = e_x e_y e_z."""
    e = np.asarray(E, float)
    H = {}
    for a in range(3):
        for b in range(3):
            if a != b:
                H[(a, b)] = e[:, a] * (e[:, b] ** 2 - CS2)
    H["xyz"] = e[:, 0] * e[:, 1] * e[:, 2]
    return H


@pytest.mark.parametrize("L", ["D3Q19", "D3Q27"])
@pytest.mark.parametrize("tau_31", [0.6, 1.6])
def test_third_order_trace_rate(L, tau_31):
    """eq:domg at order 3 with its own rate for the trace S^(3,1): about rest, for any
    perturbation, the collision scales each axis's trace pair H_abb + H_acc by
    1 - 1/tau_31 and the differences H_abb - H_acc and H_xyz by 1 - 1/tau3 (moments taken
    with the Hermite polynomials written out, not the oracle's tables); the spectrum has
    exactly three eigenvalues at 1 - 1/tau_31."""
    tau2, tau3 = 0.8, 1.0
    o = Oracle(L, "smrt", (1, 1, 1), tau=(tau2, tau3, 1.0), tau_31=tau_31)
    J = _collision_jacobian(o)
    H = _hermite3(lat.velocities(L))
    q3, q31 = 1 - 1 / tau3, 1 - 1 / tau_31
    rng = np.random.default_rng(4)
    for _ in range(4):
        d = rng.standard_normal(o.Q)
        d2 = J @ d
        for a in range(3):
            b, c = (a + 1) % 3, (a + 2) % 3
            s0 = H[(a, b)] @ d + H[(a, c)] @ d
            s1 = H[(a, b)] @ d2 + H[(a, c)] @ d2
            t0 = H[(a, b)] @ d - H[(a, c)] @ d
            t1 = H[(a, b)] @ d2 - H[(a, c)] @ d2
            assert abs(s1 - q31 * s0) < 1e-8 and abs(t1 - q3 * t0) < 1e-8, (a, s0, s1, t0, t1)
        if L == "D3Q27":
            assert abs(H["xyz"] @ d2 - q3 * (H["xyz"] @ d)) < 1e-8
    n2 = 6
    n3 = ORDER3[L]
    lam = np.sort(np.linalg.eigvals(J).real)
    want = ([1.0] * 4 + [1 - 1 / tau2] * n2 + [q31] * 3 + [q3] * (n3 - 3)
            + [0.0] * (o.Q - 4 - n2 - n3))
    assert np.max(np.abs(lam - np.sort(want))) < 1e-8, (lam, sorted(want))


def _central_hermite(E, f, u, m):
    """sum_i f_i H_m(e_i - u) with the one-dimensional Hermite polynomials at c_s^2 = 1/3
    written out (1, x, x^2 - 1/3): the Hermite central moment of f about u."""
    he = (lambda x: np.ones_like(x), lambda x: x, lambda x: x * x - CS2)
    h = np.ones(len(E))
    for a in range(3):
        h = h * he[m[a]](E[:, a] - u[a])
    return h @ f


@pytest.mark.parametrize("max_order", [4, 6])
@pytest.mark.parametrize("seed", range(3))
def test_high_orders_on_d3q27(max_order, seed):
    """D3Q27 carries Hermite orders up to 6.  After an unforced collision (u = j/rho), the
    central moments about u of orders 2 and 3 are the relaxed ones (1 - 1/tau_n times the
    pre-collision value) and order 4 is trimmed to zero.  With max_order 4 the raw moments
    of orders 5 and 6 are zero (the reconstruction sums to order 4) while their central
    moments are not; with max_order 6 the central moments of orders 5 and 6 are zero too
    (trimmed like order 4, Galilean invariant).  All moments are taken with the Hermite
    polynomials written out, not the oracle's tables."""
    tau2, tau3 = 0.8, 0.9
    o = Oracle("D3Q27", "smrt", (1, 1, 1), tau=(tau2, tau3, 1.0), max_order=max_order)
    E = np.array(lat.velocities("D3Q27"), float)
    rng = np.random.default_rng(seed)
    u0 = rng.uniform(-0.08, 0.08, 3)
    f = o.init_node(1.02, u0, [0, 0, 0]) + 1e-3 * rng.standard_normal(27)
    rho = f.sum()
    u = (E.T @ f) / rho
    fs = o.collide_node(f, [0, 0, 0])
    assert abs(fs.sum() - rho) < 1e-14 and np.max(np.abs(E.T @ fs - rho * u)) < 1e-15
    raw = {}
    for m in itertools.product(range(3), repeat=3):
        n = sum(m)
        c_post = _central_hermite(E, fs, u, m)
        if n in (2, 3):
            q = 1 - 1 / (tau2 if n == 2 else tau3)
            assert abs(c_post - q * _central_hermite(E, f, u, m)) < 1e-14, m
        elif n == 4 or (n > 4 and max_order == 6):
            assert abs(c_post) < 1e-15, (m, c_post)
        elif n > 4:
            raw[m] = (_central_hermite(E, fs, np.zeros(3), m), c_post)
    if max_order == 4:
        assert all(abs(r) < 1e-15 for r, _ in raw.values()), raw
        assert max(abs(c) for _, c in raw.values()) > 1e-8, raw


@pytest.mark.parametrize("L", lat.ALL_LATTICES)
@pytest.mark.parametrize("tau_b", [0.0, 0.9, 1.7])
def test_bulk_rate_sound_attenuation(L, tau_b):
    """Hydrodynamic limit of the linearised step at small wavenumber k (along x): the
    sound pair decays as exp(-Gamma k^2 t) with Gamma = ((2 - 2/D) nu + zeta)/2, the
    shear modes as exp(-nu k^2 t), with nu = c_s^2 (tau2 - 1/2) and the bulk viscosity
    zeta = (2/D) c_s^2 (tau_bulk - 1/2) (zeta = 2 nu / D with one rate, the textbook
    value of the lattice BGK).  The step about rest is diag(exp(-i k e_ix)) J (pull
    streaming after the collision J); the O(k^2) relative error must shrink ~4x when k
    halves."""
    tau2 = 0.8
    o = Oracle(L, "smrt", (1, 1, 1), tau=(tau2, 1.0, 1.0), tau_bulk=tau_b)
    D = o.D
    J = _collision_jacobian(o)
    ex = np.array(lat.velocities(L))[:, 0]
    c2 = _cs2(L)
    cs = math.sqrt(c2)
    nu = c2 * (tau2 - 0.5)
    zeta = (2.0 / D) * c2 * ((tau_b or tau2) - 0.5)
    gam = 0.5 * ((2 - 2.0 / D) * nu + zeta)
    errs = []
    for k in (2 * math.pi / 64, 2 * math.pi / 128):
        ev = np.linalg.eigvals(np.diag(np.exp(-1j * k * ex)) @ J)
        sound = ev[(np.abs(np.abs(np.angle(ev)) - cs * k) < 0.2 * cs * k) & (np.abs(ev) > 0.5)]
        shear = ev[(np.abs(np.angle(ev)) < 1e-6) & (np.abs(ev) > 0.5) & (np.abs(ev) < 1 - 1e-12)]
        assert sound.size == 2 and shear.size == D - 1, (sound, shear)
        g_meas = -np.log(np.abs(sound)) / k ** 2
        n_meas = -np.log(np.abs(shear)) / k ** 2
        assert np.max(np.abs(n_meas / nu - 1)) < 5e-4
        errs.append(np.max(np.abs(g_meas / gam - 1)))
    # second-order convergence to the hydrodynamic rate; D3Q39's O(k^2) coefficient is
    # larger (measured 7.4e-4 at tau_bulk 1.7, k = 2 pi / 128)
    bound = 2e-4 if L in lat.LATTICES else 1e-3
    assert errs[1] < bound and errs[1] < 0.3 * errs[0], errs


@pytest.mark.parametrize("L", lat.LATTICES)
@pytest.mark.parametrize("coll", ["bgk", "smrt"])
def test_staggered_momentum_mode_never_decays(L, coll):
    """u_x = eps (-1)^x at rest density is an equilibrium, so collision keeps it; streaming
    carries every population with e_x = +-1 to the other sublattice and keeps the e_x = 0
    ones, whose equilibrium is even in u_x, so the state becomes the equilibrium of
    -u_x: the checkerboard flips sign every step for ever, whatever the relaxation
    times (the eigenvalue -1 of the step at wavenumber (pi, 0, 0))."""
    shape = (4, 3, 1) if lat.dim(L) == 2 else (4, 3, 2)
    o = Oracle(L, coll, shape, tau=(0.6, 0.9, 1.0))
    x = np.arange(o.N) % shape[0]
    eps = 0.01
    u = np.zeros((3, o.N))
    u[0] = eps * (-1.0) ** x
    f = o.init(1.0, u, None)
    for t in range(1, 4):
        f = o.step(f, None)
        rho, ut = o.moments(f, None)
        assert np.max(np.abs(rho - 1.0)) < 1e-14
        assert np.max(np.abs(ut[0] - eps * (-1.0) ** (x + t))) < 1e-15
        assert np.max(np.abs(ut[1:])) < 1e-15


@pytest.mark.parametrize("L", lat.ALL_LATTICES)
@pytest.mark.parametrize("seed", range(3))
def test_third_order_force_content(L, seed):
    """force_order 3 (eq:Frc at theta = 1, d_F^(3) = 3 g d^(2)): against force_order 1 the
    post-collision state changes only in the raw third-order Hermite moments on the
    lattice's index set, by (1 - omega_3/2) sum_a m_a g_a d_{m-e_a} with d = (1 -
    omega_2/2) D, D the central non-equilibrium second moment of the pre-collision state
    -- here recomputed from the populations with numpy, not through the oracle's tables
    (the order-4 raw moments move too, by the shift of the changed central moments)."""
    rho, u, g = _setup(L, seed)
    tau2, tau3 = 0.7, 0.9
    o1 = Oracle(L, "smrt", (1, 1, 1), tau=(tau2, tau3, 1.0))
    o3 = Oracle(L, "smrt", (1, 1, 1), tau=(tau2, tau3, 1.0), force_order=3)
    D = lat.dim(L)
    Lt = lat.tables(L, np.float64)
    e = np.asarray(Lt["e"], np.float64).reshape(o1.Q, -1)
    e3 = np.zeros((o1.Q, 3))
    e3[:, :D] = e[:, :D]
    rng = np.random.default_rng(seed + 40)
    f = o1.init_node(rho, u, g) * (1 + 0.05 * rng.uniform(-1, 1, o1.Q))
    diff = o3.collide_node(f, g) - o1.collide_node(f, g)
    # pre-collision macroscopic state (eq:half_F) and central non-equilibrium second moment
    r = f.sum()
    j = e3.T @ f
    uu = j / r + g / 2
    F = r * g
    c2 = _cs2(L)
    A2 = np.einsum("i,ia,ib->ab", f, e3, e3) - r * np.eye(3) * c2 * (np.arange(3) < D)[:, None]
    N2 = A2 - r * np.outer(uu, uu)
    N1 = -F / 2
    Dc = N2 - np.outer(uu, N1) - np.outer(N1, uu)
    d2 = (1 - 0.5 / tau2) * Dc
    mi = np.asarray(Lt["mi"]).reshape(-1, 3)
    biggest = 0.0
    for m in mi[mi.sum(1) == 3]:
        want = 0.0
        for a in range(3):
            if m[a]:
                b = m.copy()
                b[a] -= 1
                pair = [c for c in range(3) for _ in range(b[c])]
                want += m[a] * g[a] * d2[pair[0], pair[1]]
        want *= (1 - 0.5 / tau3)
        # raw third-order Hermite moment of the change: sum_i diff_i H_m(e_i)
        H = np.ones(o1.Q)
        for c in range(3):
            x = e3[:, c]
            H *= {0: 1.0, 1: x, 2: x * x - c2, 3: x ** 3 - 3 * c2 * x}[int(m[c])]
        got = float(diff @ H)
        assert abs(got - want) <= 1e-13 + 1e-9 * abs(want), (m, got, want)
        biggest = max(biggest, abs(want))
    assert biggest > 1e-7  # the term is exercised
    # mass, momentum and the second-order moments are untouched
    assert abs(diff.sum()) < 1e-16
    assert np.max(np.abs(e3.T @ diff)) < 1e-16
    # (D3Q39 rebuilds the whole state from its moments, so both outputs carry their own
    # rounding: bound by the rounding of the second-moment sums instead)
    tol2 = 1e-16 if o1.L["NM"] == o1.Q else 32 * np.finfo(float).eps * float(
        np.max(np.einsum("i,ia,ib->ab", np.abs(f), np.abs(e3), np.abs(e3))))
    assert np.max(np.abs(np.einsum("i,ia,ib->ab", diff, e3, e3))) < tol2


@pytest.mark.parametrize("L", lat.ALL_LATTICES)
@pytest.mark.parametrize("seed", range(3))
def test_raw_moment_mrt_against_central(L, seed):
    """The appendix's raw-moment MRT (RMRT) against the central-moment SMRT on one node:
    post-collision moments of orders 0..2 agree for any rates (at order 2 the central
    shift of the force, (1 + q_2)/2, equals the raw force factor 1 - omega_2/2); with every
    tau-hat = 1 the two collisions are the same map; with tau3 != 1 their third-order
    moments differ (the frames of relaxation differ by u-dependent terms)."""
    rho, u, g = _setup(L, seed)
    rng = np.random.default_rng(seed + 70)
    D = lat.dim(L)
    Lt = lat.tables(L, np.float64)
    e = np.zeros((len(Lt["w"]), 3))
    e[:, :D] = np.asarray(Lt["e"], np.float64).reshape(len(Lt["w"]), -1)[:, :D]

    def moments(f):
        return (f.sum(), e.T @ f, np.einsum("i,ia,ib->ab", f, e, e))

    for tau, third_differs in (((0.7, 0.9, 1.0), True), ((1.0, 1.0, 1.0), False)):
        cm = Oracle(L, "smrt", (1, 1, 1), tau=tau)
        rm = Oracle(L, "rmrt", (1, 1, 1), tau=tau)
        f = cm.init_node(rho, u, g) * (1 + 0.05 * rng.uniform(-1, 1, cm.Q))
        a, b = cm.collide_node(f, g), rm.collide_node(f, g)
        for x, y in zip(moments(a), moments(b)):
            assert np.max(np.abs(np.asarray(x) - np.asarray(y))) < 1e-15
        if third_differs:
            assert np.max(np.abs(a - b)) > 1e-9
        else:
            assert np.max(np.abs(a - b)) < 1e-15
