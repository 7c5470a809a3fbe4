"""The explicit collisions against the implicit (trapezoidal) rule they come from.

Sec. II.B integrates the discrete-velocity equation with force along a characteristic by
the trapezoid rule (eq:implicityeq) and removes the implicitness with the change of
variable f-bar = f - Omega/2 - F/2 (eq:newf); the explicit update is then f-bar* = f-bar +
Omega + F (eq:evolution), with Omega and F evaluated at the distribution f itself.  From
those two relations alone, f = (f-bar + f-bar*)/2: the distribution at the node is the mean
of the stored populations before and after the collision.

These tests take the oracle's collision as a black box, form f from its input and
output, and check the implicit rule in the continuous-time rates tau = tau-hat - 1/2
(Sec. II.B), with every moment recomputed from the populations by numpy:

* BGK (eq:collision_BGK with the second-order force below eq:Fr): f-bar* - f-bar =
  -(f - f_eq(rho, u))/tau + F(rho, u, g), population by population.
* SMRT (eq:domg, eq:RHS): in Hermite central moments about the velocity u of f, order n
  changes by -d^(n)(f)/tau_n + d_F^(n); with the force in the first central moment only
  d_F^(n) = 0 for n >= 2, with the third-order content d_F^(3) = 3 g d^(2) (eq:Frc at
  theta = 1), d^(2) the central second moment of f itself, and with the fourth-order
  content also d_F^(4) = 4 g d^(3).  Separate rates for the trace at order 2 and for the
  trace pairs at order 3 change the rate of those parts only.  Order 4 is trimmed
  (tau-hat_4 = 1, i.e. tau_4 = 1/2).
* RMRT (the appendix, eq:RHS_a): the same in raw Hermite moments about rest, with the raw
  force moments a_F = sum_a m_a u^{m-e_a} F_a.

On the high-order lattice D3Q39 (c_s^2 = 2/3, quadrature exact to degree 7) the moments of
orders 0 to 3 are checked; its fourth-order moments are not all independent on the 39
velocities, so the rule at order 4 is not a statement about them.

Nowhere is the explicit factor 1 - omega/2 or the relation d = (1 - omega/2) d-bar typed
in: they follow from the collision's own output.  A dropped term, a wrong rate or
factor, or a sign error in any of the collisions fails these tests.  They run on both
oracle builds (the operation-order twin and the plain one).
"""
import itertools

import numpy as np
import pytest

from oracle import Oracle
from oracle import lattice as lat

BUILDS = [False, True]  # plain?


def _cs2(L):
    return float(lat.cs2(L))


def _velocities(L):
    D = lat.dim(L)
    E = np.zeros((len(lat.velocities(L)), 3))
    E[:, :D] = np.asarray(lat.velocities(L), float)[:, :D]
    return E


def _weights(L):
    return np.asarray(lat.tables(L, np.float64)["w"], float)


def _hermite(x, n, c2):
    """One-dimensional lattice Hermite polynomial of degree n at c_s^2 = c2."""
    return {0: np.ones_like(x), 1: x, 2: x * x - c2, 3: x ** 3 - 3 * c2 * x,
            4: x ** 4 - 6 * c2 * x * x + 3 * c2 * c2}[n]


def _moment(E, f, m, about, c2):
    """sum_i f_i prod_a H_{m_a}(e_ia - about_a)."""
    h = np.ones(len(E))
    for a in range(3):
        h = h * _hermite(E[:, a] - about[a], m[a], c2)
    return float(h @ f)


def _top_order(L):
    """Highest Hermite order whose moments the lattice resolves exactly."""
    return 3 if L in lat.HIGH_ORDER else 4


def _index_set(L):
    return [tuple(int(v) for v in m) for m in np.asarray(lat.tables(L, np.float64)["mi"]).reshape(-1, 3)]


def _state(L, seed, amp=0.1):
    rng = np.random.default_rng(seed)
    D = lat.dim(L)
    rho = 1.0 + 0.05 * rng.uniform(-1, 1)
    u = np.zeros(3)
    g = np.zeros(3)
    u[:D] = rng.uniform(-0.1, 0.1, D)
    g[:D] = rng.uniform(-1e-2, 1e-2, D)
    return rho, u, g, rng


def _mean_state(o, fbar, g):
    """f = (f-bar + f-bar*)/2 and its density and velocity (eq:newf, eq:evolution)."""
    fstar = o.collide_node(fbar, g)
    f = 0.5 * (fbar + fstar)
    E = _velocities(o.lattice)
    rho = f.sum()
    u = (E.T @ f) / rho
    return fstar, f, rho, u


def _tol(*arrays):
    return 64 * np.finfo(float).eps * max(np.max(np.abs(a)) for a in arrays)


@pytest.mark.parametrize("plain", BUILDS)
@pytest.mark.parametrize("L", lat.ALL_LATTICES)
@pytest.mark.parametrize("seed", range(3))
def test_bgk_is_the_trapezoid_rule(L, seed, plain):
    rho0, u0, g, rng = _state(L, seed)
    tau_hat = 0.63
    o = Oracle(L, "bgk", (1, 1, 1), tau=(tau_hat, tau_hat, 1.0), plain=plain)
    fbar = o.init_node(rho0, u0, g) * (1 + 0.1 * rng.uniform(-1, 1, o.Q))
    fstar, f, rho, u = _mean_state(o, fbar, g)
    E, w = _velocities(L), _weights(L)
    eu = E @ u
    c2 = _cs2(L)
    feq = w * rho * (1 + eu / c2 + (eu ** 2 - c2 * (u @ u)) / (2 * c2 ** 2))
    F = rho * g
    Fi = w * (((E - u) @ F) / c2 + (E @ F) * eu / c2 ** 2)
    tau = tau_hat - 0.5
    rhs = -(f - feq) / tau + Fi
    assert np.max(np.abs((fstar - fbar) - rhs)) <= _tol(fbar, fstar), (fstar - fbar, rhs)


SMRT_CASES = [
    # (force_order, tau2, tau3, tau_bulk, tau_31)
    (1, 0.7, 0.9, 0.0, 0.0),
    (1, 0.56, 1.0, 0.0, 0.0),
    (3, 0.7, 0.9, 0.0, 0.0),
    (3, 1.3, 0.6, 0.0, 0.0),
    (1, 0.7, 0.9, 1.4, 0.0),
    (1, 0.7, 0.9, 0.0, 1.6),
    (3, 0.7, 0.9, 1.4, 0.0),
    (4, 0.7, 0.9, 0.0, 0.0),
    (4, 1.3, 0.6, 0.0, 0.0),
    (4, 0.6, 1.1, 1.7, 0.0),
]


def _force_content(m, g, cen):
    """d_F^(n) of eq:Frc at theta = 1 for multi-index m: sum_a m_a g_a d_{m - e_a}, with d
    the central moment of f itself (its non-equilibrium part: the equilibrium's central
    moments vanish)."""
    dF = 0.0
    for a in range(3):
        if m[a]:
            ml = list(m)
            ml[a] -= 1
            dF += m[a] * g[a] * cen[tuple(ml)][2]
    return dF


@pytest.mark.parametrize("plain", BUILDS)
@pytest.mark.parametrize("L", lat.ALL_LATTICES)
@pytest.mark.parametrize("case", SMRT_CASES)
def test_smrt_is_the_trapezoid_rule(L, case, plain):
    fo, tau2h, tau3h, taubh, tau31h = case
    if tau31h and L == "D2Q9":
        pytest.skip("D2Q9 carries no traceless third-order part")
    if tau31h and L in lat.HIGH_ORDER:
        pytest.skip("tau_31 is defined on the lattices that lack D_aaa")
    if fo == 4 and L in lat.HIGH_ORDER:
        pytest.skip("the fourth-order force content needs independent fourth-order moments")
    rho0, u0, g, rng = _state(L, 7 + fo)
    o = Oracle(L, "smrt", (1, 1, 1), tau=(tau2h, tau3h, 1.0), force_order=fo, tau_bulk=taubh,
               tau_31=tau31h, plain=plain)
    fbar = o.init_node(rho0, u0, g) * (1 + 0.1 * rng.uniform(-1, 1, o.Q))
    fstar, f, rho, u = _mean_state(o, fbar, g)
    E = _velocities(L)
    D = lat.dim(L)
    I = _index_set(L)
    tau = {2: tau2h - 0.5, 3: tau3h - 0.5, 4: 0.5}
    c2 = _cs2(L)
    cen = {m: (_moment(E, fbar, m, u, c2), _moment(E, fstar, m, u, c2), _moment(E, f, m, u, c2))
           for m in I}
    tol = _tol(fbar, fstar)
    # orders 0 and 1: mass kept, momentum gains F; the first central moment of f is 0
    F = rho * g
    assert abs(fstar.sum() - fbar.sum()) <= tol
    assert np.max(np.abs(E.T @ fstar - E.T @ fbar - F)) <= tol
    assert np.max(np.abs(E.T @ f - rho * u)) <= tol
    # order 2: trace (bulk) and traceless (shear) parts
    diag = [m for m in I if sum(m) == 2 and max(m) == 2]
    trace = sum(cen[m][2] for m in diag)
    for m in I:
        n = sum(m)
        if n < 2 or n > _top_order(L):
            continue
        before, after, mean = cen[m]
        if n == 2:
            rhs = -mean / tau[2]
            if taubh and m in diag:
                rhs = -(mean - trace / D) / tau[2] - (trace / D) / (taubh - 0.5)
        elif n == 3:
            rhs = -mean / tau[3]
            if tau31h:
                # the trace pair of this index: a + 2b and a + 2c carry sum_b D_abb
                a = m.index(1) if 1 in m else None
                if a is not None and 2 in m:
                    b = m.index(2)
                    c = 3 - a - b
                    mp = [0, 0, 0]
                    mp[a], mp[c] = 1, 2
                    s = mean + cen[tuple(mp)][2]
                    rhs = -(mean - s / 2) / tau[3] - (s / 2) / (tau31h - 0.5)
            if fo >= 3:
                rhs += _force_content(m, g, cen)
        else:
            rhs = -mean / tau[4]
            if fo == 4:
                rhs += _force_content(m, g, cen)
        assert abs((after - before) - rhs) <= tol, (m, after - before, rhs)


@pytest.mark.parametrize("plain", BUILDS)
@pytest.mark.parametrize("L", lat.ALL_LATTICES)
@pytest.mark.parametrize("taus", [(0.7, 0.9), (0.58, 1.3)])
def test_rmrt_is_the_trapezoid_rule(L, taus, plain):
    tau2h, tau3h = taus
    rho0, u0, g, rng = _state(L, 11)
    o = Oracle(L, "rmrt", (1, 1, 1), tau=(tau2h, tau3h, 1.0), plain=plain)
    fbar = o.init_node(rho0, u0, g) * (1 + 0.1 * rng.uniform(-1, 1, o.Q))
    fstar, f, rho, u = _mean_state(o, fbar, g)
    E = _velocities(L)
    F = rho * g
    zero = np.zeros(3)
    tau = {2: tau2h - 0.5, 3: tau3h - 0.5, 4: 0.5}
    tol = _tol(fbar, fstar)
    c2 = _cs2(L)
    for m in _index_set(L):
        n = sum(m)
        if n < 2 or n > _top_order(L):
            continue
        um = np.prod([u[a] ** m[a] for a in range(3)])
        aF = 0.0
        for a in range(3):
            if m[a]:
                ml = list(m)
                ml[a] -= 1
                aF += m[a] * np.prod([u[b] ** ml[b] for b in range(3)]) * F[a]
        neq = _moment(E, f, m, zero, c2) - rho * um
        rhs = -neq / tau[n] + aF
        got = _moment(E, fstar, m, zero, c2) - _moment(E, fbar, m, zero, c2)
        assert abs(got - rhs) <= tol, (m, got, rhs)


@pytest.mark.parametrize("L", lat.ALL_LATTICES)
@pytest.mark.parametrize("coll", ["bgk", "smrt", "rmrt"])
def test_plain_and_twin_builds_agree_to_rounding(L, coll):
    """The operation-order twin and the plain build compute the same step: on a walled
    lattice (periodic for D3Q39) with a random state and force, after 1 and 40 steps they
    differ by rounding only (bound 1e-14 max |f|; measured about 4e-16)."""
    shape = (12, 10, 1) if L == "D2Q9" else (8, 6, 5)
    kw = dict(walls=(0, 0, 0) if L in lat.HIGH_ORDER else (0, 1, 0), tau=(0.7, 0.9, 1.0))
    a = Oracle(L, coll, shape, **kw)
    b = Oracle(L, coll, shape, plain=True, **kw)
    rng = np.random.default_rng(3)
    f = a.init(1.0, None, None) * (1 + 0.05 * rng.uniform(-1, 1, (a.Q, a.N)))
    g = np.array([1e-4, -3e-5, 2e-5])
    for n in (1, 40):
        fa, fb = a.run(f, g, n), b.run(f, g, n)
        assert np.max(np.abs(fa - fb)) <= 1e-14 * np.max(np.abs(fb)), n
        if coll == "bgk":
            assert np.array_equal(fa, fb)  # BGK has no moment transforms to reorder
