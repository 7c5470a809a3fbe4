"""Closed-form and brute-force steady states used to pin the oracle (test infrastructure).

None of this calls the oracle's step; the pins compare the oracle against these.

Setting: D2Q9, flow invariant along x, acceleration g(y) along x, density 1 and
u_y = 0 throughout (these hold exactly for such flows: every even-in-e_x source
of the step has zero mass inside each e_y group, so the y-momentum and density
never change).  What remains is linear and lives in the odd-in-e_x sector:
per row y the three differences h_c(y) = f(1, c) - f(-1, c), c in {-1, 0, 1}, or
equivalently the moments
    X = sum f e_x = h_-1 + h_0 + h_1                 (x momentum j_x)
    Y = sum f e_x e_y = h_1 - h_-1                   (shear stress moment)
    Z = sum f e_x (3 e_y^2 - 1) = 2 h_1 + 2 h_-1 - h_0
(Z/3 is the third-order Hermite moment H_xyy in lattice units).

Collision in this sector (paper Sec. II.B and II.C):
  * BGK with Guo force (eq:explict_eq, second-order force): the odd part of the
    equilibrium is 3 w e_x u_x and of the force 3 w e_x g, so per group
    h* = h - omega (h - 6 w_c u_x) + (1 - omega/2) 6 w_c g, u_x = X + g/2,
    with w_0 = 1/9 and w_{+-1} = 1/36.
  * SMRT: the first moment gains F (post-collision a^(1) = rho u + F/2 with
    rho u = j + F/2), the second- and third-order central moments (here equal to
    Y and Z/3 because u_y = 0 and the yy moment vanishes) relax with q_n = 1 - omega_n:
    X' = X + g, Y' = q2 Y, Z' = q3 Z.
Streaming moves group c by c rows; at a halfway bounce-back wall the leaving
population returns in the opposite direction, so h_c at the boundary row takes
-h*_(-c) of the same row.
"""
from __future__ import annotations

import math

import numpy as np


def nu_of(tau2: float) -> float:
    """Kinematic viscosity c_s^2 (tau-hat - 1/2) in lattice units."""
    return (tau2 - 0.5) / 3.0


# ---- closed forms ---------------------------------------------------------------------

def poiseuille_profile(n: int, g: float, tau2: float, tau3: float) -> np.ndarray:
    """Exact discrete steady u_x on rows y = 1..n between halfway walls.

    Parabola with curvature -g/nu plus a constant slip u_s = g (16 L - 3) / (8 (tau2 - 1/2)),
    L = (tau2 - 1/2)(tau3 - 1/2) (BGK: tau3 = tau2).
    """
    y = np.arange(1, n + 1, dtype=np.float64)
    nu = nu_of(tau2)
    lam = (tau2 - 0.5) * (tau3 - 0.5)
    us = g * (16 * lam - 3) / (8 * (tau2 - 0.5))
    return g / (2 * nu) * ((n / 2) ** 2 - (y - (n + 1) / 2) ** 2) + us


def kolmogorov_amplitude(G: float, k: float, tau2: float, tau3: float) -> float:
    """Exact discrete steady amplitude U of u_x = U sin(k y) for g_x = G sin(k y), SMRT.

    With c = cos k, s = sin k, q_n = 1 - 1/tau_n:
      R = c - s^2 q2 / (1 - c q2),  X = [R G + (2G/omega3)(1 - R q3)] / (1 - R),  U = X + G/2.
    """
    q2 = 1 - 1 / tau2
    q3 = 1 - 1 / tau3
    w3 = 1 / tau3
    c = math.cos(k)
    s = math.sin(k)
    one_m_c = 2 * math.sin(k / 2) ** 2
    den = (1 / tau2) + q2 * one_m_c  # 1 - c q2
    R = c - s * s * q2 / den
    one_m_R = one_m_c + s * s * q2 / den
    X = (R * G + (2 * G / w3) * (1 - R * q3)) / one_m_R
    return X + G / 2


def kolmogorov_amplitude_bgk(G: float, k: float, tau: float) -> float:
    """Same for BGK, derived from populations: U = G [4 tau + 1 + Z (1 - omega/2)] / (2 - omega Z),
    Z = 2 (c - q) / (1 - 2 q c + q^2).  Equals the SMRT form at tau3 = tau2."""
    w = 1 / tau
    q = 1 - w
    c = math.cos(k)
    Z = 2 * (c - q) / (1 - 2 * q * c + q * q)
    return G * (4 * tau + 1 + Z * (1 - w / 2)) / (2 - w * Z)


def kolmogorov_amplitude_continuum(G: float, k: float, tau2: float) -> float:
    return G / (nu_of(tau2) * k * k)


# ---- brute force: dense steady solve of the odd sector --------------------------------

def odd_sector_affine(g: np.ndarray, tau2: float, tau3: float, collision: str,
                      walls: bool):
    """One step of the odd sector as an affine map h -> A h + b s, for the acceleration
    g (per row, length n) scaled by s that step.  Unknowns: h_c(y) for c in (-1, 0, 1)
    after streaming (pre-collision), ordered c-major.  Returns (A, b)."""
    g = np.asarray(g, dtype=np.float64)
    n = g.size
    cs = (-1, 0, 1)
    wc = {-1: 1 / 36, 0: 1 / 9, 1: 1 / 36}
    nv = 3 * n

    def idx(c, y):
        return cs.index(c) * n + y

    # collision: h* = C h + d, built row by row
    Cm = np.zeros((nv, nv))
    d = np.zeros(nv)
    for y in range(n):
        if collision == "bgk":
            om = 1 / tau2
            for c in cs:
                r = idx(c, y)
                Cm[r, r] += 1 - om
                # + omega * 6 w_c u_x, u_x = X + g/2, X = sum_c' h_c'
                for c2 in cs:
                    Cm[r, idx(c2, y)] += om * 6 * wc[c]
                d[r] += om * 6 * wc[c] * g[y] / 2 + (1 - om / 2) * 6 * wc[c] * g[y]
        else:
            q2 = 1 - 1 / tau2
            q3 = 1 - 1 / tau3
            # moments of h: X = h-1 + h0 + h1, Y = h1 - h-1, Z = 2h1 + 2h-1 - h0
            T = np.array([[1, 1, 1], [-1, 0, 1], [2, -1, 2]], dtype=np.float64)
            Ti = np.linalg.inv(T)
            K = Ti @ np.diag([1.0, q2, q3]) @ T
            off = Ti @ np.array([g[y], 0.0, 0.0])
            rows = [idx(c, y) for c in cs]
            for a, ra in enumerate(rows):
                for b, rb in enumerate(rows):
                    Cm[ra, rb] += K[a, b]
                d[ra] += off[a]
    # streaming with walls / periodic
    S = np.zeros((nv, nv))
    for c in cs:
        for y in range(n):
            src = y - c
            if 0 <= src < n:
                S[idx(c, y), idx(c, src)] = 1
            elif not walls:
                S[idx(c, y), idx(c, src % n)] = 1
            else:
                # population leaving row y toward the wall returns as -c: h_c(y) <- -h*_{-c}(y)
                S[idx(c, y), idx(-c, y)] = -1
    return S @ Cm, S @ d


def _sector_velocity(h, g, s):
    n = g.size
    return h[: n] + h[n: 2 * n] + h[2 * n:] + np.asarray(g) * s / 2


def odd_sector_steady(g: np.ndarray, tau2: float, tau3: float, collision: str,
                      walls: bool) -> np.ndarray:
    """Steady u_x(y) of the odd sector by one dense linear solve of (I - A) h = b."""
    g = np.asarray(g, dtype=np.float64)
    A, b = odd_sector_affine(g, tau2, tau3, collision, walls)
    nv = b.size
    if walls:
        h = np.linalg.solve(np.eye(nv) - A, b)
    else:
        # periodic: uniform x-momentum is a free (neutral) mode; fix it by the total
        # momentum sum_y X = -sum_y g/2 of a flow whose mean physical velocity is zero.
        con = np.zeros((1, nv))
        con[0, :] = 1.0
        M = np.vstack([np.eye(nv) - A, con])
        r = np.concatenate([b, [-g.sum() / 2]])
        h = np.linalg.lstsq(M, r, rcond=None)[0]
    return _sector_velocity(h, g, 1.0)


def odd_sector_periodic(g: np.ndarray, omega: float, tau2: float, tau3: float, collision: str,
                        walls: bool) -> np.ndarray:
    """Time-periodic response of the odd sector to the acceleration g(y) cos(omega t):
    with s_t = Re(exp(i omega t)) the step h_{t+1} = A h_t + b s_t has the periodic
    solution h_t = Re(H exp(i omega t)), (exp(i omega) I - A) H = b.  Returns the complex
    amplitude of u_x(y): u_x(y, t) = Re(U(y) exp(i omega t)) (u = X + g s / 2)."""
    g = np.asarray(g, dtype=np.float64)
    A, b = odd_sector_affine(g, tau2, tau3, collision, walls)
    H = np.linalg.solve(np.exp(1j * omega) * np.eye(b.size) - A, b.astype(complex))
    return _sector_velocity(H, g.astype(complex), 1.0)


def odd_sector_evolve(g: np.ndarray, s, tau2: float, tau3: float, collision: str,
                      walls: bool) -> np.ndarray:
    """u_x(y) after len(s) - 1 steps from rest (rho = 1, u = 0) with the acceleration
    g(y) s_t at step t (s_0 .. s_{k-1}) and s_k for the final velocity.  The rest state
    holds f-bar = f_eq - F/2 with the first-order force term F_i = 3 w_i rho e_i . g, whose
    odd part is h_c = -3 w_c g s_0."""
    g = np.asarray(g, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    import scipy.sparse
    A, b = odd_sector_affine(g, tau2, tau3, collision, walls)
    As = scipy.sparse.csr_matrix(A)  # a few entries per row: the recursion is cheap
    h = np.concatenate([-3 * w * g * s[0] for w in (1 / 36, 1 / 9, 1 / 36)])
    for t in range(s.size - 1):
        h = As @ h + b * s[t]
    return _sector_velocity(h, g, s[-1])


def womersley_profile(ny: int, nu: float, amp: float, omega: float, t: float,
                      rho0: float = 1.0) -> np.ndarray:
    """Continuum Womersley flow between plates at y = -1/2 and ny - 1/2 (halfway walls,
    width 2L = ny) under the uniform force -amp cos(omega t) (paper Sec. III.B):
    U = Re(i amp/(rho0 omega) {1 - cosh((1+i) y sqrt(omega/2nu)) / cosh((1+i) L
    sqrt(omega/2nu))} exp(i omega t)), y measured from the mid-plane, at the ny nodes."""
    y = np.arange(ny) - (ny - 1) / 2.0
    L = ny / 2.0
    k = (1 + 1j) * math.sqrt(omega / (2 * nu))
    prof = 1j * amp / (rho0 * omega) * (1 - np.cosh(k * y) / np.cosh(k * L))
    return np.real(prof * np.exp(1j * omega * t))


def taylor_green_velocity(shape, u0: float, nu: float, t: float):
    """2-D decaying Taylor-Green field of the paper's Sec. III.A (k1 = k2 = 2 pi / L):
    u = -u0 [cos(k x) sin(k y), -sin(k x) cos(k y)] exp(-(k1^2 + k2^2) nu t)."""
    nx, ny = shape
    k1 = 2 * math.pi / nx
    k2 = 2 * math.pi / ny
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    decay = math.exp(-(k1 * k1 + k2 * k2) * nu * t)
    ux = -u0 * np.cos(k1 * x) * np.sin(k2 * y) * decay
    uy = u0 * (k1 / k2) * np.sin(k1 * x) * np.cos(k2 * y) * decay
    return ux, uy


def e2_error(u, ua) -> float:
    """Relative L2 velocity error of the paper's Sec. III.A."""
    u = np.asarray(u, dtype=np.float64)
    ua = np.asarray(ua, dtype=np.float64)
    return math.sqrt(float(np.sum((u - ua) ** 2) / np.sum(ua ** 2)))


def fourier_perturbative_steady(box: int, tau2: float, modes, order: int = 2, rho0: float = 1.0):
    """Steady periodic flow of the incompressible equations forced by solenoidal Fourier
    modes g = sum_j amp_j p_j sin(theta_j), theta_j = 2 pi k_j . x / box + phase_j, in
    powers of the forcing (this is not from the paper: it is the analytic start the warm
    start is measured against).

    order 1 (Stokes): nu lap u1 = -g, so u1 = sum_j s_j p_j sin(theta_j) with
    s_j = amp_j / (nu K_j^2).  order 2: nu lap u2 = (u1 . grad) u1 + grad p2 / rho0; the
    advection of mode j by mode i is s_i s_j (p_i . K_j) p_j sin(theta_i) cos(theta_j),
    half a wave at theta_i + theta_j and half at theta_i - theta_j; for a wave
    A sin(q . x + phi) the solenoidal part P_q A = A - q (q . A) / |q|^2 gives
    u2 = -P_q A sin(.) / (nu |q|^2) and the rest the pressure p2 = rho0 (q . A) cos(.) /
    |q|^2 (q = 0 waves are uniform and drop out).  Density rho0 + p2 / c_s^2.

    Returns (rho (N,), u (3, N)) on the box^3 lattice, x fastest."""
    nu = (tau2 - 0.5) / 3.0
    x, y, z = (np.arange(box ** 3) % box, (np.arange(box ** 3) // box) % box,
               np.arange(box ** 3) // box ** 2)
    pos = np.stack([x, y, z]).astype(np.float64)
    kp = 2.0 * math.pi / box
    ks = [kp * np.asarray(m["k"], np.float64) for m in modes]
    ps = [np.asarray(m["p"], np.float64) for m in modes]
    th = [k @ pos + m["phase"] for k, m in zip(ks, modes)]
    s = [m["amp"] / (nu * float(k @ k)) for k, m in zip(ks, modes)]
    u = np.zeros((3, box ** 3))
    rho = np.full(box ** 3, rho0)
    for j in range(len(modes)):
        u += s[j] * np.outer(ps[j], np.sin(th[j]))
    if order >= 2:
        for i in range(len(modes)):
            for j in range(len(modes)):
                if i == j:
                    continue
                A = 0.5 * s[i] * s[j] * float(ps[i] @ ks[j]) * ps[j]
                for sg in (1.0, -1.0):
                    q = ks[i] + sg * ks[j]
                    q2 = float(q @ q)
                    if q2 < 1e-300:
                        continue
                    phase = th[i] + sg * th[j]
                    PA = A - q * float(q @ A) / q2
                    u -= np.outer(PA / (nu * q2), np.sin(phase))
                    rho += 3.0 * rho0 * float(q @ A) / q2 * np.cos(phase)
    return rho, u
