"""Closed-form solutions used to pin the oracle (test infrastructure only).

Coordinates: walls are halfway between nodes, so node j of an n-node channel
sits at y = j + 1/2 with the walls at y = 0 and y = H = n.
"""
from __future__ import annotations

import numpy as np


def node_coords(n: int) -> np.ndarray:
    return np.arange(n) + 0.5


def brinkman_channel(n: int, a: float, K: float, nu: float, nu_e: float, phi: float) -> np.ndarray:
    """Steady unidirectional flow driven by a uniform acceleration a between
    no-slip walls, Brinkman-extended Darcy model (Eq. 2 with Eq. 4, F_phi = 0):
    nu_e u'' - (phi nu / K) u + phi a = 0, u(0) = u(H) = 0, so
    u = (a K / nu) [1 - cosh(r (y - H/2)) / cosh(r H / 2)], r = sqrt(phi nu / (K nu_e))."""
    H = float(n)
    y = node_coords(n)
    r = np.sqrt(phi * nu / (K * nu_e))
    return a * K / nu * (1.0 - np.cosh(r * (y - H / 2)) / np.cosh(r * H / 2))


def forchheimer_channel(n: int, a: float, K: float, nu: float, nu_e: float, phi: float,
                        F_phi: float, refine: int = 64) -> np.ndarray:
    """Same channel with the Forchheimer drag (Eq. 4 in full), which has no
    closed form: nu_e u'' - (phi nu/K) u - (phi F_phi/sqrt K) |u| u + phi a = 0.
    Solved by Newton's method on a fine second-order finite-difference grid
    (refine cells per lattice spacing), then Richardson-extrapolated from two
    grids and sampled at the lattice nodes."""

    def solve(m):
        H = float(n)
        h = H / m
        y = (np.arange(1, m) * h)
        u = np.zeros(m - 1)
        c1 = phi * nu / K
        c2 = phi * F_phi / np.sqrt(K)
        for _ in range(60):
            up = np.concatenate(([0.0], u, [0.0]))
            lap = (up[2:] - 2 * up[1:-1] + up[:-2]) / (h * h)
            R = nu_e * lap - c1 * u - c2 * np.abs(u) * u + phi * a
            main = -2 * nu_e / (h * h) - c1 - 2 * c2 * np.abs(u)
            off = nu_e / (h * h) * np.ones(m - 2)
            # tridiagonal Newton step
            A = np.diag(main) + np.diag(off, 1) + np.diag(off, -1)
            du = np.linalg.solve(A, -R)
            u = u + du
            if np.max(np.abs(du)) < 1e-16 * max(1.0, np.max(np.abs(u))):
                break
        return np.concatenate(([0.0], y, [H])), np.concatenate(([0.0], u, [0.0]))

    m1 = n * refine
    y1, u1 = solve(m1)
    y2, u2 = solve(2 * m1)
    yn = node_coords(n)
    a1 = np.interp(yn, y1, u1)
    a2 = np.interp(yn, y2, u2)
    return a2 + (a2 - a1) / 3.0


def mixed_convection_channel(n: int, u0: float, u1: float, nu: float, nu_e: float,
                             alpha_e: float, phi: float, J: float, Da: float,
                             T_c: float, T_h: float):
    """Eqs. 48-50: porous channel with injection u1 through the cold lower wall,
    withdrawal through the hot upper wall moving at u0.  Returns u_x(y), T(y)."""
    H = float(n)
    y = node_coords(n)
    Re = H * u1 / nu
    Pr_e = nu / alpha_e
    th1 = Re / (2 * phi * J)
    th2 = np.sqrt(Re * Re + 4 * phi ** 3 * J / Da) / (2 * phi * J)
    ux = u0 * np.exp(th1 * (y / H - 1)) * np.sinh(th2 * y / H) / np.sinh(th2)
    T = T_c + (T_h - T_c) * np.expm1(Pr_e * Re * y / H) / np.expm1(Pr_e * Re)
    return ux, T


def mixed_convection_accel(n: int, u1: float, nu: float, K: float, gbeta: float, dT: float,
                           alpha_e: float) -> np.ndarray:
    """Eq. 47: the wall-normal external acceleration a_y(y) at the nodes."""
    H = float(n)
    y = node_coords(n)
    return nu / K * u1 - gbeta * dT * np.expm1(y * u1 / alpha_e) / np.expm1(H * u1 / alpha_e)


def relative_global_error(a: np.ndarray, b: np.ndarray) -> float:
    """Eq. 52: E = sqrt(sum |a - b|^2) / sqrt(sum |a|^2), a the analytical field."""
    return float(np.sqrt(np.sum((a - b) ** 2)) / np.sqrt(np.sum(a ** 2)))


# ---------------------------------------------------------------- two-region melting (Sec. 4.3)
def melting_eta(alpha_l: float, alpha_s: float, k_l: float, k_s: float, T_hot: float, T_melt: float,
                T_init: float, latent: float, c_pl: float) -> float:
    """Root eta of the transcendental Eq. 59 of the two-region melting problem
    (bisection on the bracket where its two sides cross)."""
    from scipy.special import erf, erfc
    r = alpha_l / alpha_s
    theta = (T_init - T_melt) / (T_hot - T_melt)

    def residual(eta):
        lhs = (np.exp(-eta * eta) / erf(eta)
               + (k_s / k_l) * np.sqrt(r) * theta * np.exp(-eta * eta * r) / erfc(eta * np.sqrt(r)))
        return lhs - eta * latent * np.sqrt(np.pi) / (c_pl * (T_hot - T_melt))

    lo, hi = 1e-6, 1.0
    while residual(hi) > 0.0:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if residual(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def two_region_melting(x, t: float, alpha_l: float, alpha_s: float, k_l: float, k_s: float, T_hot: float,
                       T_melt: float, T_init: float, latent: float, c_pl: float):
    """Temperature of Eqs. 57 (liquid, x <= x_m) and 58 (solid) and the front
    x_m(t) = 2 eta sqrt(alpha_l t), with eta from Eq. 59."""
    from scipy.special import erf, erfc
    eta = melting_eta(alpha_l, alpha_s, k_l, k_s, T_hot, T_melt, T_init, latent, c_pl)
    x = np.asarray(x, dtype=np.float64)
    xm = 2.0 * eta * np.sqrt(alpha_l * t)
    liquid = T_hot - (T_hot - T_melt) * erf(x / (2.0 * np.sqrt(alpha_l * t))) / erf(eta)
    solid = T_init + (T_melt - T_init) * erfc(x / (2.0 * np.sqrt(alpha_s * t))) / erfc(eta * np.sqrt(alpha_l / alpha_s))
    return np.where(x <= xm, liquid, solid), xm, eta
