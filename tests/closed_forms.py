"""Closed-form Kerr results used to pin the oracle (test-side only).

These are textbook results for the Kerr metric in Boyer-Lindquist form (the
line element printed at the start of Sec. 2.1), written independently of the
oracle: spherical photon orbits (the orbits of Sec. 3.1 / Table tab:tests),
Bardeen's shadow boundary, the radial potential that decides capture,
circular-orbit frequencies (Sec. 3.2) and the Keplerian emitter.  G = c = M = 1.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate


def r_horizon(a):
    return 1.0 + np.sqrt(max(1.0 - a * a, 0.0))


def r_prograde_photon(a):
    """Sec. 3.1: r_p = 2{1 + cos[(2/3) arccos(-|a|)]}."""
    return 2.0 * (1.0 + np.cos(2.0 / 3.0 * np.arccos(-abs(a))))


def r_retrograde_photon(a):
    """Sec. 3.1: r_r = 2{1 + cos[(2/3) arccos(|a|)]}."""
    return 2.0 * (1.0 + np.cos(2.0 / 3.0 * np.arccos(abs(a))))


def r_isco(a):
    z1 = 1 + (1 - a * a) ** (1 / 3) * ((1 + a) ** (1 / 3) + (1 - a) ** (1 / 3))
    z2 = np.sqrt(3 * a * a + z1 * z1)
    return 3 + z2 - np.sqrt((3 - z1) * (3 + z1 + 2 * z2))


def spherical_xi_eta(r, a):
    """Angular momentum xi = L_z/E and Carter constant eta = Q/E^2 of the
    spherical photon orbit of radius r (from R(r) = R'(r) = 0)."""
    xi = (r * r * (3 - r) - a * a * (r + 1)) / (a * (r - 1))
    eta = r ** 3 * (4 * a * a - r * (r - 3) ** 2) / (a * a * (r - 1) ** 2)
    return xi, eta


def _u_roots(xi, eta, a):
    s = eta + xi * xi - a * a
    disc = np.sqrt(s * s + 4 * a * a * eta)
    up = (-s + disc) / (2 * a * a)
    um = (s + disc) / (2 * a * a)
    return up, um


def spherical_max_cos(r, a):
    xi, eta = spherical_xi_eta(r, a)
    up, _ = _u_roots(xi, eta, a)
    return np.sqrt(min(up, 1.0))


def spherical_dphi(r, a):
    """Azimuth advance over one full latitude period of a spherical photon orbit.

    With Mino time, dphi = (a P / Delta - a) + xi / sin^2(theta) and
    dtheta = sqrt(Theta); substituting cos(theta) = sqrt(u+) sin(chi) makes
    both period integrals regular.
    """
    xi, eta = spherical_xi_eta(r, a)
    up, um = _u_roots(xi, eta, a)
    up = min(up, 1.0)
    delta = r * r - 2 * r + a * a
    P = r * r + a * a - a * xi

    def w(chi):
        return 1.0 / (a * np.sqrt(up * np.sin(chi) ** 2 + um))

    T = 4 * integrate.quad(w, 0, np.pi / 2, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
    if xi == 0.0 or abs(xi) < 1e-14:
        I = 0.0
    else:
        I = 4 * integrate.quad(lambda c: w(c) / (1 - up * np.sin(c) ** 2), 0, np.pi / 2, epsabs=1e-13,
                               epsrel=1e-12, limit=200)[0]
    return (a * P / delta - a) * T + xi * I


def spherical_orbit_tests():
    return {"A": 1.8, "B": 2.0, "C": 1 + np.sqrt(2), "D": 1 + np.sqrt(3), "E": 3.0, "F": 1 + 2 * np.sqrt(2)}


def bardeen_beta2(r, a, incl):
    """beta^2 on the shadow boundary parametrised by the photon-orbit radius r."""
    xi, eta = spherical_xi_eta(r, a)
    return eta + a * a * np.cos(incl) ** 2 - xi * xi / np.tan(incl) ** 2


def bardeen_alpha(r, a, incl):
    xi, _ = spherical_xi_eta(r, a)
    return -xi / np.sin(incl)


def bardeen_beta0_edges(a, incl):
    """alpha of the two shadow edges on the beta = 0 line (a > 0)."""
    from scipy.optimize import brentq

    rp, rr = r_prograde_photon(a), r_retrograde_photon(a)
    rs = np.linspace(rp + 1e-9, rr - 1e-9, 4001)
    b2 = np.array([bardeen_beta2(r, a, incl) for r in rs])
    roots = []
    for i in range(len(rs) - 1):
        if b2[i] == 0 or b2[i] * b2[i + 1] < 0:
            roots.append(brentq(lambda r: bardeen_beta2(r, a, incl), rs[i], rs[i + 1], xtol=1e-14))
    al = sorted(bardeen_alpha(r, a, incl) for r in roots)
    return al[0], al[-1]


def radial_potential_has_turning_point(xi, eta, a):
    """True if R(r) = (r^2 + a^2 - a xi)^2 - Delta (eta + (xi - a)^2) has a real root
    outside the outer horizon, i.e. a photon from infinity turns back (escapes)."""
    A = a * a - a * xi
    B = eta + (xi - a) ** 2
    coeffs = [1.0, 0.0, 2 * A - B, 2 * B, A * A - a * a * B]
    roots = np.roots(coeffs)
    rH = r_horizon(a)
    real = roots[np.abs(roots.imag) < 1e-9 * np.maximum(1, np.abs(roots))].real
    return bool(np.any(real > rH))


def omega_kepler(r, a):
    return 1.0 / (r ** 1.5 + a)


def ut_kepler(r, a):
    return (r ** 1.5 + a) / (r ** 0.75 * np.sqrt(r ** 1.5 - 3 * np.sqrt(r) + 2 * a))


def omega_vertical(r, a):
    """Vertical epicyclic frequency (observer at infinity), prograde orbit."""
    om = omega_kepler(r, a)
    return om * np.sqrt(1 - 4 * a * r ** -1.5 + 3 * a * a * r ** -2)


def bl_metric(r, th, a):
    """Boyer-Lindquist line element as printed at the start of Sec. 2.1,
    coordinates (t, r, theta, phi)."""
    rho2 = r * r + a * a * np.cos(th) ** 2
    delta = r * r - 2 * r + a * a
    s2 = np.sin(th) ** 2
    g = np.zeros((4, 4))
    g[0, 0] = -(1 - 2 * r / rho2)
    g[0, 3] = g[3, 0] = -2 * r * a * s2 / rho2
    g[1, 1] = rho2 / delta
    g[2, 2] = rho2
    g[3, 3] = (r * r + a * a + 2 * r * a * a * s2 / rho2) * s2
    return g


def schwarzschild_crossings(x0, v0, k_max, r_capture, r_escape):
    """Equatorial crossings of a Schwarzschild (a = 0) photon from the orbit
    equation, independently of any integrator.

    x0, v0: initial Cartesian position and spatial velocity dx^i/dlambda (the
    spatial coordinates of the Kerr-Schild chart are those of Schwarzschild
    at a = 0, so the path is the textbook one).  The photon moves in the plane
    of x0 and v0; with u = 1/r and the in-plane angle psi from x0,
    (du/dpsi)^2 = P(u) = 1/b^2 - u^2 + 2 u^3, where b^2 = L^2 / (rdot^2 +
    L^2 u^2 (1 - 2u)) (null condition), L = |x0 x v0|.  Crossings of z = 0 are
    at psi_j = psi_1 + (j - 1) pi.  The angle integrals are taken with the
    cubic's roots factored out (smooth integrands through the turning point).
    Returns [(r_j, azimuth_j)] for the crossings reached before the photon
    falls below r_capture or leaves past r_escape.
    """
    from scipy.optimize import brentq

    x0, v0 = np.asarray(x0, float), np.asarray(v0, float)
    r0 = np.linalg.norm(x0)
    xh = x0 / r0
    rdot = v0 @ xh
    assert rdot < 0.0, "the photon must start inward"
    w = v0 - rdot * xh
    Lw = np.linalg.norm(w)
    if Lw < 1e-12 * np.linalg.norm(v0):
        return []  # radial: the photon keeps the sign of z until r = 0
    wh = w / Lw
    L = r0 * Lw
    u0 = 1.0 / r0
    b2 = L * L / (rdot * rdot + L * L * u0 * u0 * (1.0 - 2.0 * u0))
    c = 1.0 / b2
    th = np.arctan2(-xh[2], wh[2])
    psi1 = th % np.pi
    if psi1 == 0.0:
        psi1 = np.pi
    roots = np.sort(np.roots([2.0, -1.0, 0.0, c]).real[np.abs(np.roots([2.0, -1.0, 0.0, c]).imag) < 1e-12])
    u_cap, u_esc = 1.0 / r_capture, 1.0 / r_escape
    out = []

    def point(psi, u):
        p = np.cos(psi) * xh + np.sin(psi) * wh
        return (1.0 / u, float(np.arctan2(p[1], p[0])))

    if c < 1.0 / 27.0 and len(roots) == 3 and roots[1] > u0:
        rn, ut, r3 = roots  # P(u) = 2 (u - rn)(u - ut)(u - r3), u0 < ut < r3
        g = lambda s: 2.0 / np.sqrt(2.0 * (ut - s * s - rn) * (r3 - ut + s * s))  # noqa: E731
        G = lambda s: integrate.quad(g, 0.0, s, epsabs=1e-14, epsrel=1e-13, limit=200)[0]  # noqa: E731
        s0 = np.sqrt(ut - u0)
        G0 = G(s0)
        s_esc = np.sqrt(ut - u_esc)
        G_esc = G(s_esc)
        for j in range(k_max):
            psi = psi1 + j * np.pi
            if psi <= G0:  # inward branch: psi = G0 - G(s)
                s = brentq(lambda s: G0 - G(s) - psi, 0.0, s0, xtol=1e-15)
            elif psi - G0 < G_esc:  # outward branch: psi = G0 + G(s)
                s = brentq(lambda s: G0 + G(s) - psi, 0.0, s_esc, xtol=1e-15)
            else:
                break
            out.append(point(psi, ut - s * s))
    else:  # no turning point: the photon falls in
        f = lambda u: 1.0 / np.sqrt(c - u * u + 2.0 * u ** 3)  # noqa: E731
        F = lambda u: integrate.quad(f, u0, u, epsabs=1e-14, epsrel=1e-13, limit=200)[0]  # noqa: E731
        F_cap = F(u_cap)
        for j in range(k_max):
            psi = psi1 + j * np.pi
            if psi >= F_cap:
                break
            u = brentq(lambda u: F(u) - psi, u0, u_cap, xtol=1e-16)
            out.append(point(psi, u))
    return out
