"""Property tests of the oracle's right-hand side on states drawn by hypothesis.

The geodesic acceleration of `eq:geo` in the Kerr-Schild chart of `def:CKS`
has symmetries and invariants that hold at every point outside the horizon:
it is quadratic in the momentum, does not depend on t, commutes with
rotations about the spin axis and with the reflection z -> -z, turns into
the acceleration of the hole of spin -a under the mirror y -> -y, and keeps
E, L_z, Carter's Q and g k k constant along the flow.  Hypothesis draws spins
in [-1, 1] (the extremes and zero included), radii from just outside the
horizon to 200 M, polar angles down to the axis, and null or time-like
momenta; a dropped term, a wrong sign of a, or x and y exchanged anywhere in
the metric, its derivatives or the contraction breaks one of them.
"""
import numpy as np
from hypothesis import HealthCheck, assume, given, settings, strategies as st

import oracle as O

SETTINGS = settings(max_examples=120, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.filter_too_much, HealthCheck.too_slow])

spins = st.one_of(st.sampled_from([-1.0, 0.0, 1.0]), st.floats(-1.0, 1.0))
angles = st.floats(0.0, np.pi)


def _state(a, dr, th, ph, kdir, kmag, timelike):
    """(x, k) at Boyer-Lindquist-like (r, theta, phi) with r = r_H + dr, in the
    Cartesian Kerr-Schild chart (x + iy = (r + ia) e^{i phi} sin theta,
    z = r cos theta), the spatial momentum kmag * kdir and k^0 from the null or
    unit time-like condition (future-directed root); None inside the ergoregion."""
    r = 1.0 + np.sqrt(max(1.0 - a * a, 0.0)) + dr
    c = (r + 1j * a) * np.exp(1j * ph) * np.sin(th)
    x = np.array([0.0, c.real, c.imag, r * np.cos(th)])
    kd = np.asarray(kdir, dtype=float)
    nrm = np.linalg.norm(kd)
    if nrm < 1e-3:
        return None
    k = np.zeros(4)
    k[1:] = kmag * kd / nrm
    g, _ = O.metric(a, x)
    A = g[0, 0]
    B = g[0, 1:] @ k[1:]
    C = k[1:] @ g[1:, 1:] @ k[1:] + (1.0 if timelike else 0.0)
    if not A < -1e-3:
        return None
    disc = B * B - A * C
    if disc < 0:
        return None
    k[0] = (B + np.sqrt(disc)) / (-A)
    return x, k


@st.composite
def states(draw):
    """(a, x, k): a spin and a state outside its horizon and ergoregion."""
    a = draw(spins)
    s = _state(a, draw(st.floats(0.05, 200.0)), draw(angles), draw(angles),
               draw(st.tuples(st.floats(-1, 1), st.floats(-1, 1), st.floats(-1, 1))), draw(st.floats(0.05, 5.0)),
               draw(st.booleans()))
    assume(s is not None)
    return (a, *s)


def _close(got, want, rtol=1e-10):
    scale = max(1.0, float(np.abs(want).max()))
    np.testing.assert_allclose(got, want, rtol=rtol, atol=rtol * scale)


@SETTINGS
@given(states(), st.floats(0.1, 10.0))
def test_rhs_is_quadratic_in_the_momentum(s0, lam):
    a, x, k = s0
    _close(O.rhs(a, x, lam * k), lam * lam * O.rhs(a, x, k))


@SETTINGS
@given(states(), st.floats(-1e4, 1e4))
def test_rhs_does_not_depend_on_t(s0, t):
    a, x, k = s0
    xt = x.copy()
    xt[0] = t
    _close(O.rhs(a, xt, k), O.rhs(a, x, k), rtol=1e-14)


def _rot(al):
    R = np.eye(4)
    R[1:3, 1:3] = [[np.cos(al), -np.sin(al)], [np.sin(al), np.cos(al)]]
    return R


@SETTINGS
@given(states(), st.floats(-np.pi, np.pi))
def test_rhs_commutes_with_rotations_about_the_spin_axis(s0, al):
    a, x, k = s0
    R = _rot(al)
    _close(O.rhs(a, R @ x, R @ k), R @ O.rhs(a, x, k))


@SETTINGS
@given(states())
def test_rhs_commutes_with_the_equatorial_reflection(s0):
    a, x, k = s0
    Z = np.diag([1.0, 1.0, 1.0, -1.0])
    _close(O.rhs(a, Z @ x, Z @ k), Z @ O.rhs(a, x, k))


@SETTINGS
@given(states())
def test_mirror_maps_spin_a_to_spin_minus_a(s0):
    a, x, k = s0
    P = np.diag([1.0, 1.0, -1.0, 1.0])
    _close(O.rhs(-a, P @ x, P @ k), P @ O.rhs(a, x, k))


@SETTINGS
@given(states())
def test_constants_of_motion_are_conserved_by_the_flow(s0):
    """d/dl of (E, L_z, Q, g k k) along (x, k) -> (x + e k, k + e acc), by a
    fourth-order central difference, vanishes to the difference's error."""
    a, x, k = s0
    acc = O.rhs(a, x, k)
    r = O.radius(a, *x[1:])
    # a step well inside the scale of variation (r, and the distance to the horizon)
    hh = 1e-4 * min(1.0, r - (1.0 + np.sqrt(max(1.0 - a * a, 0.0)))) / max(1.0, np.abs(k).max())

    def C(e):
        return O.constants(a, x + e * k, k + e * acc)

    d = (-C(2 * hh) + 8 * C(hh) - 8 * C(-hh) + C(-2 * hh)) / (12 * hh)
    scale = np.maximum(np.abs(C(0.0)), 1.0) * max(1.0, np.abs(k).max()) * max(1.0, np.abs(acc).max())
    assert np.all(np.abs(d) < 1e-6 * scale), (d, scale)



@SETTINGS
@given(spins, st.floats(0.05, 50.0), st.booleans(), st.floats(-3, 3), st.floats(-3, 3), st.floats(-3, 3),
       st.booleans())
def test_carter_constant_is_continuous_onto_the_axis(a, dr, south, kx, ky, kz, timelike):
    """On the spin axis both quotients of Carter's Q are 0/0; the oracle takes
    the limit.  Approached from eight directions, the off-axis formula tends to
    the on-axis value, whatever the direction: the largest difference falls at
    least 20-fold from a distance of 1e-5 to 1e-7 (it is linear in the
    distance), so a wrong on-axis value would stay put."""
    r = 1.0 + np.sqrt(max(1.0 - a * a, 0.0)) + dr
    z = -r if south else r

    def state(x, y):
        xx = np.array([0.0, x, y, z])
        k = np.array([0.0, kx, ky, kz])
        g, _ = O.metric(a, xx)
        A, B = g[0, 0], g[0, 1:] @ k[1:]
        C = k[1:] @ g[1:, 1:] @ k[1:] + (1.0 if timelike else 0.0)
        assume(A < -1e-3 and B * B - A * C > 0)
        k[0] = (B + np.sqrt(B * B - A * C)) / (-A)
        return xx, k

    x0, k0 = state(0.0, 0.0)
    q0 = O.constants(a, x0, k0)[2]
    assert np.isfinite(q0)
    scale = max(1.0, abs(q0), (r * r + a * a) * (kx * kx + ky * ky))
    d = {}
    for eps in (1e-5, 1e-7):
        d[eps] = max(abs(O.constants(a, np.array([0.0, eps * np.cos(t), eps * np.sin(t), z]), k0)[2] - q0)
                     for t in np.linspace(0.0, 2 * np.pi, 8, endpoint=False))
    assert d[1e-7] <= 0.05 * d[1e-5] + 1e-10 * scale, (d, q0)
