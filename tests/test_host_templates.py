"""CPU checks of the GPU library's device arithmetic.

The right-hand side, the Runge-Kutta steps, the constants and the Hermite root
are __host__ __device__ templates; tests/host/host_templates.cpp instantiates
them for the host so their arithmetic can be compared with the oracle here,
without a GPU.  (The same templates are what the kernels run.)
"""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "host", "host_templates.cpp")
LIB = os.path.join(HERE, "host", "libhost_templates.so")
CSRC = os.path.join(ROOT, "paper_1706_07062_amd", "csrc")


@pytest.fixture(scope="module")
def H():
    deps = [SRC] + [os.path.join(CSRC, f) for f in ("ks_math.hpp", "bl_math.hpp", "steppers.hpp")]
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(d) for d in deps):
        subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__",
                        "-I/opt/rocm/include", "-I" + CSRC, "-o", LIB, SRC], check=True)
    L = C.CDLL(LIB)
    pd = C.POINTER(C.c_double)
    L.host_rhs.argtypes = [C.c_int, C.c_int, C.c_double, pd, pd, pd]
    L.host_dp5.argtypes = [C.c_double, pd, pd, C.c_double, C.c_double, C.c_double, pd]
    L.host_rk4.argtypes = [C.c_double, pd, pd, C.c_double, pd]
    L.host_rk4_bl.argtypes = [C.c_double, pd, pd, C.c_double, pd]
    L.host_hermite_zero.argtypes = [C.c_double] * 5
    L.host_hermite_zero.restype = C.c_double
    L.host_constants.argtypes = [C.c_double, pd, pd, pd]
    L.host_redshift.argtypes = [C.c_double] * 3
    L.host_redshift.restype = C.c_double
    L.host_atan2_est.argtypes = [C.c_double] * 2
    L.host_atan2_est.restype = C.c_double
    return L


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


rng = np.random.default_rng(1706070621)


def _states(n, a, rmin=1.3, rmax=200.0):
    out = []
    while len(out) < n:
        x = rng.uniform(-1, 1, 3) * rng.choice([3.0, 20.0, rmax])
        r = O.radius(a, *x)
        rh = 1 + np.sqrt(max(1 - a * a, 0))
        if not (max(rmin, 1.02 * rh) < r < rmax):
            continue
        k = rng.normal(size=3)
        y = np.array([rng.uniform(0, 100), *x, 0.0, *k])
        g, _ = O.metric(a, y[:4])
        A, B, Cq = g[0, 0], g[0, 1:] @ k, k @ g[1:, 1:] @ k
        if A >= 0:
            continue
        y[4] = (B + np.sqrt(B * B - A * Cq)) / (-A)
        out.append(y)
    return out


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("a", [0.0, -0.5, 0.99, -0.99, 1.0])
def test_rhs_matches_oracle(H, form, a):
    """The regrouped eq:opt0/opti evaluation equals the plain Christoffel form."""
    for y in _states(40, a):
        acc = np.zeros(6)
        H.host_rhs(form, 0, a, _p(y[:4].copy()), _p(y[4:].copy()), _p(acc))
        want = O.rhs(a, y[:4], y[4:])
        scale = np.abs(want).max() + 1e-300
        np.testing.assert_allclose(acc[:4], want, rtol=0, atol=2e-12 * scale)
        assert acc[4] == pytest.approx(O.radius(a, *y[1:4]), rel=1e-14)


@pytest.mark.parametrize("form", [0, 1])
def test_rhs_fp32_close_to_oracle(H, form):
    a = -0.99
    for y in _states(40, a, rmax=50.0):
        acc = np.zeros(6)
        H.host_rhs(form, 1, a, _p(y[:4].copy()), _p(y[4:].copy()), _p(acc))
        want = O.rhs(a, y[:4], y[4:])
        scale = np.abs(want).max()
        assert np.abs(acc[:4] - want).max() < 2e-4 * scale


def test_dopri5_attempt_matches_oracle_first_step(H):
    """The Nystrom-form DOPRI5 attempt reproduces the oracle's first-order form."""
    a = -0.9
    n = 0
    for y in _states(30, a, rmin=2.5, rmax=60.0):
        p = O.Params(method=O.DOPRI5, rtol=1e-8, atol=1e-8, h_coeff=0.01, hmax_coeff=0.1, r_escape=1e9,
                     r_h_factor=0.5)
        tr = O.trajectory(p, a, y, max_out=2)
        if len(tr) < 2:
            continue
        h = tr[1, 0] - tr[0, 0]
        out = np.zeros(15)
        H.host_dp5(a, _p(y[:4].copy()), _p(y[4:].copy()), h, 1e-8, 1e-8, _p(out))
        if out[12] > 1.0:
            continue  # oracle rejected this h first; the accepted step is not comparable
        np.testing.assert_allclose(out[:8], tr[1, 1:], rtol=1e-13, atol=1e-13 * np.abs(tr[1, 1:]).max())
        n += 1
    assert n >= 10


def test_rk4_step_matches_oracle(H):
    a = 0.7
    for y in _states(20, a, rmin=2.0, rmax=40.0):
        h = 0.05
        p = O.Params(method=O.RK4, h_coeff=h, r_escape=1e9, r_h_factor=0.5)
        tr = O.trajectory(p, a, y, max_out=2)
        out = np.zeros(8)
        H.host_rk4(a, _p(y[:4].copy()), _p(y[4:].copy()), h, _p(out))
        np.testing.assert_allclose(out, tr[1, 1:], rtol=1e-13, atol=1e-13 * np.abs(tr[1, 1:]).max())


def test_constants_and_redshift_match_oracle(H):
    for a in (0.0, 0.6, -0.99):
        # random states, and states on the spin axis (where Q is a limit)
        axis = [np.array([0.0, 0.0, 0.0, z, 0.0, *rng.normal(size=3)]) for z in (2.5, -7.0, 40.0)]
        for y in _states(20, a) + axis:
            if y[1] == 0.0 and y[2] == 0.0:
                g, _ = O.metric(a, y[:4])
                k = y[5:]
                A, B, Cq = g[0, 0], g[0, 1:] @ k, k @ g[1:, 1:] @ k
                y[4] = (B + np.sqrt(B * B - A * Cq)) / (-A)
            out = np.zeros(4)
            H.host_constants(a, _p(y[:4].copy()), _p(y[4:].copy()), _p(out))
            want = O.constants(a, y[:4], y[4:])
            assert np.all(np.isfinite(out)) and np.all(np.isfinite(want))
            np.testing.assert_allclose(out, want, rtol=1e-11, atol=1e-11 * np.abs(want).max())
    for r, xi, a in [(6.0, 2.0, 0.0), (2.0, -3.0, 0.99), (30.0, 5.0, 0.5), (1.2, 1.0, 0.9)]:
        g1, g2 = H.host_redshift(r, xi, a), O.redshift(r, xi, a)
        assert (np.isnan(g1) and np.isnan(g2)) or g1 == pytest.approx(g2, rel=1e-14)


def test_hermite_zero_is_the_cubic_root(H):
    for _ in range(200):
        y0, y1 = rng.uniform(0.1, 2), -rng.uniform(0.1, 2)
        if rng.random() < 0.5:
            y0, y1 = -y0, -y1
        m0, m1, h = rng.normal(), rng.normal(), rng.uniform(0.1, 3)
        th = H.host_hermite_zero(y0, m0, y1, m1, h)
        assert 0 <= th <= 1
        t2, t3 = th * th, th ** 3
        p = (2 * t3 - 3 * t2 + 1) * y0 + (t3 - 2 * t2 + th) * h * m0 + (-2 * t3 + 3 * t2) * y1 + (t3 - t2) * h * m1
        assert abs(p) < 1e-12 * (abs(y0) + abs(y1) + h * (abs(m0) + abs(m1)))


def test_azimuth_estimate_recovers_winding(H):
    """The integrator rebuilds the winding count w of a stored unwrapped azimuth
    phi = atan2(y, x) + 2 pi w by rounding (phi - est) / 2 pi, so the estimate
    must stay within pi of atan2 everywhere, including on the axes and for
    signed zeros (where atan2 is +-pi or +-0)."""
    pts = [(y, x) for y in (0.0, -0.0, 1.0, -1.0, 1e-300, -1e-300) for x in (0.0, -0.0, 2.0, -2.0, 1e-300, -1e-300)]
    ang = rng.uniform(-np.pi, np.pi, 20000)
    rad = 10 ** rng.uniform(-8, 8, ang.size)
    pts += list(zip(rad * np.sin(ang), rad * np.cos(ang)))
    worst = 0.0
    for i, (y, x) in enumerate(pts):
        true = np.arctan2(y, x)
        est = H.host_atan2_est(y, x)
        if i >= 36:  # off the origin (the first 36 points include zeros and FP32 underflow)
            worst = max(worst, abs(est - true))
        for w in (-3, -1, 0, 2, 5):
            phi = true + 2 * np.pi * w
            assert int(np.rint((phi - est) / (2 * np.pi))) == w, (y, x, w)
    assert worst < 0.08 + 1e-6  # away from the origin the estimate is within 0.08 rad


# ---------------------------------------------------------------------------
# Boyer-Lindquist form (chart comparison of Sec. 4).
# ---------------------------------------------------------------------------
def _bl_states(n, a):
    out = []
    rh = 1 + np.sqrt(1 - a * a)
    while len(out) < n:
        r = rh * 1.02 + rng.choice([2.0, 20.0, 1000.0]) * rng.uniform()
        th = rng.uniform(0.05, np.pi - 0.05)
        k = rng.normal(size=4)
        out.append(np.array([rng.uniform(0, 10), r, th, rng.uniform(-3, 3), *k]))
    return out


@pytest.mark.parametrize("a", [0.0, 0.5, -0.9, 0.999])
def test_bl_rhs_matches_oracle(H, a):
    """The contracted Boyer-Lindquist form equals the Christoffel form on the
    Boyer-Lindquist line element."""
    for y in _bl_states(60, a):
        acc = np.zeros(6)
        H.host_rhs(2, 0, a, _p(y[:4].copy()), _p(y[4:].copy()), _p(acc))
        want = O.bl_rhs(a, y[:4], y[4:])
        scale = np.abs(want).max()
        np.testing.assert_allclose(acc[:4], want, rtol=0, atol=1e-12 * scale)
        assert acc[4] == y[1] and acc[5] == y[5]


def test_bl_rhs_fp32_error(H):
    a = 0.999
    errs = []
    for y in _bl_states(200, a):
        a64, a32 = np.zeros(6), np.zeros(6)
        H.host_rhs(2, 0, a, _p(y[:4].copy()), _p(y[4:].copy()), _p(a64))
        H.host_rhs(2, 1, a, _p(y[:4].copy()), _p(y[4:].copy()), _p(a32))
        errs.append(np.abs(a32[:4] - a64[:4]).max() / np.abs(a64[:4]).max())
    assert np.median(errs) < 1e-5


def test_bl_rk4_step_matches_oracle(H):
    a = -0.999
    for y in _bl_states(30, abs(a)):
        y[6:] /= y[1]  # angular rates of order 1/r, as for a ray of unit energy
        hc = 1 / 64
        out = np.zeros(8)
        H.host_rk4_bl(a, _p(y[:4].copy()), _p(y[4:].copy()), hc * y[1], _p(out))
        want, st, _ = O.rk4_fixed("bl", a, hc, 0.0, 1e30, 1, y[:, None])
        if st[0] != O.ACTIVE:
            continue
        np.testing.assert_allclose(out, want[:, 0], rtol=1e-11, atol=1e-11 * np.abs(y).max())
