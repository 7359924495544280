"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (tests/golden), textbook closed forms (tests/closed_forms.py),
an independent Hamiltonian formulation, conservation laws, symmetry, and the
convergence order the paper reports.
"""
import os

import numpy as np
import pytest

import closed_forms as cf
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tab_tests():
    rows = {}
    with open(os.path.join(GOLDEN, "tab_tests.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            rows[p[0]] = dict(a=float(p[1]), r=float(p[2]), Phi=float(p[3]), Q=float(p[4]), maxcos=float(p[5]),
                              dphi=float(p[6]))
    return rows


TAB = _tab_tests()
rng = np.random.default_rng(1706070620)


def random_states(n, a, rmin=1.6, rmax=30.0):
    """Random positions outside the horizon and random null momenta."""
    out = []
    while len(out) < n:
        x = rng.uniform(-rmax, rmax, 3)
        r = O.radius(a, *x)
        if not (rmin < r < rmax):
            continue
        k = rng.normal(size=3)
        y = np.array([0.0, *x, 0.0, *k])
        g, _ = O.metric(a, y[:4])
        A = g[0, 0]
        B = g[0, 1:] @ k
        Cq = k @ g[1:, 1:] @ k
        if A >= 0:
            continue
        y[4] = (B + np.sqrt(B * B - A * Cq)) / (-A)
        out.append(y)
    return out


# ---------------------------------------------------------------------------
# The closed forms themselves against the paper's printed table.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("label", list("ABCDEF"))
def test_closed_forms_reproduce_tab_tests(label):
    row = TAB[label]
    xi, eta = cf.spherical_xi_eta(row["r"], row["a"])
    assert round(xi, 2) == pytest.approx(row["Phi"], abs=1e-9)
    assert round(eta, 4) == pytest.approx(row["Q"], abs=1e-9)
    assert round(cf.spherical_max_cos(row["r"], row["a"]), 4) == pytest.approx(row["maxcos"], abs=1e-9)
    assert round(cf.spherical_dphi(row["r"], row["a"]), 4) == pytest.approx(row["dphi"], abs=1e-9)


def test_photon_orbit_radius_bounds():
    # Sec. 3.1: M <= r_p <= 3M <= r_r <= 4M for every spin.
    for a in np.linspace(0, 1, 11):
        rp, rr = cf.r_prograde_photon(a), cf.r_retrograde_photon(a)
        assert 1 - 1e-12 <= rp <= 3 + 1e-12 <= rr + 2e-12 <= 4 + 3e-12


# ---------------------------------------------------------------------------
# Metric (def:CKS) against the textbook forms.
# ---------------------------------------------------------------------------
def test_metric_schwarzschild_limit_is_ingoing_eddington_finkelstein():
    # a = 0: -dt^2 + |dx|^2 + (2/r)(dt + n.dx)^2 with n = x/r.
    for _ in range(20):
        x = rng.uniform(-20, 20, 3)
        r = np.linalg.norm(x)
        if r < 2.5:
            continue
        g, _ = O.metric(0.0, np.array([0.0, *x]))
        l = np.array([1.0, *(x / r)])
        want = np.diag([-1.0, 1, 1, 1]) + (2.0 / r) * np.outer(l, l)
        np.testing.assert_allclose(g, want, rtol=0, atol=1e-14)


@pytest.mark.parametrize("a", [0.3, 0.9, 0.99, 1.0])
def test_metric_pullback_equals_boyer_lindquist(a):
    """Pull the Cartesian metric back to Boyer-Lindquist coordinates through
    x + i y = (r + i a) e^{i phi_KS} sin(theta), z = r cos(theta),
    t_KS = t_BL + int 2r/Delta dr, phi_KS = phi_BL + int a/Delta dr,
    and compare with the BL line element printed in Sec. 2.1."""
    for r, th, ph in [(2.5, 0.7, 0.3), (5.0, 1.3, 2.0), (12.0, 2.6, -1.1), (1.9, 1.57, 4.0), (40.0, 0.2, 0.9)]:
        if r <= cf.r_horizon(a) + 0.05:
            continue
        delta = r * r - 2 * r + a * a
        st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
        X = st * (r * cp - a * sp)
        Y = st * (r * sp + a * cp)
        Z = r * ct
        dxyz_dr = np.array([st * cp, st * sp, ct])
        dxyz_dth = np.array([ct * (r * cp - a * sp), ct * (r * sp + a * cp), -r * st])
        dxyz_dph = np.array([-Y, X, 0.0])
        J = np.zeros((4, 4))  # rows: (t, x, y, z); columns: BL (t, r, theta, phi)
        J[0, 0] = 1.0
        J[0, 1] = 2 * r / delta
        J[1:, 1] = dxyz_dr + dxyz_dph * a / delta
        J[1:, 2] = dxyz_dth
        J[1:, 3] = dxyz_dph
        g, _ = O.metric(a, np.array([0.0, X, Y, Z]))
        gbl = J.T @ g @ J
        np.testing.assert_allclose(gbl, cf.bl_metric(r, th, a), rtol=1e-11, atol=1e-11)


def test_radius_solves_implicit_definition():
    # eq:CKSr: x^2 + y^2 + z^2 = r^2 + a^2 (1 - z^2 / r^2), including R < a.
    for a in (0.0, 0.5, 0.999):
        for _ in range(50):
            x = rng.uniform(-3, 3, 3)
            r = O.radius(a, *x)
            lhs = x @ x
            rhs = r * r + a * a * (1 - x[2] ** 2 / r ** 2)
            assert abs(lhs - rhs) <= 8e-16 * max(lhs, 1.0)


def test_metric_derivatives_match_finite_differences():
    a = 0.9
    for y in random_states(10, a):
        x = y[:4]
        _, dg = O.metric(a, x)
        for c in (1, 2, 3):
            e = np.zeros(4)
            hh = 1e-4
            e[c] = hh
            gp2, _ = O.metric(a, x + 2 * e)
            gp1, _ = O.metric(a, x + e)
            gm1, _ = O.metric(a, x - e)
            gm2, _ = O.metric(a, x - 2 * e)
            fd = (-gp2 + 8 * gp1 - 8 * gm1 + gm2) / (12 * hh)
            np.testing.assert_allclose(dg[c], fd, atol=1e-9 * max(1.0, np.abs(dg[c]).max()))
        assert np.all(dg[0] == 0.0)


# ---------------------------------------------------------------------------
# Right-hand side (eq:geo) against independent formulations.
# ---------------------------------------------------------------------------
def _ginv(a, x):
    g, _ = O.metric(a, x)
    return np.linalg.inv(g)


@pytest.mark.parametrize("a", [0.0, 0.7, 0.99])
def test_rhs_equals_hamiltonian_form(a):
    """H = g^{ab} p_a p_b / 2: dp_m/dl = -1/2 d_m g^{ab} p_a p_b and
    k^m = g^{mn} p_n, so dk^m/dl = (d_c g^{mn}) k^c p_n + g^{mn} dp_n/dl.
    The inverse metric comes from numpy and its derivatives from finite
    differences; no Christoffel symbol is formed."""
    for y in random_states(8, a):
        x, k = y[:4], y[4:]
        g, _ = O.metric(a, x)
        p = g @ k
        gi = np.linalg.inv(g)
        dgi = np.zeros((4, 4, 4))
        hh = 1e-4
        for c in (1, 2, 3):
            e = np.zeros(4)
            e[c] = hh
            dgi[c] = (-_ginv(a, x + 2 * e) + 8 * _ginv(a, x + e) - 8 * _ginv(a, x - e) + _ginv(a, x - 2 * e)) / (
                12 * hh)
        pdot = np.array([-0.5 * p @ dgi[m] @ p for m in range(4)])
        want = np.einsum("c,cmn,n->m", k, dgi, p) + gi @ pdot
        got = O.rhs(a, x, k)
        np.testing.assert_allclose(got, want, atol=2e-8 * max(1.0, np.abs(want).max()))


@pytest.mark.parametrize("a", [0.0, 0.6, 0.99, 1.0])
def test_rhs_conserves_constants_of_motion(a):
    """Along the flow (x, k) -> (x + e k, k + e acc), E, L_z, Carter's Q and
    g k k have zero derivative."""
    for y in random_states(8, a):
        x, k = y[:4], y[4:]
        acc = O.rhs(a, x, k)
        hh = 1e-4

        def C(e):
            return O.constants(a, x + e * k, k + e * acc)

        d = (-C(2 * hh) + 8 * C(hh) - 8 * C(-hh) + C(-2 * hh)) / (12 * hh)
        scale = np.maximum(np.abs(C(0.0)), 1.0) * max(1.0, np.abs(k).max()) ** 2
        assert np.all(np.abs(d) < 1e-7 * scale), d


def test_rhs_schwarzschild_radial_infall():
    # a = 0, radial null ray: the affine parameter is linear in r (dr/dl = const).
    x = np.array([0.0, 7.0, 0.0, 0.0])
    k = np.array([0.0, -1.0, 0.0, 0.0])
    g, _ = O.metric(0.0, x)
    k[0] = (g[0, 1:] @ k[1:] + np.sqrt((g[0, 1:] @ k[1:]) ** 2 - g[0, 0] * (k[1:] @ g[1:, 1:] @ k[1:]))) / -g[0, 0]
    acc = O.rhs(0.0, x, k)
    assert abs(acc[1]) < 1e-15 and abs(acc[2]) < 1e-15 and abs(acc[3]) < 1e-15


def test_carter_constant_schwarzschild_is_total_angular_momentum():
    # a = 0: Q + L_z^2 = |x cross k_i|^2 (covariant spatial components).
    for y in random_states(10, 0.0):
        x, k = y[:4], y[4:]
        g, _ = O.metric(0.0, x)
        kl = g @ k
        L = np.cross(x[1:], kl[1:])
        c = O.constants(0.0, x, k)
        assert c[1] == pytest.approx(L[2], rel=1e-12, abs=1e-12)
        assert c[2] + c[1] ** 2 == pytest.approx(L @ L, rel=1e-10)


def test_null_initial_data_norm():
    init = O.camera_rays(0.99, 1000.0, np.radians(60), -12, 12, -12, 12, 1024, 1024,
                         pix=np.arange(0, 1024 * 1024, 9973))
    for i in range(init["s"].shape[1]):
        y = init["s"][:, i]
        c = O.constants(-0.99, y[:4], y[4:])
        assert abs(c[3]) < 1e-15 * max(1.0, y[4] ** 2)  # order 1e-16, as the paper reports
        assert y[4] > 0


# ---------------------------------------------------------------------------
# Steppers.
# ---------------------------------------------------------------------------
def test_dopri5_order_on_harmonic_oscillator():
    """Global error of the 5th-order solution falls as h^5 on y'' = -y, and the
    embedded error estimate behaves as h^5 per step."""
    y0 = np.array([1.0, 0.0, 0.5, -0.3, 0.0, 1.0, 0.2, 0.7])
    T = 2.0
    errs, ests = [], []
    for n in (20, 40, 80):
        h = T / n
        y, est = O.dopri5_sho(y0, h, n, rtol=1.0)
        ex = np.concatenate([y0[:4] * np.cos(T) + y0[4:] * np.sin(T), -y0[:4] * np.sin(T) + y0[4:] * np.cos(T)])
        errs.append(np.abs(y - ex).max())
        ests.append(est)
    o1 = np.log2(errs[0] / errs[1])
    o2 = np.log2(errs[1] / errs[2])
    assert 4.6 < o1 < 5.6 and 4.6 < o2 < 5.6, (errs, o1, o2)
    e1 = np.log2(ests[0] / ests[1])
    assert 4.3 < e1 < 5.7, ests


def _spherical_initial_state(label):
    """Sec. 3.1: start on the equator at +x moving upward.  a = 1, E = 1,
    contravariant k^x = 0 (dr/dl = 0), covariant k_t = -1, k_y = xi / x,
    k_z = sqrt(eta) / r; (k^t, k^y) from the 2x2 system k_m = g_mn k^n."""
    row = TAB[label]
    a, r = row["a"], row["r"]
    xi, eta = cf.spherical_xi_eta(r, a)
    X = np.sqrt(r * r + a * a)
    x = np.array([0.0, X, 0.0, 0.0])
    g, _ = O.metric(a, x)
    M = np.array([[g[0, 0], g[0, 2]], [g[2, 0], g[2, 2]]])
    kt, ky = np.linalg.solve(M, np.array([-1.0, xi / X]))
    kz = np.sqrt(eta) / r
    return np.array([0.0, X, 0.0, 0.0, kt, 0.0, ky, kz]), a


def test_spherical_orbit_launch_constants():
    # Test B at launch: Phi = L_z/E = 1, Q = 16, null (printed in Table tab:tests).
    for label in "ABCDEF":
        y, a = _spherical_initial_state(label)
        c = O.constants(a, y[:4], y[4:])
        assert c[0] == pytest.approx(1.0, abs=1e-13)
        assert c[1] == pytest.approx(TAB[label]["Phi"], abs=1e-12)
        assert round(c[2], 4) == pytest.approx(TAB[label]["Q"], abs=1e-9)
        assert abs(c[3]) < 1e-14


def _rk4_run(label, dl, lam_max):
    y, a = _spherical_initial_state(label)
    p = O.Params(method=O.RK4, h_coeff=dl, r_escape=1e30, r_h_factor=0.5)
    return O.trajectory(p, a, y, max_out=int(lam_max / dl) + 2), a


def _first_peak_cos(tr):
    cos = tr[:, 4] / np.array([O.radius(1.0, *row[2:5]) for row in tr])
    i = int(np.argmax(cos[: len(cos) // 2]))
    # quadratic through the largest three samples (the paper's peak fit)
    yy = cos[i - 1:i + 2]
    den = yy[0] - 2 * yy[1] + yy[2]
    return yy[1] - (yy[2] - yy[0]) ** 2 / (8 * den)


@pytest.mark.parametrize("label", ["B", "D"])
def test_rk4_max_cos_theta_converges_fourth_order(label):
    """Sec. 3.1 / Fig. z-conv: the fitted first peak of cos(theta) converges at
    4th order to max|cos(theta)| of Table tab:tests."""
    exact = cf.spherical_max_cos(TAB[label]["r"], 1.0)
    errs = []
    for dl in (1 / 16, 1 / 32, 1 / 64):
        tr, _ = _rk4_run(label, dl, 12.0)
        errs.append(abs(_first_peak_cos(tr) - exact))
    assert round(exact, 4) == TAB[label]["maxcos"]
    # the printed 4 decimals are already reached at dl = 1/64
    assert errs[-1] < 5e-5
    ratio = errs[1] / errs[2]
    assert 9 < ratio < 28, errs


@pytest.mark.parametrize("label", ["A", "B", "D", "F"])
def test_rk4_null_norm_converges_fourth_order(label):
    """Fig. uu-conv: max |u^2| over the run falls by ~16 per halving of the step."""
    m = []
    for dl in (1 / 16, 1 / 32):
        tr, a = _rk4_run(label, dl, 8.0)
        u2 = [abs(O.constants(a, row[1:5], row[5:9])[3]) for row in tr]
        m.append(max(u2))
    assert 10 < m[0] / m[1] < 24, m


def _dphi_full_period(tr):
    """Unwrapped Cartesian azimuth at the second upward equatorial crossing
    (one complete latitude oscillation), with linear interpolation in z."""
    x, y, z = tr[:, 2], tr[:, 3], tr[:, 4]
    dpsi = np.arctan2(x[:-1] * y[1:] - y[:-1] * x[1:], x[:-1] * x[1:] + y[:-1] * y[1:])
    psi = np.concatenate([[np.arctan2(y[0], x[0])], np.arctan2(y[0], x[0]) + np.cumsum(dpsi)])
    ups = np.where((z[:-1] < 0) & (z[1:] >= 0))[0]
    i = ups[0]
    f = -z[i] / (z[i + 1] - z[i])
    return psi[i] + f * (psi[i + 1] - psi[i]) - psi[0]


@pytest.mark.parametrize("label", ["B", "D", "E", "F", "C"])
def test_dphi_one_latitude_period(label):
    """Fig. dphi-conv: the azimuth advance over one complete latitude period
    matches Table tab:tests (Test C passes the poles, where the Cartesian
    azimuth jumps by pi, so it is compared modulo pi)."""
    exact = cf.spherical_dphi(TAB[label]["r"], 1.0)
    errs = []
    for dl in (1 / 256, 1 / 512):
        tr, _ = _rk4_run(label, dl, 40.0)
        d = _dphi_full_period(tr) - exact
        if label == "C":
            d = (d + np.pi / 2) % np.pi - np.pi / 2
        errs.append(abs(d))
    assert errs[-1] < 2e-4, errs
    assert round(exact, 4) == TAB[label]["dphi"]


def test_test_c_passes_the_poles():
    # Sec. 3.1: Test C passes the poles at x = y = 0, z ~ +-2.41.
    tr, _ = _rk4_run("C", 1 / 1024, 6.0)
    rho = np.hypot(tr[:, 2], tr[:, 3])
    i = int(np.argmin(rho))
    assert rho[i] < 2e-3
    assert abs(abs(tr[i, 4]) - 2.41) < 0.01


# ---------------------------------------------------------------------------
# Image rays: capture, shadow, constants.
# ---------------------------------------------------------------------------
def test_schwarzschild_capture_matches_sqrt27():
    """a = 0 (the 64x64, 60 deg, RK4 h = 0.01 r workload): a ray is captured iff
    its impact parameter b = sqrt(L_z^2 + Q)/E < sqrt(27), away from b = sqrt(27)."""
    init = O.camera_rays(0.0, 1000.0, np.radians(60), -10, 10, -10, 10, 64, 64, pix=np.arange(0, 4096, 5))
    out = O.integrate(init, O.Params(method=O.RK4, h_coeff=0.01, r_escape=1000.0))
    E, Lz, Q = out["c0"][0], out["c0"][1], out["c0"][2]
    b = np.sqrt(Lz ** 2 + Q) / E
    far = np.abs(b - np.sqrt(27)) > 0.02
    cap = out["status"] == O.CAPTURED
    assert np.all(np.isin(out["status"], [O.CAPTURED, O.ESCAPED]))
    assert np.array_equal(cap[far], (b < np.sqrt(27))[far])
    assert far.sum() > 0.95 * len(b)


def test_kerr_capture_matches_radial_potential():
    """a = 0.99: captured iff the radial potential has no turning point outside
    the horizon, for rays away from the critical curve."""
    a = 0.99
    init = O.camera_rays(a, 1000.0, np.radians(60), -12, 12, -12, 12, 1024, 1024,
                         pix=np.arange(0, 1024 * 1024, 1499))
    out = O.integrate(init, O.Params(method=O.DOPRI5, rtol=1e-8, atol=1e-8))
    E, Lz, Q = out["c0"][0], out["c0"][1], out["c0"][2]
    ac = -a  # chart spin
    agree = 0
    for i in range(len(E)):
        xi, eta = Lz[i] / E[i], Q[i] / E[i] ** 2
        esc = cf.radial_potential_has_turning_point(xi, eta, ac)
        # skip rays within 1e-3 of the critical curve in eta
        near = any(cf.radial_potential_has_turning_point(xi, eta + d, ac) != esc for d in (-1e-3, 1e-3))
        if near:
            continue
        assert (out["status"][i] == O.ESCAPED) == esc, (i, xi, eta)
        agree += 1
    assert agree > 600


def test_bardeen_shadow_edges_beta0():
    """a = 0.99, i = 60 deg, beta = 0: bisect the capture boundary along alpha
    with the oracle and compare with Bardeen's closed-form edges."""
    a, incl = 0.99, np.radians(60)
    lo_edge, hi_edge = cf.bardeen_beta0_edges(a, incl)
    p = O.Params(method=O.DOPRI5, rtol=1e-10, atol=1e-10)

    def captured(al):
        init = O.list_rays([a], [incl], [al], [0.0], 1000.0)
        return O.integrate(init, p, nthreads=1)["status"][0] == O.CAPTURED

    def bisect(x0, x1):
        c0 = captured(x0)
        for _ in range(22):
            m = 0.5 * (x0 + x1)
            if captured(m) == c0:
                x0 = m
            else:
                x1 = m
        return 0.5 * (x0 + x1)

    assert captured(2.0) and not captured(-4.0) and not captured(9.0)
    # The image is at r_obs = 1000, not infinity: allow O(1/r_obs) offsets.
    assert bisect(-4.0, 2.0) == pytest.approx(lo_edge, abs=1e-2)
    assert bisect(2.0, 9.0) == pytest.approx(hi_edge, abs=1e-2)


def test_image_constants_conserved_and_mirror_symmetry():
    """a = 0.99 DOPRI5 rtol 1e-8: E, L_z, Q and g k k drift stay below 1e2 rtol.
    a = 0: the image is mirror symmetric under alpha -> -alpha (y -> -y)."""
    init = O.camera_rays(0.99, 1000.0, np.radians(17), -12, 12, -12, 12, 1024, 1024,
                         pix=np.arange(0, 1024 * 1024, 2311))
    out = O.integrate(init, O.Params(method=O.DOPRI5, k_cross=4))
    d = np.abs(out["c1"] - out["c0"]) / np.maximum(np.abs(out["c0"]), 1.0)
    assert np.nanmax(d[:3]) < 1e-6
    # g k k scales with the square of the momentum, which grows near the horizon
    assert np.nanmax(d[3] / np.maximum(out["s"][4], 1.0) ** 2) < 1e-6

    W = 64
    rows, cols = np.meshgrid(np.arange(8, 56, 7), np.arange(0, 32, 3), indexing="ij")
    pix = (rows * W + cols).ravel()
    mir = (rows * W + (W - 1 - cols)).ravel()
    p = O.Params(method=O.DOPRI5, k_cross=4)
    o1 = O.integrate(O.camera_rays(0.0, 1000.0, np.radians(60), -12, 12, -12, 12, W, W, pix=pix), p)
    o2 = O.integrate(O.camera_rays(0.0, 1000.0, np.radians(60), -12, 12, -12, 12, W, W, pix=mir), p)
    assert np.array_equal(o1["status"], o2["status"])
    assert np.array_equal(o1["n_cross"], o2["n_cross"])
    np.testing.assert_allclose(o1["cross"][..., 0], o2["cross"][..., 0], rtol=1e-9)
    # y -> -y flips the azimuth; the redshift is not mirror symmetric (the
    # emitting disk rotates prograde), so it is not compared.
    np.testing.assert_allclose(o1["cross"][..., 1], -o2["cross"][..., 1], rtol=1e-9, atol=1e-12)


def test_schwarzschild_crossings_match_orbit_equation():
    """a = 0: every equatorial-crossing record (count, radius, azimuth) of the
    oracle equals the crossings of the textbook photon orbit, found by
    quadrature of (du/dpsi)^2 = 1/b^2 - u^2 + 2u^3 in the plane of the initial
    position and velocity (tests/closed_forms.py).  Rays of a 41x41 image
    over [-8, 8]^2 at 60 deg (direct, captured and once-wound rays) and a
    beta = 0 cut through the photon ring, b in [5.0, 5.6] and a finer one
    in [5.18, 5.26] (up to four crossings); rays within 2e-3 of b = sqrt(27)
    are left out (there the crossing radius changes by more than the
    tolerance per 1e-10 of b).  DOPRI5 rtol 1e-12 with the
    step cap at 0.01 r keeps the Hermite localisation error below the
    tolerances."""
    rays = [O.camera_rays(0.0, 1000.0, np.radians(60), -8, 8, -8, 8, 41, 41, pix=np.arange(0, 41 * 41, 13)),
            O.camera_rays(0.0, 1000.0, np.radians(60), 5.0, 5.6, -0.5, 0.5, 61, 1),
            O.camera_rays(0.0, 1000.0, np.radians(60), 5.18, 5.26, -0.5, 0.5, 41, 1)]
    p = O.Params(method=O.DOPRI5, k_cross=4, rtol=1e-12, atol=1e-12, hmax_coeff=0.01)
    n_checked = n_multi = 0
    for init in rays:
        out = O.integrate(init, p)
        s = init["s"]
        for i in range(s.shape[1]):
            x, v = s[1:4, i], s[5:8, i]
            L = np.linalg.norm(np.cross(x, v))
            rdot = x @ v / np.linalg.norm(x)
            u0 = 1 / np.linalg.norm(x)
            b = L / np.sqrt(rdot ** 2 + L * L * u0 * u0 * (1 - 2 * u0))
            if abs(b - np.sqrt(27.0)) < 2e-3:
                continue
            want = cf.schwarzschild_crossings(x, v, 4, 2.02, 1000.0)
            assert min(out["n_cross"][i], 4) == len(want), (i, b)
            for j, (r, ph) in enumerate(want):
                got = out["cross"][i, j]
                assert abs(got[0] - r) <= 1e-8 * r, (i, j, got[0], r)
                assert abs((got[1] - ph + np.pi) % (2 * np.pi) - np.pi) < 1e-9, (i, j)
            n_checked += 1
            n_multi += len(want) >= 3
    assert n_checked > 150 and n_multi >= 5


def test_negative_spin_is_the_mirror_image():
    """A hole of spin -a is the hole of spin a seen in a mirror: reflecting
    y -> -y maps Kerr(a) to Kerr(-a) and the camera's alpha to -alpha (the
    observer sits in the x-z plane).  So the a = -0.9 image equals the
    a = 0.9 image with its columns reversed: same statuses and crossing
    counts, final positions and crossing radii with y negated, crossing
    azimuths negated.  (The redshift is not mirrored: its emitter orbits
    about +z for either sign of the spin.)"""
    W_, H = 31, 23
    p = O.Params(method=O.DOPRI5, k_cross=2)
    cols, rows = np.meshgrid(np.arange(W_), np.arange(H))
    pix = (rows * W_ + cols).ravel()
    mir = (rows * W_ + (W_ - 1 - cols)).ravel()
    o1 = O.integrate(O.camera_rays(0.9, 1000.0, np.radians(40), -10, 10, -8, 8, W_, H, pix=pix), p)
    o2 = O.integrate(O.camera_rays(-0.9, 1000.0, np.radians(40), -10, 10, -8, 8, W_, H, pix=mir), p)
    assert np.array_equal(o1["status"], o2["status"])
    assert np.array_equal(o1["n_cross"], o2["n_cross"])
    flip = np.array([1, 1, -1, 1, 1, 1, -1, 1])[:, None]
    np.testing.assert_allclose(o1["s"] * flip, o2["s"], rtol=1e-6, atol=1e-6 * 1000)
    np.testing.assert_allclose(o1["cross"][..., 0], o2["cross"][..., 0], rtol=1e-8)
    np.testing.assert_allclose(o1["cross"][..., 1], -o2["cross"][..., 1], rtol=1e-8, atol=1e-10)
    assert np.sum(o1["status"] == O.CAPTURED) > 20


def test_redshift_formula_matches_normalised_four_velocity():
    """The Keplerian u^t in the redshift equals the normalisation of
    u = u^t (1, Omega zhat x x) in the Cartesian metric (prograde, spin +a)."""
    for a in (0.0, 0.5, 0.99):
        for r in (4.0, 6.0, 25.0):
            om = cf.omega_kepler(r, a)
            rho = np.sqrt(r * r + a * a)
            x = np.array([0.0, rho, 0.0, 0.0])
            v = np.array([1.0, 0.0, om * rho, 0.0])
            g, _ = O.metric(a, x)
            ut = 1 / np.sqrt(-(v @ g @ v))
            assert ut == pytest.approx(cf.ut_kepler(r, a), rel=1e-13)
            xi = 1.7
            assert O.redshift(r, xi, a) == pytest.approx(1 / (ut * (1 - om * xi)), rel=1e-13)


def test_crossing_redshift_uses_conserved_xi():
    """The recorded g equals the closed form at the recorded r with the photon's
    xi = -L_z/E taken from the initial data (the chart runs with spin -a)."""
    a = 0.9
    init = O.camera_rays(a, 1000.0, np.radians(60), -12, 12, -12, 12, 1024, 1024,
                         pix=np.arange(0, 1024 * 1024, 7919))
    out = O.integrate(init, O.Params(method=O.DOPRI5, k_cross=4))
    xi = -out["c0"][1] / out["c0"][0]
    n = 0
    for i in range(len(xi)):
        for j in range(min(out["n_cross"][i], 4)):
            r, g = out["cross"][i, j, 0], out["cross"][i, j, 2]
            if np.isnan(g):
                continue
            want = 1 / (cf.ut_kepler(r, a) * (1 - cf.omega_kepler(r, a) * xi[i]))
            assert g == pytest.approx(want, rel=1e-6)
            n += 1
    assert n > 50


# ---------------------------------------------------------------------------
# Time-like geodesics (Sec. 3.2).
# ---------------------------------------------------------------------------
def _circular(a, r, vz=0.0):
    om = cf.omega_kepler(r, a)
    rho = np.sqrt(r * r + a * a)
    return O.timelike([a], np.array([[rho], [0.0], [0.0]]), np.array([[0.0], [om * rho], [vz]]))


def test_circular_orbit_frequency():
    """Stable circular orbits: r stays put and the azimuthal frequency is
    Omega = 1/(r^{3/2} + a) (observer at infinity)."""
    for a, r in ((0.0, 8.0), (0.5, 6.0), (0.998, 3.0)):
        init = _circular(a, r)
        T = 2 * np.pi / cf.omega_kepler(r, a)
        p = O.Params(method=O.DOPRI5, rtol=1e-10, atol=1e-10, t_end=3 * T, r_escape=1e4)
        out = O.integrate(init, p)
        assert out["status"][0] == O.T_END
        s = out["s"][:, 0]
        assert s[0] == pytest.approx(3 * T, rel=1e-12)
        assert O.radius(a, *s[1:4]) == pytest.approx(r, rel=1e-7)
        psi = np.arctan2(s[2], s[1])
        assert abs(psi) < 1e-6  # three full turns


def test_vertical_epicyclic_frequency():
    """Sec. 3.2 / Fig. OmegaV: a = 1, nearly circular orbit with v_z = 1e-12; the
    vertical oscillation frequency matches the closed form."""
    a = 1.0
    for r in (1.3, 1.5, 3.0):
        init = _circular(a, r, vz=1e-12)
        y0 = init["s"][:, 0]
        p = O.Params(method=O.DOPRI5, rtol=1e-12, atol=1e-30, hmax_coeff=0.05, r_escape=1e4, r_h_factor=0.5)
        tr = O.trajectory(p, a, y0, max_out=20000)
        t, z = tr[:, 1], tr[:, 4]
        vz = tr[:, 8] / tr[:, 5]
        ups = np.where((z[:-1] < 0) & (z[1:] >= 0))[0]
        assert len(ups) >= 6
        # cubic Hermite zero of z(t) in each bracketing step
        tz = []
        for i in ups:
            h = t[i + 1] - t[i]
            from scipy.optimize import brentq

            def H(s):
                return ((2 * s ** 3 - 3 * s ** 2 + 1) * z[i] + (s ** 3 - 2 * s ** 2 + s) * h * vz[i]
                        + (-2 * s ** 3 + 3 * s ** 2) * z[i + 1] + (s ** 3 - s ** 2) * h * vz[i + 1])

            tz.append(t[i] + h * brentq(H, 0, 1, xtol=1e-15))
        period = (tz[-1] - tz[0]) / (len(tz) - 1)
        want = cf.omega_vertical(r, a)
        assert 2 * np.pi / period == pytest.approx(want, rel=1e-9)


def test_t_end_landing():
    a = 0.7
    init = _circular(a, 9.0, vz=0.01)
    out = O.integrate(init, O.Params(method=O.DOPRI5, t_end=1234.5, r_escape=1e4))
    assert out["status"][0] == O.T_END
    assert abs(out["s"][0, 0] - 1234.5) <= 1e-12 * 1234.5
    d = np.abs(out["c1"] - out["c0"]) / np.maximum(np.abs(out["c0"]), 1.0)
    assert d.max() < 1e-6


# ---------------------------------------------------------------------------
# Coordinate-time integration (the coordinate-time subsection of Sec. 2.2):
# the six-variable state (x^i, v^i = dx^i/dt) with t as independent variable.
# ---------------------------------------------------------------------------
def test_coordinate_time_circular_orbit_frequency():
    """In coordinate time a circular equatorial orbit keeps its radius and
    turns at exactly Omega = 1/(r^{3/2} + a) per unit t: three periods end on
    the starting azimuth (the Cartesian azimuth differs from the spheroidal
    one by a constant on a circle)."""
    for a, r in ((0.0, 8.0), (0.5, 6.0), (0.998, 3.0)):
        init = _circular(a, r)
        T = 2 * np.pi / cf.omega_kepler(r, a)
        p = O.Params(method=O.DOPRI5_T, rtol=1e-10, atol=1e-10, t_end=3 * T, r_escape=1e4)
        out = O.integrate(init, p)
        assert out["status"][0] == O.T_END
        s = out["s"][:, 0]
        assert s[0] == 3 * T  # the last step is clipped onto t_end exactly
        assert O.radius(a, *s[1:4]) == pytest.approx(r, rel=1e-7)
        assert abs(np.arctan2(s[2], s[1])) < 1e-6
        # the energy is restored exactly (it fixes k^0); L_z and mu^2 drift at the tolerance
        assert out["c1"][0, 0] == pytest.approx(out["c0"][0, 0], rel=1e-14)
        assert out["c1"][1, 0] == pytest.approx(out["c0"][1, 0], rel=1e-8)
        assert out["c1"][3, 0] == pytest.approx(out["c0"][3, 0], rel=1e-8)


def test_coordinate_time_agrees_with_affine_integration():
    """The two formulations integrate the same curve: particles landed on the
    same t_end and photons scattered to the same escape direction agree to
    the tolerance, though their step sequences differ completely."""
    a = 0.9
    # time-like: a tilted, slightly eccentric orbit
    init = _circular(a, 9.0, vz=0.02)
    pa = O.Params(method=O.DOPRI5, rtol=1e-10, atol=1e-10, t_end=700.0, r_escape=1e4)
    pt = O.Params(method=O.DOPRI5_T, rtol=1e-10, atol=1e-10, t_end=700.0, r_escape=1e4)
    oa, ot = O.integrate(init, pa), O.integrate(init, pt)
    assert oa["status"][0] == ot["status"][0] == O.T_END
    np.testing.assert_allclose(ot["s"][:4, 0], oa["s"][:4, 0], rtol=1e-7, atol=1e-7)
    np.testing.assert_allclose(ot["s"][4:, 0], oa["s"][4:, 0], rtol=1e-6, atol=1e-8)
    # null: image rays passing at a few impact parameters
    rays = O.camera_rays(a, 1000.0, np.radians(60.0), -12.0, 12.0, -12.0, 12.0, 9, 9)
    pa = O.Params(method=O.DOPRI5, rtol=1e-10, atol=1e-10)
    pt = O.Params(method=O.DOPRI5_T, rtol=1e-10, atol=1e-10)
    oa, ot = O.integrate(rays, pa), O.integrate(rays, pt)
    assert np.array_equal(oa["status"], ot["status"])
    esc = oa["status"] == O.ESCAPED
    assert esc.sum() >= 40
    da = oa["s"][5:8, esc] / np.linalg.norm(oa["s"][5:8, esc], axis=0)
    dt = ot["s"][5:8, esc] / np.linalg.norm(ot["s"][5:8, esc], axis=0)
    assert np.abs(da - dt).max() < 1e-6
    # the escaped photon's k in coordinate time is rescaled to the entry energy
    np.testing.assert_allclose(ot["c1"][0, esc], ot["c0"][0, esc], rtol=1e-13)
    np.testing.assert_allclose(ot["c1"][3, esc], 0.0, atol=1e-8)  # still null


# ---------------------------------------------------------------------------
# Dense output at coordinate times (method (ii) of Sec. 2.2).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("method", [O.DOPRI5, O.DOPRI5_T])
def test_dense_output_on_a_circular_orbit(method):
    """States at ten coordinate times of a circular equatorial orbit: each lies
    on the circle at the azimuth Omega t_j (plus the start's), with the target
    time itself in x^0; targets beyond the end stay NaN.  The states come from
    the cubic Hermite interpolant of a step, whose error on a circle is at most
    (h Omega)^4 / 384 relative: 2.3e-7 at the step cap h = 0.1 r^{3/2}, r = 7."""
    a, r = 0.5, 7.0
    init = _circular(a, r)
    om = cf.omega_kepler(r, a)
    T = 2 * np.pi / om
    bound = (0.1 * r ** 1.5 * om) ** 4 / 384
    t_out = np.linspace(0.0, 1.9 * T, 10)
    p = O.Params(method=method, rtol=1e-10, atol=1e-10, t_end=1.9 * T - 1.0, r_escape=1e4)
    out = O.integrate(init, p, t_out=t_out)
    so = out["s_out"][0]
    phi0 = np.arctan2(init["s"][2, 0], init["s"][1, 0])
    for j, tj in enumerate(t_out[:-1]):
        assert so[j, 0] == tj
        assert O.radius(a, *so[j, 1:4]) == pytest.approx(r, rel=bound)
        dphi = np.angle(np.exp(1j * (np.arctan2(so[j, 2], so[j, 1]) - phi0 - om * tj)))
        assert abs(dphi) < bound + 1e-8, j
    assert np.all(np.isnan(so[-1]))  # the last target lies past t_end


def test_dense_output_agrees_between_variables():
    """An eccentric, tilted orbit sampled at 25 times by the affine and the
    coordinate-time integration: the same states to the tolerance."""
    a = 0.8
    init = _circular(a, 12.0, vz=0.03)
    init["s"][5:8] *= 1.05
    t_out = np.linspace(5.0, 900.0, 25)
    pa = O.Params(method=O.DOPRI5, rtol=1e-10, atol=1e-10, t_end=1000.0, r_escape=1e4)
    pt = O.Params(method=O.DOPRI5_T, rtol=1e-10, atol=1e-10, t_end=1000.0, r_escape=1e4)
    sa = O.integrate(init, pa, t_out=t_out)["s_out"][0]
    st = O.integrate(init, pt, t_out=t_out)["s_out"][0]
    assert np.all(np.isfinite(sa)) and np.all(np.isfinite(st))
    # interpolation error of either side, (h / period)^4-small (see above)
    np.testing.assert_allclose(st[:, :4], sa[:, :4], rtol=1e-7, atol=5e-7)
    np.testing.assert_allclose(st[:, 4:], sa[:, 4:], rtol=1e-6, atol=1e-8)
