"""GPU results against closed forms of the Kerr geometry (not against the
oracle): the edges of the black-hole shadow on the beta = 0 line, and the
equatorial crossings of Schwarzschild photons.

The rays come from the library's own initialisation (kh_init_rays_list,
kh_init_rays) and are integrated by kh_integrate in FP64."""
import numpy as np
import pytest
import torch

import closed_forms as cf
import paper_1706_07062_amd as K
from paper_1706_07062_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _capture_edge(ctx, a, incl, lo, hi, n=32768, r_obs=1e4):
    """alpha of the capture / escape transition on beta = 0 inside [lo, hi],
    sampled at n points; returns the midpoint of the transition and the
    spacing."""
    f64 = dict(dtype=torch.float64, device="cuda")
    al = torch.linspace(lo, hi, n, **f64)
    st = K.State(n, constants=False)
    ctx.kh_init_rays_list(torch.full((n,), a, **f64), torch.full((n,), incl, **f64), al, torch.zeros(n, **f64),
                          r_obs, st)
    p = K.kh_default_params(rtol=1e-10, atol=1e-10, r_escape=2 * r_obs)
    ctx.kh_integrate(p, st)
    status = st.status.cpu().numpy()
    assert np.all((status == K.CAPTURED) | (status == K.ESCAPED))
    cap = status == K.CAPTURED
    flips = np.nonzero(cap[1:] != cap[:-1])[0]
    assert len(flips) == 1, flips  # one clean transition inside the window
    alc = al.cpu().numpy()
    i = flips[0]
    return 0.5 * (alc[i] + alc[i + 1]), alc[1] - alc[0]


@pytest.mark.parametrize("a, incl_deg", [(0.0, 60.0), (0.99, 60.0), (0.99, 17.0), (0.5, 85.0)])
def test_shadow_edges_on_beta_zero_match_bardeen(a, incl_deg):
    """Bardeen's shadow boundary (spherical photon orbits projected on the
    observer's sky) crosses beta = 0 at two alpha; for a = 0 they are
    +-sqrt(27).  Rays 2e-2 wide around each edge, 32,768 per window, switch
    from escape to capture within one sample spacing of the closed form
    (the observer sits at r = 1e4, where the finite distance moves the edges
    by ~1e-9)."""
    torch.cuda.set_device(0)
    ctx = K.Context(0)
    incl = np.radians(incl_deg)
    if a == 0.0:
        edges = (-np.sqrt(27.0), np.sqrt(27.0))
    else:
        edges = cf.bardeen_beta0_edges(a, incl)
    for e in edges:
        got, d = _capture_edge(ctx, a, incl, e - 1e-2, e + 1e-2)
        say(f"  a {a} i {incl_deg}: edge {got:.8f} closed form {e:.8f} (spacing {d:.1e})")
        assert abs(got - e) <= 1.5 * d
    ctx.close()


def test_schwarzschild_crossing_records_match_orbit_equation():
    """a = 0: the GPU's equatorial-crossing records (count, radius, azimuth)
    equal the crossings of the textbook photon orbit from the quadrature of
    (du/dpsi)^2 = 1/b^2 - u^2 + 2u^3 (tests/closed_forms.py), for a 41x41
    image over [-8, 8]^2 and a beta = 0 cut through the photon ring at 60 deg;
    FP64 DOPRI5 rtol 1e-12 with the step cap at 0.01 r.  Radii to 1e-8
    relative, azimuths to 1e-9 rad; rays within 2e-3 of b = sqrt(27) are left
    out."""
    torch.cuda.set_device(0)
    ctx = K.Context(0)
    cams = [W.Camera(0.0, 1000.0, 60.0, -8.0, 8.0, -8.0, 8.0, 41, 41),
            W.Camera(0.0, 1000.0, 60.0, 5.0, 5.6, -0.5, 0.5, 61, 1),
            W.Camera(0.0, 1000.0, 60.0, 5.18, 5.26, -0.5, 0.5, 41, 1)]
    n = sum(c.n for c in cams)
    st = K.State(n, k_cross=4)
    ctx.kh_init_rays([K.kh_camera(c.a, c.r_obs, c.incl, c.alpha_min, c.alpha_max, c.beta_min, c.beta_max,
                                  c.width, c.height) for c in cams], st)
    s0 = st.s.cpu().numpy()
    p = K.kh_default_params(k_cross=4, rtol=1e-12, atol=1e-12, hmax_coeff=0.01)
    ctx.kh_integrate(p, st)
    g = st.numpy()
    counts = {}
    worst = 0.0
    for i in range(n):
        x, v = s0[1:4, i], s0[5:8, i]
        L = np.linalg.norm(np.cross(x, v))
        rdot = x @ v / np.linalg.norm(x)
        u0 = 1 / np.linalg.norm(x)
        b = L / np.sqrt(rdot ** 2 + L * L * u0 * u0 * (1 - 2 * u0))
        if abs(b - np.sqrt(27.0)) < 2e-3:
            continue
        want = cf.schwarzschild_crossings(x, v, 4, 2.02, 1000.0)
        assert min(g["n_cross"][i], 4) == len(want), (i, b)
        counts[len(want)] = counts.get(len(want), 0) + 1
        for j, (r, ph) in enumerate(want):
            got = g["cross"][i, j]
            worst = max(worst, abs(got[0] - r) / r)
            assert abs(got[0] - r) <= 1e-8 * r, (i, j, got[0], r)
            assert abs((got[1] - ph + np.pi) % (2 * np.pi) - np.pi) < 1e-9, (i, j)
    say(f"  rays by crossing count {sorted(counts.items())}, worst relative radius {worst:.1e}")
    assert counts.get(3, 0) >= 5
    ctx.close()
