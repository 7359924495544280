"""GPU results against closed forms of the Kerr geometry (not against the
oracle): the edges of the black-hole shadow on the beta = 0 line.

The rays come from the library's own initialisation (kh_init_rays_list) and
are integrated by kh_integrate in FP64; only the capture flag is read."""
import numpy as np
import pytest
import torch

import closed_forms as cf
import paper_1706_07062_amd as K

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
