"""GPU parity of the fixed-step RK4 kernel of the chart / data-layout
comparison (Sec. 4, tab:elapse): Cartesian Kerr-Schild and Boyer-Lindquist
states, structure-of-arrays and array-of-structures, FP64 and FP32, through
the C ABI (kh_pack_fixed, kh_rk4_fixed) against the oracle's fixed-step RK4
on the same seeded camera.

Tolerance policy as for the adaptive integrator: identical statuses and step
counts, final positions within 1e-6 relative (Boyer-Lindquist: r relative,
theta and phi absolute), except on rays the oracle itself flags as
ill-conditioned (a 1e-12 relative move of alpha and beta changes its own
result by more than 1e-7 or changes the status)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import paper_1706_07062_amd as K
from paper_1706_07062_amd import workloads as W
from parity_util import kcam

pytestmark = pytest.mark.gpu

POS_TOL = 1e-6
ILL_TOL = 1e-7
CHARTS = {K.RHS_FACTORED: "ks", K.RHS_PAPER: "ks", K.RHS_BL: "bl"}


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = K.Context(0)
    yield c
    c.close()


def _small_camera():
    return W.Camera(0.999, 1024.0, 60.0, -12.0, 12.0, -12.0, 12.0, 37, 23)  # 851 rays: 3 blocks + 83


def _r_stop(a):
    return 1.01 * (1 + np.sqrt(1 - a * a))


def _gpu_start(ctx, cam, params):
    st = K.State(cam.n, constants=False)
    ctx.kh_init_rays([kcam(cam)], st)
    return K.FixedState(ctx, params, st.s, st.status)


def _gpu_run(ctx, fs, params, per_call=300, max_calls=40):
    p = K.kh_fixed_params.from_buffer_copy(params)
    p.nsteps = per_call
    for _ in range(max_calls):
        ctx.kh_rk4_fixed(p, fs.y, fs.status, fs.steps)
        if not bool((fs.status == K.ACTIVE).any()):
            break
    torch.cuda.synchronize()
    return fs.components().double().cpu().numpy(), fs.status.cpu().numpy(), fs.steps.cpu().numpy()


def _oracle_start(cam, chart, perturb=0.0, pix=None):
    init = O.camera_rays(cam.a, cam.r_obs, cam.incl, cam.alpha_min, cam.alpha_max, cam.beta_min, cam.beta_max,
                         cam.width, cam.height, pix=pix, perturb=perturb)
    assert np.all(init["status"] == O.ACTIVE)
    s = init["s"]
    return s if chart == "ks" else O.ks_to_bl(-cam.a, s)


def _chart_pos_err(chart, s, ref):
    """Per-ray position difference: Cartesian relative norm, or for
    Boyer-Lindquist max(|dr| / r, |dtheta|, |dphi| / (1 + |phi|))."""
    if chart == "ks":
        return np.linalg.norm(s[1:4] - ref[1:4], axis=0) / np.linalg.norm(ref[1:4], axis=0)
    return np.maximum.reduce([np.abs(s[1] - ref[1]) / ref[1], np.abs(s[2] - ref[2]),
                              np.abs(s[3] - ref[3]) / (1 + np.abs(ref[3]))])


def _params(form, layout=K.SOA, precision=K.P64, cam=None, h_coeff=1 / 64):
    cam = cam or _small_camera()
    return K.fixed_params(rhs_form=form, layout=layout, precision=precision, nsteps=0, spin=-cam.a,
                          h_coeff=h_coeff, r_stop=_r_stop(cam.a), r_escape=cam.r_obs)


@pytest.mark.parametrize("form", [K.RHS_FACTORED, K.RHS_BL])
def test_pack_matches_oracle(ctx, form):
    """Kerr-Schild copy, and the Kerr-Schild -> Boyer-Lindquist map, of the
    camera's initial states, in every layout and precision."""
    cam = _small_camera()
    chart = CHARTS[form]
    say(f"pack form={form}")
    ref = _oracle_start(cam, chart)
    soa = _gpu_start(ctx, cam, _params(form, K.SOA))
    aos = _gpu_start(ctx, cam, _params(form, K.AOS))
    f32 = _gpu_start(ctx, cam, _params(form, K.AOS, K.P32))
    g = soa.components().cpu().numpy()
    assert torch.equal(soa.components(), aos.components())
    assert torch.equal(f32.components(), soa.components().float())
    scale = np.maximum(np.abs(ref).max(axis=1, keepdims=True), 1e-300)  # x^0 starts at 0
    err = np.abs(g - ref) / scale
    say(f"  max component error / component scale: {err.max():.2e}")
    assert err.max() < 1e-13


@pytest.mark.parametrize("form", [K.RHS_FACTORED, K.RHS_PAPER, K.RHS_BL])
def test_rk4_fixed_parity_fp64(ctx, form):
    cam = _small_camera()
    chart = CHARTS[form]
    params = _params(form)
    say(f"fixed-step RK4 parity form={form} ({chart}), {cam.width}x{cam.height}")
    g, gst, gsp = _gpu_run(ctx, _gpu_start(ctx, cam, params), params)
    args = (chart, -cam.a, params.h_coeff, params.r_stop, params.r_escape, 100000)
    o, ost, osp = O.rk4_fixed(*args, _oracle_start(cam, chart))
    op, opst, _ = O.rk4_fixed(*args, _oracle_start(cam, chart, perturb=1e-12))
    assert np.all(ost != O.ACTIVE) and np.all(gst != K.ACTIVE)
    # Boyer-Lindquist rays that reach the horizon's neighbourhood blow up there
    # (k^r grows like 1/Delta at a fixed step h = r / 64): the oracle ends them
    # as failed, and such rays are not compared
    failed = (ost == O.FAILED) | (opst == O.FAILED)
    ill = (_chart_pos_err(chart, op, o) > ILL_TOL) | (opst != ost) | failed
    well = ~ill
    d = _chart_pos_err(chart, g, o)
    say(f"  ill {int(ill.sum())} (failed {int(failed.sum())}), status {np.bincount(gst, minlength=6)}, "
        f"steps median {np.median(gsp):.0f} max {gsp.max()}, max pos err {d[well].max():.2e}")
    if chart == "ks":
        assert not failed.any() and ill.sum() <= 0.01 * cam.n
    assert ill.sum() <= 0.05 * cam.n
    assert np.array_equal(gst[well], ost[well])
    assert np.array_equal(gsp[well], osp[well])
    assert d[well].max() < POS_TOL


@pytest.mark.parametrize("form", [K.RHS_FACTORED, K.RHS_BL])
def test_layouts_and_resume_are_bitwise(ctx, form):
    """Structure-of-arrays and array-of-structures run the same arithmetic, and
    a run split over calls equals one call."""
    cam = _small_camera()
    say(f"layouts and resume form={form}")
    for prec in (K.P64, K.P32):
        res = []
        for layout in (K.SOA, K.AOS):
            params = _params(form, layout, prec)
            res.append(_gpu_run(ctx, _gpu_start(ctx, cam, params), params, per_call=500, max_calls=1))
        for a, b in zip(res[0], res[1]):
            assert np.array_equal(a, b, equal_nan=True)
        params = _params(form, K.SOA, prec)
        fs = _gpu_start(ctx, cam, params)
        _gpu_run(ctx, fs, params, per_call=200, max_calls=1)
        split = _gpu_run(ctx, fs, params, per_call=300, max_calls=1)
        for a, b in zip(split, res[0]):
            assert np.array_equal(a, b, equal_nan=True)


@pytest.mark.parametrize("form", [K.RHS_FACTORED, K.RHS_BL])
def test_rk4_fixed_fp32_error_reported(ctx, form):
    cam = _small_camera()
    chart = CHARTS[form]
    params = _params(form, K.SOA, K.P32)
    say(f"fixed-step RK4 FP32 form={form}")
    g, gst, _ = _gpu_run(ctx, _gpu_start(ctx, cam, params), params)
    o, ost, _ = O.rk4_fixed(chart, -cam.a, params.h_coeff, params.r_stop, params.r_escape, 100000,
                            _oracle_start(cam, chart))
    agree = float(np.mean(gst == ost))
    both = (gst == ost) & (ost != O.FAILED)
    d = _chart_pos_err(chart, g, o)[both]
    say(f"  status agreement {agree:.4f}, position error median {np.median(d):.2e} p90 {np.quantile(d, 0.9):.2e}")
    assert agree > 0.97
    assert np.median(d) < 1e-3


@pytest.mark.parametrize("form", [K.RHS_FACTORED, K.RHS_BL])
def test_full_size_launch_sampled(ctx, form):
    """The benchmark launch (1024x1024 image, 1024 steps of h = r / 256) keeps
    every ray active for the whole launch; 256 sampled rays match the oracle
    in FP64 and are reported in FP32."""
    cam = W.elapse_image(1024)
    chart = CHARTS[form]
    rng = np.random.default_rng(17060706)
    pix = np.sort(rng.choice(cam.n, 256, replace=False))
    o0 = _oracle_start(cam, chart, pix=pix)
    o, ost, osp = O.rk4_fixed(chart, -cam.a, W.ELAPSE_H_COEFF, _r_stop(cam.a), cam.r_obs, W.ELAPSE_STEPS, o0)
    assert np.all(ost == O.ACTIVE) and np.all(osp == W.ELAPSE_STEPS)
    for prec, tol in ((K.P64, 1e-10), (K.P32, 1e-3)):
        say(f"full-size launch form={form} precision={prec}")
        params = _params(form, K.SOA, prec, cam=cam, h_coeff=W.ELAPSE_H_COEFF)
        fs = _gpu_start(ctx, cam, params)
        g, gst, gsp = _gpu_run(ctx, fs, params, per_call=W.ELAPSE_STEPS, max_calls=1)
        assert np.all(gst == K.ACTIVE) and np.all(gsp == W.ELAPSE_STEPS)
        d = _chart_pos_err(chart, g[:, pix], o)
        say(f"  sampled position error max {d.max():.2e} median {np.median(d):.2e}")
        assert d.max() < tol
        del fs


def test_fixed_argument_errors(ctx):
    say("fixed-step argument errors")
    cam = _small_camera()
    good = _params(K.RHS_BL)
    fs = _gpu_start(ctx, cam, good)
    for field, bad in (("rhs_form", 7), ("layout", 3), ("precision", K.PMIXED), ("nsteps", -1),
                       ("h_coeff", 0.0), ("h_coeff", float("nan")), ("spin", 1.0), ("r_stop", float("inf"))):
        p = K.kh_fixed_params.from_buffer_copy(good)
        setattr(p, field, bad)
        with pytest.raises(K.KerrHipError):
            ctx.kh_rk4_fixed(p, fs.y, fs.status, fs.steps)
    # a host pointer is refused before any launch
    host = torch.zeros(8 * cam.n, dtype=torch.float64)
    rc = K.lib().kh_rk4_fixed(ctx.handle, ctypes.byref(good), host.data_ptr(), fs.status.data_ptr(),
                              fs.steps.data_ptr(), cam.n, None)
    assert rc == K.KH_EINVAL
    # negative and oversized counts are refused from the size alone
    for n_bad in (-1, 1 << 31):
        rc = K.lib().kh_rk4_fixed(ctx.handle, ctypes.byref(good), fs.y.data_ptr(), fs.status.data_ptr(),
                                  fs.steps.data_ptr(), n_bad, None)
        assert rc == K.KH_EINVAL and b"2^31" in K.lib().kh_last_error(ctx.handle), n_bad
    # n = 0 is a no-op
    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    ctx.kh_rk4_fixed(good, torch.zeros(0, dtype=torch.float64, device="cuda"), e, e)
    torch.cuda.synchronize()
