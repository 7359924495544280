"""The two-queue mixed-precision policy (kh_params.mixed_split = 1) against the
FP64 oracle, against the library's other policies at the radii where it must
reduce to them exactly, and for independence of the launch shape.

Mixed precision (FP32 right-hand sides and stage sums away from the hole,
FP64 inside r_fp64, FP64 state and error norm) is not in the paper; its
errors are reported quantities (parity unpinned), so the oracle comparisons
bound them loosely and print them."""
import numpy as np
import pytest
import torch

import paper_1706_07062_amd as K
from paper_1706_07062_amd import workloads as W
from parity_util import gpu_image, kcam, oracle_image, oracle_params, reduced_precision_errors

pytestmark = pytest.mark.gpu

FIELDS = ("s", "h", "lam", "phi", "status", "n_acc", "n_rej", "cross", "n_cross", "c1")


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = K.Context(0)
    yield c
    c.close()


def _same(g, h, fields=FIELDS):
    for f in fields:
        assert np.array_equal(g[f], h[f], equal_nan=g[f].dtype.kind == "f"), f


def _mixed(**kw):
    return K.kh_default_params(precision=K.PMIXED, k_cross=4, **kw)


def test_split_with_every_ray_parked_equals_fp64(ctx):
    """r_fp64 above the camera distance parks every ray before its first
    attempt, so the FP64 pass integrates the whole image from the state the
    first pass wrote back: bitwise the FP64 run (state, step size, affine
    parameter, azimuth, crossing records, counters and constants)."""
    say("split, everything parked")
    cam = W.Camera(0.99, 1000.0, 60.0, -12, 12, -12, 12, 100, 77)
    ref = gpu_image(ctx, [cam], K.kh_default_params(k_cross=4), k_cross=4).numpy()
    g = gpu_image(ctx, [cam], _mixed(mixed_split=1, r_fp64=1e9), k_cross=4).numpy()
    _same(g, ref)


def test_split_with_no_ray_parked_equals_the_per_wave_switch(ctx):
    """r_fp64 = 0 parks nothing and switches no wave to FP64: the two policies
    run the same FP32 arithmetic, bitwise."""
    say("split, nothing parked")
    cam = W.Camera(0.99, 1000.0, 17.0, -12, 12, -12, 12, 100, 77)
    a = gpu_image(ctx, [cam], _mixed(mixed_split=0, r_fp64=0.0), k_cross=4).numpy()
    b = gpu_image(ctx, [cam], _mixed(mixed_split=1, r_fp64=0.0), k_cross=4).numpy()
    _same(a, b)


def test_split_results_do_not_depend_on_the_launch_shape(ctx):
    """With the split each ray's arithmetic is fixed by its own path (FP32 until
    it first comes inside r_fp64, FP64 after), so block size, grid, refill
    threshold, queue partitions and the tile order give bitwise identical
    results, which the per-wave switch does not promise."""
    say("split, launch shapes")
    cam = W.kerr_image(60.0, side=96)
    base = gpu_image(ctx, [cam], _mixed(mixed_split=1), k_cross=4).numpy()
    assert np.sum(base["status"] == K.CAPTURED) > 100
    for bs, gb, rf, qp, wpe in ((64, 0, 1, 1, 1), (128, 7, 64, 3, 3), (256, 1, 16, 8, 1), (192, 3, 5, 2, 3)):
        p = _mixed(mixed_split=1, block_size=bs, grid_blocks=gb, refill_min=rf, queue_parts=qp, waves_per_eu=wpe)
        g = gpu_image(ctx, [cam], p, k_cross=4).numpy()
        _same(g, base)
    # natural order instead of the longest-first tile order
    st = K.State(cam.n, k_cross=4, schedule=None)
    ctx.kh_init_rays([kcam(cam)], st)
    ctx.kh_integrate(_mixed(mixed_split=1), st)
    _same(st.numpy(), base)


@pytest.mark.parametrize("incl", [17.0, 60.0])
def test_split_error_against_the_fp64_oracle(ctx, incl):
    """A 128x128 a = 0.99 image at rtol 1e-8 under the split against the FP64
    oracle on 800 pixels: statuses, first crossing and escape direction."""
    say(f"split vs oracle incl={incl}")
    cam = W.kerr_image(incl, side=128)
    st = gpu_image(ctx, [cam], _mixed(mixed_split=1), k_cross=4)
    g = st.numpy()
    assert set(np.unique(g["status"])) <= {K.CAPTURED, K.ESCAPED}
    pix = W.strided_pixels(cam.n, 800)
    o = oracle_image(cam, oracle_params(K.kh_default_params(k_cross=4)), pix=pix, conditioning=False)
    rep = reduced_precision_errors(g, o, pix)
    say(f"  {rep}")
    assert rep["status_agree"] > 0.99
    assert rep["cross_r_median"] < 1e-6 and rep["cross_g_median"] < 1e-6
    assert rep["escape_angle_median"] < 1e-6


def test_split_coordinate_time_against_fp64(ctx):
    """Coordinate time (DOPRI5_T) under the split on a 64x64 image against the
    library's FP64 coordinate-time run: same statuses, first crossings within
    the mixed tolerance; with every ray parked the two agree to rounding (the
    parked state is written back in the affine form and read again)."""
    say("split, coordinate time")
    cam = W.kerr_image(60.0, side=64)
    ref = gpu_image(ctx, [cam], K.kh_default_params(method=K.DOPRI5_T, k_cross=4), k_cross=4).numpy()
    for r64, tol in ((3.0, 1e-5), (1e9, 1e-9)):
        g = gpu_image(ctx, [cam], _mixed(method=K.DOPRI5_T, mixed_split=1, r_fp64=r64), k_cross=4).numpy()
        agree = np.mean(g["status"] == ref["status"])
        both = (g["n_cross"] > 0) & (ref["n_cross"] > 0)
        d = np.abs(g["cross"][both, 0, 0] - ref["cross"][both, 0, 0]) / ref["cross"][both, 0, 0]
        say(f"  r_fp64={r64}: status agree {agree:.4f}, crossing r max {d.max():.2e}, median {np.median(d):.2e}")
        assert agree > 0.99 and np.median(d) < tol


def test_split_step_cap_pauses_and_resumes(ctx):
    """max_steps under the split: a ray paused by the first pass stays paused
    (KH_MAX_STEPS, not continued in FP64); a parked ray gets the cap again in
    the FP64 pass.  No internal status leaks out, and a second call finishes
    every ray.  The camera sits at r = 30, so rays reach r_fp64 = 3 within the
    cap of 30 steps."""
    say("split, step cap")
    cam = W.Camera(0.99, 30.0, 17.0, -8, 8, -8, 8, 64, 64)
    cap = 30
    st = K.State(cam.n, k_cross=4)
    ctx.kh_init_rays([kcam(cam)], st)
    ctx.kh_integrate(_mixed(mixed_split=1, max_steps=cap), st)
    g = st.numpy()
    assert set(np.unique(g["status"])) <= {K.CAPTURED, K.ESCAPED, K.MAX_STEPS}
    paused = g["status"] == K.MAX_STEPS
    assert paused.sum() > 100
    assert g["n_acc"].max() <= 2 * cap
    # a ray past the cap was parked and continued in FP64; paused rays never pass the cap twice
    assert np.any(g["n_acc"] > cap)
    stats = ctx.kh_stats(st)
    assert stats["status_counts"][K.MAX_STEPS] == int(paused.sum())
    ctx.kh_integrate(_mixed(mixed_split=1), st)
    g2 = st.numpy()
    assert set(np.unique(g2["status"])) <= {K.CAPTURED, K.ESCAPED}
    full = gpu_image(ctx, [cam], _mixed(mixed_split=1), k_cross=4).numpy()
    assert np.mean(g2["status"] == full["status"]) > 0.99


def test_split_argument_errors(ctx):
    say("split argument errors")
    st = K.State(16)
    with pytest.raises(K.KerrHipError, match="mixed_split"):
        ctx.kh_integrate(K.kh_default_params(precision=K.PMIXED, mixed_split=2), st)
    with pytest.raises(K.KerrHipError, match="mixed_split"):
        ctx.kh_integrate(K.kh_default_params(precision=K.P64, mixed_split=1), st)
    with pytest.raises(K.KerrHipError, match="DOPRI5"):
        ctx.kh_integrate(K.kh_default_params(method=K.RK4, precision=K.PMIXED, mixed_split=1), st)
