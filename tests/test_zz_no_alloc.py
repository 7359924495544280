"""GPU: kh_integrate_noalloc, the entry point for callers that cannot
allocate (static work-queue counters, no context), gives bitwise the results
of kh_integrate on the same states: two calls in a row, the second on a
smaller state, so the shared counters must be cleared between calls; a
paused-and-resumed run; and its argument errors, which come before any
launch."""
import numpy as np
import pytest
import torch

import paper_1706_07062_amd as K
from paper_1706_07062_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("s", "h", "lam", "phi", "status", "n_acc", "n_rej", "cross", "n_cross", "c0", "c1")


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)


def kcam(cam):
    return K.kh_camera(cam.a, cam.r_obs, cam.incl, cam.alpha_min, cam.alpha_max, cam.beta_min, cam.beta_max,
                       cam.width, cam.height)


def assert_same(a, b, what):
    for f in FIELDS:
        x, y = a[f], b[f]
        assert x.shape == y.shape, (what, f)
        assert np.array_equal(x, y, equal_nan=np.issubdtype(x.dtype, np.floating)), (what, f)


def test_noalloc_equals_integrate_on_two_calls_and_a_resume():
    torch.cuda.set_device(0)
    ctx = K.Context(0)
    try:
        p = K.kh_default_params(k_cross=4)
        # 96^2 = 9,216 rays (144 tiles), then 37 x 23 = 851 rays (a ragged tile)
        for cam in (W.kerr_image(60.0, side=96), W.Camera(0.99, 1000.0, 17.0, -12.0, 12.0, -9.0, 9.0, 37, 23)):
            say(f"noalloc vs kh_integrate: {cam.width}x{cam.height} at {cam.incl_deg} deg")
            ref = K.State(cam.n, k_cross=4)
            ctx.kh_init_rays([kcam(cam)], ref)
            ctx.kh_integrate(p, ref)
            got = K.State(cam.n, k_cross=4)
            ctx.kh_init_rays([kcam(cam)], got)
            K.kh_integrate_noalloc(p, got)
            torch.cuda.synchronize()
            a, b = ref.numpy(), got.numpy()
            assert (b["status"] != K.ACTIVE).all()
            assert_same(a, b, f"{cam.width}x{cam.height}")
        # a run paused after 40 accepted steps and resumed by the other entry point
        cam = W.kerr_image(17.0, side=48)
        say("noalloc: paused and resumed run")
        ref = K.State(cam.n, k_cross=4)
        ctx.kh_init_rays([kcam(cam)], ref)
        ctx.kh_integrate(p, ref)
        got = K.State(cam.n, k_cross=4)
        ctx.kh_init_rays([kcam(cam)], got)
        K.kh_integrate_noalloc(K.kh_default_params(k_cross=4, max_steps=40), got)
        torch.cuda.synchronize()
        assert (got.status == K.MAX_STEPS).any()
        K.kh_integrate_noalloc(p, got)
        torch.cuda.synchronize()
        assert_same(ref.numpy(), got.numpy(), "resumed")
    finally:
        ctx.close()


def test_noalloc_two_queue_mixed_split_equals_integrate():
    """The two-queue mixed policy enqueues two launches, each clearing the
    shared counters first: the allocation-free entry point gives bitwise the
    context entry point's results."""
    torch.cuda.set_device(0)
    ctx = K.Context(0)
    try:
        p = K.kh_default_params(k_cross=4, precision=K.PMIXED, mixed_split=1)
        cam = W.kerr_image(17.0, side=64)
        say("noalloc vs kh_integrate: two-queue mixed split, 64x64")
        ref = K.State(cam.n, k_cross=4)
        ctx.kh_init_rays([kcam(cam)], ref)
        ctx.kh_integrate(p, ref)
        got = K.State(cam.n, k_cross=4)
        ctx.kh_init_rays([kcam(cam)], got)
        K.kh_integrate_noalloc(p, got)
        torch.cuda.synchronize()
        assert (got.status == K.CAPTURED).sum() > 100
        assert_same(ref.numpy(), got.numpy(), "split")
    finally:
        ctx.close()


def test_noalloc_argument_errors():
    torch.cuda.set_device(0)
    st = K.State(128, k_cross=4)
    for bad, what in ((dict(rtol=0.0), "rtol"), (dict(queue_parts=9), "queue_parts"),
                      (dict(k_cross=5), "k_cross")):
        p = K.kh_default_params(k_cross=4)
        for name, value in bad.items():
            setattr(p, name, value)
        with pytest.raises(K.KerrHipError) as e:
            K.kh_integrate_noalloc(p, st)
        say(f"noalloc refuses {what}: {e.value}")
        assert "(-1)" in str(e.value) or "(-3)" in str(e.value)
    # nothing was launched: the state is untouched
    assert (st.n_acc == 0).all() and (st.status == 0).all()
