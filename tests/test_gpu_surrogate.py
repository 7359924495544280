"""GPU: the surrogate network's BF16-MFMA kernels against the FP64 numpy
reference, and a small end-to-end training + fallback run."""
import numpy as np
import pytest
import torch

import paper_1706_07062_amd as K
from oracle import mlp as M
from paper_1706_07062_amd import surrogate as S
from paper_1706_07062_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = K.Context(0)
    yield c
    c.close()


rng = np.random.default_rng(1706070627)


def _random_biases(p, seed):
    """Every layer's bias set to N(0, 0.3) draws (the initialisation leaves
    them zero), so the kernels' bias handling is exercised."""
    q = p.copy()
    g = np.random.default_rng(seed)
    off = 0
    for nin, nout in M.LAYERS:
        off += nin * nout
        q[off:off + nout] = g.normal(0.0, 0.3, nout)
        off += nout
    return q


def _batch(n):
    x = np.stack([rng.uniform(-12, 12, n), rng.uniform(-12, 12, n), rng.uniform(0, 0.998, n),
                  np.radians(rng.uniform(5, 85, n))], axis=1).astype(np.float32)
    t = np.stack([rng.normal(size=n), rng.normal(size=n), rng.normal(size=n), (rng.random(n) < 0.3) * 1.0],
                 axis=1).astype(np.float32)
    mask = rng.integers(0, 4, n).astype(np.uint8)
    return x, t, mask


def test_forward_matches_reference(ctx):
    """Raw outputs for 1000 rays (31 full waves and a ragged one), with
    nonzero biases in every layer, equal the FP64 reference with BF16 storage
    of weights and activations, to the FP32 accumulation-order level."""
    say("mlp forward")
    p = _random_biases(S.init_params(11), 21)
    net = K.Mlp(p, train=False)
    ctx.kh_mlp_sync(net)
    x, _, _ = _batch(1000)
    y = torch.empty((1000, 4), dtype=torch.float32, device="cuda")
    ctx.kh_mlp_forward(net, torch.from_numpy(x).cuda(), y)
    got = y.cpu().numpy()
    want, _ = M.forward(p.astype(np.float64), x.astype(np.float64), bf16_storage=True)
    err = np.abs(got - want).max() / np.abs(want).max()
    col = np.abs(got - want).max(axis=0) / np.abs(want).max(axis=0)
    say(f"  max abs err / max |y| = {err:.2e}; per output {np.array2string(col, precision=2)}")
    assert err < 2e-2
    # and the plain FP64 network is close too (BF16 storage costs ~1e-2)
    plain, _ = M.forward(p.astype(np.float64), x.astype(np.float64))
    assert np.abs(got - plain).max() / np.abs(plain).max() < 5e-2


def test_gradient_matches_reference(ctx):
    """kh_mlp_grad on a 512-ray batch against the FP64 reference gradient
    (BF16 storage of weights and activations; the GPU also stores the
    back-propagated errors as BF16)."""
    say("mlp gradient")
    p = _random_biases(S.init_params(12) * 0.7, 23)
    net = K.Mlp(p, train=True)
    ctx.kh_mlp_sync(net)
    x, t, mask = _batch(512)
    work = torch.empty(K.kh_mlp_work_bytes(512), dtype=torch.uint8, device="cuda")
    grad = torch.empty(K.MLP_NPARAMS, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ctx.kh_mlp_grad(net, work, 512, torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(),
                    torch.from_numpy(mask).cuda(), 512, grad, loss)
    g = grad.cpu().numpy().astype(np.float64)
    lw, gw = M.loss_and_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64), mask,
                             bf16_storage=True)
    rel = np.linalg.norm(g - gw) / np.linalg.norm(gw)
    cos = g @ gw / (np.linalg.norm(g) * np.linalg.norm(gw))
    say(f"  loss {loss.item():.6f} vs {lw:.6f}; grad rel err {rel:.2e}, cosine {cos:.6f}")
    assert loss.item() == pytest.approx(lw, rel=1e-2)
    assert rel < 3e-2 and cos > 0.9995
    # every layer's weight and bias block agrees in direction
    off = 0
    for nin, nout in M.LAYERS:
        for size in (nin * nout, nout):
            a, b = g[off:off + size], gw[off:off + size]
            say(f"  block {nin}x{nout} size {size}: max |dg| / max |g| = "
                f"{np.abs(a - b).max() / max(np.abs(b).max(), 1e-300):.2e}, "
                f"max |dg| / (|g| + max|g|/10) = {np.max(np.abs(a - b) / (np.abs(b) + 0.1 * np.abs(b).max())):.2e}")
            if np.linalg.norm(b) > 0:
                assert a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300) > 0.995, (nin, nout, size)
            off += size


def test_image_kernel_decodes_forward_and_lists_fallback(ctx):
    """The camera-image kernel on a ragged 37x23 camera (6 full blocks of 128
    rays + 83): its decoded outputs equal the forward kernel's raw outputs,
    decoded on the host, on the same pixel features; they match the FP64
    reference with BF16 storage; and the fallback list is exactly the set of
    pixels whose capture probability lies in (tau, 1 - tau), in any order."""
    say("mlp image kernel")
    p = _random_biases(S.init_params(12), 22)
    net = K.Mlp(p, train=False)
    ctx.kh_mlp_sync(net)
    cam = W.Camera(0.9, 1000.0, 45.0, -12.0, 12.0, -9.0, 9.0, 37, 23)
    n = cam.n
    col, row = np.arange(n) % cam.width, np.arange(n) // cam.width
    al = cam.alpha_min + (col + 0.5) * (cam.alpha_max - cam.alpha_min) / cam.width
    be = cam.beta_min + (row + 0.5) * (cam.beta_max - cam.beta_min) / cam.height
    x = np.stack([al, be, np.full(n, cam.a), np.full(n, cam.incl)], axis=1).astype(np.float32)
    raw = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    ctx.kh_mlp_forward(net, torch.from_numpy(x).cuda(), raw)
    raw = raw.cpu().numpy().astype(np.float64)
    for tau in (0.2, 0.45, 0.0):
        out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
        ids = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
        ctx.kh_mlp_image(net, S.camera_struct(cam), tau, out, ids, cnt)
        img = out.cpu().numpy().astype(np.float64)
        dec = np.stack([np.exp(2 * raw[:, 0] + 2), np.pi * raw[:, 1], 0.3 * raw[:, 2] + 0.8,
                        1 / (1 + np.exp(-raw[:, 3]))], axis=1)
        np.testing.assert_allclose(img, dec, rtol=2e-6, atol=2e-6)
        k = int(cnt.item())
        listed = np.sort(ids.cpu().numpy()[:k])
        pc = img[:, 3]
        want = np.nonzero((pc > tau) & (pc < 1 - tau))[0]
        say(f"  tau {tau}: {k} fallback pixels")
        assert np.array_equal(listed, want)
    ref, _ = M.forward(p.astype(np.float64), x.astype(np.float64), bf16_storage=True)
    assert np.abs(raw - ref).max() / np.abs(ref).max() < 2e-2


def test_image_kernel_full_size_sampled(ctx):
    """The image kernel at the inference size the benchmark renders (the
    4096x4096 camera at a = 0.9, 45 deg): 4,096 pixels spread over the image
    match the FP64 reference network with BF16 storage, decoded; and the
    fallback list holds exactly the pixels whose capture probability lies in
    (tau, 1 - tau), each once."""
    say("mlp image kernel, 4096^2")
    p = _random_biases(S.init_params(14), 24)
    net = K.Mlp(p, train=False)
    ctx.kh_mlp_sync(net)
    cam = W.surrogate_eval_camera()
    n = cam.n
    tau = 0.05
    out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    ids = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.kh_mlp_image(net, S.camera_struct(cam), tau, out, ids, cnt)
    torch.cuda.synchronize()
    img = out.cpu().numpy().astype(np.float64)
    assert np.isfinite(img).all()
    pix = W.strided_pixels(n, 4096, offset=17)
    col, row = pix % cam.width, pix // cam.width
    al = cam.alpha_min + (col + 0.5) * (cam.alpha_max - cam.alpha_min) / cam.width
    be = cam.beta_min + (row + 0.5) * (cam.beta_max - cam.beta_min) / cam.height
    x = np.stack([al, be, np.full(len(pix), cam.a), np.full(len(pix), cam.incl)], axis=1).astype(np.float32)
    ref, _ = M.forward(p.astype(np.float64), x.astype(np.float64), bf16_storage=True)
    # compare in the raw (pre-decode) outputs: invert the decode of the kernel
    got = img[pix]
    raw = np.stack([(np.log(got[:, 0]) - 2) / 2, got[:, 1] / np.pi, (got[:, 2] - 0.8) / 0.3,
                    np.log(got[:, 3] / (1 - got[:, 3]))], axis=1)
    err = np.abs(raw - ref).max() / np.abs(ref).max()
    say(f"  sampled raw-output error / max |y| = {err:.2e}")
    assert err < 2e-2
    pc = img[:, 3]
    # a second threshold that lists about half of the image
    tau2 = float(np.quantile(np.minimum(pc, 1 - pc), 0.5))
    for t_, first in ((tau, True), (tau2, False)):
        if not first:
            ids.fill_(-1)
            cnt.zero_()
            ctx.kh_mlp_image(net, S.camera_struct(cam), t_, out, ids, cnt)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), img.astype(np.float32))
        k = int(cnt.item())
        listed = ids.cpu().numpy()[:k]
        want = np.nonzero((pc > t_) & (pc < 1 - t_))[0]
        say(f"  tau {t_:.4f}: {k} fallback pixels of {n}")
        assert len(np.unique(listed)) == k
        assert np.array_equal(np.sort(listed), want)


def test_pixel_init_targets_and_image_from_state(ctx):
    """The surrogate pipeline's data calls on a ragged 23x19 camera:
    kh_init_rays_pixels gives bitwise the kh_init_rays states of the listed
    pixels; after integration, kh_image_from_state (in place and scattered
    through a pixel list) and kh_mlp_targets equal their definitions
    evaluated on the host from the state (first crossing, capture flag,
    normalised targets, validity mask); kh_stats_device equals kh_stats."""
    say("pixel init, targets, image from state")
    cam = W.Camera(0.9, 1000.0, 45.0, -12.0, 12.0, -9.0, 9.0, 23, 19)
    n = cam.n
    kc = S.camera_struct(cam)
    st = K.State(n, k_cross=1)
    ctx.kh_init_rays([kc], st)
    init_s = st.s.cpu().numpy()
    pix = np.random.default_rng(5).permutation(n)[:200].astype(np.int32)
    sp = K.State(len(pix), k_cross=1)
    ctx.kh_init_rays_pixels(kc, torch.from_numpy(pix).cuda(), sp)
    assert np.array_equal(sp.s.cpu().numpy(), init_s[:, pix])
    ctx.kh_integrate(K.kh_default_params(k_cross=1), st)
    torch.cuda.synchronize()
    g = st.numpy()
    cross = g["n_cross"] > 0
    c0 = g["cross"][:, 0, :]
    want_img = np.stack([np.where(cross, c0[:, 0], np.nan), np.where(cross, c0[:, 1], np.nan),
                         np.where(cross, c0[:, 2], np.nan), (g["status"] == K.CAPTURED) * 1.0],
                        axis=1).astype(np.float32)
    out = torch.full((n, 4), -1.0, dtype=torch.float32, device="cuda")
    ctx.kh_image_from_state(st, None, out)
    assert np.array_equal(out.cpu().numpy(), want_img, equal_nan=True)
    # scattered: state entry i goes to pixel rev[i]
    rev = np.arange(n)[::-1].astype(np.int32).copy()
    out2 = torch.full((n, 4), -1.0, dtype=torch.float32, device="cuda")
    ctx.kh_image_from_state(st, torch.from_numpy(rev).cuda(), out2)
    assert np.array_equal(out2.cpu().numpy()[rev], want_img, equal_nan=True)
    # training targets
    col, row = np.arange(n) % cam.width, np.arange(n) // cam.width
    al = cam.alpha_min + (col + 0.5) * (cam.alpha_max - cam.alpha_min) / cam.width
    be = cam.beta_min + (row + 0.5) * (cam.beta_max - cam.beta_min) / cam.height
    f64 = dict(dtype=torch.float64, device="cuda")
    x = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    t = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    mask = torch.empty(n, dtype=torch.uint8, device="cuda")
    ctx.kh_mlp_targets(st, torch.from_numpy(al).to(**f64), torch.from_numpy(be).to(**f64),
                       torch.full((n,), cam.a, **f64), torch.full((n,), cam.incl, **f64), x, t, mask)
    want_x = np.stack([al, be, np.full(n, cam.a), np.full(n, cam.incl)], axis=1).astype(np.float32)
    assert np.array_equal(x.cpu().numpy(), want_x)
    r, ph, gg = c0[:, 0], c0[:, 1], c0[:, 2]
    rok = cross & (np.nan_to_num(r) > 0) & np.isfinite(r) & np.isfinite(ph)
    gok = rok & np.isfinite(gg)
    with np.errstate(invalid="ignore", divide="ignore"):
        want_t = np.stack([np.where(rok, (np.log(r) - 2) * 0.5, 0), np.where(rok, ph / np.pi, 0),
                           np.where(gok, (gg - 0.8) / 0.3, 0), (g["status"] == K.CAPTURED) * 1.0], axis=1)
    np.testing.assert_allclose(t.cpu().numpy(), want_t.astype(np.float32), rtol=1e-6, atol=1e-7)
    assert np.array_equal(mask.cpu().numpy(), (rok * 1 + gok * 2).astype(np.uint8))
    say(f"  {int(rok.sum())} rays with a crossing, {int(gok.sum())} with a finite redshift, "
        f"{int((g['status'] == K.CAPTURED).sum())} captured")
    assert rok.sum() > n // 4 and (g["status"] == K.CAPTURED).sum() > 0
    dev = torch.zeros(8, dtype=torch.int64, device="cuda")
    ctx.kh_stats_device(st, dev)
    host = ctx.kh_stats(st)
    assert dev.cpu().tolist() == host["status_counts"] + [host["n_acc"], host["n_rej"]]


def test_forward_single_ray_and_one_past_a_block(ctx):
    p = _random_biases(S.init_params(13), 25)
    net = K.Mlp(p, train=False)
    ctx.kh_mlp_sync(net)
    x, _, _ = _batch(129)
    full = torch.empty((129, 4), dtype=torch.float32, device="cuda")
    ctx.kh_mlp_forward(net, torch.from_numpy(x).cuda(), full)
    for m in (1, 128, 129):
        y = torch.full((m, 4), float("nan"), dtype=torch.float32, device="cuda")
        ctx.kh_mlp_forward(net, torch.from_numpy(x[:m].copy()).cuda(), y)
        assert torch.equal(y, full[:m])


def test_training_and_fallback_image(ctx):
    """Train on 2^18 integrated rays for 600 steps, then render a 256x256 image
    at a = 0.9, i = 45 deg: the loss falls, the fallback integrates a minority
    of pixels, and the merged image's capture map matches the integrator's."""
    say("surrogate small end-to-end")
    sur = S.Surrogate(ctx, seed=1, max_batch=4096)
    x, t, mask, t_data = sur.make_data(1 << 18)
    m = mask.cpu().numpy()
    assert (m & 1).mean() > 0.5
    hist = sur.train(x, t, mask, steps=600, batch=4096, lr=2e-3, log_every=100)
    say(f"  data {t_data:.2f} s; loss history {[round(v, 4) for _, v in hist]}")
    assert hist[-1][1] < 0.5 * hist[0][1]
    cam = W.surrogate_eval_camera(side=256)
    ref, _ = S.integrate_image(ctx, cam)
    img, tm = sur.render(cam, tau=0.02)
    err = S.image_error(img, ref)
    say(f"  fallback fraction {tm['fallback_fraction']:.3f}; error {err}")
    assert tm["fallback_fraction"] < 0.6
    assert err["capture_mismatch"] < 0.02
