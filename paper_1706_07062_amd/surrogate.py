"""Learned surrogate for the image workload, with integrator fallback.

Pipeline (all device work in the library's kernels, see include/kerrhip_mlp.h):

1. data: rays with random (alpha, beta, a, inclination) are integrated by the
   geodesic integrator (FP64 DOPRI5, one crossing slot) and turned into
   normalised targets: first equatorial crossing (log r, azimuth, redshift)
   and the capture flag;
2. training: mini-batch Adam on the BF16 matrix cores, FP32 master weights;
3. image: the network evaluates every pixel of a camera; pixels whose capture
   probability is within tau of 1/2, pixels near the camera's critical curve
   (the shadow edge, where the map is discontinuous and rays wind around the
   hole) and pixels whose predicted crossing lies deep in the potential well
   are compacted into a list, integrated, and merged back.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import (DOPRI5, P64, Context, Mlp, State, kh_adam, kh_camera, kh_default_params, kh_mlp_work_bytes)
from . import workloads as W

LAYERS = [(4, 256), (256, 256), (256, 256), (256, 256), (256, 4)]

# Weights of the (log r, phi, g, capture) loss terms for training: the image
# error that matters is the redshift's (and the capture flag, which the
# fallback band settles), so g weighs 16 and the azimuth and the capture term
# a quarter (a training sweep on the 4096^2 image at a = 0.9, 45 deg: p99 |dg|
# without fallback 1.8e-3 with unit weights, 0.93e-3 with these).
LOSS_WEIGHTS = (1.0, 0.25, 16.0, 0.25)


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights (scale sqrt(2 / fan_in)), zero biases, in the flat layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for nin, nout in LAYERS:
        parts.append(rng.normal(0.0, math.sqrt(2.0 / nin), (nout, nin)).ravel())
        parts.append(np.zeros(nout))
    return np.concatenate(parts).astype(np.float32)


def camera_struct(cam) -> kh_camera:
    return kh_camera(cam.a, cam.r_obs, cam.incl, cam.alpha_min, cam.alpha_max, cam.beta_min, cam.beta_max,
                     cam.width, cam.height)


def integrator_params():
    return kh_default_params(method=DOPRI5, precision=P64, k_cross=1)


class Surrogate:
    def __init__(self, ctx: Context, seed: int = 0, max_batch: int = 8192):
        self.ctx = ctx
        self.net = Mlp(init_params(seed), train=True)
        ctx.kh_mlp_sync(self.net)
        self.max_batch = max_batch
        self.work = torch.empty(kh_mlp_work_bytes(max_batch), dtype=torch.uint8, device="cuda")
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.step = 0

    # ------------------------------------------------------------------ data
    def make_data(self, n: int, seed: int = W.SEED_SURROGATE, chunk: int = 1 << 21, params=None):
        """Integrate n random rays and return device tensors x [n][4], t [n][4],
        mask [n] plus the integration time."""
        rays = W.surrogate_rays(n, seed)
        dev = {k: torch.from_numpy(rays[k]).cuda() for k in ("alpha", "beta", "a", "incl")}
        x = torch.empty((n, 4), dtype=torch.float32, device="cuda")
        t = torch.empty((n, 4), dtype=torch.float32, device="cuda")
        mask = torch.empty(n, dtype=torch.uint8, device="cuda")
        p = params or integrator_params()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(0, n, chunk):
            e = min(n, s + chunk)
            st = State(e - s, k_cross=1, constants=False)
            sl = {k: v[s:e] for k, v in dev.items()}
            self.ctx.kh_init_rays_list(sl["a"], sl["incl"], sl["alpha"], sl["beta"], 1000.0, st)
            self.ctx.kh_integrate(p, st)
            self.ctx.kh_mlp_targets(st, sl["alpha"], sl["beta"], sl["a"], sl["incl"], x[s:e], t[s:e], mask[s:e])
        torch.cuda.synchronize()
        return x, t, mask, time.perf_counter() - t0

    # -------------------------------------------------------------- training
    def train(self, x, t, mask, steps: int, batch: int = 8192, lr: float = 2e-3, lr_min: float = 5e-5, log=None,
              log_every: int = 500, loss_w=None):
        """Adam with a cosine learning-rate decay; batches are consecutive slices
        of the (already random) data, wrapping around.  loss_w: weights of the
        (r, phi, g, capture) loss terms (None: all 1)."""
        n = x.shape[0]
        batch = min(batch, self.max_batch)
        nb = n // batch
        if nb < 1:
            raise ValueError("need at least one full batch")
        hist = []
        self.loss.zero_()
        for i in range(steps):
            j = (self.step + i) % nb
            s = j * batch
            lr_i = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * i / max(steps - 1, 1)))
            opt = kh_adam(lr_i, 0.9, 0.999, 1e-8, self.step + i + 1)
            self.ctx.kh_mlp_train_step(self.net, self.work, self.max_batch, x[s:s + batch], t[s:s + batch],
                                       mask[s:s + batch], batch, opt, self.loss, loss_w=loss_w)
            if (i + 1) % log_every == 0 or i + 1 == steps:
                v = float(self.loss.item()) / log_every if (i + 1) % log_every == 0 else float(self.loss.item()) / (
                    (i + 1) % log_every)
                hist.append((i + 1, v))
                self.loss.zero_()
                if log:
                    log(f"surrogate step {i + 1}/{steps}: loss {v:.5f}")
        self.step += steps
        return hist

    # ----------------------------------------------------------------- image
    def image(self, cam, tau: float, shadow_band: float = 0.0, r_min: float = 0.0):
        npix = cam.width * cam.height
        out = torch.empty((npix, 4), dtype=torch.float32, device="cuda")
        ids = torch.empty(npix, dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.ctx.kh_mlp_image(self.net, camera_struct(cam), tau, out, ids, cnt, shadow_band=shadow_band, r_min=r_min)
        return out, ids, cnt

    def render(self, cam, tau: float, params=None, shadow_band: float = 0.0, r_min: float = 0.0):
        """Surrogate image with the pixels the fallback rules select (capture
        band tau, shadow-edge band, strong-field radius) integrated.  Returns
        the image [npix][4] = (r, phi, g, captured or p) and a timing dict."""
        p = params or integrator_params()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out, ids, cnt = self.image(cam, tau, shadow_band, r_min)
        n_fb = int(cnt.item())  # one 4-byte read-back sizes the fallback launch
        t1 = time.perf_counter()
        if n_fb > 0:
            st = State(n_fb, k_cross=1, constants=False)
            pix = ids[:n_fb]
            self.ctx.kh_init_rays_pixels(camera_struct(cam), pix, st)
            self.ctx.kh_integrate(p, st)
            self.ctx.kh_image_from_state(st, pix, out)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return out, dict(mlp_s=t1 - t0, fallback_s=t2 - t1, total_s=t2 - t0, n_fallback=n_fb,
                         fallback_fraction=n_fb / (cam.width * cam.height))


    def audit(self, cam, img, n: int, seed: int = 0, params=None):
        """The integrator judging a rendered image without a full reference:
        n pixels drawn uniformly (seeded) are integrated and compared with the
        image, pixels that went to the fallback included (there the error is
        zero, as in the full comparison).  Returns the estimated image error
        (image_error's fields on the sample), the audit's run time and n."""
        p = params or integrator_params()
        npix = cam.width * cam.height
        n = min(int(n), npix)
        pix = np.sort(np.random.default_rng(seed).choice(npix, n, replace=False)).astype(np.int32)
        dev = torch.from_numpy(pix).cuda()
        ref = torch.empty((n, 4), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = State(n, k_cross=1, constants=False)
        self.ctx.kh_init_rays_pixels(camera_struct(cam), dev, st)
        self.ctx.kh_integrate(p, st)
        self.ctx.kh_image_from_state(st, None, ref)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        est = image_error(img[dev.long()], ref)
        return dict(est, audit_rays=n, audit_s=dt)


def integrate_image(ctx: Context, cam, params=None):
    """The integrator's image of a camera in the surrogate's format, and its time."""
    p = params or integrator_params()
    st = State(cam.width * cam.height, k_cross=1, constants=False)
    out = torch.empty((cam.width * cam.height, 4), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.kh_init_rays([camera_struct(cam)], st)
    ctx.kh_integrate(p, st)
    ctx.kh_image_from_state(st, None, out)
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def image_error(img, ref) -> dict:
    """Image-level error of a surrogate image against the integrator's:
    capture mismatch (surrogate p > 1/2 vs captured), and on pixels where both
    have a crossing: |delta g|, |delta r| / r, |delta phi|."""
    a = img.cpu().numpy()
    b = ref.cpu().numpy()
    cap_a = a[:, 3] > 0.5
    cap_b = b[:, 3] > 0.5
    both = np.isfinite(b[:, 0]) & np.isfinite(a[:, 0]) & ~cap_b
    bothg = both & np.isfinite(b[:, 2]) & np.isfinite(a[:, 2])
    dg = np.abs(a[bothg, 2] - b[bothg, 2])
    dr = np.abs(a[both, 0] - b[both, 0]) / b[both, 0]
    dphi = np.abs(a[both, 1] - b[both, 1])
    q = lambda v, p: float(np.quantile(v, p)) if len(v) else float("nan")  # noqa: E731
    return dict(capture_mismatch=float(np.mean(cap_a != cap_b)), g_abs_median=q(dg, 0.5), g_abs_p99=q(dg, 0.99),
                r_rel_median=q(dr, 0.5), r_rel_p99=q(dr, 0.99), phi_abs_median=q(dphi, 0.5),
                phi_abs_p99=q(dphi, 0.99), pixels_compared=int(bothg.sum()))
