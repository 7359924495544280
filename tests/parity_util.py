"""Helpers shared by the GPU parity tests: run the library through its C ABI,
run the oracle on the same seeded inputs, and compare.

Tolerance policy (the a = 0.99 image target): final positions agree to 1e-6
relative and statuses are identical, except for rays the oracle itself flags as
ill-conditioned: the oracle re-integrates each ray with alpha and beta moved by
1e-12 (relative); if the two oracle runs differ by more than 1e-7 (relative) in
final position or in status, the ray winds near the photon shell, where
round-off is amplified ~e^{2 pi} per orbit, and the comparison is not decidable.
"""
from __future__ import annotations

import numpy as np
import torch

import oracle as O
import paper_1706_07062_amd as K

POS_TOL = 1e-6
ILL_TOL = 1e-7
PERTURB = 1e-12


def kcam(cam):
    return K.kh_camera(cam.a, cam.r_obs, cam.incl, cam.alpha_min, cam.alpha_max, cam.beta_min, cam.beta_max,
                       cam.width, cam.height)


def oracle_params(p: "K.kh_params") -> O.Params:
    return O.Params(method=p.method, k_cross=p.k_cross, h_coeff=p.h_coeff, rtol=p.rtol, atol=p.atol,
                    hmax_coeff=p.hmax_coeff, r_h_factor=p.r_h_factor, r_escape=p.r_escape, t_end=p.t_end,
                    max_steps=p.max_steps)


def gpu_image(ctx, cams, params, k_cross=0):
    n = sum(c.n for c in cams)
    st = K.State(n, k_cross=k_cross)
    ctx.kh_init_rays([kcam(c) for c in cams], st)
    ctx.kh_integrate(params, st)
    torch.cuda.synchronize()
    return st


def oracle_image(cam, params: O.Params, pix=None, conditioning=True):
    init = O.camera_rays(cam.a, cam.r_obs, cam.incl, cam.alpha_min, cam.alpha_max, cam.beta_min, cam.beta_max,
                         cam.width, cam.height, pix=pix)
    out = O.integrate(init, params)
    if conditioning:
        initp = O.camera_rays(cam.a, cam.r_obs, cam.incl, cam.alpha_min, cam.alpha_max, cam.beta_min, cam.beta_max,
                              cam.width, cam.height, pix=pix, perturb=PERTURB)
        outp = O.integrate(initp, params)
        d = rel_pos(out["s"], outp["s"])
        out["ill"] = (d > ILL_TOL) | (out["status"] != outp["status"])
    else:
        out["ill"] = np.zeros(len(out["status"]), bool)
    return out


def rel_pos(s_a, s_b):
    """Relative difference of the final spatial positions, per ray."""
    num = np.linalg.norm(s_a[1:4] - s_b[1:4], axis=0)
    den = np.linalg.norm(s_b[1:4], axis=0)
    return num / np.maximum(den, 1e-300)


def compare(g: dict, o: dict, idx=None, pos_tol=POS_TOL):
    """Compare GPU arrays g (full state, numpy) against oracle results o (for
    rays idx of g).  Returns a report dict; asserts nothing."""
    sel = slice(None) if idx is None else idx
    gs = g["s"][:, sel]
    well = ~o["ill"]
    d = rel_pos(gs, o["s"])
    st_eq = g["status"][sel] == o["status"]
    rep = dict(n=len(o["status"]), ill=int((~well).sum()), status_mismatch=int((~st_eq & well).sum()),
               max_rel_pos=float(np.max(d[well])) if well.any() else 0.0,
               n_pos_bad=int((d[well] > pos_tol).sum()))
    t_ref = np.abs(o["s"][0]) + 1.0
    rep["max_rel_t"] = float(np.max(np.abs(gs[0] - o["s"][0])[well] / t_ref[well])) if well.any() else 0.0
    kn = np.linalg.norm(o["s"][4:], axis=0)
    rep["max_rel_k"] = float(np.max((np.linalg.norm(gs[4:] - o["s"][4:], axis=0) / kn)[well])) if well.any() else 0.0
    return rep


def reduced_precision_errors(g, o, idx):
    """Step-independent errors of a reduced-precision run against FP64: status,
    first equatorial crossing (r, g; interpolated at z = 0, so independent of
    where the steps fall) and the escape direction k^i/|k|.  Final positions
    are not comparable: an escaping ray stops anywhere within its last step
    (up to 0.1 r), and different step sequences stop at different places."""
    gs, gst = g["s"][:, idx], g["status"][idx]
    agree = float(np.mean(gst == o["status"]))
    both = (g["n_cross"][idx] > 0) & (o["n_cross"] > 0)
    cr = np.abs(g["cross"][idx, 0, 0] - o["cross"][:, 0, 0])[both] / o["cross"][both, 0, 0]
    okg = both & ~np.isnan(o["cross"][:, 0, 2])
    cg = np.abs(g["cross"][idx, 0, 2] - o["cross"][:, 0, 2])[okg] / o["cross"][okg, 0, 2]
    esc = (gst == K.ESCAPED) & (o["status"] == K.ESCAPED)
    ug = gs[5:8, esc] / np.linalg.norm(gs[5:8, esc], axis=0)
    uo = o["s"][5:8, esc] / np.linalg.norm(o["s"][5:8, esc], axis=0)
    ang = np.arccos(np.clip(np.sum(ug * uo, axis=0), -1, 1))
    return dict(status_agree=agree, cross_r_median=float(np.median(cr)), cross_r_p99=float(np.quantile(cr, 0.99)),
                cross_g_median=float(np.median(cg)), escape_angle_median=float(np.median(ang)),
                escape_angle_p99=float(np.quantile(ang, 0.99)))
