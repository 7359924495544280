#!/usr/bin/env python3
"""Benchmark: rays/s and right-hand-side evaluations/s for the a = 0.99,
1024x1024 Kerr image pair (inclinations 17 and 60 deg, observer at 1000 M,
[-12, 12]^2, adaptive DOPRI5 rtol = atol = 1e-8 in FP64, four equatorial
crossing records per ray).

One step = one pass of the whole path over both images: kh_init_rays (both
cameras, one launch) + kh_integrate (one persistent launch over 2^21 rays).
Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X vector FP64 (256 CU x 64 lanes x 2 flop x 2.4 GHz)
FP32_PEAK_TFLOPS = 157.3  # MI355X vector FP32, published (packed FP32; non-packed FMAs issue at the FP64 rate)
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# The sources the integrator kernel is compiled from (its translation unit and
# the headers it includes).
INTEGRATOR_SOURCES = ("kerrhip.hip", "internal.hpp", "ks_math.hpp", "bl_math.hpp", "steppers.hpp")


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1706_07062_amd", "csrc")
    for f in INTEGRATOR_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# From the committed rocprofv3 runs of the FP64 DOPRI5 kernel on this workload
# (profiles/k_integrate_dopri5_fp64_kerr1024.md): HBM bytes per launch
# (FETCH_SIZE, WRITE_SIZE, calibrated against a plain copy) and hardware FP64
# FLOP per launch (SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes), valid only for the
# kernel source they were taken on.
PROFILED = {"source_hash": "2567e0131d51ac69",
            "traffic_bytes": (120546.5 * 2.0 + 318639.5 * 1.0) * 1024,
            "hw_fp64_flops": 5804555000.0 * 64}


def algorithmic_flops(K, stats, n_rays, method, form):
    """Operation count of one integrate launch: per DOPRI5 attempt 6 right-hand
    sides plus the stage combinations and error norm; one extra right-hand side
    per ray for its first stage."""
    f = K.kh_flops(method, form)
    rhs = f["add"] + f["mul"] + f["div"] + f["sqrt"]
    step = f["step_add"] + f["step_mul"] + f["step_div"] + f["step_sqrt"]
    attempts = stats["n_acc"] + stats["n_rej"]
    if method in (K.DOPRI5, K.DOPRI5_T):
        n_rhs = 6 * attempts + n_rays
        flops = attempts * (6 * rhs + step) + n_rays * rhs
    else:
        n_rhs = 4 * stats["n_acc"] + n_rays
        flops = stats["n_acc"] * (4 * rhs + step) + n_rays * rhs
    return flops, n_rhs, rhs, step


# Final states of the GPU runs on the rays the CPU leg integrates with the
# oracle (filled by the GPU legs, read by cpu_baseline).
SAMPLES = {}


def headline_sample_ids(cpu_sample):
    """Ray ids (in the two-image state) of the oracle's sample: strided pixels
    of each 1024x1024 image, half of the sample each."""
    from paper_1706_07062_amd import workloads as W

    per_img = cpu_sample // 2
    return [W.strided_pixels(cam.n, per_img, offset=j) + j * cam.n for j, cam in enumerate(W.kerr_1024())]


def keep_sample(name, st, ids, **extra):
    import torch

    idx = torch.from_numpy(np.ascontiguousarray(ids, dtype=np.int64)).cuda()
    SAMPLES[name] = dict(s=st.s[:, idx].cpu().numpy(), status=st.status[idx].cpu().numpy(),
                         n_cross=st.n_cross[idx].cpu().numpy() if st.n_cross is not None else None,
                         cross=st.cross[idx].cpu().numpy() if st.cross is not None else None, **extra)


def result_errors(g, o):
    """Errors of a GPU result against the FP64 oracle on the same rays:
    status agreement; final position (relative); the first equatorial
    crossing's radius and redshift (relative; interpolated at z = 0, so they
    do not depend on where the steps fall); the direction of escape (rad).
    Final positions of reduced-precision runs are not comparable (an escaping
    ray stops anywhere within its last step), the crossing and the escape
    direction are."""
    st_eq = g["status"] == o["status"]
    out = dict(rays=int(len(st_eq)), status_agree=float(st_eq.mean()))
    d = np.linalg.norm(g["s"][1:4] - o["s"][1:4], axis=0) / np.linalg.norm(o["s"][1:4], axis=0)
    out["position_rel_median"] = float(np.median(d[st_eq]))
    out["position_within_1e-6"] = float(np.mean(d[st_eq] <= 1e-6))
    if g.get("n_cross") is not None and "n_cross" in o:
        both = (g["n_cross"] > 0) & (o["n_cross"] > 0)
        cr = np.abs(g["cross"][both, 0, 0] - o["cross"][both, 0, 0]) / o["cross"][both, 0, 0]
        okg = both & np.isfinite(o["cross"][:, 0, 2]) & np.isfinite(g["cross"][:, 0, 2])
        cg = np.abs(g["cross"][okg, 0, 2] - o["cross"][okg, 0, 2]) / o["cross"][okg, 0, 2]
        out.update(cross_count_agree=float(np.mean(g["n_cross"] == o["n_cross"])),
                   cross_r_rel_median=float(np.median(cr)), cross_r_rel_p99=float(np.quantile(cr, 0.99)),
                   cross_g_rel_median=float(np.median(cg)), cross_g_rel_p99=float(np.quantile(cg, 0.99)))
    esc = (g["status"] == 2) & (o["status"] == 2)
    ug = g["s"][5:8, esc] / np.linalg.norm(g["s"][5:8, esc], axis=0)
    uo = o["s"][5:8, esc] / np.linalg.norm(o["s"][5:8, esc], axis=0)
    ang = 2 * np.arcsin(np.clip(np.linalg.norm(ug - uo, axis=0) / 2, 0, 1))
    out.update(escape_angle_median=float(np.median(ang)), escape_angle_p99=float(np.quantile(ang, 0.99)))
    return out


def run_gpu(args):
    import torch

    import paper_1706_07062_amd as K
    from paper_1706_07062_amd import workloads as W

    torch.cuda.set_device(0)
    ctx = K.Context(0)
    cams = W.kerr_1024()
    kc = [K.kh_camera(c.a, c.r_obs, c.incl, c.alpha_min, c.alpha_max, c.beta_min, c.beta_max, c.width, c.height)
          for c in cams]
    n = sum(c.n for c in cams)
    st = K.State(n, k_cross=4)
    params = K.kh_default_params(k_cross=4)
    stream = torch.cuda.current_stream()

    def one_step():
        ctx.kh_init_rays(kc, st)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.kh_integrate(params, st)
        e1.record(stream)
        return e0, e1

    for i in range(args.warmup):
        one_step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [one_step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in evs]
    stats = ctx.kh_stats(st)
    log(f"timed {args.steps} steps: {wall:.3f} s; integrate kernel {np.mean(kern_ms):.2f} ms avg; stats {stats}")
    keep_sample("fp64", st, np.concatenate(headline_sample_ids(args.cpu_sample)))
    flops, n_rhs, rhs_f, step_f = algorithmic_flops(K, stats, n, K.DOPRI5, K.RHS_FACTORED)
    ms_step = 1e3 * wall / args.steps
    kern_s = np.mean(kern_ms) / 1e3
    tflops = flops / kern_s / 1e12
    profiled = kernel_source_hash() == PROFILED["source_hash"]
    hw_tflops = PROFILED["hw_fp64_flops"] / kern_s / 1e12 if profiled else None
    out = dict(
        metric="rays/s and RHS evals/s at a=0.99 1024^2; surrogate vs integrator at fixed error",
        value=n * args.steps / wall,
        unit="rays/s",
        n_gpus=1,
        steps=args.steps,
        warmup=args.warmup,
        ms_per_step=ms_step,
        higher_is_better=True,
        scaling="weak",
        vs_baseline=None,
        dtype="f64",
        data="synthetic",
        config={"workload": "kerr a=0.99 1024x1024 images at incl 17 and 60 deg, r_obs=1000, alpha,beta in "
                            "[-12,12], DOPRI5 rtol=atol=1e-8 FP64, 4 equatorial crossings",
                "rays_per_step": n, "parallelism": "single GPU, persistent kernel"},
        rhs_evals_per_s=n_rhs * args.steps / wall,
        useful_rhs_evals_per_s=(6 * stats["n_acc"] + n) * args.steps / wall,

        rhs_evals_per_step=n_rhs,
        accepted_steps_per_ray=stats["n_acc"] / n,
        rejected_steps_per_ray=stats["n_rej"] / n,
        integrate_kernel_ms=float(np.mean(kern_ms)),
        roofline=dict(bound="alu", achieved=tflops, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                      frac=tflops / FP64_PEAK_TFLOPS,
                      traffic=PROFILED["traffic_bytes"] if profiled else None,
                      traffic_unit="bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
                      flops_per_launch=flops, flop_per_rhs=rhs_f, flop_per_attempt_overhead=step_f,
                      hw_achieved=hw_tflops, hw_frac=(hw_tflops / FP64_PEAK_TFLOPS if hw_tflops else None),
                      hw_note="hardware-counted FP64 FLOP (FMA = 2, all lanes of issued instructions) of the "
                              "profiled build / this run's kernel time"),
    )
    # frames of the same image pair streamed: each frame's copy to page-locked
    # host memory overlaps the next frame's integration (two streams).  Taken
    # before the extras: the runtime spreads streams over a few hardware
    # queues, and once the extras have made more streams the two can share
    # one, which serialises them.
    from paper_1706_07062_amd.batched import ImageStream

    frames = 8
    ims = ImageStream(0, n, params, k_cross=params.k_cross)
    ims.run([cams] * 2, lambda *a: None)  # untimed
    t_e = time.perf_counter()
    ims.run([cams] * frames, lambda *a: None)
    e2e_s = (time.perf_counter() - t_e) / frames
    ims.close()
    out["end_to_end_streamed"] = dict(rays_per_s=n / e2e_s, ms=e2e_s * 1e3, frames=frames,
                                      includes="init + integrate of each frame on one stream, its read-back into "
                                               "page-locked host buffers on another, overlapping the next frame")
    if not args.no_extras:
        out["extras"] = extras(args, ctx, K, W, torch)
    # one more step, after everything else, end to end: init, integrate and
    # the copy of every final state and status to (pageable) host memory
    torch.cuda.synchronize()
    t_e = time.perf_counter()
    ctx.kh_init_rays(kc, st)
    ctx.kh_integrate(params, st)
    ctx.kh_read_state(st)
    e2e_s = time.perf_counter() - t_e
    out["end_to_end"] = dict(rays_per_s=n / e2e_s, ms=e2e_s * 1e3,
                             includes="kh_init_rays + kh_integrate + kh_read_state of all 2^21 states and statuses "
                                      "to pageable host memory (PCIe), one step outside the timed ones")
    # the same step into page-locked host buffers allocated beforehand
    pinned = (torch.empty((n, 8), dtype=torch.float64, pin_memory=True),
              torch.empty(n, dtype=torch.int32, pin_memory=True))
    torch.cuda.synchronize()
    t_e = time.perf_counter()
    ctx.kh_init_rays(kc, st)
    ctx.kh_integrate(params, st)
    ctx.kh_read_state(st, out=pinned)
    e2e_s = time.perf_counter() - t_e
    out["end_to_end_pinned"] = dict(rays_per_s=n / e2e_s, ms=e2e_s * 1e3,
                                    includes="as end_to_end, into page-locked host buffers allocated beforehand")
    ctx.close()
    return out, st


def PRECISION_RUNS(K):
    """(name, precision, rtol = atol, method, mixed_split) of the secondary
    precision figures on the benchmark images.  The two-queue split goes last:
    a launch that follows one of its launches directly measures several per
    cent slower."""
    return (("fp32", K.P32, 1e-6, K.DOPRI5, 0), ("mixed", K.PMIXED, 1e-8, K.DOPRI5, 0),
            ("coordinate_time_fp64", K.P64, 1e-8, K.DOPRI5_T, 0), ("mixed_split", K.PMIXED, 1e-8, K.DOPRI5, 1))


def extras(args, ctx, K, W, torch):  # noqa: C901
    """Secondary figures on the same images: FP32 and mixed precision, and the
    fixed-step RK4 time per step per ray (the paper's benchmark unit)."""
    res = {}
    cams = W.kerr_1024()
    kc = [K.kh_camera(c.a, c.r_obs, c.incl, c.alpha_min, c.alpha_max, c.beta_min, c.beta_max, c.width, c.height)
          for c in cams]
    n = sum(c.n for c in cams)
    for name, prec, tol, method, split in PRECISION_RUNS(K):
        st = K.State(n, k_cross=4)
        p = K.kh_default_params(k_cross=4, precision=prec, rtol=tol, atol=tol, method=method, mixed_split=split)
        ctx.kh_init_rays(kc, st)
        ctx.kh_integrate(p, st)
        torch.cuda.synchronize()
        ctx.kh_init_rays(kc, st)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.kh_integrate(p, st)
        e1.record()
        torch.cuda.synchronize()
        dt = e0.elapsed_time(e1) / 1e3  # HIP events on the launch's stream, as for the headline
        s = ctx.kh_stats(st)
        flops = algorithmic_flops(K, s, n, method, K.RHS_FACTORED)[0]
        tf = flops / dt / 1e12
        res[name] = dict(rays_per_s=n / dt, kernel_ms=dt * 1e3, rtol=tol,
                         rhs_evals_per_s=(6 * (s["n_acc"] + s["n_rej"]) + n) / dt, alg_tflops=tf,
                         frac_fp64_peak=tf / FP64_PEAK_TFLOPS, frac_fp32_peak=tf / FP32_PEAK_TFLOPS)
        log(f"{name}: {n / dt:.3e} rays/s, {tf:.1f} TFLOP/s")
        keep_sample(name, st, np.concatenate(headline_sample_ids(args.cpu_sample)))
    # Fixed-step RK4 (h = 0.01 r) on the paper's benchmark geometry: a = 0.999,
    # image at r = 1024 M, 1024x1024.
    cam = W.Camera(0.999, 1024.0, 60.0, -12, 12, -12, 12, 1024, 1024)
    kc1 = [K.kh_camera(cam.a, cam.r_obs, cam.incl, cam.alpha_min, cam.alpha_max, cam.beta_min, cam.beta_max,
                       cam.width, cam.height)]
    st = K.State(cam.n)
    p = K.kh_default_params(method=K.RK4, h_coeff=0.01, r_escape=1024.0)
    for prec, name in ((K.P64, "rk4_fp64"), (K.P32, "rk4_fp32")):
        p.precision = prec
        ctx.kh_init_rays(kc1, st)
        ctx.kh_integrate(p, st)
        torch.cuda.synchronize()
        ctx.kh_init_rays(kc1, st)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.kh_integrate(p, st)
        e1.record()
        torch.cuda.synchronize()
        dt = e0.elapsed_time(e1) / 1e3
        s = ctx.kh_stats(st)
        res[name] = dict(ns_per_step_per_ray=dt * 1e9 / s["n_acc"], steps=s["n_acc"], kernel_ms=dt * 1e3,
                         workload="a=0.999, 1024x1024, r_obs=1024, 60 deg, h=0.01r")
        log(f"{name}: {res[name]['ns_per_step_per_ray']:.4f} ns per RK4 step per ray")
    res["elapse_table"] = elapse_extra(ctx, K, W, torch)
    res["batched_256_images"] = batched_extra(ctx, K, W, torch)
    res["particles_2p20"] = particles_extra(ctx, K, W, torch)
    res["surrogate_4096"] = surrogate_extra(ctx, K, W, torch, args)
    return res


# Sec. 4, tab:elapse, last column (nVidia Titan Black), ns per RK4 step per ray.
PAPER_TITAN_BLACK_NS = {"fp32_bl_aos": 0.167, "fp32_bl_soa": 0.175, "fp32_ks_aos": 0.297, "fp32_ks_soa": 0.309,
                        "fp64_bl_aos": 1.65, "fp64_bl_soa": 1.66, "fp64_ks_aos": 1.15, "fp64_ks_soa": 1.15}


def elapse_extra(ctx, K, W, torch, reps=5):
    """The chart / data-layout comparison of Sec. 4 (tab:elapse) on one MI355X:
    the 1024x1024 image at r = 1024 toward a = 0.999, one launch of 1024
    fixed RK4 steps (h = r / 256) per ray, in Kerr-Schild and Boyer-Lindquist
    coordinates, array-of-structures and structure-of-arrays, FP32 and FP64.
    ns per step per ray = shortest of `reps` launches / (1024 x rays), as in
    the paper; every ray stays active for the whole launch (checked)."""
    cam = W.elapse_image(1024)
    kc = [K.kh_camera(cam.a, cam.r_obs, cam.incl, cam.alpha_min, cam.alpha_max, cam.beta_min, cam.beta_max,
                      cam.width, cam.height)]
    st = K.State(cam.n, constants=False, schedule=False)
    ctx.kh_init_rays(kc, st)
    r_stop = 1.01 * (1 + (1 - cam.a ** 2) ** 0.5)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    for prec, pname, peak in ((K.P32, "fp32", FP32_PEAK_TFLOPS), (K.P64, "fp64", FP64_PEAK_TFLOPS)):
        for form, chart in ((K.RHS_BL, "bl"), (K.RHS_FACTORED, "ks")):
            f = K.kh_flops(K.RK4, form)
            flop_step = 4 * (f["add"] + f["mul"]) + f["step_add"] + f["step_mul"]
            for layout, lname in ((K.AOS, "aos"), (K.SOA, "soa")):
                params = K.fixed_params(form, layout, prec, W.ELAPSE_STEPS, -cam.a, W.ELAPSE_H_COEFF, r_stop,
                                        cam.r_obs)
                fs = K.FixedState(ctx, params, st.s)
                y0 = fs.y.clone()
                times = []
                for _ in range(reps):
                    fs.y.copy_(y0)
                    fs.status.zero_()
                    fs.steps.zero_()
                    e0.record()
                    ctx.kh_rk4_fixed(params, fs.y, fs.status, fs.steps)
                    e1.record()
                    torch.cuda.synchronize()
                    times.append(e0.elapsed_time(e1))
                taken = int(fs.steps.sum().item())
                if taken != W.ELAPSE_STEPS * cam.n:
                    raise RuntimeError(f"elapse {pname}/{chart}/{lname}: {taken} steps, not 1024 per ray")
                ms = min(times)
                tflops = flop_step * taken / (ms * 1e-3) / 1e12
                key = f"{pname}_{chart}_{lname}"
                out[key] = dict(ns_per_step_per_ray=ms * 1e6 / taken, launch_ms=ms, alg_tflops=tflops,
                                alg_frac_fp_vector_peak=tflops / peak, flop_per_step=flop_step,
                                paper_titan_black_ns=PAPER_TITAN_BLACK_NS[key])
                log(f"elapse {key}: {ms * 1e6 / taken:.4f} ns per RK4 step per ray ({tflops:.1f} TFLOP/s)")
                del fs, y0
    out["workload"] = ("a=0.999, 1024x1024 image at r=1024 M, 60 deg, [-12,12]^2; one launch of 1024 RK4 steps "
                       "(h = r/256) per ray; shortest of 5 launches")
    out["peak_note"] = ("vector peaks FP32 157.3 (published, packed FP32) and FP64 78.6 TFLOP/s; the FP32 "
                        "kernels are built without packed FP32, whose FMAs issue at the FP64 rate, so their "
                        "arithmetic is held near 78.6; alg_frac_fp_vector_peak uses 157.3 for FP32")
    return out


def surrogate_extra(ctx, K, W, torch, args):
    """Learned surrogate: integrate 1e7 random rays (FP64 DOPRI5), train the
    BF16-MFMA network on them, then render the 4096x4096 a = 0.9, 45 deg image
    with integrator fallback under several fallback settings, against the
    integrator's own image of the same camera."""
    from paper_1706_07062_amd import surrogate as S

    sur = S.Surrogate(ctx, seed=0, max_batch=8192)
    x, t, mask, t_data = sur.make_data(args.surrogate_rays)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = sur.train(x, t, mask, steps=args.surrogate_steps, batch=8192, lr=2e-3,
                     log_every=max(1, args.surrogate_steps // 8), log=log, loss_w=S.LOSS_WEIGHTS)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    cam = W.surrogate_eval_camera()
    S.integrate_image(ctx, cam)  # warm-up
    ref, t_int = S.integrate_image(ctx, cam)
    curve = []
    # (tau, shadow_band [M], r_min [M]): capture band alone, then with the
    # shadow-edge and strong-field rules
    for tau, band, r_min in ((0.45, 0.0, 0.0), (0.2, 0.0, 0.0), (0.05, 0.0, 0.0), (0.01, 0.0, 0.0),
                             (0.2, 0.1, 0.0), (0.2, 0.3, 0.0), (0.2, 0.3, 3.0), (0.05, 0.3, 4.0)):
        # the clocks settle over the first launches of a new kernel: three
        # untimed renders, then the median of five (the outputs are identical)
        for _ in range(3):
            sur.render(cam, tau, shadow_band=band, r_min=r_min)
        runs = [sur.render(cam, tau, shadow_band=band, r_min=r_min) for _ in range(5)]
        img, tm = sorted(runs, key=lambda rt: rt[1]["total_s"])[2]
        err = S.image_error(img, ref)
        curve.append(dict(tau=tau, shadow_band=band, r_min=r_min, speedup=t_int / tm["total_s"], **tm, **err))
        log(f"surrogate tau {tau} band {band} r_min {r_min}: speedup {t_int / tm['total_s']:.2f}, fallback "
            f"{tm['fallback_fraction']:.4f}, capture mismatch {err['capture_mismatch']:.2e}, "
            f"|dg| p99 {err['g_abs_p99']:.2e}")
    # fixed-error point: the fastest setting with no more than 1e-4 capture
    # mismatches and p99 |dg| <= 1e-3; None when no setting meets both
    ok = [c for c in curve if c["capture_mismatch"] <= 1e-4 and c["g_abs_p99"] <= 1e-3]
    best = max(ok, key=lambda c: c["speedup"]) if ok else None
    # the integrator judging the image without the full reference: an audit
    # of 2^17 random pixels at the fixed-error setting, against the full error
    audit = None
    if best is not None:
        img, _ = sur.render(cam, best["tau"], shadow_band=best["shadow_band"], r_min=best["r_min"])
        audit = sur.audit(cam, img, 1 << 17, seed=1)
        log(f"surrogate audit of {audit['audit_rays']} pixels ({audit['audit_s'] * 1e3:.2f} ms): capture mismatch "
            f"{audit['capture_mismatch']:.2e}, |dg| p99 {audit['g_abs_p99']:.2e} (full image "
            f"{best['capture_mismatch']:.2e}, {best['g_abs_p99']:.2e})")
    return dict(train_rays=args.surrogate_rays, data_s=t_data, train_steps=args.surrogate_steps, batch=8192,
                loss_weights=dict(zip(("r", "phi", "g", "capture"), S.LOSS_WEIGHTS)), train_s=t_train,
                loss_history=hist, integrator_s=t_int, image=f"{cam.width}x{cam.height}", curve=curve,
                at_fixed_error=best, fixed_error_met=best is not None, audit_at_fixed_error=audit,
                fixed_error="capture-flag mismatch <= 1e-4 of pixels and p99 |dg| <= 1e-3 on pixels where both "
                            "images have a crossing; r and phi errors stated alongside")


def batched_extra(ctx, K, W, torch):
    """256 images of uneven size (32^2 .. 1024^2, spins and inclinations drawn)
    in one persistent, autotuned, graph-captured launch, MIXED precision at
    rtol 1e-6; against one launch per image."""
    from paper_1706_07062_amd.batched import BatchedImages, camera_struct

    cams = W.batched_images()
    p = K.kh_default_params(precision=K.PMIXED, rtol=1e-6, atol=1e-6)
    b = BatchedImages(ctx, cams, p, constants=False, tune=True, log=None)
    b.capture()
    times = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.replay()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    st = b.stats()
    n = b.n
    # every 16384th ray, for the error against the FP64 oracle on the host
    offs = np.concatenate([[0], np.cumsum([c.n for c in cams])])
    ids = np.arange(0, n, 16384)
    cam_of = np.searchsorted(offs, ids, side="right") - 1
    keep_sample("batched_mixed", b.state, ids, cam_of=cam_of, pix=ids - offs[cam_of])
    # one launch per image (eager), same precision and default launch shape
    states = [K.State(c.n, constants=False) for c in cams]
    kc = [camera_struct(c) for c in cams]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, s in zip(kc, states):
        ctx.kh_init_rays([c], s)
        ctx.kh_integrate(p, s)
    torch.cuda.synchronize()
    t_per = time.perf_counter() - t0
    del states
    out = dict(rays=n, images=len(cams), graph_replay_s=min(times), rays_per_s=n / min(times),
               per_image_launches_s=t_per, per_image_rays_per_s=n / t_per,
               accepted_steps_per_ray=st["n_acc"] / n, tuned_launch=b.choice, precision="mixed", rtol=1e-6)
    log(f"batched: {n} rays in {min(times):.3f} s (graph, one launch) vs {t_per:.3f} s (per-image launches)")
    return out


def particles_extra(ctx, K, W, torch):
    """2^20 time-like geodesics to t = 1e4 M: FP64 (rtol 1e-8) and FP32
    (rtol 1e-6), each with the affine parameter and in coordinate time,
    constants-of-motion drift per particle.  The states carry the
    per-geodesic schedule (longest expected first); each timed launch follows
    an untimed one of the same kind."""
    pw = W.particles()
    n = len(pw["a"])
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()  # noqa: E731
    spin, x3, v3 = t(pw["a"]), t(pw["x3"]), t(pw["v3"])
    out = {}
    finals = {}
    for name, prec, tol, method in (("fp64", K.P64, 1e-8, K.DOPRI5), ("fp32", K.P32, 1e-6, K.DOPRI5),
                                    ("fp64_coordinate_time", K.P64, 1e-8, K.DOPRI5_T),
                                    ("fp32_coordinate_time", K.P32, 1e-6, K.DOPRI5_T)):
        st = K.State(n, schedule="geodesics")
        p = K.kh_default_params(precision=prec, rtol=tol, atol=tol, t_end=1e4, r_escape=1e4, method=method)
        ctx.kh_init_geodesics(K.TIMELIKE, spin, x3, v3, st)
        ctx.kh_integrate(p, st)  # untimed warm-up launch
        ctx.kh_init_geodesics(K.TIMELIKE, spin, x3, v3, st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.kh_integrate(p, st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s = ctx.kh_stats(st)
        c0, c1 = st.c0.cpu().numpy(), st.c1.cpu().numpy()
        landed = st.status.cpu().numpy() == K.T_END
        drift = (np.abs(c1 - c0) / np.maximum(np.abs(c0), 1.0))[:, landed]
        cnames = ("E", "Lz", "Q", "mu2")
        out[name] = dict(seconds=dt, particles_per_s=n / dt, steps_per_particle=s["n_acc"] / n,
                         status_counts=s["status_counts"],
                         drift_median={k: float(np.median(drift[i])) for i, k in enumerate(cnames)},
                         drift_p99={k: float(np.quantile(drift[i], 0.99)) for i, k in enumerate(cnames)})
        finals[name] = (st.s.cpu().numpy(), landed)
        log(f"particles {name}: {dt:.3f} s, {s['n_acc'] / n:.0f} steps/particle")
    (s64, l64), (s32, l32) = finals["fp64"], finals["fp32"]
    both = l64 & l32
    d = np.linalg.norm(s32[1:4, both] - s64[1:4, both], axis=0) / np.linalg.norm(s64[1:4, both], axis=0)
    out["fp32_vs_fp64_position"] = dict(median=float(np.median(d)), p99=float(np.quantile(d, 0.99)))
    # dense output: the FP64 coordinate-time run again with states at 100 times
    t_out = np.linspace(100.0, 1e4, 100)
    st = K.State(n, t_out=t_out, schedule="geodesics")
    p = K.kh_default_params(method=K.DOPRI5_T, t_end=1e4, r_escape=1e4)
    ctx.kh_init_geodesics(K.TIMELIKE, spin, x3, v3, st)
    ctx.kh_integrate(p, st)  # untimed warm-up launch
    st.s_out.fill_(float("nan"))
    ctx.kh_init_geodesics(K.TIMELIKE, spin, x3, v3, st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.kh_integrate(p, st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    reached = float(torch.isfinite(st.s_out[:, :, 0]).float().mean().item())
    out["fp64_coordinate_time_dense_100"] = dict(seconds=dt, particles_per_s=n / dt, targets=100,
                                                 fraction_reached=reached,
                                                 output_bytes=int(st.s_out.numel() * 8))
    log(f"particles fp64 coordinate time + 100 dense outputs: {dt:.3f} s ({reached:.3f} of targets reached)")
    del st
    (sct, lct) = finals["fp64_coordinate_time"]
    both = l64 & lct
    d = np.linalg.norm(sct[1:4, both] - s64[1:4, both], axis=0) / np.linalg.norm(s64[1:4, both], axis=0)
    out["coordinate_time_vs_affine_position"] = dict(median=float(np.median(d)), p99=float(np.quantile(d, 0.99)))
    return out


def copy_probe(mib):
    """A plain device-to-device copy of known size (reads and writes `mib` MiB),
    run before the workload so a counter-collection run sees a reference for
    the HBM-byte counters."""
    import torch

    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy probe: 3 copies of {mib} MiB")


def cpu_baseline(args):
    """The oracle on a bounded sample of the same workload: strided pixels of
    both images, all host threads (timed: the CPU baseline).  Its results are
    also the FP64 reference against which every GPU result of this run states
    its error on the same rays: the FP64 headline, the FP32 and MIXED runs of
    the same images, and (one more, untimed oracle run) every 16384th ray of
    the 256-image MIXED batch."""
    import oracle as O
    from paper_1706_07062_amd import workloads as W

    cores = O.default_threads()
    outs = []
    done, t_total, attempts = 0, 0.0, 0
    cams = W.kerr_1024()
    for j, (cam, ids) in enumerate(zip(cams, headline_sample_ids(args.cpu_sample))):
        pix = ids - j * cam.n
        init = O.camera_rays(cam.a, cam.r_obs, cam.incl, cam.alpha_min, cam.alpha_max, cam.beta_min, cam.beta_max,
                             cam.width, cam.height, pix=pix)
        t0 = time.perf_counter()
        outs.append(O.integrate(init, O.Params(method=O.DOPRI5, k_cross=4), nthreads=cores))
        t_total += time.perf_counter() - t0
        done += len(pix)
        attempts += int(outs[-1]["n_acc"].sum()) + int(outs[-1]["n_rej"].sum())
    log(f"cpu oracle: {done} rays in {t_total:.2f} s on {cores} threads")
    ref = {k: np.concatenate([o[k] for o in outs], axis=-1 if k == "s" else 0) for k in ("s", "status", "n_cross",
                                                                                        "cross")}
    errors = {}
    for name in ("fp64", "fp32", "mixed", "mixed_split", "coordinate_time_fp64"):
        if name in SAMPLES:
            errors[name] = result_errors(SAMPLES[name], ref)
            log(f"error vs oracle, {name}: {errors[name]}")
    if "batched_mixed" in SAMPLES:
        g = SAMPLES["batched_mixed"]
        bcams = W.batched_images()
        parts = []
        for c in np.unique(g["cam_of"]):
            sel = np.nonzero(g["cam_of"] == c)[0]
            cam = bcams[c]
            init = O.camera_rays(cam.a, cam.r_obs, cam.incl, cam.alpha_min, cam.alpha_max, cam.beta_min,
                                 cam.beta_max, cam.width, cam.height, pix=g["pix"][sel])
            parts.append((sel, O.integrate(init, O.Params(method=O.DOPRI5), nthreads=cores)))
        o = dict(s=np.zeros_like(g["s"]), status=np.zeros_like(g["status"]))
        for sel, r in parts:
            o["s"][:, sel] = r["s"]
            o["status"][sel] = r["status"]
        gb = dict(s=g["s"], status=g["status"])
        errors["batched_mixed"] = result_errors(gb, o)
        log(f"error vs oracle, batched_mixed: {errors['batched_mixed']}")
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    # a DOPRI5 attempt evaluates six right-hand sides, plus one first stage per ray
    rhs = 6 * attempts + done
    return dict(value=done / t_total, unit="rays/s", cores=cores, kind="oracle",
                sample=f"{done} strided pixels of the two 1024x1024 a=0.99 images (half each), FP64 DOPRI5 "
                       f"rtol 1e-8, {t_total:.1f} s wall",
                rhs_evals_per_s=rhs / t_total,
                ns_per_attempt_per_ray_one_core=t_total * cores / attempts * 1e9,
                host=dict(cpu=model, logical_cpus=os.cpu_count())), errors


def precision_only(args):
    """The benchmark images integrated in FP32 (rtol 1e-6), MIXED (rtol 1e-8, both policies)
    and FP64 coordinate time, each `--steps` times after one untimed launch;
    one JSON line of HIP-event times."""
    import torch

    import paper_1706_07062_amd as K
    from paper_1706_07062_amd import workloads as W

    torch.cuda.set_device(0)
    ctx = K.Context(0)
    cams = W.kerr_1024()
    kc = [K.kh_camera(c.a, c.r_obs, c.incl, c.alpha_min, c.alpha_max, c.beta_min, c.beta_max, c.width, c.height)
          for c in cams]
    st = K.State(sum(c.n for c in cams), k_cross=4)
    res = {}
    for name, prec, tol, method, split in PRECISION_RUNS(K):
        p = K.kh_default_params(k_cross=4, precision=prec, rtol=tol, atol=tol, method=method, mixed_split=split)
        ms = []
        for i in range(max(1, args.steps) + 1):
            ctx.kh_init_rays(kc, st)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ctx.kh_integrate(p, st)
            e1.record()
            torch.cuda.synchronize()
            if i > 0:
                ms.append(e0.elapsed_time(e1))
        res[name] = dict(kernel_ms=ms, stats=ctx.kh_stats(st))
        log(f"{name}: {np.mean(ms):.3f} ms")
    print(json.dumps({"precision": res}), flush=True)
    ctx.close()


def surrogate_image_only():
    """The surrogate image kernel alone (timing and counters do not depend on
    the weights; the fallback count does)."""
    import torch

    import paper_1706_07062_amd as K
    from paper_1706_07062_amd import surrogate as SU, workloads as W

    torch.cuda.set_device(0)
    ctx = K.Context(0)
    sur = SU.Surrogate(ctx, seed=0)
    cam = W.surrogate_eval_camera()
    ms = []
    for _ in range(8):  # the clocks settle over the first few launches
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _, _, cnt = sur.image(cam, 0.2)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    log(f"surrogate image {cam.width}x{cam.height}: {', '.join(f'{m:.2f}' for m in ms)} ms; "
        f"fallback {int(cnt.item())}")
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=131072)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, help="MiB; plain copy before the run (counter reference)")
    ap.add_argument("--surrogate-rays", type=int, default=10_000_000)
    ap.add_argument("--surrogate-steps", type=int, default=40000)
    ap.add_argument("--precision-only", action="store_true",
                    help="only the FP32, MIXED and coordinate-time launches on the benchmark images (for profilers)")
    ap.add_argument("--elapse-only", action="store_true",
                    help="only the fixed-step chart / layout comparison (Sec. 4's tab:elapse), for profilers")
    ap.add_argument("--surrogate-image-only", action="store_true",
                    help="only the network's 4096^2 image, eight times, with untrained seed-0 weights (for profilers)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the integrator shards by ray range with no exchange on the hot "
              "path, and this build runs on a single MI355X (use --gpus 1).", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
    if args.surrogate_image_only:
        surrogate_image_only()
        return
    if args.precision_only:
        precision_only(args)
        return
    if args.elapse_only:
        import torch

        import paper_1706_07062_amd as K
        from paper_1706_07062_amd import workloads as W

        torch.cuda.set_device(0)
        ctx = K.Context(0)
        print(json.dumps({"elapse_table": elapse_extra(ctx, K, W, torch, reps=max(1, args.steps))}), flush=True)
        ctx.close()
        return
    out, _ = run_gpu(args)
    if not args.no_cpu:
        out["cpu_baseline"], out["error_vs_oracle"] = cpu_baseline(args)
        out["error_vs_oracle"]["reference"] = ("FP64 oracle (DOPRI5 rtol 1e-8) on the cpu_baseline sample of the "
                                               "two images; batched_mixed: every 16384th ray of the 256 images")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
