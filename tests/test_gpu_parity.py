"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Positions must agree to 1e-6 relative with identical
statuses on every ray the oracle does not flag as ill-conditioned
(tests/parity_util.py states the policy)."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
import paper_1706_07062_amd as K
from paper_1706_07062_amd import workloads as W
from parity_util import (POS_TOL, compare, gpu_image, kcam, oracle_image, oracle_params,
                         reduced_precision_errors, rel_pos)

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = K.Context(0)
    yield c
    c.close()


def _random_states(n, a, seed):
    """Random points outside the horizon with null momenta (oracle's metric)."""
    rng = np.random.default_rng(seed)
    ys = []
    while len(ys) < n:
        x = rng.uniform(-1, 1, 3) * rng.choice([3.0, 15.0, 300.0])
        r = O.radius(a, *x)
        if not (1.05 * (1 + np.sqrt(1 - a * a)) < r < 500):
            continue
        k = rng.normal(size=3)
        y = np.array([0.0, *x, 0.0, *k])
        g, _ = O.metric(a, y[:4])
        A, B, Cq = g[0, 0], g[0, 1:] @ k, k @ g[1:, 1:] @ k
        if A >= 0:
            continue
        y[4] = (B + np.sqrt(B * B - A * Cq)) / (-A)
        ys.append(y)
    return np.array(ys).T.copy()


@pytest.mark.parametrize("form", [K.RHS_FACTORED, K.RHS_PAPER])
def test_rhs_point_parity(ctx, form):
    """The right-hand side (metric, derivatives, eq:opt0/opti) at 3001 random
    points (a ragged multiple of the block) equals the oracle's Christoffel form."""
    say(f"rhs point parity form={form}")
    for a in (0.0, -0.99):
        s = _random_states(3001, a, seed=11 + form)
        spin = torch.full((s.shape[1],), a, dtype=torch.float64, device="cuda")
        acc = ctx.kh_rhs(K.P64, form, spin, torch.from_numpy(s).cuda()).cpu().numpy()
        for i in range(0, s.shape[1], 7):
            want = O.rhs(a, s[:4, i], s[4:, i])
            assert np.abs(acc[:, i] - want).max() <= 2e-12 * np.abs(want).max(), i
        acc32 = ctx.kh_rhs(K.P32, form, spin, torch.from_numpy(s).cuda()).cpu().numpy()
        for i in range(0, s.shape[1], 31):
            want = O.rhs(a, s[:4, i], s[4:, i])
            assert np.abs(acc32[:, i] - want).max() <= 5e-4 * np.abs(want).max(), i


def test_init_rays_matches_oracle(ctx):
    """Image-plane initial data of several concatenated cameras (ragged sizes)."""
    say("init rays")
    cams = [W.Camera(0.99, 1000.0, 17.0, -12, 12, -12, 12, 37, 29), W.Camera(0.0, 500.0, 85.0, -5, 7, -3, 9, 64, 3),
            W.Camera(-0.5, 1000.0, 60.0, -12, 12, -12, 12, 1, 1)]
    n = sum(c.n for c in cams)
    st = K.State(n, k_cross=2)
    ctx.kh_init_rays([kcam(c) for c in cams], st)
    g = st.numpy()
    off = 0
    for c in cams:
        o = O.camera_rays(c.a, c.r_obs, c.incl, c.alpha_min, c.alpha_max, c.beta_min, c.beta_max, c.width,
                          c.height)
        np.testing.assert_allclose(g["s"][:, off:off + c.n], o["s"], rtol=1e-14, atol=1e-13)
        assert np.all(g["status"][off:off + c.n] == K.ACTIVE)
        assert np.all(g["kind"][off:off + c.n] == K.NULL)
        assert np.all(g["spin"][off:off + c.n] == c.a)
        off += c.n
    assert np.all(np.isnan(g["cross"]))
    # constants at init: null norm of order 1e-16
    assert np.abs(g["c0"][3]).max() < 1e-14


def test_init_list_and_timelike_match_oracle(ctx):
    say("init list + timelike")
    rw = W.surrogate_rays(1000)
    st = K.State(1000)
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()  # noqa: E731
    ctx.kh_init_rays_list(t(rw["a"]), t(rw["incl"]), t(rw["alpha"]), t(rw["beta"]), 1000.0, st)
    o = O.list_rays(rw["a"], rw["incl"], rw["alpha"], rw["beta"], 1000.0)
    np.testing.assert_allclose(st.s.cpu().numpy(), o["s"], rtol=1e-14, atol=1e-13)
    pw = W.particles(777)
    st = K.State(777)
    ctx.kh_init_geodesics(K.TIMELIKE, t(pw["a"]), t(pw["x3"]), t(pw["v3"]), st)
    o = O.timelike(pw["a"], pw["x3"], pw["v3"])
    np.testing.assert_allclose(st.s.cpu().numpy(), o["s"], rtol=1e-13, atol=1e-13)
    assert np.array_equal(st.status.cpu().numpy(), o["status"])
    assert np.abs(st.c0.cpu().numpy()[3] - 1.0).max() < 1e-12  # mu^2 = 1


def _null_from_positions(a, x3, v3):
    """Initial states of null geodesics from positions and spatial momenta,
    built here from the definition: k^0 is the positive root of
    g_{mu nu} k^mu k^nu = 0 with the oracle's metric of chart spin -a (the
    time-reversed chart of the traced rays)."""
    n = len(a)
    s = np.zeros((8, n))
    for i in range(n):
        x = np.array([0.0, *x3[:, i]])
        g, _ = O.metric(-a[i], x)
        kv = v3[:, i]
        A = g[0, 0]
        B = 2.0 * g[0, 1:] @ kv
        Cc = kv @ g[1:, 1:] @ kv
        disc = np.sqrt(B * B - 4 * A * Cc)
        k0 = max((-B + disc) / (2 * A), (-B - disc) / (2 * A))
        s[:, i] = [0.0, *x3[:, i], k0, *kv]
    return dict(s=s, spin=np.array(a, float), kind=np.full(n, O.NULL, np.int32), status=np.zeros(n, np.int32))


def test_null_geodesics_from_positions_parity(ctx):
    """kh_init_geodesics with KH_NULL (rays that do not start on a camera):
    300 rays from r = 20 .. 60 in random directions, half with random unit
    spatial momenta and half aimed near the hole, a ~ U[0, 0.998].  The initial states equal the ones built from
    the null condition on the host; after DOPRI5 (rtol 1e-8, two crossing
    slots) statuses are identical and positions agree to 1e-6 on every ray
    whose oracle result is stable under a 1e-12 change of the momentum."""
    say("null geodesics from positions")
    rng = np.random.default_rng(1706070631)
    n = 300
    a = rng.uniform(0.0, 0.998, n)
    d = rng.normal(size=(3, n))
    x3 = rng.uniform(20.0, 60.0, n) * d / np.linalg.norm(d, axis=0)
    v = rng.normal(size=(3, n))
    # half of the rays aimed near the hole (about a third of those are captured)
    aim = np.arange(n) < n // 2
    v[:, aim] = -x3[:, aim] / np.linalg.norm(x3[:, aim], axis=0) + 0.12 * v[:, aim]
    v3 = v / np.linalg.norm(v, axis=0)
    t = lambda u: torch.from_numpy(np.ascontiguousarray(u)).cuda()  # noqa: E731
    st = K.State(n, k_cross=2)
    ctx.kh_init_geodesics(K.NULL, t(a), t(x3), t(v3), st)
    init = _null_from_positions(a, x3, v3)
    np.testing.assert_allclose(st.s.cpu().numpy(), init["s"], rtol=1e-13, atol=1e-13)
    p = K.kh_default_params(k_cross=2)
    ctx.kh_integrate(p, st)
    g = st.numpy()
    o = O.integrate(init, oracle_params(p))
    o2 = O.integrate(_null_from_positions(a, x3, v3 * (1.0 + 1e-12) + 1e-12 * np.roll(v3, 1, axis=0)),
                     oracle_params(p))
    ill = (rel_pos(o["s"], o2["s"]) > 1e-7) | (o["status"] != o2["status"])
    dpos = rel_pos(g["s"], o["s"])
    say(f"  statuses {np.bincount(g['status'], minlength=6).tolist()}, ill {ill.sum()}, "
        f"max rel pos {dpos[~ill].max():.2e}")
    assert ill.sum() <= 6
    assert np.array_equal(g["status"][~ill], o["status"][~ill])
    assert dpos[~ill].max() < POS_TOL
    assert np.array_equal(g["n_cross"][~ill], o["n_cross"][~ill])
    assert np.sum(g["status"] == K.CAPTURED) > 10 and np.sum(g["status"] == K.ESCAPED) > 10


def test_schwarzschild_64_rk4_parity(ctx):
    """a = 0, 64x64 at 60 deg, fixed-step RK4 h = 0.01 r: full image."""
    say("schwarzschild 64x64 RK4")
    cam = W.schwarzschild_64()
    p = K.kh_default_params(method=K.RK4, h_coeff=0.01, r_escape=1000.0)
    st = gpu_image(ctx, [cam], p)
    g = st.numpy()
    o = oracle_image(cam, oracle_params(p))
    rep = compare(g, o)
    say(f"  {rep}")
    assert rep["status_mismatch"] == 0 and rep["n_pos_bad"] == 0
    assert rep["ill"] < 0.01 * rep["n"]
    assert np.array_equal(g["n_acc"][~o["ill"]], o["n_acc"][~o["ill"]])
    assert set(np.unique(g["status"])) <= {K.CAPTURED, K.ESCAPED}


@pytest.mark.parametrize("incl", [17.0, 60.0])
def test_kerr_ragged_image_dopri5_parity(ctx, incl):
    """a = 0.99, 100x77 image (several blocks plus a ragged tail), DOPRI5
    rtol 1e-8, four crossing slots: full element-wise comparison."""
    say(f"kerr 100x77 DOPRI5 incl={incl}")
    cam = W.Camera(0.99, 1000.0, incl, -12, 12, -12, 12, 100, 77)
    p = K.kh_default_params(k_cross=4)
    st = gpu_image(ctx, [cam], p, k_cross=4)
    g = st.numpy()
    o = oracle_image(cam, oracle_params(p))
    rep = compare(g, o)
    say(f"  {rep}")
    well = ~o["ill"]
    assert rep["status_mismatch"] == 0 and rep["n_pos_bad"] == 0
    assert rep["ill"] < 0.01 * rep["n"]
    assert rep["max_rel_t"] < POS_TOL and rep["max_rel_k"] < 1e-5
    # crossings: same count, same (r, phi, g)
    assert np.array_equal(g["n_cross"][well], o["n_cross"][well])
    gc, oc = g["cross"][well], o["cross"][well]
    both = ~np.isnan(oc)
    assert np.array_equal(np.isnan(gc), np.isnan(oc))
    assert np.max(np.abs(gc[both] - oc[both]) / np.maximum(np.abs(oc[both]), 1.0)) < POS_TOL
    # constants of motion conserved to the tolerance
    d = np.abs(g["c1"][:3] - g["c0"][:3]) / np.maximum(np.abs(g["c0"][:3]), 1.0)
    assert np.max(d[:, well]) < 1e-6


@pytest.mark.parametrize("a, incl", [(1.0, 75.0), (-0.9, 40.0), (0.5, 90.0)])
def test_extremal_negative_spin_and_edge_on_parity(ctx, a, incl):
    """Edge cases of the geometry against the oracle, element by element: the
    extremal hole a = 1 (degenerate horizon r_H = 1), a negative spin (hole
    rotating about -z, so the chart spin flips sign), and an edge-on camera
    (inclination 90 deg: the image plane contains the spin axis and every ray
    starts in the equatorial plane's normal direction, z0 = beta).  41x29
    images, DOPRI5 rtol 1e-8, two crossing slots."""
    say(f"edge geometry a={a} incl={incl}")
    cam = W.Camera(a, 1000.0, incl, -10, 10, -8, 8, 41, 29)
    p = K.kh_default_params(k_cross=2)
    g = gpu_image(ctx, [cam], p, k_cross=2).numpy()
    o = oracle_image(cam, oracle_params(p))
    rep = compare(g, o)
    say(f"  {rep}")
    well = ~o["ill"]
    assert rep["status_mismatch"] == 0 and rep["n_pos_bad"] == 0
    assert rep["ill"] < 0.02 * rep["n"]
    assert np.sum(g["status"] == K.CAPTURED) > 20 and np.sum(g["status"] == K.ESCAPED) > 20
    assert np.array_equal(g["n_cross"][well], o["n_cross"][well])
    gc, oc = g["cross"][well], o["cross"][well]
    both = ~np.isnan(oc)
    assert np.array_equal(np.isnan(gc), np.isnan(oc))
    assert np.max(np.abs(gc[both] - oc[both]) / np.maximum(np.abs(oc[both]), 1.0)) < POS_TOL


def test_kerr_1024_both_inclinations_sampled(ctx):
    """The full workload (a = 0.99, 1024x1024 at 17 and 60 deg in one launch, the
    benchmark's launch configuration), checked on 600 pixels of each image."""
    say("kerr 2x1024^2 sampled")
    cams = W.kerr_1024()
    p = K.kh_default_params(k_cross=4)
    st = gpu_image(ctx, cams, p, k_cross=4)
    g = st.numpy()
    stats = ctx.kh_stats(st)
    assert sum(stats["status_counts"]) == 2 * 1024 * 1024
    assert stats["status_counts"][K.ACTIVE] == 0 and stats["status_counts"][K.MAX_STEPS] == 0
    assert stats["n_acc"] == int(g["n_acc"].astype(np.int64).sum())
    for j, cam in enumerate(cams):
        pix = W.strided_pixels(cam.n, 600, offset=j * 17)
        o = oracle_image(cam, oracle_params(p), pix=pix)
        rep = compare(g, o, idx=pix + j * cam.n)
        say(f"  incl={cam.incl_deg}: {rep}")
        assert rep["status_mismatch"] == 0 and rep["n_pos_bad"] == 0
        assert rep["ill"] < 0.02 * rep["n"]
        well = ~o["ill"]
        assert np.array_equal(g["n_cross"][pix + j * cam.n][well], o["n_cross"][well])


@pytest.mark.parametrize("prec", [K.P32, K.PMIXED])
def test_reduced_precision_error_reported(ctx, prec):
    """FP32 and mixed FP32/FP64 runs of a 128x128 a = 0.99 image against the
    FP64 oracle.  These errors are reported quantities (parity unpinned); the
    bounds only guard against gross breakage."""
    say(f"reduced precision {prec}")
    cam = W.kerr_image(60.0, side=128)
    tol = 1e-6 if prec == K.P32 else 1e-8
    p = K.kh_default_params(precision=prec, k_cross=4, rtol=tol, atol=tol)
    st = gpu_image(ctx, [cam], p, k_cross=4)
    g = st.numpy()
    pix = W.strided_pixels(cam.n, 800)
    o = oracle_image(cam, oracle_params(K.kh_default_params(k_cross=4)), pix=pix, conditioning=False)
    rep = reduced_precision_errors(g, o, pix)
    say(f"  {rep}")
    assert rep["status_agree"] > 0.97
    assert rep["cross_r_median"] < (1e-3 if prec == K.P32 else 1e-5)
    assert rep["escape_angle_median"] < (1e-3 if prec == K.P32 else 1e-5)


def test_resume_is_bitwise(ctx):
    """Pausing every ray after 17 accepted steps and resuming gives exactly the
    uninterrupted result (FP64), and MAX_STEPS is reported in between."""
    say("resume bitwise")
    cam = W.kerr_image(60.0, side=48)
    p = K.kh_default_params(k_cross=4)
    ref = gpu_image(ctx, [cam], p, k_cross=4).numpy()
    st = K.State(cam.n, k_cross=4)
    ctx.kh_init_rays([kcam(cam)], st)
    p17 = K.kh_default_params(k_cross=4, max_steps=17)
    ctx.kh_integrate(p17, st)
    torch.cuda.synchronize()
    mid = st.status.cpu().numpy()
    assert np.all(mid == K.MAX_STEPS) or np.mean(mid == K.MAX_STEPS) > 0.9
    for _ in range(200):
        ctx.kh_integrate(p17, st)
        if ctx.kh_stats(st)["status_counts"][K.MAX_STEPS] == 0:
            break
    g = st.numpy()
    say(f"  max |resumed - uninterrupted| / |x|: {np.max(rel_pos(g['s'], ref['s'])):.3e}")
    for name in ("s", "status", "n_acc", "n_rej", "lam", "phi", "n_cross"):
        assert np.array_equal(g[name], ref[name]), name
    assert np.array_equal(np.nan_to_num(g["cross"], nan=-7.0), np.nan_to_num(ref["cross"], nan=-7.0))


def test_resume_from_a_checkpoint_file_is_bitwise(ctx, tmp_path):
    """The state is the checkpoint: pause a particle set (per-geodesic
    schedule, constants, dense output) and an image (tile order, crossing
    records) after 40 accepted steps, write the state to disk, load it into a
    new State in a fresh context and finish: bitwise the uninterrupted run."""
    say("resume from a checkpoint file")
    pw = W.particles()
    idx = np.arange(0, 1 << 20, 8191)[:128]
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()  # noqa: E731
    cam = W.kerr_image(17.0, side=32)
    cases = []
    for kind in ("particles", "image"):
        if kind == "particles":
            mk = lambda: K.State(len(idx), schedule="geodesics", t_out=[10.0, 500.0, 5000.0])  # noqa: E731
            init = lambda c, s: c.kh_init_geodesics(K.TIMELIKE, t(pw["a"][idx]), t(pw["x3"][:, idx]),  # noqa: E731
                                                     t(pw["v3"][:, idx]), s)
            prm = dict(t_end=1e4, r_escape=1e4)
        else:
            mk = lambda: K.State(cam.n, k_cross=4)  # noqa: E731
            init = lambda c, s: c.kh_init_rays([kcam(cam)], s)  # noqa: E731
            prm = dict(k_cross=4)
        ref = mk()
        init(ctx, ref)
        ctx.kh_integrate(K.kh_default_params(**prm), ref)
        st = mk()
        init(ctx, st)
        ctx.kh_integrate(K.kh_default_params(max_steps=40, **prm), st)
        torch.cuda.synchronize()
        assert ctx.kh_stats(st)["status_counts"][K.MAX_STEPS] > 0
        path = tmp_path / f"{kind}.npz"
        st.save(path)
        cases.append((kind, path, prm, ref.numpy()))
    ctx2 = K.Context(0)
    try:
        for kind, path, prm, want in cases:
            st2 = K.State.load(path)
            ctx2.kh_integrate(K.kh_default_params(**prm), st2)
            got = st2.numpy()
            say(f"  {kind}: statuses {np.bincount(got['status'], minlength=6).tolist()}")
            for name, a in got.items():
                if a is None or name in ("order", "perm"):
                    continue
                assert np.array_equal(np.nan_to_num(a, nan=-7.0), np.nan_to_num(want[name], nan=-7.0)), (kind, name)
    finally:
        ctx2.close()


def test_launch_shape_does_not_change_results(ctx):
    """Each lane's arithmetic is independent of scheduling: block size, grid size
    and refill threshold give bitwise identical FP64 results."""
    say("launch shape determinism")
    cam = W.kerr_image(17.0, side=64)
    base = gpu_image(ctx, [cam], K.kh_default_params(k_cross=4), k_cross=4).numpy()
    for bs, gb, rf in ((64, 0, 1), (128, 7, 64), (256, 1, 16), (192, 3, 5)):
        g = gpu_image(ctx, [cam], K.kh_default_params(k_cross=4, block_size=bs, grid_blocks=gb, refill_min=rf),
                      k_cross=4).numpy()
        assert np.array_equal(g["s"], base["s"]), (bs, gb, rf)
        assert np.array_equal(g["n_acc"], base["n_acc"])


def test_particles_to_t_end_parity(ctx):
    """Time-like geodesics of the particle workload (a strided sample of 256 of
    its 2^20 draws), DOPRI5 rtol 1e-8 to t = 1e4 M with exact landing."""
    say("particles t_end")
    pw = W.particles()
    idx = np.arange(0, 1 << 20, 4099)[:256]
    a, x3, v3 = pw["a"][idx], pw["x3"][:, idx].copy(), pw["v3"][:, idx].copy()
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()  # noqa: E731
    st = K.State(len(idx))
    ctx.kh_init_geodesics(K.TIMELIKE, t(a), t(x3), t(v3), st)
    p = K.kh_default_params(t_end=1e4, r_escape=1e4)
    ctx.kh_integrate(p, st)
    g = st.numpy()
    o = O.integrate(O.timelike(a, x3, v3), oracle_params(p))
    assert np.array_equal(g["status"], o["status"])
    # a few low-energy draws near r0 = 6 plunge; every other particle lands on t_end
    landed = g["status"] == K.T_END
    assert landed.mean() > 0.95 and np.all(np.isin(g["status"], [K.T_END, K.CAPTURED]))
    assert np.abs(g["s"][0, landed] - 1e4).max() <= 1e-12 * 1e4
    d = rel_pos(g["s"], o["s"])
    say(f"  max rel pos {d.max():.2e}, median {np.median(d):.2e}")
    assert d.max() < 1e-6
    # Constant-of-motion drift grows with the number of accepted steps (each
    # adds a local error of order rtol): per particle and per constant the
    # oracle's drift on this sample stays below 1.92 n_acc rtol (Q; E 0.16,
    # L_z 0.96, mu^2 0.44), and the GPU's must stay below twice that.
    drift = (np.abs(g["c1"] - g["c0"]) / np.maximum(np.abs(g["c0"]), 1.0))[:, landed]
    per_step = drift / (g["n_acc"][landed] * p.rtol)
    say(f"  drift median/max E {np.median(drift[0]):.1e}/{drift[0].max():.1e} Lz {np.median(drift[1]):.1e}/"
        f"{drift[1].max():.1e} Q {np.median(drift[2]):.1e}/{drift[2].max():.1e} mu2 {np.median(drift[3]):.1e}/"
        f"{drift[3].max():.1e}; max drift / (n_acc rtol) {np.array2string(per_step.max(axis=1), precision=3)}")
    assert np.all(per_step < 4.0)


def test_particles_full_size_sampled(ctx):
    """The whole particle workload (2^20 time-like geodesics to t = 1e4 M, FP64
    DOPRI5 rtol 1e-8) in the launch bench.py times (per-geodesic schedule,
    default launch shape).  64 particles spread over the set and the 8 that
    take the most steps (up to ~16,000) are integrated by the oracle one by
    one: identical statuses, positions within 1e-6 relative, exact landing on
    t_end.  Particles whose oracle result moves by more than 1e-7 when the
    initial velocity is scaled by 1 + 1e-12 would be ill-conditioned and
    excluded (their count is reported)."""
    say("particles full size, sampled")
    pw = W.particles()
    n = len(pw["a"])
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()  # noqa: E731
    st = K.State(n, schedule="geodesics")
    ctx.kh_init_geodesics(K.TIMELIKE, t(pw["a"]), t(pw["x3"]), t(pw["v3"]), st)
    p = K.kh_default_params(t_end=1e4, r_escape=1e4)
    ctx.kh_integrate(p, st)
    torch.cuda.synchronize()
    status = st.status.cpu().numpy()
    nacc = st.n_acc.cpu().numpy()
    s = st.s.cpu().numpy()
    assert np.all(np.isin(status, [K.T_END, K.CAPTURED]))
    landed = status == K.T_END
    assert np.abs(s[0, landed] - 1e4).max() <= 1e-12 * 1e4
    pick = np.unique(np.concatenate([np.arange(0, n, n // 64), np.argsort(nacc, kind="stable")[-8:]]))
    op = oracle_params(p)
    a, x3, v3 = pw["a"][pick], pw["x3"][:, pick].copy(), pw["v3"][:, pick].copy()
    o = O.integrate(O.timelike(a, x3, v3), op)
    op_ = O.integrate(O.timelike(a, x3, v3 * (1.0 + 1e-12)), op)
    ill = (rel_pos(o["s"], op_["s"]) > 1e-7) | (o["status"] != op_["status"])
    d = rel_pos(s[:, pick], o["s"])
    say(f"  {len(pick)} particles (steps up to {nacc[pick].max()}), ill {ill.sum()}, "
        f"max rel pos {d[~ill].max():.2e}")
    assert ill.sum() <= len(pick) // 16
    assert np.array_equal(status[pick][~ill], o["status"][~ill])
    assert d[~ill].max() < 1e-6


def test_failure_statuses_forced_from_the_host(ctx):
    """Planted NaN state -> FAILED; max_steps = 1 -> MAX_STEPS; rays already
    terminal are left untouched."""
    say("failure statuses")
    cam = W.kerr_image(60.0, side=8)
    st = K.State(cam.n)
    ctx.kh_init_rays([kcam(cam)], st)
    st.s[1, 3] = float("nan")
    st.status[5] = K.CAPTURED
    before5 = st.s[:, 5].clone()
    ctx.kh_integrate(K.kh_default_params(max_steps=1), st)
    g = st.numpy()
    assert g["status"][3] == K.FAILED
    assert g["status"][5] == K.CAPTURED and torch.equal(st.s[:, 5], before5)
    others = np.setdiff1d(np.arange(cam.n), [3, 5])
    assert np.all(g["status"][others] == K.MAX_STEPS)
    assert np.all(g["n_acc"][others] == 1)


def test_argument_errors(ctx):
    say("argument errors")
    st = K.State(16)
    bad = K.kh_default_params(rtol=-1.0)
    with pytest.raises(K.KerrHipError, match="rtol"):
        ctx.kh_integrate(bad, st)
    with pytest.raises(K.KerrHipError, match="k_cross"):
        ctx.kh_integrate(K.kh_default_params(k_cross=4), st)
    with pytest.raises(K.KerrHipError):
        ctx.kh_integrate(K.kh_default_params(method=K.RK4, t_end=5.0), st)
    cam = W.Camera(1.5, 1000.0, 60.0, -1, 1, -1, 1, 4, 4)
    with pytest.raises(K.KerrHipError, match="camera"):
        ctx.kh_init_rays([kcam(cam)], st)
    cam = W.Camera(0.5, 1000.0, 60.0, -1, 1, -1, 1, 4, 3)
    with pytest.raises(K.KerrHipError, match="state.n"):
        ctx.kh_init_rays([kcam(cam)], st)
    # a host pointer is refused before any launch
    host = torch.zeros(16, dtype=torch.float64)
    saved = st.c.h
    st.c.h = host.data_ptr()
    with pytest.raises(K.KerrHipError, match="device memory"):
        ctx.kh_integrate(K.kh_default_params(), st)
    st.c.h = saved
    # empty and oversized states are refused from the size alone (no pointer is touched)
    for n_bad in (0, -5, 1 << 31):
        fake = K.kh_state.from_buffer_copy(st.c)
        fake.n = n_bad
        rc = K.lib().kh_integrate(ctx.handle, C.byref(K.kh_default_params()), C.byref(fake), None)
        assert rc == K.KH_EINVAL, n_bad
        assert b"state.n" in K.lib().kh_last_error(ctx.handle)
    # unknown method / precision / form; the Boyer-Lindquist form is for the fixed-step kernel only
    for field, val, msg in (("method", 9, "method"), ("precision", 7, "precision"), ("rhs_form", 5, "rhs_form"),
                            ("rhs_form", K.RHS_BL, "rhs_form"), ("k_cross", 9, "k_cross")):
        with pytest.raises(K.KerrHipError, match=msg):
            ctx.kh_integrate(K.kh_default_params(**{field: val}), st)


def test_tile_order_is_a_permutation_and_does_not_change_results(ctx):
    """kh_init_rays orders the 64-ray tiles longest-expected-first.  The order is
    a permutation of the tiles (also with a ragged last tile), the tiles it puts
    first really are the expensive ones, and integrating in that order gives
    bitwise the results of the natural order."""
    say("tile order")
    cams = [W.Camera(0.99, 1000.0, 60.0, -12.0, 12.0, -12.0, 12.0, 97, 83),
            W.Camera(0.5, 1000.0, 30.0, -9.0, 11.0, -10.0, 10.0, 61, 45)]
    n = sum(c.n for c in cams)
    assert n % 64 != 0
    p = K.kh_default_params(k_cross=4)
    ordered = gpu_image(ctx, cams, p, k_cross=4)
    order = ordered.order.cpu().numpy()
    n_tiles = (n + 63) // 64
    assert np.array_equal(np.sort(order), np.arange(n_tiles))
    st = K.State(n, k_cross=4, schedule=False)
    ctx.kh_init_rays([kcam(c) for c in cams], st)
    ctx.kh_integrate(p, st)
    torch.cuda.synchronize()
    a, b = ordered.numpy(), st.numpy()
    for name in ("s", "status", "n_acc", "n_rej", "cross", "n_cross", "phi", "lam", "h"):
        assert np.array_equal(a[name], b[name], equal_nan=True), name
    # the first tenth of the order holds the costliest tiles
    cost = (a["n_acc"] + a["n_rej"]).astype(np.float64)
    tile_cost = np.array([cost[64 * t:64 * t + 64].max() for t in range(n_tiles)])
    head = tile_cost[order[:max(1, n_tiles // 10)]]
    say(f"  max steps: first tenth of the order {head.mean():.0f}, all tiles {tile_cost.mean():.0f}")
    assert head.mean() > tile_cost.mean()
    assert tile_cost.max() in head


def test_out_of_range_tile_order_is_skipped(ctx):
    """A caller-written order with entries out of range: the integrator skips
    those positions (no access outside the state) and leaves the rays active."""
    say("bad tile order")
    cam = W.kerr_image(60.0, side=16)
    st = K.State(cam.n)
    ctx.kh_init_rays([kcam(cam)], st)
    st.order.copy_(torch.tensor([1, 1000, -5, 2], dtype=torch.int32))  # tiles 0 and 3 never handed out
    ctx.kh_integrate(K.kh_default_params(), st)
    torch.cuda.synchronize()
    g = st.numpy()
    assert np.all(g["status"][0:64] == K.ACTIVE) and np.all(g["status"][192:256] == K.ACTIVE)
    assert np.all(g["status"][64:192] != K.ACTIVE)


def test_read_state_copies_ranges_to_the_host(ctx):
    """kh_read_state: [count][8] host rows and statuses equal the device
    arrays for the whole state, an inner range and a one-ray range; statuses
    alone with host_s NULL; an empty range is a no-op; a range past the end
    is refused; a state of more than 2^20 rays (two packing chunks) and a
    range that starts near 2^20."""
    say("read state")
    cam = W.Camera(0.9, 1000.0, 45.0, -12.0, 12.0, -12.0, 12.0, 37, 29)
    st = gpu_image(ctx, [cam], K.kh_default_params())
    s = st.s.cpu().numpy()
    status = st.status.cpu().numpy()
    for first, count in ((0, cam.n), (101, 517), (cam.n - 1, 1)):
        hs, hst = ctx.kh_read_state(st, first, count)
        assert np.array_equal(hs, s[:, first:first + count].T)
        assert np.array_equal(hst, status[first:first + count])
    only = np.full(50, -7, np.int32)
    rc = K.lib().kh_read_state(ctx.handle, C.byref(st.c), 10, 50, None, only.ctypes.data, None)
    assert rc == K.KH_OK and np.array_equal(only, status[10:60])
    hs, hst = ctx.kh_read_state(st, 5, 0)
    assert hs.shape == (0, 8) and hst.shape == (0,)
    with pytest.raises(K.KerrHipError, match="range"):
        ctx.kh_read_state(st, cam.n - 3, 4)
    # more rays than one 2^20-row chunk of the device-side packing
    big = W.Camera(0.9, 1000.0, 45.0, -12.0, 12.0, -12.0, 12.0, 1025, 1024)
    sb = K.State(big.n, constants=False)
    ctx.kh_init_rays([kcam(big)], sb)
    s = sb.s.cpu().numpy()
    for first, count in ((0, big.n), ((1 << 20) - 5, 100)):
        hs, hst = ctx.kh_read_state(sb, first, count)
        assert np.array_equal(hs, s[:, first:first + count].T)
        assert np.array_equal(hst, sb.status.cpu().numpy()[first:first + count])
    # into caller-provided page-locked host tensors (the whole state: two chunks)
    pinned = (torch.full((big.n, 8), -1.0, dtype=torch.float64, pin_memory=True),
              torch.full((big.n,), -7, dtype=torch.int32, pin_memory=True))
    hs, hst = ctx.kh_read_state(sb, 0, big.n, out=pinned)
    assert hs is pinned[0] and hst is pinned[1]
    assert np.array_equal(hs.numpy(), s.T) and np.array_equal(hst.numpy(), sb.status.cpu().numpy())
    with pytest.raises(ValueError):
        ctx.kh_read_state(sb, 0, 10, out=pinned)


def _is_permutation(perm, n):
    return perm.shape == (n,) and np.array_equal(np.sort(perm), np.arange(n))


def test_geodesic_schedule_orders_particles_longest_first(ctx):
    """kh_init_geodesics with a per-geodesic schedule: perm is a permutation of
    the geodesics (several sort blocks of 8192 and a ragged tail), its keys
    descend (the key is recomputed here from the energy E in c0:
    255 - 16 log2(1 / (2 (1 - E))), truncated), the geodesics it puts first
    take more steps, and the results are bitwise those of the natural order."""
    say("geodesic schedule, particles")
    n = 3 * 8192 + 77
    pw = W.particles(n=n)
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()  # noqa: E731
    p = K.kh_default_params(t_end=1e4, r_escape=1e4)
    runs = {}
    for sched in ("geodesics", None):
        st = K.State(n, schedule=sched)
        ctx.kh_init_geodesics(K.TIMELIKE, t(pw["a"]), t(pw["x3"]), t(pw["v3"]), st)
        if sched:
            perm0 = st.perm.cpu().numpy()
        ctx.kh_integrate(p, st)
        torch.cuda.synchronize()
        runs[sched] = st.numpy()
    a, b = runs["geodesics"], runs[None]
    for name in ("s", "status", "n_acc", "n_rej", "lam", "h", "c1"):
        assert np.array_equal(a[name], b[name], equal_nan=True), name
    assert _is_permutation(perm0, n)
    E = a["c0"][0]
    bound = (E > 0) & (E < 1)
    kf = np.where(bound, 255.0 - 16.0 * np.log2(np.maximum(0.5 / np.where(bound, 1.0 - E, 1.0), 1.0)), 0.0)
    kf = np.clip(kf, 0.0, 255.0)
    kh = np.floor(kf)[perm0]
    near_int = np.abs(kf - np.round(kf))[perm0] < 1e-9
    drops = np.diff(kh)
    assert np.all((drops <= 0) | near_int[1:] | near_int[:-1])
    # resumed in calls of at most 500 accepted steps: bitwise the single run
    st = K.State(n, schedule="geodesics")
    ctx.kh_init_geodesics(K.TIMELIKE, t(pw["a"]), t(pw["x3"]), t(pw["v3"]), st)
    calls = 0
    while True:
        ctx.kh_integrate(K.kh_default_params(t_end=1e4, r_escape=1e4, max_steps=500), st)
        calls += 1
        if ctx.kh_stats(st)["status_counts"][K.MAX_STEPS] == 0 or calls > 100:
            break
    c = st.numpy()
    say(f"  resumed in {calls} calls")
    for name in ("s", "status", "n_acc", "n_rej", "lam"):
        assert np.array_equal(c[name], a[name], equal_nan=True), name
    cost = (a["n_acc"] + a["n_rej"]).astype(np.float64)[perm0]
    head, tail = cost[: n // 10].mean(), cost[-n // 10:].mean()
    say(f"  mean steps: first tenth of the schedule {head:.0f}, last tenth {tail:.0f}, max {cost.max():.0f}")
    assert head > 4 * tail
    assert cost.argmax() < n // 10


def test_geodesic_schedule_for_rays_and_images(ctx):
    """The per-ray schedule from kh_init_rays_list and kh_init_rays is a
    permutation, puts the costliest rays first, and leaves the results
    bitwise unchanged (against the tile order of the same image)."""
    say("geodesic schedule, rays")
    cams = [W.Camera(0.99, 1000.0, 60.0, -12.0, 12.0, -12.0, 12.0, 97, 83),
            W.Camera(0.5, 1000.0, 30.0, -9.0, 11.0, -10.0, 10.0, 61, 45)]
    n = sum(c.n for c in cams)
    p = K.kh_default_params(k_cross=4)
    tiles = gpu_image(ctx, cams, p, k_cross=4).numpy()
    st = K.State(n, k_cross=4, schedule="geodesics")
    ctx.kh_init_rays([kcam(c) for c in cams], st)
    perm = st.perm.cpu().numpy()
    ctx.kh_integrate(p, st)
    torch.cuda.synchronize()
    g = st.numpy()
    assert _is_permutation(perm, n)
    for name in ("s", "status", "n_acc", "n_rej", "cross", "n_cross", "phi", "lam", "h"):
        assert np.array_equal(g[name], tiles[name], equal_nan=True), name
    cost = (g["n_acc"] + g["n_rej"]).astype(np.float64)
    head = cost[perm[: n // 10]]
    say(f"  mean steps: first tenth of the schedule {head.mean():.0f}, all rays {cost.mean():.0f}")
    assert head.mean() > cost.mean()
    assert cost.max() in head
    # the list form (one spin and inclination per ray): scheduled and natural
    # order give the same bits
    c = cams[0]
    f64 = dict(dtype=torch.float64, device="cuda")
    col = np.arange(c.n) % c.width
    row = np.arange(c.n) // c.width
    args = (torch.full((c.n,), c.a, **f64), torch.full((c.n,), c.incl, **f64),
            torch.from_numpy(c.alpha_min + (col + 0.5) * (c.alpha_max - c.alpha_min) / c.width).cuda(),
            torch.from_numpy(c.beta_min + (row + 0.5) * (c.beta_max - c.beta_min) / c.height).cuda(), c.r_obs)
    out = {}
    for sched in ("geodesics", None):
        sl = K.State(c.n, k_cross=4, schedule=sched)
        ctx.kh_init_rays_list(*args, sl)
        if sched:
            assert _is_permutation(sl.perm.cpu().numpy(), c.n)
        ctx.kh_integrate(p, sl)
        torch.cuda.synchronize()
        out[sched] = sl.numpy()
    for name in ("s", "status", "n_acc", "cross"):
        assert np.array_equal(out["geodesics"][name], out[None][name], equal_nan=True), name


def test_out_of_range_geodesic_schedule_is_skipped(ctx):
    """A caller-written perm with entries out of range: those positions are
    skipped (no access outside the state) and the geodesics they would have
    named stay active; the tile order is ignored while perm is set."""
    say("bad geodesic schedule")
    cam = W.kerr_image(60.0, side=16)
    st = K.State(cam.n, schedule="geodesics")
    ctx.kh_init_rays([kcam(cam)], st)
    bad = torch.arange(cam.n, dtype=torch.int32, device="cuda")
    bad[10] = cam.n
    bad[20] = -1
    bad[30] = 1 << 30
    st.perm.copy_(bad)
    ctx.kh_integrate(K.kh_default_params(), st)
    torch.cuda.synchronize()
    status = st.status.cpu().numpy()
    skipped = np.array([10, 20, 30])
    assert np.all(status[skipped] == K.ACTIVE)
    assert np.all(np.delete(status, skipped) != K.ACTIVE)


def test_coordinate_time_image_parity(ctx):
    """Null rays of a ragged a = 0.99 image integrated in coordinate time
    (KH_DOPRI5_T, rtol 1e-8, four crossing slots) against the oracle's
    coordinate-time integration, element by element."""
    say("kerr 61x47 DOPRI5_T")
    cam = W.Camera(0.99, 1000.0, 60.0, -12, 12, -12, 12, 61, 47)
    p = K.kh_default_params(method=K.DOPRI5_T, k_cross=4)
    g = gpu_image(ctx, [cam], p, k_cross=4).numpy()
    o = oracle_image(cam, oracle_params(p))
    rep = compare(g, o)
    say(f"  {rep}")
    well = ~o["ill"]
    assert rep["status_mismatch"] == 0 and rep["n_pos_bad"] == 0
    assert rep["ill"] < 0.01 * rep["n"]
    assert rep["max_rel_t"] < POS_TOL and rep["max_rel_k"] < 1e-5
    assert np.array_equal(g["n_cross"][well], o["n_cross"][well])
    gc, oc = g["cross"][well], o["cross"][well]
    both = ~np.isnan(oc)
    assert np.array_equal(np.isnan(gc), np.isnan(oc))
    assert np.max(np.abs(gc[both] - oc[both]) / np.maximum(np.abs(oc[both]), 1.0)) < POS_TOL
    # k^0 is restored from the entry energy: E is kept to rounding
    e = np.abs(g["c1"][0] - g["c0"][0]) / np.abs(g["c0"][0])
    assert np.max(e[g["status"] != K.FAILED]) < 1e-12


def test_coordinate_time_particles_parity(ctx):
    """Time-like geodesics of the particle workload (a strided sample of 256 of
    its 2^20 draws) in coordinate time to t = 1e4 M: against the oracle's
    coordinate-time integration, and against the library's own affine
    integration of the same particles (the same curves by a different
    variable and step sequence)."""
    say("particles DOPRI5_T")
    pw = W.particles()
    idx = np.arange(0, 1 << 20, 4099)[:256]
    a, x3, v3 = pw["a"][idx], pw["x3"][:, idx].copy(), pw["v3"][:, idx].copy()
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()  # noqa: E731
    st = K.State(len(idx))
    ctx.kh_init_geodesics(K.TIMELIKE, t(a), t(x3), t(v3), st)
    p = K.kh_default_params(method=K.DOPRI5_T, t_end=1e4, r_escape=1e4)
    ctx.kh_integrate(p, st)
    g = st.numpy()
    o = O.integrate(O.timelike(a, x3, v3), oracle_params(p))
    assert np.array_equal(g["status"], o["status"])
    landed = g["status"] == K.T_END
    assert landed.mean() > 0.95
    assert np.all(g["s"][0, landed] == 1e4)  # the clipped last step ends on t_end exactly
    d = rel_pos(g["s"], o["s"])
    say(f"  vs oracle: max rel pos {d.max():.2e}, median {np.median(d):.2e}")
    assert d.max() < 1e-6
    # against the affine integration of the same particles
    sa = K.State(len(idx))
    ctx.kh_init_geodesics(K.TIMELIKE, t(a), t(x3), t(v3), sa)
    ctx.kh_integrate(K.kh_default_params(t_end=1e4, r_escape=1e4), sa)
    ga = sa.numpy()
    both = landed & (ga["status"] == K.T_END)
    da = rel_pos(g["s"][:, both], ga["s"][:, both])
    say(f"  vs affine: max rel pos {da.max():.2e}, median {np.median(da):.2e}, p90 {np.quantile(da, 0.9):.2e}")
    # Different variable, different steps: the two agree to the global error
    # of an rtol 1e-8 integration over up to a few hundred orbits.  The phase
    # error of orbits near r0 = 6 grows with the orbit count in either
    # formulation, so the tail reaches 1e-2; the bulk agrees to ~1e-7.
    assert np.median(da) < 1e-5 and np.quantile(da, 0.9) < 1e-4
    e = np.abs(g["c1"][0] - g["c0"][0]) / np.abs(g["c0"][0])
    assert np.max(e[landed]) < 1e-12


@pytest.mark.parametrize("method", [K.DOPRI5, K.DOPRI5_T])
def test_dense_output_parity(ctx, method):
    """Dense output at 40 coordinate times (method (ii) of Sec. 2.2) for a
    sample of the particle workload and for the rays of a small image, in the
    affine parameter and in coordinate time, against the oracle's dense
    output element by element; targets a ray does not reach stay NaN."""
    say(f"dense output method={method}")
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()  # noqa: E731
    # particles
    pw = W.particles()
    idx = np.arange(0, 1 << 20, 8191)[:128]
    a, x3, v3 = pw["a"][idx], pw["x3"][:, idx].copy(), pw["v3"][:, idx].copy()
    t_out = np.concatenate([[0.0], np.sort(np.random.default_rng(5).uniform(1.0, 3000.0, 38)), [3000.0]])
    st = K.State(len(idx), t_out=t_out)
    ctx.kh_init_geodesics(K.TIMELIKE, t(a), t(x3), t(v3), st)
    p = K.kh_default_params(method=method, t_end=3000.0, r_escape=1e4)
    ctx.kh_integrate(p, st)
    g = st.numpy()
    o = O.integrate(O.timelike(a, x3, v3), oracle_params(p), t_out=t_out)
    assert np.array_equal(g["status"], o["status"])
    assert np.array_equal(np.isnan(g["s_out"]), np.isnan(o["s_out"]))
    fin = ~np.isnan(o["s_out"])
    assert fin[:, :, 0].sum() >= 0.9 * fin[:, :, 0].size
    assert np.all(g["s_out"][:, :, 0][fin[:, :, 0]] == np.broadcast_to(t_out, fin.shape[:2])[fin[:, :, 0]])
    d = np.abs(g["s_out"] - o["s_out"])[fin] / np.maximum(np.abs(o["s_out"][fin]), 1.0)
    say(f"  particles: max rel {d.max():.2e}")
    assert d.max() < 1e-6
    # image rays (null): targets along the way in
    cam = W.Camera(0.9, 1000.0, 40.0, -8, 8, -8, 8, 23, 19)
    t_img = np.linspace(0.0, 1900.0, 20)
    st = K.State(cam.n, t_out=t_img)
    ctx.kh_init_rays([kcam(cam)], st)
    pi = K.kh_default_params(method=method)
    ctx.kh_integrate(pi, st)
    g = st.numpy()
    init = O.camera_rays(cam.a, cam.r_obs, cam.incl, cam.alpha_min, cam.alpha_max, cam.beta_min, cam.beta_max,
                         cam.width, cam.height)
    oo = O.integrate(init, oracle_params(pi), t_out=t_img)
    assert np.array_equal(g["status"], oo["status"])
    assert np.array_equal(np.isnan(g["s_out"]), np.isnan(oo["s_out"]))
    fin = ~np.isnan(oo["s_out"])
    d = np.abs(g["s_out"] - oo["s_out"])[fin] / np.maximum(np.abs(oo["s_out"][fin]), 1.0)
    say(f"  image: max rel {d.max():.2e}, targets reached {fin[:, :, 0].mean():.2f}")
    assert d.max() < 1e-6
