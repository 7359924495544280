"""Python binding of libkerrhip (the C ABI in include/kerrhip.h).

Argument marshalling only: every step of the geodesic integration runs in the
library's HIP kernels.  PyTorch supplies device memory and streams.  The
functions ``kh_*`` mirror the C entry points one for one; ``Context`` and
``State`` are conveniences that allocate the structure-of-arrays tensors and
raise on error codes.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # loaded first so the library binds to the same HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkerrhip.so")

KH_OK, KH_EINVAL, KH_EHIP, KH_EUNSUPPORTED, KH_ENOMEM = 0, -1, -2, -3, -4
ACTIVE, CAPTURED, ESCAPED, T_END, MAX_STEPS, FAILED = range(6)
NULL, TIMELIKE = 0, 1
RK4, DOPRI5, DOPRI5_T = 0, 1, 2
P64, P32, PMIXED = 0, 1, 2
RHS_FACTORED, RHS_PAPER, RHS_BL = 0, 1, 2
SOA, AOS = 0, 1


class kh_camera(C.Structure):
    _fields_ = [("a", C.c_double), ("r_obs", C.c_double), ("incl", C.c_double), ("alpha_min", C.c_double),
                ("alpha_max", C.c_double), ("beta_min", C.c_double), ("beta_max", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32)]


class kh_state(C.Structure):
    _fields_ = [("n", C.c_int64), ("s", C.c_void_p), ("spin", C.c_void_p), ("kind", C.c_void_p),
                ("h", C.c_void_p), ("lam", C.c_void_p), ("phi", C.c_void_p), ("status", C.c_void_p),
                ("n_acc", C.c_void_p), ("n_rej", C.c_void_p), ("cross", C.c_void_p), ("n_cross", C.c_void_p),
                ("k_cross", C.c_int32), ("c0", C.c_void_p), ("c1", C.c_void_p), ("order", C.c_void_p),
                ("n_out", C.c_int32), ("t_out", C.c_void_p), ("s_out", C.c_void_p), ("perm", C.c_void_p)]


class kh_params(C.Structure):
    _fields_ = [("method", C.c_int32), ("precision", C.c_int32), ("rhs_form", C.c_int32), ("k_cross", C.c_int32),
                ("h_coeff", C.c_double), ("rtol", C.c_double), ("atol", C.c_double), ("hmax_coeff", C.c_double),
                ("r_h_factor", C.c_double), ("r_escape", C.c_double), ("t_end", C.c_double),
                ("r_fp64", C.c_double), ("max_steps", C.c_int64), ("block_size", C.c_int32),
                ("grid_blocks", C.c_int32), ("refill_min", C.c_int32), ("waves_per_eu", C.c_int32),
                ("queue_parts", C.c_int32), ("mixed_split", C.c_int32)]


class kh_flop_counts(C.Structure):
    _fields_ = [("add", C.c_int64), ("mul", C.c_int64), ("div", C.c_int64), ("sqrt", C.c_int64),
                ("step_add", C.c_int64), ("step_mul", C.c_int64), ("step_div", C.c_int64),
                ("step_sqrt", C.c_int64), ("trig", C.c_int64)]


class kh_fixed_params(C.Structure):
    _fields_ = [("rhs_form", C.c_int32), ("layout", C.c_int32), ("precision", C.c_int32), ("nsteps", C.c_int32),
                ("spin", C.c_double), ("h_coeff", C.c_double), ("r_stop", C.c_double), ("r_escape", C.c_double)]


class kh_mlp(C.Structure):
    _fields_ = [("params", C.c_void_p), ("adam_m", C.c_void_p), ("adam_v", C.c_void_p), ("wb", C.c_void_p),
                ("wbt", C.c_void_p)]


class kh_mlp_loss_w(C.Structure):
    _fields_ = [("r", C.c_float), ("phi", C.c_float), ("g", C.c_float), ("capture", C.c_float)]


class kh_mlp_fallback(C.Structure):
    _fields_ = [("tau", C.c_float), ("shadow_band", C.c_float), ("r_min", C.c_float)]


class kh_adam(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("step", C.c_int32)]


MLP_NPARAMS = 199684
MLP_WB_ELEMS = 208896
MLP_WBT_ELEMS = 204800

EXPORTS = ["kh_create", "kh_destroy", "kh_last_error", "kh_default_params", "kh_init_rays", "kh_init_rays_list",
           "kh_init_geodesics", "kh_integrate", "kh_integrate_noalloc", "kh_read_state", "kh_stats", "kh_stats_device",
           "kh_rhs", "kh_flops", "kh_rk4_fixed", "kh_pack_fixed"]
MLP_EXPORTS = ["kh_mlp_work_bytes", "kh_mlp_sync", "kh_mlp_forward", "kh_mlp_image", "kh_mlp_targets", "kh_mlp_grad",
               "kh_mlp_train_step", "kh_init_rays_pixels", "kh_image_from_state"]

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(hipcc --offload-arch=gfx950); there is no fallback path")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        P = C.POINTER
        L.kh_create.argtypes = [P(vp), C.c_int]
        L.kh_destroy.argtypes = [vp]
        L.kh_last_error.argtypes = [vp]
        L.kh_last_error.restype = C.c_char_p
        L.kh_default_params.argtypes = [P(kh_params)]
        L.kh_default_params.restype = None
        L.kh_init_rays.argtypes = [vp, P(kh_camera), i32, P(kh_state), vp]
        L.kh_init_rays_list.argtypes = [vp, vp, vp, vp, vp, d, P(kh_state), vp]
        L.kh_init_geodesics.argtypes = [vp, i32, vp, vp, vp, P(kh_state), vp]
        L.kh_integrate.argtypes = [vp, P(kh_params), P(kh_state), vp]
        L.kh_integrate_noalloc.argtypes = [P(kh_params), P(kh_state), vp, C.c_char_p, i32]
        L.kh_read_state.argtypes = [vp, P(kh_state), i64, i64, vp, vp, vp]
        L.kh_stats.argtypes = [vp, P(kh_state), P(i64), vp]
        L.kh_stats_device.argtypes = [vp, P(kh_state), vp, vp]
        L.kh_rhs.argtypes = [vp, i32, i32, vp, vp, vp, i64, vp]
        L.kh_flops.argtypes = [i32, i32, P(kh_flop_counts)]
        L.kh_rk4_fixed.argtypes = [vp, P(kh_fixed_params), vp, vp, vp, i64, vp]
        L.kh_pack_fixed.argtypes = [vp, P(kh_fixed_params), vp, vp, i64, vp]
        L.kh_mlp_work_bytes.argtypes = [i32]
        L.kh_mlp_work_bytes.restype = i64
        L.kh_mlp_sync.argtypes = [vp, P(kh_mlp), vp]
        L.kh_mlp_forward.argtypes = [vp, P(kh_mlp), vp, vp, i64, vp]
        L.kh_mlp_image.argtypes = [vp, P(kh_mlp), P(kh_camera), P(kh_mlp_fallback), vp, vp, vp, vp]
        L.kh_mlp_targets.argtypes = [vp, P(kh_state), vp, vp, vp, vp, vp, vp, vp, vp]
        L.kh_mlp_grad.argtypes = [vp, P(kh_mlp), vp, i32, vp, vp, vp, i32, P(kh_mlp_loss_w), vp, vp, vp]
        L.kh_mlp_train_step.argtypes = [vp, P(kh_mlp), vp, i32, vp, vp, vp, i32, P(kh_mlp_loss_w), P(kh_adam), vp,
                                        vp]
        L.kh_init_rays_pixels.argtypes = [vp, P(kh_camera), vp, P(kh_state), vp]
        L.kh_image_from_state.argtypes = [vp, P(kh_state), vp, vp, vp]
        for name in EXPORTS + MLP_EXPORTS:
            if name not in ("kh_last_error", "kh_default_params", "kh_mlp_work_bytes"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


class KerrHipError(RuntimeError):
    pass


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------------------
# One-for-one entry points.
# ---------------------------------------------------------------------------
def kh_default_params(**overrides) -> kh_params:
    p = kh_params()
    lib().kh_default_params(C.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def kh_integrate_noalloc(params: kh_params, st: "State", stream=None):
    """kh_integrate without a context or any allocation (static work-queue
    counters on the current device); raises KerrHipError on an error code."""
    err = C.create_string_buffer(256)
    rc = lib().kh_integrate_noalloc(C.byref(params), C.byref(st.c), _stream(stream), err, len(err))
    if rc != KH_OK:
        raise KerrHipError(f"kh_integrate_noalloc failed ({rc}): {err.value.decode()}")


def kh_flops(method=DOPRI5, rhs_form=RHS_FACTORED) -> dict:
    out = kh_flop_counts()
    rc = lib().kh_flops(method, rhs_form, C.byref(out))
    if rc != KH_OK:
        raise KerrHipError(f"kh_flops failed ({rc})")
    return {f: getattr(out, f) for f, _ in kh_flop_counts._fields_}


class Context:
    """A library context bound to one device (``kh_create`` / ``kh_destroy``)."""

    def __init__(self, device: int = 0):
        self.handle = C.c_void_p()
        rc = lib().kh_create(C.byref(self.handle), device)
        if rc != KH_OK:
            raise KerrHipError(f"kh_create failed ({rc})")
        self.device = device

    def close(self):
        if self.handle:
            lib().kh_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != KH_OK:
            msg = lib().kh_last_error(self.handle)
            raise KerrHipError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")

    def kh_init_rays(self, cams, st: "State", stream=None, n_cams=None):
        """cams: list of kh_camera, or None to reuse the table of the last call
        (then pass n_cams; this form is a single kernel launch)."""
        if cams is None:
            self._check(lib().kh_init_rays(self.handle, None, n_cams, C.byref(st.c), _stream(stream)),
                        "kh_init_rays")
            return
        arr = (kh_camera * len(cams))(*cams)
        self._check(lib().kh_init_rays(self.handle, arr, len(cams), C.byref(st.c), _stream(stream)), "kh_init_rays")

    def kh_stats_device(self, st: "State", out, stream=None):
        if out.dtype != torch.int64 or not out.is_cuda or out.numel() < 8:
            raise ValueError("out must be an int64 CUDA tensor with 8 elements")
        self._check(lib().kh_stats_device(self.handle, C.byref(st.c), out.data_ptr(), _stream(stream)),
                    "kh_stats_device")

    def kh_init_rays_list(self, spin, incl, alpha, beta, r_obs, st: "State", stream=None):
        for t in (spin, incl, alpha, beta):
            _check_vec(t, st.n)
        self._check(lib().kh_init_rays_list(self.handle, spin.data_ptr(), incl.data_ptr(), alpha.data_ptr(),
                                            beta.data_ptr(), float(r_obs), C.byref(st.c), _stream(stream)),
                    "kh_init_rays_list")

    def kh_init_geodesics(self, kind, spin, x3, v3, st: "State", stream=None):
        _check_vec(spin, st.n)
        for t in (x3, v3):
            if t.dtype != torch.float64 or not t.is_cuda or tuple(t.shape) != (3, st.n) or not t.is_contiguous():
                raise ValueError("x3, v3 must be contiguous float64 CUDA tensors of shape (3, n)")
        self._check(lib().kh_init_geodesics(self.handle, kind, spin.data_ptr(), x3.data_ptr(), v3.data_ptr(),
                                            C.byref(st.c), _stream(stream)), "kh_init_geodesics")

    def kh_integrate(self, params: kh_params, st: "State", stream=None):
        self._check(lib().kh_integrate(self.handle, C.byref(params), C.byref(st.c), _stream(stream)),
                    "kh_integrate")

    def kh_read_state(self, st: "State", first=0, count=None, stream=None, out=None):
        """Rows [first, first + count) of the state ([count][8] float64) and
        their statuses (int32) in host memory.  out: optional (states,
        statuses) pair of contiguous CPU torch tensors of those shapes and
        dtypes to fill instead of new numpy arrays; page-locked ones
        (pin_memory=True) are copied into directly, without the runtime's
        staging through its own pinned buffers."""
        import numpy as np

        count = st.n - first if count is None else count
        if out is None:
            hs = np.zeros((count, 8))
            hst = np.zeros(count, np.int32)
            ptrs = (hs.ctypes.data, hst.ctypes.data)
        else:
            hs, hst = out
            if (hs.device.type != "cpu" or hs.dtype != torch.float64 or tuple(hs.shape) != (count, 8)
                    or not hs.is_contiguous()):
                raise ValueError("out[0] must be a contiguous CPU float64 tensor of shape (count, 8)")
            if hst.device.type != "cpu" or hst.dtype != torch.int32 or tuple(hst.shape) != (count,) \
                    or not hst.is_contiguous():
                raise ValueError("out[1] must be a contiguous CPU int32 tensor of shape (count,)")
            ptrs = (hs.data_ptr(), hst.data_ptr())
        self._check(lib().kh_read_state(self.handle, C.byref(st.c), first, count, ptrs[0], ptrs[1],
                                        _stream(stream)), "kh_read_state")
        return hs, hst

    def kh_stats(self, st: "State", stream=None):
        out = (C.c_int64 * 8)()
        self._check(lib().kh_stats(self.handle, C.byref(st.c), out, _stream(stream)), "kh_stats")
        v = list(out)
        return dict(status_counts=v[:6], n_acc=v[6], n_rej=v[7])

    def kh_rhs(self, precision, rhs_form, spin_chart, s, stream=None):
        n = spin_chart.numel()
        _check_vec(spin_chart, n)
        if s.dtype != torch.float64 or tuple(s.shape) != (8, n) or not s.is_contiguous() or not s.is_cuda:
            raise ValueError("s must be a contiguous float64 CUDA tensor of shape (8, n)")
        acc = torch.empty((4, n), dtype=torch.float64, device=s.device)
        self._check(lib().kh_rhs(self.handle, precision, rhs_form, spin_chart.data_ptr(), s.data_ptr(),
                                 acc.data_ptr(), n, _stream(stream)), "kh_rhs")
        return acc


    def kh_pack_fixed(self, params: kh_fixed_params, s, y, stream=None):
        """Kerr-Schild states s (float64 CUDA tensor (8, n)) into y, a CUDA
        tensor of 8 n values in the chart, precision and layout of params."""
        n = s.shape[1] if s.dim() == 2 else 0
        if s.dtype != torch.float64 or tuple(s.shape) != (8, n) or not s.is_contiguous() or not s.is_cuda:
            raise ValueError("s must be a contiguous float64 CUDA tensor of shape (8, n)")
        _check_fixed_y(params, y, n)
        self._check(lib().kh_pack_fixed(self.handle, C.byref(params), s.data_ptr(), y.data_ptr(), n,
                                        _stream(stream)), "kh_pack_fixed")

    def kh_rk4_fixed(self, params: kh_fixed_params, y, status, steps, stream=None):
        """params.nsteps RK4 steps on y (8 n values, chart / precision / layout
        of params); status and steps: int32 CUDA tensors of n elements."""
        n = status.numel()
        for t in (status, steps):
            if t.dtype != torch.int32 or not t.is_cuda or t.numel() != n or not t.is_contiguous():
                raise ValueError("status and steps must be contiguous int32 CUDA tensors of one length")
        _check_fixed_y(params, y, n)
        self._check(lib().kh_rk4_fixed(self.handle, C.byref(params), y.data_ptr(), status.data_ptr(),
                                       steps.data_ptr(), n, _stream(stream)), "kh_rk4_fixed")


class FixedState:
    """Device arrays of ``kh_rk4_fixed`` for the n geodesics of Kerr-Schild
    states ``s_ks`` (float64 CUDA (8, n), e.g. ``State.s`` after an init call),
    converted by ``kh_pack_fixed`` to the chart, precision and layout of
    ``params``.  ``status`` starts as given (default all active)."""

    def __init__(self, ctx: "Context", params: kh_fixed_params, s_ks, status=None, stream=None):
        n = s_ks.shape[1]
        self.n = n
        self.params = params
        dt = torch.float64 if params.precision == P64 else torch.float32
        self.y = torch.empty(8 * n, dtype=dt, device=s_ks.device)
        i32 = dict(dtype=torch.int32, device=s_ks.device)
        self.status = torch.zeros(n, **i32) if status is None else status.to(**i32).clone()
        self.steps = torch.zeros(n, **i32)
        ctx.kh_pack_fixed(params, s_ks, self.y, stream)

    def components(self):
        """(8, n) view of y whatever its layout."""
        return self.y.view(8, self.n) if self.params.layout == SOA else self.y.view(self.n, 8).t()


def fixed_params(rhs_form=RHS_FACTORED, layout=SOA, precision=P64, nsteps=1024, spin=0.0, h_coeff=1.0 / 256,
                 r_stop=0.0, r_escape=1e30) -> kh_fixed_params:
    return kh_fixed_params(rhs_form, layout, precision, nsteps, spin, h_coeff, r_stop, r_escape)


def _check_fixed_y(params, y, n):
    dt = {P64: torch.float64, P32: torch.float32}.get(params.precision, y.dtype)  # else the library refuses
    if y.dtype != dt or not y.is_cuda or y.numel() != 8 * n or not y.is_contiguous():
        raise ValueError(f"y must be a contiguous {dt} CUDA tensor of 8 n = {8 * n} elements")


def _check_vec(t, n):
    if t.dtype != torch.float64 or not t.is_cuda or t.numel() != n or not t.is_contiguous():
        raise ValueError(f"expected a contiguous float64 CUDA tensor with {n} elements")


def _dev(t, dtype, n=None, align=16):
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or (n is not None and t.numel() != n):
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor" + (f" with {n} elements" if n else ""))
    if t.data_ptr() % align:
        raise ValueError(f"tensor must be {align}-byte aligned")
    return t.data_ptr()


class Mlp:
    """Surrogate network tensors (FP32 master weights, Adam moments, BF16 copies)."""

    def __init__(self, params=None, train=True, device="cuda"):
        import numpy as np

        f32 = dict(dtype=torch.float32, device=device)
        if params is None:
            params = np.zeros(MLP_NPARAMS, np.float32)
        self.params = torch.tensor(np.asarray(params, np.float32), **f32)
        self.adam_m = torch.zeros(MLP_NPARAMS, **f32) if train else None
        self.adam_v = torch.zeros(MLP_NPARAMS, **f32) if train else None
        self.wb = torch.zeros(MLP_WB_ELEMS, dtype=torch.int16, device=device)
        self.wbt = torch.zeros(MLP_WBT_ELEMS, dtype=torch.int16, device=device) if train else None
        p = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
        self.c = kh_mlp(p(self.params), p(self.adam_m), p(self.adam_v), p(self.wb), p(self.wbt))


def kh_mlp_work_bytes(max_batch: int) -> int:
    return lib().kh_mlp_work_bytes(max_batch)


def _mlp_methods():
    def kh_mlp_sync(self, net: Mlp, stream=None):
        self._check(lib().kh_mlp_sync(self.handle, C.byref(net.c), _stream(stream)), "kh_mlp_sync")

    def kh_mlp_forward(self, net: Mlp, x, y, stream=None):
        m = x.shape[0]
        _dev(x, torch.float32, 4 * m)
        _dev(y, torch.float32, 4 * m)
        self._check(lib().kh_mlp_forward(self.handle, C.byref(net.c), x.data_ptr(), y.data_ptr(), m,
                                         _stream(stream)), "kh_mlp_forward")

    def kh_mlp_image(self, net: Mlp, cam: kh_camera, tau, out, fb_ids, fb_count, stream=None, shadow_band=0.0,
                     r_min=0.0):
        """Fallback rules: capture band tau, shadow-edge band (M) and strong-field
        radius r_min (M), as kh_mlp_fallback."""
        npix = cam.width * cam.height
        _dev(out, torch.float32, 4 * npix)
        _dev(fb_ids, torch.int32, npix, align=4)
        _dev(fb_count, torch.int32, 1, align=4)
        fb = kh_mlp_fallback(float(tau), float(shadow_band), float(r_min))
        self._check(lib().kh_mlp_image(self.handle, C.byref(net.c), C.byref(cam), C.byref(fb), out.data_ptr(),
                                       fb_ids.data_ptr(), fb_count.data_ptr(), _stream(stream)), "kh_mlp_image")

    def kh_mlp_targets(self, st: "State", alpha, beta, spin, incl, x, t, mask, stream=None):
        for v in (alpha, beta, spin, incl):
            _dev(v, torch.float64, st.n, align=8)
        _dev(x, torch.float32, 4 * st.n)
        _dev(t, torch.float32, 4 * st.n)
        _dev(mask, torch.uint8, st.n, align=1)
        self._check(lib().kh_mlp_targets(self.handle, C.byref(st.c), alpha.data_ptr(), beta.data_ptr(),
                                         spin.data_ptr(), incl.data_ptr(), x.data_ptr(), t.data_ptr(),
                                         mask.data_ptr(), _stream(stream)), "kh_mlp_targets")

    def kh_mlp_grad(self, net: Mlp, work, max_batch, x, t, mask, b, grad, loss, stream=None, loss_w=None):
        """loss_w: (r, phi, g, capture) weights of the loss terms, or None for all 1."""
        _dev(grad, torch.float32, MLP_NPARAMS)
        lw = C.byref(kh_mlp_loss_w(*loss_w)) if loss_w is not None else None
        self._check(lib().kh_mlp_grad(self.handle, C.byref(net.c), work.data_ptr(), max_batch, x.data_ptr(),
                                      t.data_ptr(), mask.data_ptr(), b, lw, grad.data_ptr(), loss.data_ptr(),
                                      _stream(stream)), "kh_mlp_grad")

    def kh_mlp_train_step(self, net: Mlp, work, max_batch, x, t, mask, b, opt: kh_adam, loss, stream=None,
                          loss_w=None):
        lw = C.byref(kh_mlp_loss_w(*loss_w)) if loss_w is not None else None
        self._check(lib().kh_mlp_train_step(self.handle, C.byref(net.c), work.data_ptr(), max_batch, x.data_ptr(),
                                            t.data_ptr(), mask.data_ptr(), b, lw, C.byref(opt), loss.data_ptr(),
                                            _stream(stream)), "kh_mlp_train_step")

    def kh_init_rays_pixels(self, cam: kh_camera, pix, st: "State", stream=None):
        _dev(pix, torch.int32, st.n, align=4)
        self._check(lib().kh_init_rays_pixels(self.handle, C.byref(cam), pix.data_ptr(), C.byref(st.c),
                                              _stream(stream)), "kh_init_rays_pixels")

    def kh_image_from_state(self, st: "State", pix, out, stream=None):
        if pix is not None:
            _dev(pix, torch.int32, st.n, align=4)
        self._check(lib().kh_image_from_state(self.handle, C.byref(st.c), pix.data_ptr() if pix is not None else None,
                                              out.data_ptr(), _stream(stream)), "kh_image_from_state")

    for f in (kh_mlp_sync, kh_mlp_forward, kh_mlp_image, kh_mlp_targets, kh_mlp_grad, kh_mlp_train_step,
              kh_init_rays_pixels, kh_image_from_state):
        setattr(Context, f.__name__, f)


_mlp_methods()


class State:
    """Structure-of-arrays geodesic state in device memory (torch tensors).

    schedule: "tiles" (default; True is the same) allocates the 64-ray tile
    order, which keeps a wave's rays adjacent (images); "geodesics" allocates
    the per-geodesic schedule `perm` (sets in no particular order, such as
    particles); None or False: natural order."""

    def __init__(self, n: int, k_cross: int = 0, constants: bool = True, device="cuda", schedule="tiles",
                 t_out=None):
        if n < 1:
            raise ValueError("n must be >= 1")
        if schedule is True:
            schedule = "tiles"
        if schedule not in ("tiles", "geodesics", None, False):
            raise ValueError("schedule must be 'tiles', 'geodesics' or None")
        f64 = dict(dtype=torch.float64, device=device)
        i32 = dict(dtype=torch.int32, device=device)
        self.n = n
        self.k_cross = k_cross
        self.s = torch.zeros((8, n), **f64)
        self.spin = torch.zeros(n, **f64)
        self.kind = torch.zeros(n, **i32)
        self.h = torch.zeros(n, **f64)
        self.lam = torch.zeros(n, **f64)
        self.phi = torch.zeros(n, **f64)
        self.status = torch.zeros(n, **i32)
        self.n_acc = torch.zeros(n, **i32)
        self.n_rej = torch.zeros(n, **i32)
        self.cross = torch.full((n, k_cross, 3), float("nan"), **f64) if k_cross > 0 else None
        self.n_cross = torch.zeros(n, **i32) if k_cross > 0 else None
        self.c0 = torch.zeros((4, n), **f64) if constants else None
        self.c1 = torch.zeros((4, n), **f64) if constants else None
        # tile order for the integrator (written by the init calls); natural order until then
        self.order = torch.arange((n + 63) // 64, **i32) if schedule == "tiles" else None
        # per-geodesic schedule (replaces the tile order when present)
        self.perm = torch.arange(n, **i32) if schedule == "geodesics" else None
        # dense output at ascending coordinate times: s_out [n][len(t_out)][8], NaN until reached
        if t_out is not None and len(t_out) > 0:
            self.t_out = torch.as_tensor(t_out, **f64).contiguous()
            self.s_out = torch.full((n, len(self.t_out), 8), float("nan"), **f64)
        else:
            self.t_out = self.s_out = None
        n_out = 0 if self.t_out is None else len(self.t_out)
        p = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
        self.c = kh_state(n, p(self.s), p(self.spin), p(self.kind), p(self.h), p(self.lam), p(self.phi),
                          p(self.status), p(self.n_acc), p(self.n_rej), p(self.cross), p(self.n_cross), k_cross,
                          p(self.c0), p(self.c1), p(self.order), n_out, p(self.t_out), p(self.s_out), p(self.perm))

    _ARRAYS = ("s", "spin", "kind", "h", "lam", "phi", "status", "n_acc", "n_rej", "cross", "n_cross", "c0", "c1",
               "order", "t_out", "s_out", "perm")

    def numpy(self) -> dict:
        """Host copy of every array (for checks; synchronises)."""
        out = {}
        for name in self._ARRAYS:
            if name == "t_out":
                continue
            t = getattr(self, name)
            out[name] = t.cpu().numpy() if t is not None else None
        return out

    def save(self, path) -> None:
        """Checkpoint: every array of the state (positions and momenta, step
        sizes, affine parameters, statuses, counters, crossing records,
        constants, schedule, dense output) to one .npz file.  The state is the
        whole of an integration's progress, so State.load(path) followed by
        kh_integrate continues bitwise as the uninterrupted run would."""
        import numpy as np

        arrays = {name: getattr(self, name).cpu().numpy() for name in self._ARRAYS if getattr(self, name) is not None}
        np.savez(path, n=np.int64(self.n), k_cross=np.int64(self.k_cross), **arrays)

    @classmethod
    def load(cls, path, device="cuda") -> "State":
        """A State holding a checkpoint written by save() (plain arrays, read
        without unpickling)."""
        import numpy as np

        with np.load(path, allow_pickle=False) as d:
            schedule = "geodesics" if "perm" in d.files else ("tiles" if "order" in d.files else None)
            st = cls(int(d["n"]), k_cross=int(d["k_cross"]), constants="c0" in d.files, device=device,
                     schedule=schedule, t_out=d["t_out"] if "t_out" in d.files else None)
            for name in cls._ARRAYS:
                if name in d.files:
                    getattr(st, name).copy_(torch.from_numpy(d[name]))
        return st
