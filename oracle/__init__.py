"""FP64 CPU oracle for Cartesian Kerr-Schild geodesic integration.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
never imports, links or calls it, and it shares no source with the GPU path.

The numerics live in ``kerr_oracle.cpp`` (plain Christoffel form of the geodesic
equation, eq:geo of Sec. 2.1, on the metric def:CKS with dual-number
derivatives and a generic 4x4 inverse; classic RK4 of Sec. 3 and a
Dormand-Prince 5(4) pair; the same Christoffel form on the Boyer-Lindquist
line element of Sec. 2.1 for the chart comparison of Sec. 4).  This module is
argument marshalling over ctypes.

Array layouts follow the GPU library's: states are ``[8][n]`` (x^0..x^3,
k^0..k^3), constants ``[4][n]`` = (E, L_z, Q, mu^2), crossings ``[n][K][3]`` =
(r, phi, g).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kerr_oracle.cpp")
_LIB = os.path.join(_HERE, "libkerr_oracle.so")

ACTIVE, CAPTURED, ESCAPED, T_END, MAX_STEPS, FAILED = range(6)
NULL, TIMELIKE = 0, 1
RK4, DOPRI5, DOPRI5_T = 0, 1, 2  # DOPRI5_T: Dormand-Prince in coordinate time


def build(force: bool = True) -> str:
    """Compile the oracle with g++ into ``oracle/libkerr_oracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [
        ("method", C.c_int32),
        ("k_cross", C.c_int32),
        ("h_coeff", C.c_double),
        ("rtol", C.c_double),
        ("atol", C.c_double),
        ("hmax_coeff", C.c_double),
        ("r_h_factor", C.c_double),
        ("r_escape", C.c_double),
        ("t_end", C.c_double),
        ("max_steps", C.c_int64),
    ]


@dataclass
class Params:
    """Integration rules (same meaning as the GPU library's parameter block)."""

    method: int = DOPRI5
    k_cross: int = 0
    h_coeff: float = 0.01
    rtol: float = 1e-8
    atol: float = 1e-8
    hmax_coeff: float = 0.1
    r_h_factor: float = 1.01
    r_escape: float = 1000.0
    t_end: float = 0.0
    max_steps: int = 1_000_000

    def c(self) -> _Params:
        return _Params(self.method, self.k_cross, self.h_coeff, self.rtol, self.atol, self.hmax_coeff,
                       self.r_h_factor, self.r_escape, self.t_end, self.max_steps)


_lib = None


def default_threads() -> int:
    """Host threads for the oracle's pool: the CPUs this process may run on,
    at most 16."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.POINTER
        d, i32, i64 = C.c_double, C.c_int32, C.c_int64
        pd, pi32, pi64 = P(d), P(i32), P(i64)
        L.oracle_camera_rays.argtypes = [d, d, d, d, d, d, d, i32, i32, pi64, i64, d, pd, pd, pi32, pi32]
        L.oracle_list_rays.argtypes = [pd, pd, pd, pd, d, i64, pd, pd, pi32, pi32]
        L.oracle_timelike.argtypes = [pd, pd, pd, i64, pd, pd, pi32, pi32]
        L.oracle_integrate.argtypes = [P(_Params), i64, pd, pd, pi32, pd, pd, pi32, pi32, pi32, pd, pi32, pd, pd,
                                       i32]
        L.oracle_integrate_out.argtypes = [P(_Params), i64, pd, pd, pi32, pd, pd, pi32, pi32, pi32, pd, pi32, pd,
                                           pd, i32, pd, pd, i32]
        L.oracle_trajectory.argtypes = [P(_Params), d, pd, i64, pd]
        L.oracle_trajectory.restype = i64
        L.oracle_rhs.argtypes = [d, pd, pd, pd]
        L.oracle_metric.argtypes = [d, pd, pd, pd]
        L.oracle_radius.argtypes = [d, d, d, d]
        L.oracle_radius.restype = d
        L.oracle_constants.argtypes = [d, pd, pd, pd]
        L.oracle_redshift.argtypes = [d, d, d]
        L.oracle_redshift.restype = d
        L.oracle_dopri5_sho.argtypes = [pd, d, i64, d, pd]
        L.oracle_dopri5_sho_attempt.argtypes = [pd, d, d, d, pd, pd]
        L.oracle_dopri5_sho_attempt.restype = d
        L.oracle_controller_trace.argtypes = [P(_Params), d, i32, pd, i64, pd, pi32]
        L.oracle_controller_trace.restype = i64
        L.oracle_bl_metric.argtypes = [d, pd, pd, pd]
        L.oracle_bl_rhs.argtypes = [d, pd, pd, pd]
        L.oracle_bl_constants.argtypes = [d, pd, pd, pd]
        L.oracle_bl_to_ks.argtypes = [d, pd, pd, pd]
        L.oracle_ks_to_bl.argtypes = [d, i64, pd, pd]
        L.oracle_ks_to_bl.restype = i64
        L.oracle_rk4_fixed.argtypes = [i32, d, d, d, d, i32, i64, pd, pi32, pi32, i32]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def camera_rays(a, r_obs, incl, amin, amax, bmin, bmax, W, H, pix=None, perturb=0.0):
    """Initial states of image rays (pixel ids ``pix``; all pixels if None)."""
    pix = np.arange(W * H, dtype=np.int64) if pix is None else np.ascontiguousarray(pix, dtype=np.int64)
    n = len(pix)
    s = np.zeros((8, n))
    spin = np.zeros(n)
    kind = np.zeros(n, np.int32)
    status = np.zeros(n, np.int32)
    lib().oracle_camera_rays(a, r_obs, incl, amin, amax, bmin, bmax, W, H, _p(pix, C.c_int64), n, perturb,
                             _p(s, C.c_double), _p(spin, C.c_double), _p(kind, C.c_int32), _p(status, C.c_int32))
    return dict(s=s, spin=spin, kind=kind, status=status)


def list_rays(a, incl, alpha, beta, r_obs):
    a, incl, alpha, beta = map(_f64, (a, incl, alpha, beta))
    n = len(a)
    s = np.zeros((8, n))
    spin = np.zeros(n)
    kind = np.zeros(n, np.int32)
    status = np.zeros(n, np.int32)
    lib().oracle_list_rays(_p(a, C.c_double), _p(incl, C.c_double), _p(alpha, C.c_double), _p(beta, C.c_double),
                           r_obs, n, _p(s, C.c_double), _p(spin, C.c_double), _p(kind, C.c_int32),
                           _p(status, C.c_int32))
    return dict(s=s, spin=spin, kind=kind, status=status)


def timelike(a, x3, v3):
    a, x3, v3 = _f64(a), _f64(x3), _f64(v3)
    n = len(a)
    s = np.zeros((8, n))
    spin = np.zeros(n)
    kind = np.zeros(n, np.int32)
    status = np.zeros(n, np.int32)
    lib().oracle_timelike(_p(a, C.c_double), _p(x3, C.c_double), _p(v3, C.c_double), n, _p(s, C.c_double),
                          _p(spin, C.c_double), _p(kind, C.c_int32), _p(status, C.c_int32))
    return dict(s=s, spin=spin, kind=kind, status=status)


def integrate(init: dict, params: Params, nthreads: int = 0, t_out=None) -> dict:
    """Integrate every ACTIVE geodesic of ``init`` to termination.  With
    ``t_out`` (ascending coordinate times) the result also holds ``s_out``
    [n][len(t_out)][8]: the state at each time the geodesic reaches (NaN
    elsewhere)."""
    s = np.array(init["s"], dtype=np.float64, order="C", copy=True)
    n = s.shape[1]
    spin = _f64(init["spin"])
    kind = np.ascontiguousarray(init["kind"], dtype=np.int32)
    status = np.array(init["status"], dtype=np.int32, copy=True)
    lam = np.zeros(n)
    phi = np.zeros(n)
    n_acc = np.zeros(n, np.int32)
    n_rej = np.zeros(n, np.int32)
    K = max(params.k_cross, 0)
    cross = np.full((n, max(K, 1), 3), np.nan)
    n_cross = np.zeros(n, np.int32)
    c0 = np.zeros((4, n))
    c1 = np.zeros((4, n))
    cp = params.c()
    nthreads = nthreads or default_threads()
    t_out = np.zeros(0) if t_out is None else _f64(t_out)
    n_out = len(t_out)
    s_out = np.full((n, max(n_out, 1), 8), np.nan)
    rc = lib().oracle_integrate_out(C.byref(cp), n, _p(s, C.c_double), _p(spin, C.c_double), _p(kind, C.c_int32),
                                    _p(lam, C.c_double), _p(phi, C.c_double), _p(status, C.c_int32),
                                    _p(n_acc, C.c_int32), _p(n_rej, C.c_int32), _p(cross, C.c_double),
                                    _p(n_cross, C.c_int32), _p(c0, C.c_double), _p(c1, C.c_double), n_out,
                                    _p(t_out, C.c_double), _p(s_out, C.c_double), nthreads)
    if rc != 0:
        raise ValueError("oracle_integrate rejected its arguments")
    out = dict(s=s, lam=lam, phi=phi, status=status, n_acc=n_acc, n_rej=n_rej, cross=cross[:, :K],
               n_cross=n_cross, c0=c0, c1=c1)
    if n_out:
        out["s_out"] = s_out
    return out


def trajectory(params: Params, spin_chart: float, y0, max_out: int = 100000) -> np.ndarray:
    """Every accepted state of one geodesic as rows (lambda, x^0..x^3, k^0..k^3).

    With ``params.method == RK4`` the affine step is fixed to ``params.h_coeff``.
    """
    y0 = _f64(y0)
    out = np.zeros((max_out, 9))
    cp = params.c()
    m = lib().oracle_trajectory(C.byref(cp), spin_chart, _p(y0, C.c_double), max_out, _p(out, C.c_double))
    return out[:m]


def rhs(a, x, k):
    x, k = _f64(x), _f64(k)
    acc = np.zeros(4)
    lib().oracle_rhs(a, _p(x, C.c_double), _p(k, C.c_double), _p(acc, C.c_double))
    return acc


def metric(a, x):
    """(g[4][4], dg[4][4][4]) with dg[c] = d g / d x^c."""
    x = _f64(x)
    g = np.zeros(16)
    dg = np.zeros(64)
    lib().oracle_metric(a, _p(x, C.c_double), _p(g, C.c_double), _p(dg, C.c_double))
    return g.reshape(4, 4), dg.reshape(4, 4, 4)


def radius(a, x, y, z):
    return lib().oracle_radius(a, x, y, z)


def constants(a, x, k):
    x, k = _f64(x), _f64(k)
    out = np.zeros(4)
    lib().oracle_constants(a, _p(x, C.c_double), _p(k, C.c_double), _p(out, C.c_double))
    return out


def redshift(r, xi, a):
    return lib().oracle_redshift(r, xi, a)


def dopri5_sho(y0, h, nsteps, rtol=1e-8):
    y0 = _f64(y0)
    out = np.zeros(9)
    lib().oracle_dopri5_sho(_p(y0, C.c_double), h, nsteps, rtol, _p(out, C.c_double))
    return out[:8], out[8]


def dopri5_sho_attempt(y0, h, rtol, atol):
    """One Dormand-Prince attempt on y'' = -y: (y5, y4, error norm)."""
    y0 = _f64(y0)
    y5 = np.zeros(8)
    y4 = np.zeros(8)
    err = lib().oracle_dopri5_sho_attempt(_p(y0, C.c_double), h, rtol, atol, _p(y5, C.c_double),
                                          _p(y4, C.c_double))
    return y5, y4, err


def controller_trace(params: Params, spin_phys: float, kind: int, y0, max_rec: int = 100000):
    """Every Dormand-Prince attempt of one geodesic: rows (h, err, accepted,
    r after the attempt, status after the attempt), and (status, accepted
    steps, rejected attempts)."""
    y0 = _f64(y0)
    out = np.zeros((max_rec, 5))
    res = np.zeros(3, np.int32)
    m = lib().oracle_controller_trace(C.byref(params.c()), spin_phys, kind, _p(y0, C.c_double), max_rec,
                                      _p(out, C.c_double), _p(res, C.c_int32))
    if m < 0:
        raise ValueError("oracle_controller_trace rejected its arguments")
    return out[:m], tuple(int(v) for v in res)


# ---------------------------------------------------------------------------
# Boyer-Lindquist chart and fixed-step RK4 in either chart (Sec. 4, tab:elapse).
# BL states are (t, r, theta, phi, k^t, k^r, k^theta, k^phi).
# ---------------------------------------------------------------------------
CHARTS = {"ks": 0, "bl": 1}


def bl_metric(a, x):
    x = _f64(x)
    g = np.zeros(16)
    dg = np.zeros(64)
    lib().oracle_bl_metric(a, _p(x, C.c_double), _p(g, C.c_double), _p(dg, C.c_double))
    return g.reshape(4, 4), dg.reshape(4, 4, 4)


def bl_rhs(a, x, k):
    x, k = _f64(x), _f64(k)
    acc = np.zeros(4)
    lib().oracle_bl_rhs(a, _p(x, C.c_double), _p(k, C.c_double), _p(acc, C.c_double))
    return acc


def bl_constants(a, x, k):
    """(E, L_z, Q, mu^2) of a Boyer-Lindquist state."""
    x, k = _f64(x), _f64(k)
    out = np.zeros(4)
    lib().oracle_bl_constants(a, _p(x, C.c_double), _p(k, C.c_double), _p(out, C.c_double))
    return out


def bl_to_ks(a, xbl):
    """Kerr-Schild point and Jacobian d x_KS / d x_BL of a Boyer-Lindquist point."""
    xbl = _f64(xbl)
    xks = np.zeros(4)
    J = np.zeros(16)
    lib().oracle_bl_to_ks(a, _p(xbl, C.c_double), _p(xks, C.c_double), _p(J, C.c_double))
    return xks, J.reshape(4, 4)


def ks_to_bl(a, s_ks):
    """Boyer-Lindquist states [8][n] of Kerr-Schild states [8][n] (chart spin a)."""
    y = np.ascontiguousarray(np.asarray(s_ks, dtype=np.float64).T)
    out = np.zeros_like(y)
    lib().oracle_ks_to_bl(a, y.shape[0], _p(y, C.c_double), _p(out, C.c_double))
    return np.ascontiguousarray(out.T)


def rk4_fixed(chart, a, h_coeff, r_stop, r_escape, nsteps, s, status=None, steps=None, nthreads=0):
    """Up to ``nsteps`` RK4 steps of h = h_coeff * r per active geodesic.

    ``chart`` is "ks" or "bl"; ``s`` is [8][n] in that chart.  Returns
    (s, status, steps) as new arrays; ``steps`` accumulates the steps taken."""
    y = np.ascontiguousarray(np.asarray(s, dtype=np.float64).T).copy()
    n = y.shape[0]
    st = np.zeros(n, np.int32) if status is None else np.array(status, dtype=np.int32)
    sp = np.zeros(n, np.int32) if steps is None else np.array(steps, dtype=np.int32)
    lib().oracle_rk4_fixed(CHARTS[chart], a, h_coeff, r_stop, r_escape, nsteps, n, _p(y, C.c_double),
                           _p(st, C.c_int32), _p(sp, C.c_int32), nthreads or default_threads())
    return np.ascontiguousarray(y.T), st, sp
