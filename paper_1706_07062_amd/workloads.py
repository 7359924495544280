"""Seeded synthetic workloads (inputs only).

This module holds the shapes, sizes and random draws of the workloads and
nothing of the integration itself, so that the GPU path and the CPU oracle
receive identical inputs.  All random numbers come from numpy's PCG64 with
fixed seeds.  Names of the workloads follow what they are:

* ``schwarzschild_64``: a = 0, 64x64 image on [-10, 10]^2, observer at 1000 M,
  inclination 60 deg, fixed-step RK4 with h = 0.01 r.
* ``kerr_1024``: a = 0.99, 1024x1024 image on [-12, 12]^2, observer at 1000 M,
  inclinations 17 and 60 deg, adaptive DOPRI5 with rtol = 1e-8, 4 crossings.
* ``particles``: 2^20 time-like geodesics, a ~ U[0, 0.998], r0 ~ U[6, 100],
  phi0 ~ U[0, 2 pi), orbital-plane tilt ~ U[0, 30 deg], speed factor
  1 + N(0, 0.05) on the local circular speed; integrated to t = 1e4 M.
* ``batched_images``: 256 images, sides uniform in {32, 64, ..., 1024}, spin
  ~ U[0, 0.998], inclination ~ U[5, 85] deg, [-12, 12]^2, observer at 1000 M.
* ``surrogate_rays``: rays with alpha, beta ~ U[-12, 12], a ~ U[0, 0.998],
  inclination ~ U[5, 85] deg; evaluation image 4096x4096 at a = 0.9, 45 deg.
* ``elapse_image``: a = 0.999, image at r = 1024 M, inclination 60 deg,
  [-12, 12]^2, fixed-step RK4 (h = r / 256) in launches of 1024 steps, in
  Kerr-Schild and Boyer-Lindquist coordinates.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_PARTICLES = 1706070623
SEED_BATCHED = 1706070624
SEED_SURROGATE = 1706070625


@dataclass(frozen=True)
class Camera:
    a: float
    r_obs: float
    incl_deg: float
    alpha_min: float
    alpha_max: float
    beta_min: float
    beta_max: float
    width: int
    height: int

    @property
    def incl(self) -> float:
        return float(np.radians(self.incl_deg))

    @property
    def n(self) -> int:
        return self.width * self.height


def schwarzschild_64() -> Camera:
    return Camera(0.0, 1000.0, 60.0, -10.0, 10.0, -10.0, 10.0, 64, 64)


def kerr_image(incl_deg: float, side: int = 1024, a: float = 0.99) -> Camera:
    return Camera(a, 1000.0, incl_deg, -12.0, 12.0, -12.0, 12.0, side, side)


# Chart / data-layout comparison of Sec. 4 (tab:elapse): an image at r = 1024
# toward a hole of spin 0.999, fixed-step RK4 in launches of 1024 steps.  The
# inclination and the image field are not stated there; 60 degrees and
# [-12, 12]^2 (the field of the images above) are taken.
ELAPSE_STEPS = 1024
ELAPSE_H_COEFF = 1.0 / 256  # no ray reaches r < 18 or turns back within one launch


def elapse_image(side: int = 1024) -> Camera:
    return Camera(0.999, 1024.0, 60.0, -12.0, 12.0, -12.0, 12.0, side, side)


def kerr_1024() -> list[Camera]:
    return [kerr_image(17.0), kerr_image(60.0)]


def particles(n: int = 1 << 20, seed: int = SEED_PARTICLES) -> dict:
    """Positions and coordinate velocities of near-circular orbits.

    Position rho (cos phi0, sin phi0, 0) with rho = sqrt(r0^2 + a^2) (the
    equatorial Kerr-Schild radius r0); velocity (1 + eps) Omega rho times the
    unit vector (-sin phi0 cos i, cos phi0 cos i, sin i): the circular
    velocity with Omega = 1 / (r0^{3/2} + a), tilted about the radius vector.
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 0.998, n)
    r0 = rng.uniform(6.0, 100.0, n)
    phi0 = rng.uniform(0.0, 2 * np.pi, n)
    tilt = rng.uniform(0.0, np.radians(30.0), n)
    eps = rng.normal(0.0, 0.05, n)
    rho = np.sqrt(r0 * r0 + a * a)
    om = 1.0 / (r0 ** 1.5 + a)
    x3 = np.stack([rho * np.cos(phi0), rho * np.sin(phi0), np.zeros(n)])
    sp = (1.0 + eps) * om * rho
    v3 = np.stack([-sp * np.sin(phi0) * np.cos(tilt), sp * np.cos(phi0) * np.cos(tilt), sp * np.sin(tilt)])
    return dict(a=a, x3=np.ascontiguousarray(x3), v3=np.ascontiguousarray(v3), r0=r0, tilt=tilt, eps=eps)


def batched_images(n_images: int = 256, seed: int = SEED_BATCHED) -> list[Camera]:
    rng = np.random.default_rng(seed)
    sides = rng.choice(np.array([32, 64, 128, 256, 512, 1024]), size=n_images)
    a = rng.uniform(0.0, 0.998, n_images)
    incl = rng.uniform(5.0, 85.0, n_images)
    return [Camera(float(a[i]), 1000.0, float(incl[i]), -12.0, 12.0, -12.0, 12.0, int(sides[i]), int(sides[i]))
            for i in range(n_images)]


def surrogate_rays(n: int, seed: int = SEED_SURROGATE) -> dict:
    rng = np.random.default_rng(seed)
    alpha = rng.uniform(-12.0, 12.0, n)
    beta = rng.uniform(-12.0, 12.0, n)
    a = rng.uniform(0.0, 0.998, n)
    incl = np.radians(rng.uniform(5.0, 85.0, n))
    return dict(alpha=alpha, beta=beta, a=a, incl=incl)


def surrogate_eval_camera(side: int = 4096) -> Camera:
    return Camera(0.9, 1000.0, 45.0, -12.0, 12.0, -12.0, 12.0, side, side)


def strided_pixels(n_total: int, count: int, offset: int = 0) -> np.ndarray:
    """`count` pixel ids spread evenly over [0, n_total) (sample for oracle checks)."""
    step = max(1, n_total // count)
    return (np.arange(count, dtype=np.int64) * step + offset) % n_total
