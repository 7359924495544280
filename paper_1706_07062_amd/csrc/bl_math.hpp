// bl_math.hpp -- the geodesic right-hand side in Boyer-Lindquist coordinates.
//
// Only for the chart comparison of Sec. 4 (tab:elapse): the same rays are
// integrated in Cartesian Kerr-Schild and in Boyer-Lindquist coordinates
// (t, r, theta, phi).  The metric is the line element at the start of
// Sec. 2.1, M = 1, with rho^2 = r^2 + a^2 cos^2, Delta = r^2 - 2 r + a^2 and
// u = 2 r / rho^2:
//   g_tt = u - 1,  g_tphi = -a u s^2,  g_phiphi = (r^2 + a^2 + a^2 u s^2) s^2,
//   g_rr = rho^2 / Delta,  g_thth = rho^2   (s = sin(theta), c = cos(theta)).
// As in the Kerr-Schild form, the acceleration is contracted without a
// Christoffel table: with d/dlambda = k^r d_r + k^th d_th acting on the metric,
//   V_d = (d g_dc / dlambda) k^c - 1/2 d_d(g_bc) k^b k^c,   a^mu = -g^{mu d} V_d,
// and the inverse in closed form: g^rr = Delta / rho^2, g^thth = 1 / rho^2, and
// the (t, phi) block, whose determinant is -Delta s^2, gives
//   a^t = (B V_t + a u V_phi) / Delta,
//   a^phi = ((u - 1) V_phi / s^2 + a u V_t) / Delta,   B = g_phiphi / s^2.
// The 1/s^2 of a^phi is the chart's polar singularity.  sin and cos of theta
// are evaluated once per call (the library's sincos).
#pragma once

#include "ks_math.hpp"

namespace kh {

__host__ __device__ inline void ksincos(double x, double* s, double* c) {
#if defined(__HIP_DEVICE_COMPILE__)
  sincos(x, s, c);
#else
  *s = std::sin(x);
  *c = std::cos(x);
#endif
}
__host__ __device__ inline void ksincos(float x, float* s, float* c) {
#if defined(__HIP_DEVICE_COMPILE__)
  sincosf(x, s, c);
#else
  *s = std::sin(x);
  *c = std::cos(x);
#endif
}

// x = (t, r, theta, phi), k = (k^t, k^r, k^theta, k^phi).  Accel.r = r and
// Accel.rdot = k^r, as for the Kerr-Schild form.
template <typename T>
__host__ __device__ inline Accel<T> rhs_bl(T a, const T x[4], const T k[4]) {
  const T r = x[1];
  T s, c;
  ksincos(x[2], &s, &c);
  const T kt = k[0], kr = k[1], kq = k[2], kp = k[3];
  const T a2 = a * a, r2 = r * r, s2 = s * s;
  const T sc2 = T(2) * s * c;  // sin(2 theta)
  const T rho2 = r2 + a2 * (c * c);
  const T Delta = r2 - T(2) * r + a2;
  // one reciprocal for 1/rho^2, 1/Delta and 1/s^2
  const T P = krcp(rho2 * Delta * s2);
  const T rs = rho2 * s2;
  const T irho2 = Delta * s2 * P, iDelta = rs * P, iDs2 = rho2 * P;
  const T u = T(2) * r * irho2;
  // derivatives of u = 2 r / rho^2 and of w = u s^2 (g_tphi = -a w)
  const T u_r = T(2) * (a2 * (c * c) - r2) * (irho2 * irho2);
  const T u_q = u * a2 * sc2 * irho2;
  const T w = u * s2;
  const T w_r = u_r * s2;
  const T w_q = u_q * s2 + u * sc2;
  const T B = r2 + a2 + a2 * w;
  const T gpp_r = (T(2) * r + a2 * w_r) * s2;
  const T gpp_q = a2 * w_q * s2 + B * sc2;
  const T grr = rho2 * iDelta;
  const T grr_r = (T(2) * r - grr * (T(2) * r - T(2))) * iDelta;
  const T rho2_q = -a2 * sc2;
  const T grr_q = rho2_q * iDelta;
  // rates along the ray
  const T du = kr * u_r + kq * u_q;
  const T dw = kr * w_r + kq * w_q;
  const T dpp = kr * gpp_r + kq * gpp_q;
  const T drr = kr * grr_r + kq * grr_q;
  const T dqq = kr * (T(2) * r) + kq * rho2_q;
  const T tp = kt * kp;
  const T Vt = du * kt - a * dw * kp;
  const T Vp = dpp * kp - a * dw * kt;
  const T Vr = drr * kr - T(0.5) * (u_r * (kt * kt) - T(2) * a * w_r * tp + grr_r * (kr * kr) +
                                    T(2) * r * (kq * kq) + gpp_r * (kp * kp));
  const T Vq = dqq * kq - T(0.5) * (u_q * (kt * kt) - T(2) * a * w_q * tp + grr_q * (kr * kr) +
                                    rho2_q * (kq * kq) + gpp_q * (kp * kp));
  const T au = a * u;
  Accel<T> out;
  out.a[0] = (B * Vt + au * Vp) * iDelta;
  out.a[1] = -Delta * irho2 * Vr;
  out.a[2] = -irho2 * Vq;
  out.a[3] = (u - T(1)) * Vp * iDs2 + au * Vt * iDelta;
  out.r = r;
  out.rdot = kr;
  return out;
}

}  // namespace kh
