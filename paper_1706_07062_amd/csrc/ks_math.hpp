// ks_math.hpp -- Cartesian Kerr-Schild geometry and the geodesic right-hand side.
//
// Everything here is a __host__ __device__ template on the scalar type T
// (double, float, or the host-side operation counter), so the same source is
// the device code and the operation count.
//
// Metric (Sec. 2.1, def:CKS): g_ab = eta_ab + f l_a l_b with
//   f = 2 r^3 / (r^4 + a^2 z^2),
//   l = (1, (r x + a y)/(r^2 + a^2), (r y - a x)/(r^2 + a^2), z / r),
// and r the positive root of eq:CKSr, r^4 - (R^2 - a^2) r^2 - a^2 z^2 = 0.
//
// Right-hand side (Sec. 2.1, eq:opt0 / eq:opti): with xdot_{b,j} = g_{bc,j} k^c
// (only spatial derivatives: the metric is stationary) and
//   F = f (l^b k^j xdot_{b,j} - 1/2 l^j k^b xdot_{b,j}),  l^b = (-1, l_1, l_2, l_3),
//   a^0 = k^j xdot_{0,j} - F,
//   a^i = -k^j (xdot_{i,j} - 1/2 xdot_{j,i}) + F l_i.
// Two evaluations of that formula are provided:
//   * rhs_paper: forms the 12 values xdot_{b,j} and then the sums, as written;
//   * rhs_factored (default): the same acceleration contracted in another
//     order (written out above the function): about 110 operations instead
//     of 155, equal to rhs_paper up to rounding.
#pragma once

#include <hip/hip_runtime.h>

namespace kh {

// Reciprocal and reciprocal square root.  On the device: the hardware
// estimate (v_rcp_f64 / v_rsq_f64, relative error below 2^-24 on gfx950)
// refined by one Newton-Raphson iteration, r <- r + r (1 - x r) and
// y <- y + y (1/2 - x y^2 / 2), which squares the relative error: below
// 2^-47 (5e-15), i.e. within ~20 ulp of the rounded value.  The right-hand
// side built from them is then accurate to ~1e-14 relative, six orders of
// magnitude below the local error the step controller admits at rtol = 1e-8.
// FP32 estimates are already within one ulp.  On the host (operation counts,
// CPU checks) plain IEEE operations.
__host__ __device__ inline double krcp(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
#else
  return 1.0 / x;
#endif
}
__host__ __device__ inline float krcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
__host__ __device__ inline double krsqrt(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double y = __builtin_amdgcn_rsq(x);
  return fma(y, fma(-0.5 * x, y * y, 0.5), y);
#else
  return 1.0 / sqrt(x);
#endif
}
__host__ __device__ inline float krsqrt(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsqf(x);
#else
  return 1.0f / sqrtf(x);
#endif
}
// Reciprocal for the scales of the error norm (same accuracy as krcp).
__host__ __device__ inline double krcp_est(double x) { return krcp(x); }
__host__ __device__ inline float krcp_est(float x) { return krcp(x); }
// sqrt(x) for x >= 0, without a branch: the argument of the reciprocal square
// root is kept >= 1e-300 (1e-30 in FP32), so x = 0 gives 0.  On the device
// the Newton-Raphson step is taken on s = x y (y the rsq estimate) itself:
// e = 1 - s y, s <- s + s e / 2, which squares the relative error as the step
// on y does, in one instruction less.
__host__ __device__ inline double ksqrt(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double y = __builtin_amdgcn_rsq(x > 1e-300 ? x : 1e-300);
  const double s = x * y;
  return fma(0.5 * s, fma(-s, y, 1.0), s);
#else
  return x * krsqrt(x > 1e-300 ? x : 1e-300);
#endif
}
__host__ __device__ inline float ksqrt(float x) { return x * krsqrt(x > 1e-30f ? x : 1e-30f); }

// Azimuth estimate with |error| < 0.08 rad, enough to recover a winding count
// by rounding: atan(|y|/|x|) = pi/4 + atan(u), u = (|y| - |x|) / (|y| + |x|),
// with atan(u) ~ pi u / 4 on [-1, 1]; quadrants (and the sign of a zero)
// follow atan2.
__host__ __device__ inline double atan2_est(double y, double x) {
  const float ax = fabsf((float)x), ay = fabsf((float)y);
  const float s = ax + ay;
#if defined(__HIP_DEVICE_COMPILE__)
  const float u = s > 0.0f ? (ay - ax) * __builtin_amdgcn_rcpf(s) : 0.0f;
#else
  const float u = s > 0.0f ? (ay - ax) / s : 0.0f;
#endif
  float t = 0.78539816f * (1.0f + u);
  if (__builtin_signbit(x)) t = 3.14159265f - t;
  return __builtin_signbit(y) ? -(double)t : (double)t;
}

template <typename T>
struct Accel {
  T a[4];  // d k^mu / d lambda
  T r;     // Kerr-Schild radius at the point
  T rdot;  // dr / dlambda = d_j r k^j
};

// Keeps the compiler from evaluating a rarely taken branch unconditionally
// (if-conversion would run its reciprocal on every call).
__host__ __device__ inline void kh_keep_branch() {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" ::: "memory");
#endif
}

// Radius from eq:CKSr.  Both root formulas are exact; the second avoids
// cancellation when R^2 < a^2 and is a real branch (taken only inside r < a).
template <typename T>
__host__ __device__ inline T ks_r2(T a2, T X, T Y, T Z) {
  const T z2 = Z * Z;
  const T w = X * X + (Y * Y + (z2 - a2));
  const T q = ksqrt(w * w + T(4) * a2 * z2);
  T r2 = T(0.5) * (w + q);
  if (!(w >= T(0))) {
    kh_keep_branch();
    r2 = T(2) * a2 * z2 * krcp(q - w);
  }
  return r2;
}

// The paper's regrouped form, written out with its 12 temporaries.
template <typename T>
__host__ __device__ inline Accel<T> rhs_paper(T a, const T x[4], const T k[4]) {
  const T X = x[1], Y = x[2], Z = x[3];
  const T a2 = a * a;
  const T r2 = ks_r2(a2, X, Y, Z);
  const T ir = krsqrt(r2);
  const T r = r2 * ir;
  const T S = r2 + a2, D = r2 * r2 + a2 * Z * Z;
  const T iSD = krcp(S * D);
  const T iS = D * iSD, iD = S * iSD;
  const T f = T(2) * r2 * r * iD;
  const T l[4] = {T(1), (r * X + a * Y) * iS, (r * Y - a * X) * iS, Z * ir};
  // d_j r = r (r^2 x_j + a^2 z delta_jz) / D
  const T c = r * iD;
  const T dr[3] = {c * r2 * X, c * r2 * Y, c * (r2 + a2) * Z};
  // d_j f = f [3 d_j r / r - (4 r^3 d_j r + 2 a^2 z delta_jz) / D]
  const T m = f * (T(3) * ir - T(4) * r2 * r * iD);
  const T df[3] = {m * dr[0], m * dr[1], m * dr[2] - T(2) * f * a2 * Z * iD};
  // dl[i][j] = d_j l_i (i = 1..3 stored at 0..2); d_j l_0 = 0.
  const T px = (X - T(2) * r * l[1]) * iS;
  const T py = (Y - T(2) * r * l[2]) * iS;
  const T pz = -l[3] * ir;
  const T rS = r * iS, aS = a * iS;
  const T dl[3][3] = {{px * dr[0] + rS, px * dr[1] + aS, px * dr[2]},
                      {py * dr[0] - aS, py * dr[1] + rS, py * dr[2]},
                      {pz * dr[0], pz * dr[1], pz * dr[2] + ir}};
  const T K = k[0] + l[1] * k[1] + l[2] * k[2] + l[3] * k[3];
  T dK[3];
  for (int j = 0; j < 3; ++j) dK[j] = k[1] * dl[0][j] + k[2] * dl[1][j] + k[3] * dl[2][j];
  // xd[b][j] = xdot_{b,j} = (d_j f l_b + f d_j l_b) K + f l_b dK_j
  T xd[4][3];
  for (int j = 0; j < 3; ++j) xd[0][j] = df[j] * K + f * dK[j];
  for (int b = 1; b < 4; ++b)
    for (int j = 0; j < 3; ++j) xd[b][j] = (df[j] * l[b] + f * dl[b - 1][j]) * K + f * l[b] * dK[j];
  // F = f (l^b k^j xd[b][j] - 1/2 l^j k^b xd[b][j])
  T s1 = T(0), s2 = T(0);
  for (int j = 0; j < 3; ++j) {
    const T kj = k[j + 1];
    s1 = s1 + kj * (-xd[0][j] + l[1] * xd[1][j] + l[2] * xd[2][j] + l[3] * xd[3][j]);
    s2 = s2 + l[j + 1] * (k[0] * xd[0][j] + k[1] * xd[1][j] + k[2] * xd[2][j] + k[3] * xd[3][j]);
  }
  const T F = f * (s1 - T(0.5) * s2);
  Accel<T> out;
  out.a[0] = k[1] * xd[0][0] + k[2] * xd[0][1] + k[3] * xd[0][2] - F;
  // the second sum runs over all four b (xdot_{0,i} is not zero), the first
  // over spatial j only (xdot_{i,0} = 0)
  for (int i = 1; i < 4; ++i) {
    T s = T(0);
    for (int j = 0; j < 3; ++j) s = s + k[j + 1] * xd[i][j];
    T v = T(0);
    for (int b = 0; b < 4; ++b) v = v + k[b] * xd[b][i - 1];
    out.a[i] = -s + T(0.5) * v + F * l[i];
  }
  out.r = r;
  out.rdot = dr[0] * k[1] + dr[1] * k[2] + dr[2] * k[3];
  return out;
}

// Regrouped evaluation of the same right-hand side.  With Christoffel symbols
// of the first kind, dk^a/dlambda = -g^{ad} V_d where
//   V_d = k^b d_b(g_dc) k^c - 1/2 d_d(g_bc) k^b k^c,
// and for g = eta + f l l with l null (g^{ab} = eta^{ab} - f l^a l^b):
//   a^0 = V_0 - f (l^d V_d),   a^i = f l_i (l^d V_d) - V_i,   l^d V_d = l_i V_i - V_0.
// With K = l.k, the rates along the ray fdot = k^j d_j f, ldot_i = k^j d_j l_i,
// Kd = k^i ldot_i, and dK_d = k^i d_d l_i:
//   V_0 = fdot K + f Kd,
//   V_i = V_0 l_i + f K (ldot_i - dK_i) - 1/2 K^2 d_i f.
// The Jacobian d_j l_i = p_i d_j r + B_ij with B = [[r/S, a/S, 0], [-a/S, r/S, 0],
// [0, 0, 1/r]] gives ldot_i - dK_i = p_i rdot - (k.p) d_i r + ((B - B^T) k)_i,
// where (B - B^T) k = 2a/S (k_y, -k_x, 0), and Kd = (k.p) rdot + (r/S)(k_x^2 + k_y^2)
// + k_z^2 / r.  d_j f = m d_j r - delta_jz 2 f a^2 z / D.  About 110 operations,
// against 155 for the regrouping by xdot_{b,j} G_j that eq:opt0/opti suggests.
template <typename T>
__host__ __device__ inline Accel<T> rhs_factored(T a, const T x[4], const T k[4]) {
  const T X = x[1], Y = x[2], Z = x[3];
  const T k0 = k[0], k1 = k[1], k2 = k[2], k3 = k[3];
  const T a2 = a * a;
  const T r2 = ks_r2(a2, X, Y, Z);
  // one reciprocal square root gives r and 1/r; one reciprocal gives 1/S and 1/D
  const T ir = krsqrt(r2);
  const T r = r2 * ir;
  const T a2z2 = a2 * (Z * Z);
  const T S = r2 + a2, D = r2 * r2 + a2z2;
  const T iSD = krcp(S * D);
  const T iS = D * iSD, iD = S * iSD;
  const T rS = r * iS, aS = a * iS;
  const T l1 = rS * X + aS * Y, l2 = rS * Y - aS * X, l3 = Z * ir;
  // gradient of r, and of f = m d_j r - cz delta_jz: with c = r / D,
  // f = 2 r^3 / D = 2 c r^2 and d_j f = f (3 / r - 4 r^3 / D) d_j r - 2 f a^2 z / D
  // delta_jz, where 4 r^3 / D = 2 f
  const T c = r * iD;
  const T cr2 = c * r2;
  const T f = cr2 + cr2;
  const T dr1 = cr2 * X, dr2 = cr2 * Y, dr3 = c * S * Z;
  const T m = f * (T(3) * ir - T(2) * f);
  const T cz = (f * iD) * (T(2) * a2 * Z);
  // p of the Jacobian's rank-one part
  const T px = (X - T(2) * r * l1) * iS;
  const T py = (Y - T(2) * r * l2) * iS;
  const T pz = -l3 * ir;
  // rates along the ray
  const T rdot = dr1 * k1 + dr2 * k2 + dr3 * k3;
  const T fdot = m * rdot - cz * k3;
  const T kp = px * k1 + py * k2 + pz * k3;
  const T K = k0 + l1 * k1 + l2 * k2 + l3 * k3;
  const T Kd = kp * rdot + rS * (k1 * k1 + k2 * k2) + ir * (k3 * k3);
  const T fK = f * K;
  const T V0 = fdot * K + f * Kd;
  // W_i = ldot_i - dK_i
  const T a2S = T(2) * aS;
  const T W1 = px * rdot - kp * dr1 + a2S * k2;
  const T W2 = py * rdot - kp * dr2 - a2S * k1;
  const T W3 = pz * rdot - kp * dr3;
  const T hK2 = T(0.5) * K * K;
  const T hK2m = hK2 * m;
  const T V1 = V0 * l1 + fK * W1 - hK2m * dr1;
  const T V2 = V0 * l2 + fK * W2 - hK2m * dr2;
  const T V3 = V0 * l3 + fK * W3 - hK2m * dr3 + hK2 * cz;
  const T flV = f * (l1 * V1 + l2 * V2 + l3 * V3 - V0);
  Accel<T> out;
  out.a[0] = V0 - flV;
  out.a[1] = flV * l1 - V1;
  out.a[2] = flV * l2 - V2;
  out.a[3] = flV * l3 - V3;
  out.r = r;
  out.rdot = rdot;
  return out;
}

template <int FORM, typename T>
__host__ __device__ inline Accel<T> rhs(T a, const T x[4], const T k[4]) {
  if constexpr (FORM == 1)
    return rhs_paper<T>(a, x, k);
  else
    return rhs_factored<T>(a, x, k);
}

// Coordinate-time form (Sec. 2.2, the coordinate-time subsection): with
// v^mu = dx^mu/dt (v^0 = 1) the spatial equations are dv^i/dt = a^i - a^0 v^i,
// where a^mu is the affine right-hand side evaluated at k = v (it is
// quadratic in k, so the k^0 scale drops out).  Same radius and dr/dt.
template <int FORM, typename T>
__host__ __device__ inline Accel<T> rhs_ct(T a, const T x[4], const T v[4]) {
  Accel<T> out = rhs<FORM, T>(a, x, v);
  const T a0 = out.a[0];
  out.a[0] = T(0);
#pragma unroll
  for (int i = 1; i < 4; ++i) out.a[i] = out.a[i] - a0 * v[i];
  return out;
}

// Energy E = -k_t = k^0 - f K (K = k^0 + l_i k^i) in the chart of spin a.
__host__ __device__ inline double energy(double a, const double x[4], const double k[4]) {
  const double a2 = a * a;
  const double r2 = ks_r2(a2, x[1], x[2], x[3]);
  const double r = sqrt(r2);
  const double iS = 1.0 / (r2 + a2);
  const double f = 2.0 * r2 * r / (r2 * r2 + a2 * x[3] * x[3]);
  const double l1 = (r * x[1] + a * x[2]) * iS, l2 = (r * x[2] - a * x[1]) * iS, l3 = x[3] / r;
  return k[0] - f * (k[0] + l1 * k[1] + l2 * k[2] + l3 * k[3]);
}

// Null condition: k^0 = [f L + sqrt(1 - f + f L^2)] / (1 - f), L = l_i k^i with
// |k^i| = 1 scaled out: for general spatial k, the future root of
// (f - 1) k0^2 + 2 f L k0 + |k|^2 + f L^2 = 0.
__host__ __device__ inline double null_k0(double a, const double x[4], const double k[4], bool* ok) {
  const double a2 = a * a;
  const double r2 = ks_r2(a2, x[1], x[2], x[3]);
  const double r = sqrt(r2);
  const double iS = 1.0 / (r2 + a2);
  const double f = 2.0 * r2 * r / (r2 * r2 + a2 * x[3] * x[3]);
  const double l1 = (r * x[1] + a * x[2]) * iS, l2 = (r * x[2] - a * x[1]) * iS, l3 = x[3] / r;
  const double L = l1 * k[1] + l2 * k[2] + l3 * k[3];
  const double kk = k[1] * k[1] + k[2] * k[2] + k[3] * k[3];
  const double disc = f * f * L * L + (1.0 - f) * (kk + f * L * L);
  *ok = (f < 1.0) && (disc >= 0.0);
  return (f * L + sqrt(disc)) / (1.0 - f);
}

// Time-like normalisation: with v = (1, v^i), u^0 = 1 / sqrt(1 - |v|^2 - f (1 + l.v)^2).
__host__ __device__ inline double timelike_u0(double a, const double x[4], const double v[3], bool* ok) {
  const double a2 = a * a;
  const double r2 = ks_r2(a2, x[1], x[2], x[3]);
  const double r = sqrt(r2);
  const double iS = 1.0 / (r2 + a2);
  const double f = 2.0 * r2 * r / (r2 * r2 + a2 * x[3] * x[3]);
  const double l1 = (r * x[1] + a * x[2]) * iS, l2 = (r * x[2] - a * x[1]) * iS, l3 = x[3] / r;
  const double lv = 1.0 + l1 * v[0] + l2 * v[1] + l3 * v[2];
  const double nrm = 1.0 - (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) - f * lv * lv;
  *ok = nrm > 0.0;
  return 1.0 / sqrt(nrm);
}

// Constants of motion in FP64: E = -k_0, L_z = x k_y - y k_x, Carter's Q and
// mu^2 = -g k k, with covariant k_a = eta_ab k^b + f l_a (l.k).  Q uses the
// spheroidal angle of the chart: cos(th) = z/r, sin(th) = rho / sqrt(r^2 + a^2),
// p_th = cot(th)(x k_x + y k_y) - r sin(th) k_z,
// Q = p_th^2 + cos^2(th) [a^2 (mu^2 - E^2) + L_z^2 / sin^2(th)].  On the spin
// axis (rho = 0) the two quotients are 0/0 and Q is their limit,
// cos^2(th) [(r^2 + a^2)(k_x^2 + k_y^2) + a^2 (mu^2 - E^2)], the same from
// every direction.
__host__ __device__ inline void constants(double a, const double x[4], const double k[4], double out[4]) {
  const double a2 = a * a;
  const double r2 = ks_r2(a2, x[1], x[2], x[3]);
  const double r = sqrt(r2);
  const double iS = 1.0 / (r2 + a2);
  const double f = 2.0 * r2 * r / (r2 * r2 + a2 * x[3] * x[3]);
  const double l1 = (r * x[1] + a * x[2]) * iS, l2 = (r * x[2] - a * x[1]) * iS, l3 = x[3] / r;
  const double K = k[0] + l1 * k[1] + l2 * k[2] + l3 * k[3];
  const double k0 = -k[0] + f * K, kx = k[1] + f * l1 * K, ky = k[2] + f * l2 * K, kz = k[3] + f * l3 * K;
  const double E = -k0;
  const double Lz = x[1] * ky - x[2] * kx;
  const double mu2 = -(k0 * k[0] + kx * k[1] + ky * k[2] + kz * k[3]);
  const double rho = sqrt(x[1] * x[1] + x[2] * x[2]);
  const double cth = x[3] / r;
  out[0] = E;
  out[1] = Lz;
  if (rho > 1e-150) {
    const double sth = rho * sqrt(iS);
    const double pth = (cth / sth) * (x[1] * kx + x[2] * ky) - r * sth * kz;
    out[2] = pth * pth + cth * cth * (a2 * (mu2 - E * E) + Lz * Lz / (sth * sth));
  } else {
    out[2] = cth * cth * ((r2 + a2) * (kx * kx + ky * ky) + a2 * (mu2 - E * E));
  }
  out[3] = mu2;
}

// Photon's xi = L_z / E in the physical frame (null rays run time-reversed in
// the chart with spin -a: same E, opposite L_z).
__host__ __device__ inline double photon_xi(double a_chart, const double x[4], const double k[4], bool reversed) {
  const double a2 = a_chart * a_chart;
  const double r2 = ks_r2(a2, x[1], x[2], x[3]);
  const double r = sqrt(r2);
  const double iS = 1.0 / (r2 + a2);
  const double f = 2.0 * r2 * r / (r2 * r2 + a2 * x[3] * x[3]);
  const double l1 = (r * x[1] + a_chart * x[2]) * iS, l2 = (r * x[2] - a_chart * x[1]) * iS, l3 = x[3] / r;
  const double K = k[0] + l1 * k[1] + l2 * k[2] + l3 * k[3];
  const double E = k[0] - f * K;
  const double Lz = x[1] * (k[2] + f * l2 * K) - x[2] * (k[1] + f * l1 * K);
  return reversed ? -Lz / E : Lz / E;
}

// Redshift nu_obs / nu_em for an emitter on the prograde Keplerian circular
// orbit at radius r (spin a): Omega = 1/(r^{3/2} + a),
// u^t = (r^{3/2} + a) / (r^{3/4} sqrt(r^{3/2} - 3 r^{1/2} + 2a)), g = 1/(u^t (1 - Omega xi)).
// NaN inside the prograde photon orbit.
__host__ __device__ inline double redshift(double r, double xi, double a) {
  const double sr = sqrt(r);
  const double r32 = r * sr;
  const double den = r32 - 3.0 * sr + 2.0 * a;
  if (!(den > 0.0)) return __builtin_nan("");
  const double ut = (r32 + a) / (sr * sqrt(sr) * sqrt(den));  // r^{3/4} = r^{1/2} r^{1/4}
  const double om = 1.0 / (r32 + a);
  return 1.0 / (ut * (1.0 - om * xi));
}

}  // namespace kh
