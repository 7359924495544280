// steppers.hpp -- Runge-Kutta steps for the second-order geodesic system.
//
// The state is (x^mu, k^mu) with x' = k and k' = acc(x, k).  Because x' is the
// momentum itself, every stage of an explicit Runge-Kutta method can be formed
// from the stage accelerations alone (Nystrom form): with the Butcher matrix A,
//   K_i = k + h sum_l A_il acc_l,
//   X_i = x + h c_i k + h^2 sum_l (A A)_il acc_l,
// so a lane keeps 4 values per stage instead of 8.  This is the same method,
// exactly, as the first-order form (c_i = sum_j A_ij holds for both tableaux).
//
// Tableaux: classic RK4 (the paper's default integrator, Sec. 3) and
// Dormand & Prince (1980) 5(4) with first-same-as-last.  The combined
// coefficients A A, b A and e A (e = b - b*) are folded at compile time.
#pragma once

#include <type_traits>

#include "bl_math.hpp"
#include "ks_math.hpp"

namespace kh {

// Right-hand side by form: 0 / 1 = Cartesian Kerr-Schild (factored / as
// regrouped in the paper), 2 = Boyer-Lindquist (fixed-step chart comparison).
template <int FORM, typename T>
__host__ __device__ inline Accel<T> chart_rhs(T a, const T x[4], const T k[4]) {
  if constexpr (FORM == 2)
    return rhs_bl<T>(a, x, k);
  else
    return rhs<FORM, T>(a, x, k);
}

// Scalar helpers for the norm, dispatched on type.
__host__ __device__ inline double kabs(double x) { return fabs(x); }
__host__ __device__ inline float kabs(float x) { return fabsf(x); }
// The larger of two magnitudes (one v_max instruction; a NaN operand yields the
// other operand, and a NaN error estimate rejects the attempt either way).
__host__ __device__ inline double kmax(double x, double y) { return fmax(x, y); }
__host__ __device__ inline float kmax(float x, float y) { return fmaxf(x, y); }

struct DP5Tab {
  double c[7];
  double A[7][7];
  double b[7];
  double e[7];      // b - b*
  double AA[7][7];  // A A
  double bA[7];     // b A
  double eA[7];     // e A
};

constexpr DP5Tab make_dp5() {
  DP5Tab t{};
  const double A[7][7] = {
      {0, 0, 0, 0, 0, 0, 0},
      {1.0 / 5, 0, 0, 0, 0, 0, 0},
      {3.0 / 40, 9.0 / 40, 0, 0, 0, 0, 0},
      {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0, 0},
      {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0, 0},
      {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0, 0},
      {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0}};
  const double c[7] = {0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1, 1};
  const double b[7] = {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0};
  const double bs[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640, -92097.0 / 339200, 187.0 / 2100, 1.0 / 40};
  for (int i = 0; i < 7; ++i) {
    t.c[i] = c[i];
    t.b[i] = b[i];
    t.e[i] = b[i] - bs[i];
    for (int j = 0; j < 7; ++j) t.A[i][j] = A[i][j];
  }
  for (int i = 0; i < 7; ++i)
    for (int l = 0; l < 7; ++l) {
      double s = 0;
      for (int j = 0; j < 7; ++j) s += A[i][j] * A[j][l];
      t.AA[i][l] = s;
    }
  for (int l = 0; l < 7; ++l) {
    double sb = 0, se = 0;
    for (int i = 0; i < 7; ++i) {
      sb += b[i] * A[i][l];
      se += (b[i] - bs[i]) * A[i][l];
    }
    t.bA[l] = sb;
    t.eA[l] = se;
  }
  return t;
}

constexpr DP5Tab DP5 = make_dp5();

template <typename TS, typename TR>
struct Conv {
  __host__ __device__ static TR to(TS v) { return static_cast<TR>(v); }
  __host__ __device__ static TS from(TR v) { return static_cast<TS>(v); }
};

// One Dormand-Prince attempt from (x, k) with acceleration a1 = acc(x, k).
// State, the new state's sums and the error estimate in TS; the stage values
// and the stage inputs X_i, K_i in TA; the right-hand side in TR.  FP64 and
// FP32 runs use one type throughout; the mixed-precision fast path runs
// stages and right-hand side in FP32 (TA = TR = float) and keeps the state,
// its update, the error estimate and the norm in FP64.
// Outputs the 5th-order state (xn, kn), its acceleration a7 (first stage of
// the next step) and the radius / radial rate at (xn, kn); returns the mean
// square of the scaled error components, i.e. the square of the RMS error
// norm (the controller needs only err^2 <= 1 and err^{-1/5} = (err^2)^{-1/10}).
// Coefficients that are exactly zero (A A on the sub-diagonal, b_2, b A on the
// sixth stage, e_2) are skipped at compile time: IEEE rules forbid the
// compiler from dropping 0 * s itself.
// CTF: coordinate-time form (x = (t, x^i), k = (1, v^i), the right-hand side
// rhs_ct; the t and v^0 slots have zero derivative and drop out of the norm,
// which is then the RMS over the six evolved components).
template <int FORM, typename TS, typename TR, bool CTF = false, typename TA = TS>
__host__ __device__ inline TS dp5_attempt(TS a_c, const TS x[4], const TS k[4], const TS a1[4], TS h, TS rtol,
                                          TS atol, TS xn[4], TS kn[4], TS a7[4], TS& r_new, TS& rdot_new) {
  TA S[6][4];
#pragma unroll
  for (int c = 0; c < 4; ++c) S[0][c] = Conv<TS, TA>::to(a1[c]);
  const TR ac = Conv<TS, TR>::to(a_c);
  // h k and h^2 once per attempt: X_i = (x + c_i (h k)) + h^2 sum_l (A A)_il S_l
  TA xa[4], ka[4], hkv[4];
  const TA ha = Conv<TS, TA>::to(h);
  hkv[0] = TA(0);  // t: unused
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    xa[c] = Conv<TS, TA>::to(x[c]);
    ka[c] = Conv<TS, TA>::to(k[c]);
    if (c > 0) hkv[c] = ha * ka[c];
  }
  const TA hh = ha * ha;
#pragma unroll
  for (int i = 1; i < 6; ++i) {
    TR X[4], K[4];
    X[0] = TR(0);  // the metric is stationary: t never enters the right-hand side
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      TA sx = TA(0), sk = TA(0);
      bool hx = false, hk = false;
#pragma unroll
      for (int l = 0; l < i; ++l) {
        if (DP5.AA[i][l] != 0.0) {
          sx = hx ? sx + TA(DP5.AA[i][l]) * S[l][c] : TA(DP5.AA[i][l]) * S[l][c];
          hx = true;
        }
        if (DP5.A[i][l] != 0.0) {
          sk = hk ? sk + TA(DP5.A[i][l]) * S[l][c] : TA(DP5.A[i][l]) * S[l][c];
          hk = true;
        }
      }
      if (c > 0)
        X[c] = Conv<TA, TR>::to(hx ? (xa[c] + TA(DP5.c[i]) * hkv[c]) + hh * sx : xa[c] + TA(DP5.c[i]) * hkv[c]);
      K[c] = Conv<TA, TR>::to(hk ? ka[c] + ha * sk : ka[c]);
    }
    const Accel<TR> ra = CTF ? rhs_ct<FORM, TR>(ac, X, K) : rhs<FORM, TR>(ac, X, K);
#pragma unroll
    for (int c = 0; c < 4; ++c) S[i][c] = Conv<TA, TR>::from(ra.a[c]);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    TA sx = TA(0), sk = TA(0);
    bool hx = false, hk = false;
#pragma unroll
    for (int l = 0; l < 6; ++l) {
      if (DP5.bA[l] != 0.0) {
        sx = hx ? sx + TA(DP5.bA[l]) * S[l][c] : TA(DP5.bA[l]) * S[l][c];
        hx = true;
      }
      if (DP5.b[l] != 0.0) {
        sk = hk ? sk + TA(DP5.b[l]) * S[l][c] : TA(DP5.b[l]) * S[l][c];
        hk = true;
      }
    }
    xn[c] = x[c] + h * (k[c] + h * Conv<TS, TA>::from(sx));
    kn[c] = k[c] + h * Conv<TS, TA>::from(sk);
  }
  {
    TR X[4], K[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      X[c] = Conv<TS, TR>::to(xn[c]);
      K[c] = Conv<TS, TR>::to(kn[c]);
    }
    const Accel<TR> ra = CTF ? rhs_ct<FORM, TR>(ac, X, K) : rhs<FORM, TR>(ac, X, K);
#pragma unroll
    for (int c = 0; c < 4; ++c) a7[c] = Conv<TS, TR>::from(ra.a[c]);
    r_new = Conv<TS, TR>::from(ra.r);
    rdot_new = Conv<TS, TR>::from(ra.rdot);
  }
  const TS hhs = std::is_same<TA, TS>::value ? Conv<TS, TA>::from(hh) : h * h;
  TS s2;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    TS ex = TS(0), ek = TS(0);
    bool hx = false, hk = false;
#pragma unroll
    for (int l = 0; l < 6; ++l) {
      if (DP5.eA[l] != 0.0) {
        const TS v = Conv<TS, TA>::from(S[l][c]);
        ex = hx ? ex + TS(DP5.eA[l]) * v : TS(DP5.eA[l]) * v;
        hx = true;
      }
      if (DP5.e[l] != 0.0) {
        const TS v = Conv<TS, TA>::from(S[l][c]);
        ek = hk ? ek + TS(DP5.e[l]) * v : TS(DP5.e[l]) * v;
        hk = true;
      }
    }
    // the last-stage term goes last, so the stage values can die before the
    // final right-hand side is evaluated
    ek = ek + TS(DP5.e[6]) * a7[c];
    ex = hhs * ex;
    ek = h * ek;
    const TS sx = atol + rtol * kmax(kabs(x[c]), kabs(xn[c]));
    const TS sk = atol + rtol * kmax(kabs(k[c]), kabs(kn[c]));
    const TS qx = ex * krcp_est(sx), qk = ek * krcp_est(sk);
    s2 = c == 0 ? qx * qx + qk * qk : s2 + qx * qx + qk * qk;
  }
  return s2 * (CTF ? TS(1.0 / 6.0) : TS(0.125));
}

// One classic RK4 step of length h from (x, k) with acceleration a1 = acc(x, k).
template <int FORM, typename TS, typename TR>
__host__ __device__ inline void rk4_step(TS a_c, const TS x[4], const TS k[4], const TS a1[4], TS h, TS xn[4],
                                         TS kn[4]) {
  const TR ac = Conv<TS, TR>::to(a_c);
  const TS hh = TS(0.5) * h;
  TR X[4], K[4];
  TS a2[4], a3[4], a4[4];
  X[0] = TR(0);
#pragma unroll
  for (int c = 1; c < 4; ++c) X[c] = Conv<TS, TR>::to(x[c] + hh * k[c]);
#pragma unroll
  for (int c = 0; c < 4; ++c) K[c] = Conv<TS, TR>::to(k[c] + hh * a1[c]);
  {
    const Accel<TR> ra = chart_rhs<FORM, TR>(ac, X, K);
#pragma unroll
    for (int c = 0; c < 4; ++c) a2[c] = Conv<TS, TR>::from(ra.a[c]);
  }
#pragma unroll
  for (int c = 1; c < 4; ++c) X[c] = Conv<TS, TR>::to(x[c] + hh * (k[c] + hh * a1[c]));
#pragma unroll
  for (int c = 0; c < 4; ++c) K[c] = Conv<TS, TR>::to(k[c] + hh * a2[c]);
  {
    const Accel<TR> ra = chart_rhs<FORM, TR>(ac, X, K);
#pragma unroll
    for (int c = 0; c < 4; ++c) a3[c] = Conv<TS, TR>::from(ra.a[c]);
  }
#pragma unroll
  for (int c = 1; c < 4; ++c) X[c] = Conv<TS, TR>::to(x[c] + h * (k[c] + hh * a2[c]));
#pragma unroll
  for (int c = 0; c < 4; ++c) K[c] = Conv<TS, TR>::to(k[c] + h * a3[c]);
  {
    const Accel<TR> ra = chart_rhs<FORM, TR>(ac, X, K);
#pragma unroll
    for (int c = 0; c < 4; ++c) a4[c] = Conv<TS, TR>::from(ra.a[c]);
  }
  const TS h6 = h / TS(6);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    xn[c] = x[c] + h * (k[c] + h6 * (a1[c] + a2[c] + a3[c]));
    kn[c] = k[c] + h6 * (a1[c] + TS(2) * (a2[c] + a3[c]) + a4[c]);
  }
}

// Cubic Hermite interpolant on theta in [0, 1] over a step of length h.
__host__ __device__ inline double herm(double th, double y0, double m0, double y1, double m1, double h) {
  const double t2 = th * th, t3 = t2 * th;
  return (2 * t3 - 3 * t2 + 1) * y0 + (t3 - 2 * t2 + th) * h * m0 + (-2 * t3 + 3 * t2) * y1 + (t3 - t2) * h * m1;
}
__host__ __device__ inline double dherm(double th, double y0, double m0, double y1, double m1, double h) {
  const double t2 = th * th;
  return (6 * t2 - 6 * th) * y0 + (3 * t2 - 4 * th + 1) * h * m0 + (-6 * t2 + 6 * th) * y1 +
         (3 * t2 - 2 * th) * h * m1;
}

// Zero of the Hermite interpolant of (y0 - target .. y1 - target) in [0, 1]
// given a sign change or an exact zero at the end: Newton from the linear
// guess, with bisection whenever an iterate leaves the current bracket.
__host__ __device__ inline double hermite_zero(double y0, double m0, double y1, double m1, double h) {
  if (y1 == 0.0) return 1.0;
  double lo = 0.0, hi = 1.0;
  double th = y0 / (y0 - y1);
  for (int it = 0; it < 60; ++it) {
    const double p = herm(th, y0, m0, y1, m1, h);
    if (p == 0.0) break;
    if ((p < 0.0) == (y0 < 0.0))
      lo = th;
    else
      hi = th;
    const double dp = dherm(th, y0, m0, y1, m1, h);
    double tn = th - p / dp;
    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
    if (fabs(tn - th) <= 1e-15) {
      th = tn;
      break;
    }
    th = tn;
  }
  return th;
}

}  // namespace kh
