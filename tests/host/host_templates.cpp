// Host instantiation of the GPU library's device templates (right-hand sides
// in both charts, Runge-Kutta steps, Hermite root), so CPU tests can compare that arithmetic
// with the oracle without a GPU.  Test-only; not part of the library.
#include "ks_math.hpp"
#include "steppers.hpp"

extern "C" {

void host_rhs(int form, int fp32, double a, const double* x, const double* k, double* acc) {
  if (fp32) {
    float xf[4], kf[4];
    for (int c = 0; c < 4; ++c) {
      xf[c] = (float)x[c];
      kf[c] = (float)k[c];
    }
    kh::Accel<float> r = form == 2   ? kh::chart_rhs<2, float>((float)a, xf, kf)
                         : form == 1 ? kh::chart_rhs<1, float>((float)a, xf, kf)
                                     : kh::chart_rhs<0, float>((float)a, xf, kf);
    for (int c = 0; c < 4; ++c) acc[c] = r.a[c];
    acc[4] = r.r;
    acc[5] = r.rdot;
  } else {
    kh::Accel<double> r = form == 2   ? kh::chart_rhs<2, double>(a, x, k)
                          : form == 1 ? kh::chart_rhs<1, double>(a, x, k)
                                      : kh::chart_rhs<0, double>(a, x, k);
    for (int c = 0; c < 4; ++c) acc[c] = r.a[c];
    acc[4] = r.r;
    acc[5] = r.rdot;
  }
}

// One DOPRI5 attempt: out = (xn[4], kn[4], a7[4], err, r_new, rdot_new).
void host_dp5(double a, const double* x, const double* k, double h, double rtol, double atol, double* out) {
  kh::Accel<double> r1 = kh::rhs<0, double>(a, x, k);
  double xn[4], kn[4], a7[4], rn, rd;
  double err = std::sqrt(kh::dp5_attempt<0, double, double>(a, x, k, r1.a, h, rtol, atol, xn, kn, a7, rn, rd));
  for (int c = 0; c < 4; ++c) {
    out[c] = xn[c];
    out[4 + c] = kn[c];
    out[8 + c] = a7[c];
  }
  out[12] = err;
  out[13] = rn;
  out[14] = rd;
}

void host_rk4(double a, const double* x, const double* k, double h, double* out) {
  kh::Accel<double> r1 = kh::rhs<0, double>(a, x, k);
  double xn[4], kn[4];
  kh::rk4_step<0, double, double>(a, x, k, r1.a, h, xn, kn);
  for (int c = 0; c < 4; ++c) {
    out[c] = xn[c];
    out[4 + c] = kn[c];
  }
}

// One RK4 step in the Boyer-Lindquist chart: out = (xn[4], kn[4]).
void host_rk4_bl(double a, const double* x, const double* k, double h, double* out) {
  kh::Accel<double> r1 = kh::chart_rhs<2, double>(a, x, k);
  double xn[4], kn[4];
  kh::rk4_step<2, double, double>(a, x, k, r1.a, h, xn, kn);
  for (int c = 0; c < 4; ++c) {
    out[c] = xn[c];
    out[4 + c] = kn[c];
  }
}

double host_hermite_zero(double y0, double m0, double y1, double m1, double h) {
  return kh::hermite_zero(y0, m0, y1, m1, h);
}

void host_constants(double a, const double* x, const double* k, double* out) { kh::constants(a, x, k, out); }

double host_redshift(double r, double xi, double a) { return kh::redshift(r, xi, a); }

double host_atan2_est(double y, double x) { return kh::atan2_est(y, x); }
}
