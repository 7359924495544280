// kerr_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, FP64 CPU reference for batched geodesic integration in
// Cartesian Kerr-Schild coordinates (Chan, Medeiros, Ozel & Psaltis, GRay2).
// Only the test-suite, the smoke check and the CPU-baseline leg of the
// benchmark may load it.  It shares no source with the GPU library.
//
// What it computes, and from which passage:
//   * metric g = eta + f l l with f, l_alpha and the implicit radius r of
//     Sec. 2.1 (def:CKS, eq:CKSr), evaluated straightforwardly;
//   * metric derivatives g_{mu nu, alpha} by forward-mode dual numbers on that
//     evaluation (the metric is stationary, so the t-derivative is zero);
//   * the inverse metric by a generic 4x4 Gauss-Jordan elimination (the
//     Kerr-Schild closed form of the inverse is deliberately NOT used);
//   * the geodesic equation written with Christoffel symbols (the first
//     display of Sec. 2.1's geodesic discussion and eq:geo):
//         xddot^mu = -Gamma^mu_{ab} xdot^a xdot^b,
//         Gamma^mu_{ab} = 1/2 g^{mu nu} (g_{nu a,b} + g_{nu b,a} - g_{ab,nu});
//   * classic fourth-order Runge-Kutta (Sec. 3, the default integrator) and
//     the Dormand-Prince 5(4) embedded pair with the step controller, the
//     termination rules, equatorial-crossing records, redshift and constants
//     of motion that the GPU library documents in include/kerrhip.h;
//   * for the chart comparison of Sec. 4 (tab:elapse): the Boyer-Lindquist
//     line element of Sec. 2.1 through the same dual-number / Gauss-Jordan /
//     Christoffel route, the map from ingoing Kerr-Schild to Boyer-Lindquist
//     states, and fixed-step RK4 in either chart.
//
// Everything is double precision.  Parallelism is a std::thread pool over
// chunks of 64 geodesics; geodesics are independent, so results do not depend
// on the thread count.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

// ----------------------------------------------------------------------------
// Dual numbers: a value and its gradient with respect to (x, y, z).
// ----------------------------------------------------------------------------
struct Dual {
  double v;
  double d[3];
};

inline Dual mk(double c) { return Dual{c, {0.0, 0.0, 0.0}}; }
inline Dual seed(double v, int i) {
  Dual r{v, {0.0, 0.0, 0.0}};
  r.d[i] = 1.0;
  return r;
}
inline double val(const Dual& a) { return a.v; }
inline double val(double a) { return a; }

inline Dual operator+(const Dual& a, const Dual& b) {
  return Dual{a.v + b.v, {a.d[0] + b.d[0], a.d[1] + b.d[1], a.d[2] + b.d[2]}};
}
inline Dual operator-(const Dual& a, const Dual& b) {
  return Dual{a.v - b.v, {a.d[0] - b.d[0], a.d[1] - b.d[1], a.d[2] - b.d[2]}};
}
inline Dual operator*(const Dual& a, const Dual& b) {
  Dual r;
  r.v = a.v * b.v;
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r;
  r.v = a.v / b.v;
  for (int i = 0; i < 3; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
inline Dual operator+(const Dual& a, double c) { return a + mk(c); }
inline Dual operator+(double c, const Dual& a) { return mk(c) + a; }
inline Dual operator-(const Dual& a, double c) { return a - mk(c); }
inline Dual operator-(double c, const Dual& a) { return mk(c) - a; }
inline Dual operator*(const Dual& a, double c) { return a * mk(c); }
inline Dual operator*(double c, const Dual& a) { return mk(c) * a; }
inline Dual operator/(const Dual& a, double c) { return a / mk(c); }
inline Dual operator/(double c, const Dual& a) { return mk(c) / a; }
inline Dual sqrt(const Dual& a) {
  double s = std::sqrt(a.v);
  Dual r{s, {0.0, 0.0, 0.0}};
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] / (2.0 * s);
  return r;
}
inline Dual sin(const Dual& a) {
  Dual r{std::sin(a.v), {0.0, 0.0, 0.0}};
  double c = std::cos(a.v);
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] * c;
  return r;
}
inline Dual cos(const Dual& a) {
  Dual r{std::cos(a.v), {0.0, 0.0, 0.0}};
  double sn = std::sin(a.v);
  for (int i = 0; i < 3; ++i) r.d[i] = -a.d[i] * sn;
  return r;
}
inline Dual log(const Dual& a) {
  Dual r{std::log(a.v), {0.0, 0.0, 0.0}};
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] / a.v;
  return r;
}
inline Dual fabs(const Dual& a) { return a.v < 0.0 ? 0.0 - a : a; }
using std::cos;
using std::fabs;
using std::log;
using std::sin;
using std::sqrt;

const double ETA[4] = {-1.0, 1.0, 1.0, 1.0};

// ----------------------------------------------------------------------------
// Sec. 2.1: the Cartesian Kerr-Schild metric.
// ----------------------------------------------------------------------------
// r is the positive root of eq:CKSr rewritten as r^4 - (R^2 - a^2) r^2 - a^2 z^2 = 0.
// The two forms of the quadratic root are algebraically equal; the second one
// avoids cancellation when R^2 < a^2.
template <class S>
S ks_radius(double a, const S& x, const S& y, const S& z) {
  S R2 = x * x + y * y + z * z;
  S w = R2 - a * a;
  S disc = sqrt(w * w + 4.0 * a * a * z * z);
  S r2 = (val(w) >= 0.0) ? 0.5 * (w + disc) : (2.0 * a * a * z * z) / (disc - w);
  return sqrt(r2);
}

// def:CKS: g_{ab} = eta_{ab} + f l_a l_b, f = 2 r^3 / (r^4 + a^2 z^2),
// l = (1, (r x + a y)/(r^2 + a^2), (r y - a x)/(r^2 + a^2), z / r).  G = c = M = 1.
template <class S>
void ks_metric(double a, const S& x, const S& y, const S& z, S g[4][4]) {
  S r = ks_radius(a, x, y, z);
  S r2 = r * r;
  S f = 2.0 * r * r2 / (r2 * r2 + a * a * z * z);
  S one = 0.0 * x + 1.0;
  S l[4] = {one, (r * x + a * y) / (r2 + a * a), (r * y - a * x) / (r2 + a * a), z / r};
  for (int m = 0; m < 4; ++m)
    for (int n = 0; n < 4; ++n) g[m][n] = f * l[m] * l[n] + ((m == n) ? ETA[m] : 0.0);
}

// double-only overload used where no derivatives are needed.
void metric_value(double a, const double x[4], double g[4][4]) {
  Dual X = mk(x[1]), Y = mk(x[2]), Z = mk(x[3]);
  Dual gd[4][4];
  ks_metric(a, X, Y, Z, gd);
  for (int m = 0; m < 4; ++m)
    for (int n = 0; n < 4; ++n) g[m][n] = gd[m][n].v;
}

double radius(double a, const double x[4]) { return ks_radius(a, x[1], x[2], x[3]); }

// Metric and its coordinate derivatives dg[c][m][n] = d g_{mn} / d x^c.
void metric_and_derivs(double a, const double x[4], double g[4][4], double dg[4][4][4]) {
  Dual X = seed(x[1], 0), Y = seed(x[2], 1), Z = seed(x[3], 2);
  Dual gd[4][4];
  ks_metric(a, X, Y, Z, gd);
  for (int m = 0; m < 4; ++m)
    for (int n = 0; n < 4; ++n) {
      g[m][n] = gd[m][n].v;
      dg[0][m][n] = 0.0;  // stationary metric
      for (int j = 0; j < 3; ++j) dg[j + 1][m][n] = gd[m][n].d[j];
    }
}

// Generic 4x4 inverse by Gauss-Jordan elimination with partial pivoting.
bool invert4(const double A[4][4], double Ainv[4][4]) {
  double M[4][8];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      M[i][j] = A[i][j];
      M[i][j + 4] = (i == j) ? 1.0 : 0.0;
    }
  for (int c = 0; c < 4; ++c) {
    int p = c;
    for (int i = c + 1; i < 4; ++i)
      if (std::fabs(M[i][c]) > std::fabs(M[p][c])) p = i;
    if (M[p][c] == 0.0) return false;
    if (p != c)
      for (int j = 0; j < 8; ++j) std::swap(M[p][j], M[c][j]);
    double inv = 1.0 / M[c][c];
    for (int j = 0; j < 8; ++j) M[c][j] *= inv;
    for (int i = 0; i < 4; ++i) {
      if (i == c) continue;
      double fct = M[i][c];
      if (fct == 0.0) continue;
      for (int j = 0; j < 8; ++j) M[i][j] -= fct * M[c][j];
    }
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) Ainv[i][j] = M[i][j + 4];
  return true;
}

// The geodesic equation with Christoffel symbols (eq:geo), for any chart given
// its metric g and derivatives dg[c][m][n] = d g_{mn} / d x^c at the point:
//   acc^mu = -Gamma^mu_{ab} k^a k^b.
void christoffel_acc(const double g[4][4], const double dg[4][4][4], const double k[4], double acc[4]) {
  double gi[4][4];
  if (!invert4(g, gi)) {
    for (int m = 0; m < 4; ++m) acc[m] = NAN;
    return;
  }
  // Christoffel symbols of the first kind, Gamma_{n a b}.
  double G1[4][4][4];
  for (int n = 0; n < 4; ++n)
    for (int p = 0; p < 4; ++p)
      for (int q = 0; q < 4; ++q) G1[n][p][q] = 0.5 * (dg[q][n][p] + dg[p][n][q] - dg[n][p][q]);
  for (int m = 0; m < 4; ++m) {
    double s = 0.0;
    for (int p = 0; p < 4; ++p)
      for (int q = 0; q < 4; ++q) {
        double gam = 0.0;
        for (int n = 0; n < 4; ++n) gam += gi[m][n] * G1[n][p][q];
        s += gam * k[p] * k[q];
      }
    acc[m] = -s;
  }
}

// Kerr-Schild right-hand side.
void geodesic_rhs(double a, const double x[4], const double k[4], double acc[4]) {
  double g[4][4], dg[4][4][4];
  metric_and_derivs(a, x, g, dg);
  christoffel_acc(g, dg, k, acc);
}

// First-order form of the system: y = (x^mu, k^mu), y' = (k^mu, acc^mu).
void deriv(double a, const double y[8], double dy[8]) {
  for (int m = 0; m < 4; ++m) dy[m] = y[4 + m];
  geodesic_rhs(a, y, y + 4, dy + 4);
}

// ----------------------------------------------------------------------------
// Constants of motion and redshift.
// ----------------------------------------------------------------------------
void lower(double a, const double x[4], const double k[4], double kl[4]) {
  double g[4][4];
  metric_value(a, x, g);
  for (int m = 0; m < 4; ++m) {
    kl[m] = 0.0;
    for (int n = 0; n < 4; ++n) kl[m] += g[m][n] * k[n];
  }
}

// E = -k_t, L_z = x k_y - y k_x, mu^2 = -g k k and Carter's constant
// Q = p_theta^2 + cos^2(theta) [a^2 (mu^2 - E^2) + L_z^2 / sin^2(theta)], with the
// spheroidal angle of the Kerr-Schild chart: cos(theta) = z / r,
// sin(theta) = rho / sqrt(r^2 + a^2), rho = sqrt(x^2 + y^2), and
// p_theta = k_i dx^i/dtheta = cot(theta) (x k_x + y k_y) - r sin(theta) k_z.
// On the spin axis (rho = 0, where both quotients are 0/0) Q takes its limit:
// p_theta^2 + cos^2(theta) L_z^2 / sin^2(theta) tends to
// cos^2(theta) (r^2 + a^2) (k_x^2 + k_y^2) from every direction, and there
// the covariant k_x, k_y equal the contravariant ones.
void constants(double a, const double x[4], const double k[4], double out[4]) {
  double kl[4];
  lower(a, x, k, kl);
  double g[4][4];
  metric_value(a, x, g);
  double mu2 = 0.0;
  for (int m = 0; m < 4; ++m)
    for (int n = 0; n < 4; ++n) mu2 -= g[m][n] * k[m] * k[n];
  double E = -kl[0];
  double Lz = x[1] * kl[2] - x[2] * kl[1];
  double r = radius(a, x);
  double rho = std::sqrt(x[1] * x[1] + x[2] * x[2]);
  double cth = x[3] / r;
  double Q;
  if (rho > 1e-150) {
    double sth = rho / std::sqrt(r * r + a * a);
    double pth = (cth / sth) * (x[1] * kl[1] + x[2] * kl[2]) - r * sth * kl[3];
    Q = pth * pth + cth * cth * (a * a * (mu2 - E * E) + Lz * Lz / (sth * sth));
  } else {
    Q = cth * cth * ((r * r + a * a) * (kl[1] * kl[1] + kl[2] * kl[2]) + a * a * (mu2 - E * E));
  }
  out[0] = E;
  out[1] = Lz;
  out[2] = Q;
  out[3] = mu2;
}

// Redshift g = nu_obs / nu_em for an emitter on the prograde Keplerian circular
// orbit of radius r in the equatorial plane of a hole of spin a:
// Omega = 1/(r^{3/2} + a), u^t = (r^{3/2} + a) / (r^{3/4} sqrt(r^{3/2} - 3 r^{1/2} + 2a)),
// g = 1 / (u^t (1 - Omega xi)) with xi = L_z / E of the photon.
double redshift(double r, double xi, double a) {
  double sr = std::sqrt(r);
  double r32 = r * sr;
  double den = r32 - 3.0 * sr + 2.0 * a;
  if (!(den > 0.0)) return NAN;
  double ut = (r32 + a) / (std::pow(r, 0.75) * std::sqrt(den));
  double Om = 1.0 / (r32 + a);
  return 1.0 / (ut * (1.0 - Om * xi));
}

// ----------------------------------------------------------------------------
// Parameters and per-geodesic bookkeeping.
// ----------------------------------------------------------------------------
enum { ST_ACTIVE = 0, ST_CAPTURED = 1, ST_ESCAPED = 2, ST_T_END = 3, ST_MAX_STEPS = 4, ST_FAILED = 5 };
enum { KIND_NULL = 0, KIND_TIMELIKE = 1 };
enum { M_RK4 = 0, M_DOPRI5 = 1, M_DOPRI5_T = 2 };

}  // namespace

extern "C" {

typedef struct {
  int32_t method;     // 0 = classic RK4 with h = h_coeff * r; 1 = Dormand-Prince 5(4);
                      // 2 = Dormand-Prince 5(4) in coordinate time (Sec. 2.2, eq:geo_t)
  int32_t k_cross;    // crossing slots per geodesic (0 disables crossing records)
  double h_coeff;     // RK4 step and DOPRI5 initial step coefficient
  double rtol, atol;  // DOPRI5 tolerances
  double hmax_coeff;  // DOPRI5 step cap: h <= hmax_coeff * scale(r)
  double r_h_factor;  // capture when r < r_h_factor * r_H
  double r_escape;    // escape when r > r_escape and dr/dlambda > 0
  double t_end;       // > 0: stop (and land exactly) at coordinate time t_end
  int64_t max_steps;  // accepted steps per call
} oracle_params;

}  // extern "C"

namespace {

// Step-size scale: r for null geodesics, r^{3/2} for time-like ones.
double hscale(int kind, double r) { return kind == KIND_TIMELIKE ? r * std::sqrt(r) : r; }

// dr/dlambda from the implicit radius: d_j r = r (r^2 x_j + a^2 z delta_jz) / (r^4 + a^2 z^2).
double rdot(double a, const double y[8]) {
  double r = radius(a, y);
  double D = r * r * r * r + a * a * y[3] * y[3];
  return r * (r * r * (y[1] * y[5] + y[2] * y[6] + y[3] * y[7]) + a * a * y[3] * y[7]) / D;
}

// Cubic Hermite basis on theta in [0, 1] for a step of length h.
double herm(double th, double y0, double m0, double y1, double m1, double h) {
  double t2 = th * th, t3 = t2 * th;
  return (2 * t3 - 3 * t2 + 1) * y0 + (t3 - 2 * t2 + th) * h * m0 + (-2 * t3 + 3 * t2) * y1 + (t3 - t2) * h * m1;
}
double dherm(double th, double y0, double m0, double y1, double m1, double h) {
  double t2 = th * th;
  return (6 * t2 - 6 * th) * y0 + (3 * t2 - 4 * th + 1) * h * m0 + (-6 * t2 + 6 * th) * y1 + (3 * t2 - 2 * th) * h * m1;
}

// Root of the Hermite interpolant of component c on [0, 1], given a sign change
// (or an exact zero at the end): safeguarded Newton iteration started from the
// linear-interpolation guess; bisection whenever Newton leaves the bracket.
double hermite_root(int c, const double y0[8], const double f0[8], const double y1[8], const double f1[8], double h,
                    double target) {
  double z0 = y0[c] - target, z1 = y1[c] - target;
  if (z1 == 0.0) return 1.0;
  double lo = 0.0, hi = 1.0;
  double th = z0 / (z0 - z1);
  for (int it = 0; it < 60; ++it) {
    double p = herm(th, z0, f0[c], z1, f1[c], h);
    if (p == 0.0) break;
    if ((p < 0.0) == (z0 < 0.0))
      lo = th;
    else
      hi = th;
    double dp = dherm(th, z0, f0[c], z1, f1[c], h);
    double tn = th - p / dp;
    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
    if (std::fabs(tn - th) <= 1e-15) {
      th = tn;
      break;
    }
    th = tn;
  }
  return th;
}

// Dense output of all 8 components at theta: positions use dx/dlambda = k,
// momenta use dk/dlambda = acc.
void hermite_state(double th, const double y0[8], const double f0[8], const double y1[8], const double f1[8], double h,
                   double out[8]) {
  for (int c = 0; c < 8; ++c) out[c] = herm(th, y0[c], f0[c], y1[c], f1[c], h);
}

struct Geo {
  double a_chart, a_phys;
  int kind;
};

struct Ray {
  double y[8];
  double lam, phi;
  int32_t status, nacc, nrej, ncross;
  double* cross;  // k_cross * 3
  // dense output at coordinate times (method (ii) of Sec. 2.2): ascending
  // targets t_out[0..n_out), states written to s_out[j][8], next target j_out
  int32_t n_out = 0, j_out = 0;
  const double* t_out = nullptr;
  double* s_out = nullptr;
  // optional record of every Dormand-Prince attempt (controller pins):
  // kTraceFields values per attempt, at most trace_cap attempts
  double* trace = nullptr;
  int64_t trace_cap = 0, trace_len = 0;
};

// One record per attempt: the step tried, its error norm, 1 if accepted, the
// radius of the state the next attempt starts from, and the status after it.
constexpr int kTraceFields = 5;
void trace_attempt(Ray& R, double h, double err, bool accepted, double r_next) {
  if (!R.trace || R.trace_len >= R.trace_cap) return;
  double* t = R.trace + kTraceFields * R.trace_len++;
  t[0] = h;
  t[1] = err;
  t[2] = accepted ? 1.0 : 0.0;
  t[3] = r_next;
  t[4] = (double)R.status;
}

// First target at or after the entry time; a target equal to it takes the
// entry state.
void dense_out_start(Ray& R) {
  if (R.n_out == 0) return;
  while (R.j_out < R.n_out && R.t_out[R.j_out] < R.y[0]) ++R.j_out;
  if (R.j_out < R.n_out && R.t_out[R.j_out] == R.y[0]) {
    for (int c = 0; c < 8; ++c) R.s_out[8 * R.j_out + c] = R.y[c];
    ++R.j_out;
  }
}

bool any_nan(const double y[8]) {
  for (int c = 0; c < 8; ++c)
    if (std::isnan(y[c])) return true;
  return false;
}

// Equatorial crossing between two accepted states.
void detect_crossing(const oracle_params& p, const Geo& G, Ray& R, const double y0[8], const double f0[8],
                     const double y1[8], const double f1[8], double h, double phi0) {
  double z0 = y0[3], z1 = y1[3];
  bool cross = (z0 < 0.0 && z1 > 0.0) || (z0 > 0.0 && z1 < 0.0) || (z1 == 0.0 && z0 != 0.0);
  if (!cross) return;
  double th = hermite_root(3, y0, f0, y1, f1, h, 0.0);
  double yc[8];
  hermite_state(th, y0, f0, y1, f1, h, yc);
  yc[3] = 0.0;
  double a = G.a_chart;
  double rc = std::sqrt(std::max(yc[1] * yc[1] + yc[2] * yc[2] - a * a, 0.0));
  double phic = phi0 + std::atan2(y0[1] * yc[2] - y0[2] * yc[1], y0[1] * yc[1] + y0[2] * yc[2]);
  // xi is a constant of motion: take it from the accepted end state of the
  // step (an integrator node), not from the interpolant.
  double kl[4];
  lower(a, y1, y1 + 4, kl);
  double E = -kl[0];
  double Lz = y1[1] * kl[2] - y1[2] * kl[1];
  // Null rays run future-directed in the chart with reversed spin; the
  // physical photon then has the same E and the opposite L_z.
  double xi = (G.kind == KIND_NULL) ? -Lz / E : Lz / E;
  double gz = redshift(rc, xi, G.a_phys);
  if (R.ncross < p.k_cross) {
    double* c = R.cross + 3 * R.ncross;
    c[0] = rc;
    c[1] = phic;
    c[2] = gz;
  }
  R.ncross += 1;
}

// Termination checks after an accepted step.  Returns the new status.
int32_t check_end(const oracle_params& p, const Geo& G, const double y[8]) {
  double r = radius(G.a_chart, y);
  double rH = 1.0 + std::sqrt(std::max(1.0 - G.a_chart * G.a_chart, 0.0));
  if (r < p.r_h_factor * rH) return ST_CAPTURED;
  if (r > p.r_escape && rdot(G.a_chart, y) > 0.0) return ST_ESCAPED;
  return ST_ACTIVE;
}

void run_rk4(const oracle_params& p, const Geo& G, Ray& R) {
  const double a = G.a_chart;
  int64_t steps = 0;
  while (true) {
    double h = p.h_coeff * radius(a, R.y);
    double k1[8], k2[8], k3[8], k4[8], t[8];
    deriv(a, R.y, k1);
    for (int c = 0; c < 8; ++c) t[c] = R.y[c] + 0.5 * h * k1[c];
    deriv(a, t, k2);
    for (int c = 0; c < 8; ++c) t[c] = R.y[c] + 0.5 * h * k2[c];
    deriv(a, t, k3);
    for (int c = 0; c < 8; ++c) t[c] = R.y[c] + h * k3[c];
    deriv(a, t, k4);
    for (int c = 0; c < 8; ++c) R.y[c] += h / 6.0 * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
    R.lam += h;
    R.nacc += 1;
    ++steps;
    if (any_nan(R.y)) {
      R.status = ST_FAILED;
      break;
    }
    R.status = check_end(p, G, R.y);
    if (R.status != ST_ACTIVE) break;
    if (steps >= p.max_steps) {
      R.status = ST_MAX_STEPS;
      break;
    }
  }
}

// Dormand & Prince (1980) 5(4) tableau.
const double C2 = 1.0 / 5, C3 = 3.0 / 10, C4 = 4.0 / 5, C5 = 8.0 / 9;
const double A21 = 1.0 / 5;
const double A31 = 3.0 / 40, A32 = 9.0 / 40;
const double A41 = 44.0 / 45, A42 = -56.0 / 15, A43 = 32.0 / 9;
const double A51 = 19372.0 / 6561, A52 = -25360.0 / 2187, A53 = 64448.0 / 6561, A54 = -212.0 / 729;
const double A61 = 9017.0 / 3168, A62 = -355.0 / 33, A63 = 46732.0 / 5247, A64 = 49.0 / 176,
             A65 = -5103.0 / 18656;
const double B1 = 35.0 / 384, B3 = 500.0 / 1113, B4 = 125.0 / 192, B5 = -2187.0 / 6784, B6 = 11.0 / 84;
// 4th-order weights b*
const double S1 = 5179.0 / 57600, S3 = 7571.0 / 16695, S4 = 393.0 / 640, S5 = -92097.0 / 339200,
             S6 = 187.0 / 2100, S7 = 1.0 / 40;

// One Dormand-Prince attempt from y with derivative f1 = y'(y); returns the
// 5th-order solution y5, its derivative f7 (FSAL) and the RMS error norm.
template <class RHS>
double dopri5_attempt(RHS&& F, const double y[8], const double f1[8], double h, double rtol, double atol,
                      double y5[8], double f7[8], double* y4_out = nullptr) {
  double f2[8], f3[8], f4[8], f5[8], f6[8], t[8];
  for (int c = 0; c < 8; ++c) t[c] = y[c] + h * (A21 * f1[c]);
  F(t, f2);
  for (int c = 0; c < 8; ++c) t[c] = y[c] + h * (A31 * f1[c] + A32 * f2[c]);
  F(t, f3);
  for (int c = 0; c < 8; ++c) t[c] = y[c] + h * (A41 * f1[c] + A42 * f2[c] + A43 * f3[c]);
  F(t, f4);
  for (int c = 0; c < 8; ++c) t[c] = y[c] + h * (A51 * f1[c] + A52 * f2[c] + A53 * f3[c] + A54 * f4[c]);
  F(t, f5);
  for (int c = 0; c < 8; ++c)
    t[c] = y[c] + h * (A61 * f1[c] + A62 * f2[c] + A63 * f3[c] + A64 * f4[c] + A65 * f5[c]);
  F(t, f6);
  for (int c = 0; c < 8; ++c) y5[c] = y[c] + h * (B1 * f1[c] + B3 * f3[c] + B4 * f4[c] + B5 * f5[c] + B6 * f6[c]);
  F(y5, f7);
  double s = 0.0;
  for (int c = 0; c < 8; ++c) {
    double y4 = y[c] + h * (S1 * f1[c] + S3 * f3[c] + S4 * f4[c] + S5 * f5[c] + S6 * f6[c] + S7 * f7[c]);
    if (y4_out) y4_out[c] = y4;
    double sc = atol + rtol * std::max(std::fabs(y[c]), std::fabs(y5[c]));
    double e = (y5[c] - y4) / sc;
    s += e * e;
  }
  return std::sqrt(s / 8.0);
}

// Step-size controller: accept if err <= 1; the new step is
// h * min(5, max(0.2, 0.9 err^{-1/5})), with no growth right after a rejection.
double grow_factor(double err, bool after_reject) {
  double fac = (err == 0.0) ? 5.0 : std::min(5.0, std::max(0.2, 0.9 * std::pow(err, -0.2)));
  if (after_reject) fac = std::min(fac, 1.0);
  return fac;
}
double shrink_factor(double err) { return std::isnan(err) ? 0.2 : std::max(0.2, 0.9 * std::pow(err, -0.2)); }

void run_dopri5(const oracle_params& p, const Geo& G, Ray& R) {
  const double a = G.a_chart;
  dense_out_start(R);
  auto F = [a](const double* y, double* dy) { deriv(a, y, dy); };
  double f1[8];
  F(R.y, f1);
  double h = p.h_coeff * hscale(G.kind, radius(a, R.y));
  h = std::min(h, p.hmax_coeff * hscale(G.kind, radius(a, R.y)));
  bool after_reject = false;
  int64_t steps = 0;
  int64_t attempts = 0;
  R.status = ST_ACTIVE;
  while (true) {
    double y5[8], f7[8];
    double err = dopri5_attempt(F, R.y, f1, h, p.rtol, p.atol, y5, f7);
    ++attempts;
    const double h_try = h;
    auto traced = [&]() { trace_attempt(R, h_try, err, err <= 1.0, radius(a, R.y)); };
    if (err <= 1.0) {
      double y0[8], f0[8];
      std::memcpy(y0, R.y, sizeof y0);
      std::memcpy(f0, f1, sizeof f0);
      std::memcpy(R.y, y5, sizeof y0);
      std::memcpy(f1, f7, sizeof f0);
      R.lam += h;
      R.nacc += 1;
      ++steps;
      if (any_nan(R.y)) {
        R.status = ST_FAILED;
        traced();
        return;
      }
      if (p.k_cross > 0) {
        double phi0 = R.phi;
        R.phi = phi0 + std::atan2(y0[1] * R.y[2] - y0[2] * R.y[1], y0[1] * R.y[1] + y0[2] * R.y[2]);
        detect_crossing(p, G, R, y0, f0, R.y, f1, h, phi0);
      }
      // dense output: every target time passed by this step, from the Hermite
      // interpolant of t(lambda) (root) and of the state (never past t_end)
      while (R.j_out < R.n_out && R.t_out[R.j_out] <= R.y[0] && !(p.t_end > 0.0 && R.t_out[R.j_out] > p.t_end)) {
        const double tj = R.t_out[R.j_out];
        double th = hermite_root(0, y0, f0, R.y, f1, h, tj);
        double* o = R.s_out + 8 * R.j_out;
        hermite_state(th, y0, f0, R.y, f1, h, o);
        o[0] = tj;
        ++R.j_out;
      }
      int32_t st = check_end(p, G, R.y);
      if (st == ST_ACTIVE && p.t_end > 0.0 && R.y[0] >= p.t_end) {
        // Land on t = t_end with the Hermite interpolant of t(lambda).
        double th = hermite_root(0, y0, f0, R.y, f1, h, p.t_end);
        double yl[8];
        hermite_state(th, y0, f0, R.y, f1, h, yl);
        R.lam += (th - 1.0) * h;
        std::memcpy(R.y, yl, sizeof yl);
        st = ST_T_END;
      }
      if (st != ST_ACTIVE) {
        R.status = st;
        traced();
        return;
      }
      h *= grow_factor(err, after_reject);
      h = std::min(h, p.hmax_coeff * hscale(G.kind, radius(a, R.y)));
      after_reject = false;
      if (steps >= p.max_steps) {
        R.status = ST_MAX_STEPS;
        traced();
        return;
      }
    } else {
      R.nrej += 1;
      h *= shrink_factor(err);
      after_reject = true;
      if (!(h >= 1e-12 * p.h_coeff * hscale(G.kind, radius(a, R.y)))) {  // also ends a NaN step
        R.status = ST_FAILED;
        traced();
        return;
      }
    }
    if (attempts > 4 * p.max_steps + 1000) R.status = ST_MAX_STEPS;
    traced();
    if (R.status != ST_ACTIVE) return;
  }
}

// ----------------------------------------------------------------------------
// Coordinate-time integration (Sec. 2.2, the coordinate-time subsection):
// with v^mu = dx^mu/dt (v^0 = 1) the spatial equations are
//     dv^i/dt = -Gamma^i_{ab} v^a v^b + Gamma^0_{ab} v^a v^b v^i,
// the paper's first display there, written out with the same Christoffel
// symbols as eq:geo.  The state is the six numbers (x^i, v^i) and t is the
// independent variable.  Dormand-Prince 5(4) as above, the RMS error norm over
// the six components, the same controller, step scale and termination rules.
// A target time t_end is hit exactly: the step is clipped to t_end - t.
// On exit the state is returned in the affine form (x^mu, k^mu) with
// k^mu = k^0 (1, v^i); k^0 follows from the conserved energy
// E = -k_t = -k^0 (g_{0a} v^a) of the entry state, so E is preserved exactly
// and the other constants (L_z, Q, mu^2) measure the drift.  The affine
// parameter is not advanced.
// ----------------------------------------------------------------------------
void deriv_ct(double a, const double y[6], double dy[6]) {
  const double x[4] = {0.0, y[0], y[1], y[2]};
  const double v[4] = {1.0, y[3], y[4], y[5]};
  double acc[4];
  geodesic_rhs(a, x, v, acc);  // acc^mu = -Gamma^mu_{ab} v^a v^b
  for (int i = 0; i < 3; ++i) {
    dy[i] = y[3 + i];
    dy[3 + i] = acc[1 + i] - acc[0] * y[3 + i];
  }
}

double dopri5_attempt6(double a, const double y[6], const double f1[6], double h, double rtol, double atol,
                       double y5[6], double f7[6]) {
  double f2[6], f3[6], f4[6], f5[6], f6[6], t[6];
  for (int c = 0; c < 6; ++c) t[c] = y[c] + h * (A21 * f1[c]);
  deriv_ct(a, t, f2);
  for (int c = 0; c < 6; ++c) t[c] = y[c] + h * (A31 * f1[c] + A32 * f2[c]);
  deriv_ct(a, t, f3);
  for (int c = 0; c < 6; ++c) t[c] = y[c] + h * (A41 * f1[c] + A42 * f2[c] + A43 * f3[c]);
  deriv_ct(a, t, f4);
  for (int c = 0; c < 6; ++c) t[c] = y[c] + h * (A51 * f1[c] + A52 * f2[c] + A53 * f3[c] + A54 * f4[c]);
  deriv_ct(a, t, f5);
  for (int c = 0; c < 6; ++c)
    t[c] = y[c] + h * (A61 * f1[c] + A62 * f2[c] + A63 * f3[c] + A64 * f4[c] + A65 * f5[c]);
  deriv_ct(a, t, f6);
  for (int c = 0; c < 6; ++c) y5[c] = y[c] + h * (B1 * f1[c] + B3 * f3[c] + B4 * f4[c] + B5 * f5[c] + B6 * f6[c]);
  deriv_ct(a, y5, f7);
  double s = 0.0;
  for (int c = 0; c < 6; ++c) {
    double y4 = y[c] + h * (S1 * f1[c] + S3 * f3[c] + S4 * f4[c] + S5 * f5[c] + S6 * f6[c] + S7 * f7[c]);
    double sc = atol + rtol * std::max(std::fabs(y[c]), std::fabs(y5[c]));
    double e = (y5[c] - y4) / sc;
    s += e * e;
  }
  return std::sqrt(s / 6.0);
}

// The 8-slot forms used by the shared crossing and termination helpers:
// Y = (t, x^i, 1, v^i) and its t-derivative (1, v^i, 0, dv^i/dt).
void to8(double t, const double y[6], double Y[8]) {
  Y[0] = t;
  Y[4] = 1.0;
  for (int i = 0; i < 3; ++i) {
    Y[1 + i] = y[i];
    Y[5 + i] = y[3 + i];
  }
}
void to8d(const double f[6], double F[8]) {
  F[0] = 1.0;
  F[4] = 0.0;
  for (int i = 0; i < 3; ++i) {
    F[1 + i] = f[i];
    F[5 + i] = f[3 + i];
  }
}

void run_dopri5_ct(const oracle_params& p, const Geo& G, Ray& R) {
  const double a = G.a_chart;
  dense_out_start(R);
  double kl[4];
  lower(a, R.y, R.y + 4, kl);
  const double E0 = -kl[0];
  double t = R.y[0];
  double y[6] = {R.y[1], R.y[2], R.y[3], R.y[5] / R.y[4], R.y[6] / R.y[4], R.y[7] / R.y[4]};
  double f1[6];
  deriv_ct(a, y, f1);
  double Y[8];
  to8(t, y, Y);
  double h = p.h_coeff * hscale(G.kind, radius(a, Y));
  h = std::min(h, p.hmax_coeff * hscale(G.kind, radius(a, Y)));
  bool after_reject = false;
  int64_t steps = 0, attempts = 0;
  R.status = ST_ACTIVE;
  if (p.t_end > 0.0 && t >= p.t_end) R.status = ST_T_END;  // already there: no step
  while (R.status == ST_ACTIVE) {
    const bool landing = p.t_end > 0.0 && t + h >= p.t_end;
    const double hs = landing ? p.t_end - t : h;
    double y5[6], f7[6];
    double err = dopri5_attempt6(a, y, f1, hs, p.rtol, p.atol, y5, f7);
    ++attempts;
    if (err <= 1.0) {
      double Y0[8], F0[8], Y1[8], F1[8];
      to8(t, y, Y0);
      to8d(f1, F0);
      t = landing ? p.t_end : t + hs;
      std::memcpy(y, y5, sizeof y);
      std::memcpy(f1, f7, sizeof f1);
      to8(t, y, Y1);
      to8d(f1, F1);
      R.nacc += 1;
      ++steps;
      bool bad = std::isnan(t);
      for (int c = 0; c < 6; ++c) bad = bad || std::isnan(y[c]);
      int32_t st = ST_ACTIVE;
      if (bad) {
        st = ST_FAILED;
      } else {
        if (p.k_cross > 0) {
          double phi0 = R.phi;
          R.phi = phi0 + std::atan2(Y0[1] * Y1[2] - Y0[2] * Y1[1], Y0[1] * Y1[1] + Y0[2] * Y1[2]);
          detect_crossing(p, G, R, Y0, F0, Y1, F1, hs, phi0);
        }
        // dense output: in coordinate time the target sits at theta = (t_j - t0) / h;
        // k^mu = k^0 (1, v) with k^0 from the entry energy, as on exit
        while (R.j_out < R.n_out && R.t_out[R.j_out] <= t) {
          const double tj = R.t_out[R.j_out];
          double Yj[8];
          hermite_state((tj - Y0[0]) / hs, Y0, F0, Y1, F1, hs, Yj);
          Yj[0] = tj;
          Yj[4] = 1.0;
          double klj[4];
          lower(a, Yj, Yj + 4, klj);
          const double k0 = E0 / (-klj[0]);
          double* o = R.s_out + 8 * R.j_out;
          for (int c = 0; c < 4; ++c) {
            o[c] = Yj[c];
            o[4 + c] = k0 * Yj[4 + c];
          }
          ++R.j_out;
        }
        st = check_end(p, G, Y1);
        if (st == ST_ACTIVE && landing) st = ST_T_END;
      }
      if (st != ST_ACTIVE) {
        R.status = st;
        break;
      }
      h = hs * grow_factor(err, after_reject);
      h = std::min(h, p.hmax_coeff * hscale(G.kind, radius(a, Y1)));
      after_reject = false;
      if (steps >= p.max_steps) {
        R.status = ST_MAX_STEPS;
        break;
      }
    } else {
      R.nrej += 1;
      h = hs * shrink_factor(err);
      after_reject = true;
      double Yc[8];
      to8(t, y, Yc);
      if (!(h >= 1e-12 * p.h_coeff * hscale(G.kind, radius(a, Yc)))) {  // also ends a NaN step
        R.status = ST_FAILED;
        break;
      }
    }
    if (attempts > 4 * p.max_steps + 1000) {
      R.status = ST_MAX_STEPS;
      break;
    }
  }
  // back to (x^mu, k^mu): k^0 from the conserved energy of the entry state
  double Yv[8];
  to8(t, y, Yv);
  lower(a, Yv, Yv + 4, kl);  // covariant components of (1, v)
  const double k0 = E0 / (-kl[0]);
  R.y[0] = t;
  for (int i = 0; i < 3; ++i) {
    R.y[1 + i] = y[i];
    R.y[5 + i] = k0 * y[3 + i];
  }
  R.y[4] = k0;
}

template <class Fn>
void parallel_chunks(int64_t n, int nthreads, Fn&& fn) {
  if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
  std::atomic<int64_t> next{0};
  const int64_t chunk = 64;
  auto worker = [&]() {
    while (true) {
      int64_t b = next.fetch_add(chunk);
      if (b >= n) break;
      int64_t e = std::min(n, b + chunk);
      for (int64_t i = b; i < e; ++i) fn(i);
    }
  };
  if (nthreads == 1 || n <= chunk) {
    worker();
    return;
  }
  std::vector<std::thread> ts;
  for (int t = 0; t < nthreads; ++t) ts.emplace_back(worker);
  for (auto& t : ts) t.join();
}

// Null initial momentum: solve g_{ab} k^a k^b = 0 for k^0 given spatial k^i,
// taking the future-directed (k^0 > 0) root.  Returns false if none exists.
bool null_k0(double a, const double x[4], double k[4]) {
  double g[4][4];
  metric_value(a, x, g);
  double A = g[0][0], B = 0.0, C = 0.0;
  for (int i = 1; i < 4; ++i) {
    B += g[0][i] * k[i];
    for (int j = 1; j < 4; ++j) C += g[i][j] * k[i] * k[j];
  }
  double disc = B * B - A * C;
  if (!(A < 0.0) || !(disc >= 0.0)) return false;
  k[0] = (B + std::sqrt(disc)) / (-A);
  return true;
}

// Camera of the image plane: observer direction n = (sin i, 0, cos i), screen axes
// e_alpha = (0, 1, 0) and e_beta = (-cos i, 0, sin i); the ray starts at
// d n + alpha e_alpha + beta e_beta with spatial momentum -n.
void camera_ray(double a_phys, double d, double incl, double alpha, double beta, double y[8], bool* ok) {
  double si = std::sin(incl), ci = std::cos(incl);
  y[0] = 0.0;
  y[1] = d * si - beta * ci;
  y[2] = alpha;
  y[3] = d * ci + beta * si;
  y[4] = 0.0;
  y[5] = -si;
  y[6] = 0.0;
  y[7] = -ci;
  *ok = null_k0(-a_phys, y, y + 4);
}

}  // namespace

extern "C" {

// Rays of an image: pixel p = row * W + col has alpha = amin + (col + 1/2)(amax - amin)/W
// and beta = bmin + (row + 1/2)(bmax - bmin)/H.  perturb shifts alpha and beta by
// perturb * (1 + |.|) (conditioning probe).  s is [8][n] (SoA).
int oracle_camera_rays(double a_phys, double r_obs, double incl, double amin, double amax, double bmin, double bmax,
                       int32_t W, int32_t H, const int64_t* pix, int64_t n, double perturb, double* s,
                       double* spin, int32_t* kind, int32_t* status) {
  for (int64_t i = 0; i < n; ++i) {
    int64_t pid = pix ? pix[i] : i;
    int64_t row = pid / W, col = pid % W;
    double al = amin + (col + 0.5) * (amax - amin) / W;
    double be = bmin + (row + 0.5) * (bmax - bmin) / H;
    al += perturb * (1.0 + std::fabs(al));
    be += perturb * (1.0 + std::fabs(be));
    double y[8];
    bool ok;
    camera_ray(a_phys, r_obs, incl, al, be, y, &ok);
    for (int c = 0; c < 8; ++c) s[c * n + i] = y[c];
    spin[i] = a_phys;
    kind[i] = KIND_NULL;
    status[i] = ok ? ST_ACTIVE : ST_FAILED;
  }
  (void)H;
  return 0;
}

// Rays with individual (spin, inclination, alpha, beta) and a common observer distance.
int oracle_list_rays(const double* a_phys, const double* incl, const double* alpha, const double* beta, double r_obs,
                     int64_t n, double* s, double* spin, int32_t* kind, int32_t* status) {
  for (int64_t i = 0; i < n; ++i) {
    double y[8];
    bool ok;
    camera_ray(a_phys[i], r_obs, incl[i], alpha[i], beta[i], y, &ok);
    for (int c = 0; c < 8; ++c) s[c * n + i] = y[c];
    spin[i] = a_phys[i];
    kind[i] = KIND_NULL;
    status[i] = ok ? ST_ACTIVE : ST_FAILED;
  }
  return 0;
}

// Time-like geodesics from positions x3 [3][n] and coordinate velocities
// v3 = dx^i/dt [3][n]: u^0 = 1 / sqrt(-g_{ab} v^a v^b) with v^0 = 1, u^i = u^0 v^i.
int oracle_timelike(const double* a, const double* x3, const double* v3, int64_t n, double* s, double* spin,
                    int32_t* kind, int32_t* status) {
  for (int64_t i = 0; i < n; ++i) {
    double x[4] = {0.0, x3[i], x3[n + i], x3[2 * n + i]};
    double v[4] = {1.0, v3[i], v3[n + i], v3[2 * n + i]};
    double g[4][4];
    metric_value(a[i], x, g);
    double nrm = 0.0;
    for (int m = 0; m < 4; ++m)
      for (int q = 0; q < 4; ++q) nrm += g[m][q] * v[m] * v[q];
    bool ok = nrm < 0.0;
    double u0 = ok ? 1.0 / std::sqrt(-nrm) : NAN;
    for (int c = 0; c < 4; ++c) {
      s[c * n + i] = x[c];
      s[(4 + c) * n + i] = u0 * v[c];
    }
    spin[i] = a[i];
    kind[i] = KIND_TIMELIKE;
    status[i] = ok ? ST_ACTIVE : ST_FAILED;
  }
  return 0;
}

int oracle_integrate_out(const oracle_params* p, int64_t n, double* s, const double* spin, const int32_t* kind,
                         double* lam, double* phi, int32_t* status, int32_t* n_acc, int32_t* n_rej, double* cross,
                         int32_t* n_cross, double* c0, double* c1, int32_t n_out, const double* t_out,
                         double* s_out, int32_t nthreads);

// Integrate n geodesics from their current state.  s is [8][n]; cross is
// [n][k_cross][3] = (r, phi, g); c0/c1 are [4][n] = (E, L_z, Q, mu^2) at the start
// and at the end (may be NULL).  Geodesics whose status is not ACTIVE are skipped.
int oracle_integrate(const oracle_params* p, int64_t n, double* s, const double* spin, const int32_t* kind,
                     double* lam, double* phi, int32_t* status, int32_t* n_acc, int32_t* n_rej, double* cross,
                     int32_t* n_cross, double* c0, double* c1, int32_t nthreads) {
  return oracle_integrate_out(p, n, s, spin, kind, lam, phi, status, n_acc, n_rej, cross, n_cross, c0, c1, 0, nullptr,
                              nullptr, nthreads);
}

// The same, with dense output at the ascending coordinate times t_out[0..n_out):
// s_out is [n][n_out][8] (x^mu, k^mu at t_out[j]; entries the call does not
// reach are left as they are).  DOPRI5 methods only.
int oracle_integrate_out(const oracle_params* p, int64_t n, double* s, const double* spin, const int32_t* kind,
                         double* lam, double* phi, int32_t* status, int32_t* n_acc, int32_t* n_rej, double* cross,
                         int32_t* n_cross, double* c0, double* c1, int32_t n_out, const double* t_out,
                         double* s_out, int32_t nthreads) {
  if (!p || n < 0 || n_out < 0 || (n_out > 0 && (!t_out || !s_out))) return -1;
  if (p->method != M_RK4 && p->method != M_DOPRI5 && p->method != M_DOPRI5_T) return -1;
  if (n_out > 0 && p->method == M_RK4) return -1;
  parallel_chunks(n, nthreads, [&](int64_t i) {
    Geo G;
    G.kind = kind[i];
    G.a_phys = spin[i];
    G.a_chart = (G.kind == KIND_NULL) ? -spin[i] : spin[i];
    Ray R;
    for (int c = 0; c < 8; ++c) R.y[c] = s[c * n + i];
    R.lam = lam ? lam[i] : 0.0;
    R.phi = std::atan2(R.y[2], R.y[1]);
    R.status = status[i];
    R.nacc = 0;
    R.nrej = 0;
    R.ncross = 0;
    std::vector<double> cbuf(3 * std::max(p->k_cross, 1), NAN);
    R.cross = cbuf.data();
    R.n_out = n_out;
    R.t_out = t_out;
    R.s_out = n_out > 0 ? s_out + (int64_t)8 * n_out * i : nullptr;
    double cst[4];
    constants(G.a_chart, R.y, R.y + 4, cst);
    if (c0)
      for (int q = 0; q < 4; ++q) c0[q * n + i] = cst[q];
    if (R.status == ST_ACTIVE) {
      if (p->method == M_RK4)
        run_rk4(*p, G, R);
      else if (p->method == M_DOPRI5_T)
        run_dopri5_ct(*p, G, R);
      else
        run_dopri5(*p, G, R);
    }
    for (int c = 0; c < 8; ++c) s[c * n + i] = R.y[c];
    if (lam) lam[i] = R.lam;
    if (phi) phi[i] = R.phi;
    status[i] = R.status;
    if (n_acc) n_acc[i] = R.nacc;
    if (n_rej) n_rej[i] = R.nrej;
    if (n_cross) n_cross[i] = R.ncross;
    if (cross && p->k_cross > 0)
      for (int q = 0; q < 3 * p->k_cross; ++q) cross[3 * p->k_cross * i + q] = cbuf[q];
    constants(G.a_chart, R.y, R.y + 4, cst);
    if (c1)
      for (int q = 0; q < 4; ++q) c1[q * n + i] = cst[q];
  });
  return 0;
}

// One geodesic, recording every accepted state (lambda, x^mu, k^mu) -> out[max_out][9].
// Stops at termination or after max_out records.  Returns the record count.
int64_t oracle_trajectory(const oracle_params* p, double spin_chart, const double y0[8], int64_t max_out,
                          double* out) {
  Geo G;
  G.kind = KIND_NULL;
  G.a_chart = spin_chart;
  G.a_phys = -spin_chart;
  double a = spin_chart;
  double y[8];
  std::memcpy(y, y0, sizeof y);
  double lam = 0.0;
  int64_t m = 0;
  auto rec = [&](const double* yy) {
    if (m >= max_out) return;
    out[9 * m] = lam;
    for (int c = 0; c < 8; ++c) out[9 * m + 1 + c] = yy[c];
    ++m;
  };
  rec(y);
  double mu2_chk[4];
  constants(a, y, y + 4, mu2_chk);
  if (mu2_chk[3] > 1e-6) G.kind = KIND_TIMELIKE;
  if (p->method == M_RK4) {
    while (m < max_out) {
      double h = p->h_coeff;  // fixed affine step for trajectories
      double k1[8], k2[8], k3[8], k4[8], t[8];
      deriv(a, y, k1);
      for (int c = 0; c < 8; ++c) t[c] = y[c] + 0.5 * h * k1[c];
      deriv(a, t, k2);
      for (int c = 0; c < 8; ++c) t[c] = y[c] + 0.5 * h * k2[c];
      deriv(a, t, k3);
      for (int c = 0; c < 8; ++c) t[c] = y[c] + h * k3[c];
      deriv(a, t, k4);
      for (int c = 0; c < 8; ++c) y[c] += h / 6.0 * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
      lam += h;
      rec(y);
      if (any_nan(y) || check_end(*p, G, y) != ST_ACTIVE) break;
    }
    return m;
  }
  auto F = [a](const double* yy, double* dy) { deriv(a, yy, dy); };
  double f1[8];
  F(y, f1);
  double h = std::min(p->h_coeff, p->hmax_coeff) * hscale(G.kind, radius(a, y));
  bool after_reject = false;
  int64_t attempts = 0;
  while (m < max_out && attempts < 100 * max_out) {
    double y5[8], f7[8];
    double err = dopri5_attempt(F, y, f1, h, p->rtol, p->atol, y5, f7);
    ++attempts;
    if (err <= 1.0) {
      std::memcpy(y, y5, sizeof y);
      std::memcpy(f1, f7, sizeof f1);
      lam += h;
      rec(y);
      if (any_nan(y) || check_end(*p, G, y) != ST_ACTIVE) break;
      if (p->t_end > 0.0 && y[0] >= p->t_end) break;
      h *= grow_factor(err, after_reject);
      h = std::min(h, p->hmax_coeff * hscale(G.kind, radius(a, y)));
      after_reject = false;
    } else {
      h *= shrink_factor(err);
      after_reject = true;
    }
  }
  return m;
}

// Pieces exposed for the pins.
void oracle_rhs(double a, const double x[4], const double k[4], double acc[4]) { geodesic_rhs(a, x, k, acc); }

void oracle_metric(double a, const double x[4], double g[16], double dg[64]) {
  double gg[4][4], d[4][4][4];
  metric_and_derivs(a, x, gg, d);
  for (int m = 0; m < 4; ++m)
    for (int q = 0; q < 4; ++q) {
      g[4 * m + q] = gg[m][q];
      for (int c = 0; c < 4; ++c) dg[16 * c + 4 * m + q] = d[c][m][q];
    }
}

double oracle_radius(double a, double x, double y, double z) { return ks_radius(a, x, y, z); }

void oracle_constants(double a, const double x[4], const double k[4], double out[4]) { constants(a, x, k, out); }

double oracle_redshift(double r, double xi, double a) { return redshift(r, xi, a); }

// The Dormand-Prince pair on the harmonic oscillator y'' = -y, embedded in the
// same 8-component first-order layout (x' = k, k' = -x); fixed step h for
// nsteps steps.  out[0..7] = final state, out[8] = last error norm.
void oracle_dopri5_sho(const double y0[8], double h, int64_t nsteps, double rtol, double out[9]) {
  auto F = [](const double* y, double* dy) {
    for (int c = 0; c < 4; ++c) {
      dy[c] = y[4 + c];
      dy[4 + c] = -y[c];
    }
  };
  double y[8], f1[8], y5[8], f7[8];
  std::memcpy(y, y0, sizeof y);
  F(y, f1);
  double err = 0.0;
  for (int64_t i = 0; i < nsteps; ++i) {
    err = dopri5_attempt(F, y, f1, h, rtol, rtol, y5, f7);
    std::memcpy(y, y5, sizeof y);
    std::memcpy(f1, f7, sizeof f1);
  }
  std::memcpy(out, y, sizeof y);
  out[8] = err;
}

// One Dormand-Prince attempt of step h on y'' = -y (the same 8-component
// layout as above) with separate tolerances: the 5th-order solution y5, the
// embedded 4th-order solution y4 and the error norm; returns the norm.
double oracle_dopri5_sho_attempt(const double y0[8], double h, double rtol, double atol, double y5[8],
                                 double y4[8]) {
  auto F = [](const double* y, double* dy) {
    for (int c = 0; c < 4; ++c) {
      dy[c] = y[4 + c];
      dy[4 + c] = -y[c];
    }
  };
  double f1[8], f7[8];
  F(y0, f1);
  return dopri5_attempt(F, y0, f1, h, rtol, atol, y5, f7, y4);
}

// One geodesic (chart spin from the physical spin and the kind, as in
// oracle_integrate) integrated by the Dormand-Prince integrator, recording
// every attempt in out[max_rec][5] = (h, err, accepted, r after the attempt,
// status after the attempt).  res[0..2] = (status, accepted steps, rejected
// attempts).  Returns the number of records.
int64_t oracle_controller_trace(const oracle_params* p, double spin_phys, int32_t kind, const double y0[8],
                                int64_t max_rec, double* out, int32_t* res) {
  if (!p || p->method != M_DOPRI5 || max_rec < 0) return -1;
  Geo G;
  G.kind = kind;
  G.a_phys = spin_phys;
  G.a_chart = (kind == KIND_NULL) ? -spin_phys : spin_phys;
  Ray R;
  std::memcpy(R.y, y0, sizeof R.y);
  R.lam = 0.0;
  R.phi = std::atan2(R.y[2], R.y[1]);
  R.status = ST_ACTIVE;
  R.nacc = R.nrej = R.ncross = 0;
  std::vector<double> cbuf(3 * std::max(p->k_cross, 1), NAN);
  R.cross = cbuf.data();
  R.trace = out;
  R.trace_cap = max_rec;
  run_dopri5(*p, G, R);
  if (res) {
    res[0] = R.status;
    res[1] = R.nacc;
    res[2] = R.nrej;
  }
  return R.trace_len;
}

}  // extern "C"

// ============================================================================
// Boyer-Lindquist chart (the line element at the start of Sec. 2.1) and
// fixed-step RK4 in either chart: the workload of the benchmark of Sec. 4
// (tab:elapse), which integrates the same rays in both charts.
// ============================================================================
namespace {

enum { CHART_KS = 0, CHART_BL = 1 };

// Boyer-Lindquist metric in coordinates (t, r, theta, phi), M = 1, with
// rho^2 = r^2 + a^2 cos^2(theta) and Delta = r^2 - 2 r + a^2:
//   g_tt = -(1 - 2 r / rho^2),  g_t phi = -2 a r sin^2(theta) / rho^2,
//   g_rr = rho^2 / Delta,       g_theta theta = rho^2,
//   g_phi phi = (r^2 + a^2 + 2 a^2 r sin^2(theta) / rho^2) sin^2(theta).
template <class S>
void bl_metric(double a, const S& r, const S& th, S g[4][4]) {
  S s = sin(th), c = cos(th);
  S rho2 = r * r + a * a * c * c;
  S Delta = r * r - 2.0 * r + a * a;
  S zero = 0.0 * r;
  for (int m = 0; m < 4; ++m)
    for (int n = 0; n < 4; ++n) g[m][n] = zero;
  g[0][0] = 2.0 * r / rho2 - 1.0;
  g[0][3] = (-2.0 * a) * r * s * s / rho2;
  g[3][0] = g[0][3];
  g[1][1] = rho2 / Delta;
  g[2][2] = rho2;
  g[3][3] = (r * r + a * a + 2.0 * a * a * r * s * s / rho2) * s * s;
}

// Metric and derivatives dg[c][m][n] = d g_{mn} / d x^c by dual numbers in
// (r, theta); the metric depends on neither t nor phi.
void bl_metric_and_derivs(double a, const double x[4], double g[4][4], double dg[4][4][4]) {
  Dual R = seed(x[1], 0), TH = seed(x[2], 1);
  Dual gd[4][4];
  bl_metric(a, R, TH, gd);
  for (int m = 0; m < 4; ++m)
    for (int n = 0; n < 4; ++n) {
      g[m][n] = gd[m][n].v;
      dg[0][m][n] = 0.0;
      dg[1][m][n] = gd[m][n].d[0];
      dg[2][m][n] = gd[m][n].d[1];
      dg[3][m][n] = 0.0;
    }
}

void bl_rhs(double a, const double x[4], const double k[4], double acc[4]) {
  double g[4][4], dg[4][4][4];
  bl_metric_and_derivs(a, x, g, dg);
  christoffel_acc(g, dg, k, acc);
}

void deriv_bl(double a, const double y[8], double dy[8]) {
  for (int m = 0; m < 4; ++m) dy[m] = y[4 + m];
  bl_rhs(a, y, y + 4, dy + 4);
}

// E = -k_t, L_z = k_phi, mu^2 = -g k k and Carter's constant
// Q = k_theta^2 + cos^2(theta) [a^2 (mu^2 - E^2) + L_z^2 / sin^2(theta)].  On the
// axis (sin(theta) = 0), where the chart is singular, L_z = 0 and the last
// term is taken as its limit 0.
void bl_constants(double a, const double x[4], const double k[4], double out[4]) {
  double g[4][4];
  bl_metric(a, x[1], x[2], g);
  double kl[4], mu2 = 0.0;
  for (int m = 0; m < 4; ++m) {
    kl[m] = 0.0;
    for (int n = 0; n < 4; ++n) kl[m] += g[m][n] * k[n];
    mu2 -= kl[m] * k[m];
  }
  double E = -kl[0], Lz = kl[3];
  double c = std::cos(x[2]), s = std::sin(x[2]);
  out[0] = E;
  out[1] = Lz;
  out[2] = kl[2] * kl[2] + c * c * (a * a * (mu2 - E * E) + (Lz == 0.0 ? 0.0 : Lz * Lz / (s * s)));
  out[3] = mu2;
}

// Ingoing Kerr-Schild coordinates from Boyer-Lindquist ones (|a| < 1): with
// r_pm = 1 +- sqrt(1 - a^2), the time and azimuth shifts
//   F(r) = int 2 r / Delta dr = 2 (r_+ ln|r - r_+| - r_- ln|r - r_-|) / (r_+ - r_-),
//   G(r) = int a / Delta dr   = a ln|(r - r_+) / (r - r_-)| / (r_+ - r_-),
// give T = t + F(r), psi = phi + G(r) and the Cartesian form
//   x + i y = (r + i a) sin(theta) e^{i psi},  z = r cos(theta),
// which satisfies eq:CKSr and carries the metric def:CKS (pinned by pulling
// def:CKS back through this map).
template <class S>
S shift_F(double a, const S& r) {
  double rp = 1.0 + std::sqrt(1.0 - a * a), rm = 1.0 - std::sqrt(1.0 - a * a);
  return (2.0 / (rp - rm)) * (rp * log(fabs(r - rp)) - rm * log(fabs(r - rm)));
}
template <class S>
S shift_G(double a, const S& r) {
  double rp = 1.0 + std::sqrt(1.0 - a * a), rm = 1.0 - std::sqrt(1.0 - a * a);
  return (a / (rp - rm)) * log(fabs((r - rp) / (r - rm)));
}
template <class S>
void bl_to_ks(double a, const S& r, const S& th, const S& ph, S& F, S& X, S& Y, S& Z) {
  F = shift_F(a, r);
  S psi = ph + shift_G(a, r);
  S sn = sin(th);
  X = sn * (r * cos(psi) - a * sin(psi));
  Y = sn * (r * sin(psi) + a * cos(psi));
  Z = r * cos(th);
}

// Kerr-Schild point xks and Jacobian J[mu][nu] = d x_KS^mu / d x_BL^nu at the
// Boyer-Lindquist point xbl.
void bl_to_ks_jacobian(double a, const double xbl[4], double xks[4], double J[4][4]) {
  Dual R = seed(xbl[1], 0), TH = seed(xbl[2], 1), PH = seed(xbl[3], 2);
  Dual F, X, Y, Z;
  bl_to_ks(a, R, TH, PH, F, X, Y, Z);
  xks[0] = xbl[0] + F.v;
  xks[1] = X.v;
  xks[2] = Y.v;
  xks[3] = Z.v;
  const Dual* row[4] = {&F, &X, &Y, &Z};
  for (int m = 0; m < 4; ++m) {
    J[m][0] = (m == 0) ? 1.0 : 0.0;
    for (int j = 0; j < 3; ++j) J[m][j + 1] = row[m]->d[j];
  }
}

// Kerr-Schild state -> Boyer-Lindquist state: r from eq:CKSr,
// cos(theta) = z / r, psi = atan2(y, x) - atan2(a, r), phi = psi - G(r),
// t = T - F(r); the momentum is J^{-1} k with J of the map above.
bool ks_to_bl_state(double a, const double yk[8], double yb[8]) {
  double r = ks_radius(a, yk[1], yk[2], yk[3]);
  double ct = std::max(-1.0, std::min(1.0, yk[3] / r));
  double th = std::acos(ct);
  double ph = std::atan2(yk[2], yk[1]) - std::atan2(a, r) - shift_G(a, r);
  yb[0] = yk[0] - shift_F(a, r);
  yb[1] = r;
  yb[2] = th;
  yb[3] = ph;
  double xks[4], J[4][4], Ji[4][4];
  bl_to_ks_jacobian(a, yb, xks, J);
  if (!invert4(J, Ji)) return false;
  for (int m = 0; m < 4; ++m) {
    yb[4 + m] = 0.0;
    for (int n = 0; n < 4; ++n) yb[4 + m] += Ji[m][n] * yk[4 + n];
  }
  return true;
}

double chart_radius(int chart, double a, const double y[8]) { return chart == CHART_BL ? y[1] : radius(a, y); }
double chart_rdot(int chart, double a, const double y[8]) { return chart == CHART_BL ? y[5] : rdot(a, y); }

// Up to nsteps classic RK4 steps of h = h_coeff * r (r at the step's start),
// no error control.  After each step: a NaN component ends the geodesic as
// failed, r < r_stop as captured, r > r_escape with dr/dlambda > 0 as escaped.
// Only active geodesics are stepped; `steps` counts the steps taken.
void rk4_fixed(int chart, double a, double hc, double r_stop, double r_esc, int32_t nsteps, double y[8],
               int32_t& st, int32_t& steps) {
  if (st != ST_ACTIVE) return;
  auto F = [&](const double* yy, double* dy) {
    if (chart == CHART_BL)
      deriv_bl(a, yy, dy);
    else
      deriv(a, yy, dy);
  };
  for (int32_t s = 0; s < nsteps; ++s) {
    double h = hc * chart_radius(chart, a, y);
    double k1[8], k2[8], k3[8], k4[8], t[8];
    F(y, k1);
    for (int c = 0; c < 8; ++c) t[c] = y[c] + 0.5 * h * k1[c];
    F(t, k2);
    for (int c = 0; c < 8; ++c) t[c] = y[c] + 0.5 * h * k2[c];
    F(t, k3);
    for (int c = 0; c < 8; ++c) t[c] = y[c] + h * k3[c];
    F(t, k4);
    for (int c = 0; c < 8; ++c) y[c] += h / 6.0 * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
    ++steps;
    if (any_nan(y)) {
      st = ST_FAILED;
      return;
    }
    double r = chart_radius(chart, a, y);
    if (r < r_stop) {
      st = ST_CAPTURED;
      return;
    }
    if (r > r_esc && chart_rdot(chart, a, y) > 0.0) {
      st = ST_ESCAPED;
      return;
    }
  }
}

}  // namespace

extern "C" {

void oracle_bl_metric(double a, const double x[4], double g[16], double dg[64]) {
  double gg[4][4], d[4][4][4];
  bl_metric_and_derivs(a, x, gg, d);
  for (int m = 0; m < 4; ++m)
    for (int q = 0; q < 4; ++q) {
      g[4 * m + q] = gg[m][q];
      for (int c = 0; c < 4; ++c) dg[16 * c + 4 * m + q] = d[c][m][q];
    }
}

void oracle_bl_rhs(double a, const double x[4], const double k[4], double acc[4]) { bl_rhs(a, x, k, acc); }

void oracle_bl_constants(double a, const double x[4], const double k[4], double out[4]) {
  bl_constants(a, x, k, out);
}

void oracle_bl_to_ks(double a, const double xbl[4], double xks[4], double jac[16]) {
  double J[4][4];
  bl_to_ks_jacobian(a, xbl, xks, J);
  for (int m = 0; m < 4; ++m)
    for (int n = 0; n < 4; ++n) jac[4 * m + n] = J[m][n];
}

// y_ks, y_bl: [n][8].  Returns the number of states whose Jacobian was singular
// (their output is NaN).
int64_t oracle_ks_to_bl(double a, int64_t n, const double* y_ks, double* y_bl) {
  int64_t bad = 0;
  for (int64_t i = 0; i < n; ++i)
    if (!ks_to_bl_state(a, y_ks + 8 * i, y_bl + 8 * i)) {
      for (int c = 0; c < 8; ++c) y_bl[8 * i + c] = NAN;
      ++bad;
    }
  return bad;
}

// chart 0 = Kerr-Schild (Cartesian), 1 = Boyer-Lindquist; y [n][8] in place.
void oracle_rk4_fixed(int32_t chart, double a, double h_coeff, double r_stop, double r_escape, int32_t nsteps,
                      int64_t n, double* y, int32_t* status, int32_t* steps, int32_t nthreads) {
  parallel_chunks(n, nthreads, [&](int64_t i) {
    rk4_fixed(chart, a, h_coeff, r_stop, r_escape, nsteps, y + 8 * i, status[i], steps[i]);
  });
}

}  // extern "C"
