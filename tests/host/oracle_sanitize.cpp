// Driver for the oracle built with AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_oracle_sanitizers.py): runs every
// integration path of oracle/kerr_oracle.cpp on small inputs -- camera rays
// with crossing records and constants (two threads), RK4, coordinate time with
// dense output and t_end landing, a recorded trajectory, a controller trace,
// the Boyer-Lindquist map and fixed-step charts -- and checks that each call
// succeeds and ends every geodesic.  Exit status 0 on success; the sanitizers
// abort the process on any finding.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
typedef struct {
  int32_t method;
  int32_t k_cross;
  double h_coeff;
  double rtol, atol;
  double hmax_coeff;
  double r_h_factor;
  double r_escape;
  double t_end;
  int64_t max_steps;
} oracle_params;

int oracle_camera_rays(double a_phys, double r_obs, double incl, double amin, double amax, double bmin, double bmax,
                       int32_t W, int32_t H, const int64_t* pix, int64_t n, double perturb, double* s, double* spin,
                       int32_t* kind, int32_t* status);
int oracle_timelike(const double* a, const double* x3, const double* v3, int64_t n, double* s, double* spin,
                    int32_t* kind, int32_t* status);
int oracle_integrate(const oracle_params* p, int64_t n, double* s, const double* spin, const int32_t* kind,
                     double* lam, double* phi, int32_t* status, int32_t* n_acc, int32_t* n_rej, double* cross,
                     int32_t* n_cross, double* c0, double* c1, int32_t nthreads);
int oracle_integrate_out(const oracle_params* p, int64_t n, double* s, const double* spin, const int32_t* kind,
                         double* lam, double* phi, int32_t* status, int32_t* n_acc, int32_t* n_rej, double* cross,
                         int32_t* n_cross, double* c0, double* c1, int32_t n_out, const double* t_out,
                         double* s_out, int32_t nthreads);
int64_t oracle_trajectory(const oracle_params* p, double spin_chart, const double y0[8], int64_t max_out,
                          double* out);
int64_t oracle_controller_trace(const oracle_params* p, double spin_phys, int32_t kind, const double y0[8],
                                int64_t max_rec, double* out, int32_t* res);
int64_t oracle_ks_to_bl(double a, int64_t n, const double* y_ks, double* y_bl);
void oracle_rk4_fixed(int32_t chart, double a, double h_coeff, double r_stop, double r_escape, int32_t nsteps,
                      int64_t n, double* y, int32_t* status, int32_t* steps, int32_t nthreads);
}

namespace {

int failures = 0;

void check(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "check failed: %s\n", what);
    ++failures;
  }
}

struct Set {
  int64_t n;
  std::vector<double> s, spin, lam, phi, cross, c0, c1;
  std::vector<int32_t> kind, status, n_acc, n_rej, n_cross;
  Set(int64_t n_, int k) : n(n_), s(8 * n_), spin(n_), lam(n_), phi(n_), cross(n_ * k * 3 + 1), c0(4 * n_),
                           c1(4 * n_), kind(n_), status(n_), n_acc(n_), n_rej(n_), n_cross(n_) {}
  int run(const oracle_params& p, int threads) {
    return oracle_integrate(&p, n, s.data(), spin.data(), kind.data(), lam.data(), phi.data(), status.data(),
                            n_acc.data(), n_rej.data(), cross.data(), n_cross.data(), c0.data(), c1.data(), threads);
  }
  bool all_done() const {
    for (int32_t v : status)
      if (v == 0) return false;
    return true;
  }
};

oracle_params params(int method, int k_cross) {
  oracle_params p{};
  p.method = method;
  p.k_cross = k_cross;
  p.h_coeff = 0.01;
  p.rtol = 1e-8;
  p.atol = 1e-8;
  p.hmax_coeff = 0.1;
  p.r_h_factor = 1.01;
  p.r_escape = 1000.0;
  p.t_end = 0.0;
  p.max_steps = 1000000;
  return p;
}

}  // namespace

int main() {
  // camera rays at a = 0.99, 60 deg, DOPRI5 with four crossing slots, two threads
  {
    const int W = 12, H = 10;
    Set g(W * H, 4);
    check(oracle_camera_rays(0.99, 1000.0, 1.0471975511965976, -8, 8, -8, 8, W, H, nullptr, g.n, 0.0, g.s.data(),
                             g.spin.data(), g.kind.data(), g.status.data()) == 0, "camera rays");
    check(g.run(params(1, 4), 2) == 0 && g.all_done(), "DOPRI5 image");
    // the same rays by classic RK4
    Set r(W * H, 0);
    oracle_camera_rays(0.99, 1000.0, 1.0471975511965976, -8, 8, -8, 8, W, H, nullptr, r.n, 1e-12, r.s.data(),
                       r.spin.data(), r.kind.data(), r.status.data());
    check(r.run(params(0, 0), 1) == 0 && r.all_done(), "RK4 image");
    // Boyer-Lindquist map of the initial states and fixed-step charts
    std::vector<double> yks(8 * r.n), ybl(8 * r.n);
    oracle_camera_rays(0.99, 1000.0, 1.0471975511965976, -8, 8, -8, 8, W, H, nullptr, r.n, 0.0, r.s.data(),
                       r.spin.data(), r.kind.data(), r.status.data());
    for (int64_t i = 0; i < r.n; ++i)
      for (int c = 0; c < 8; ++c) yks[8 * i + c] = r.s[c * r.n + i];
    check(oracle_ks_to_bl(-0.99, r.n, yks.data(), ybl.data()) == 0, "KS -> BL");
    std::vector<int32_t> st(r.n), steps(r.n);
    oracle_rk4_fixed(0, -0.99, 1.0 / 64, 2.0, 1000.0, 300, r.n, yks.data(), st.data(), steps.data(), 2);
    oracle_rk4_fixed(1, -0.99, 1.0 / 64, 2.0, 1000.0, 300, r.n, ybl.data(), st.data(), steps.data(), 2);
    // one recorded trajectory and one controller trace
    double y0[8];
    for (int c = 0; c < 8; ++c) y0[c] = g.s[c * g.n];
    oracle_camera_rays(0.99, 1000.0, 1.0471975511965976, -8, 8, -8, 8, W, H, nullptr, 1, 0.0, y0, g.spin.data(),
                       g.kind.data(), g.status.data());
    std::vector<double> traj(4000 * 9);
    const oracle_params pd = params(1, 0);
    check(oracle_trajectory(&pd, -0.99, y0, 4000, traj.data()) > 0, "trajectory");
    std::vector<double> rec(4000 * 5);
    int32_t res[3];
    check(oracle_controller_trace(&pd, 0.99, 0, y0, 4000, rec.data(), res) > 0, "controller trace");
  }
  // time-like geodesics in coordinate time to t_end with dense output, and in
  // the affine parameter with t_end landing
  {
    const int64_t n = 16;
    std::vector<double> a(n), x3(3 * n), v3(3 * n);
    for (int64_t i = 0; i < n; ++i) {
      a[i] = 0.06 * i;
      const double r0 = 7.0 + 2.0 * i, rho = std::sqrt(r0 * r0 + a[i] * a[i]);
      const double om = 1.0 / (std::pow(r0, 1.5) + a[i]);
      x3[i] = rho;
      v3[n + i] = om * rho * std::cos(0.2);
      v3[2 * n + i] = om * rho * std::sin(0.2);
    }
    for (int method : {1, 2}) {
      Set g(n, 0);
      check(oracle_timelike(a.data(), x3.data(), v3.data(), n, g.s.data(), g.spin.data(), g.kind.data(),
                            g.status.data()) == 0, "time-like init");
      oracle_params p = params(method, 0);
      p.r_escape = 1e4;
      p.t_end = 300.0;
      const double t_out[5] = {0.0, 50.0, 100.0, 250.0, 299.0};
      std::vector<double> s_out(n * 5 * 8, NAN);
      check(oracle_integrate_out(&p, n, g.s.data(), g.spin.data(), g.kind.data(), g.lam.data(), g.phi.data(),
                                 g.status.data(), g.n_acc.data(), g.n_rej.data(), nullptr, g.n_cross.data(),
                                 g.c0.data(), g.c1.data(), 5, t_out, s_out.data(), 2) == 0 && g.all_done(),
            "time-like integration with dense output");
    }
  }
  if (failures) return 1;
  std::printf("oracle under sanitizers: all paths ran\n");
  return 0;
}
