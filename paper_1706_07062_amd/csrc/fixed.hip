// fixed.hip -- fixed-step RK4 in Cartesian Kerr-Schild or Boyer-Lindquist
// coordinates, state stored structure-of-arrays or array-of-structures: the
// workload of the chart and data-layout comparison of Sec. 4 (tab:elapse).
//
// One geodesic per lane, no refill and no scheduling: every lane loads its 8
// components once, takes up to nsteps steps in registers and stores once, so
// the kernel is bound by the right-hand side's arithmetic and the layout only
// changes the single load and store.  The step is the library's RK4 (Nystrom
// form of the classic tableau) on the chart's right-hand side; the
// acceleration at the end of a step is the first stage of the next one and
// also gives r and dr/dlambda for the termination tests.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.hpp"
#include "steppers.hpp"

using namespace khi;
using namespace kh;

namespace {

constexpr int kFixedBlock = 256;

template <int LAYOUT>
__device__ __forceinline__ int64_t comp_index(int64_t i, int c, int64_t n) {
  if constexpr (LAYOUT == KH_AOS)
    return 8 * i + c;
  else
    return c * n + i;
}

template <typename T>
__device__ __forceinline__ bool finite8(const T x[4], const T k[4]) {
  bool ok = true;
#pragma unroll
  for (int c = 0; c < 4; ++c) ok = ok && !__builtin_isnan(x[c]) && !__builtin_isnan(k[c]);
  return ok;
}

template <int FORM, int LAYOUT, typename T>
__global__ __launch_bounds__(kFixedBlock) void k_rk4_fixed(T a, T h_coeff, T r_stop, T r_escape, int32_t nsteps,
                                                           T* __restrict__ y, int32_t* __restrict__ status,
                                                           int32_t* __restrict__ steps, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kFixedBlock + threadIdx.x;
  if (i >= n || status[i] != KH_ACTIVE) return;
  T x[4], k[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    x[c] = y[comp_index<LAYOUT>(i, c, n)];
    k[c] = y[comp_index<LAYOUT>(i, 4 + c, n)];
  }
  Accel<T> acc = chart_rhs<FORM, T>(a, x, k);
  int32_t st = KH_ACTIVE, taken = 0;
  while (taken < nsteps) {
    T xn[4], kn[4];
    rk4_step<FORM, T, T>(a, x, k, acc.a, h_coeff * acc.r, xn, kn);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      x[c] = xn[c];
      k[c] = kn[c];
    }
    ++taken;
    acc = chart_rhs<FORM, T>(a, x, k);
    if (!finite8(x, k)) {
      st = KH_FAILED;
      break;
    }
    if (acc.r < r_stop) {
      st = KH_CAPTURED;
      break;
    }
    if (acc.r > r_escape && acc.rdot > T(0)) {
      st = KH_ESCAPED;
      break;
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    y[comp_index<LAYOUT>(i, c, n)] = x[c];
    y[comp_index<LAYOUT>(i, 4 + c, n)] = k[c];
  }
  status[i] = st;
  steps[i] += taken;
}

// Ingoing Kerr-Schild time and azimuth shifts (|a| < 1):
// F(r) = int 2r/Delta dr, G(r) = int a/Delta dr, Delta = (r - r_+)(r - r_-).
__device__ inline double shift_t(double a, double r) {
  const double q = sqrt(1.0 - a * a), rp = 1.0 + q, rm = 1.0 - q;
  return (rp * log(fabs(r - rp)) - rm * log(fabs(r - rm))) / q;
}
__device__ inline double shift_phi(double a, double r) {
  const double q = sqrt(1.0 - a * a), rp = 1.0 + q, rm = 1.0 - q;
  return 0.5 * a / q * log(fabs((r - rp) / (r - rm)));
}

// Kerr-Schild state (T, x, y, z, k) -> Boyer-Lindquist state.  The inverse
// Jacobian rows, from r^4 - (R^2 - a^2) r^2 - a^2 z^2 = 0, cos(theta) = z/r,
// psi = atan2(y, x) - atan2(a, r), phi = psi - G(r), t = T - F(r):
//   dr     = r (r^2 (x dx + y dy) + S z dz) / D,     S = r^2 + a^2, D = r^4 + a^2 z^2,
//   dtheta = (z dr / r - dz) / (r sin(theta)),        sin(theta) = rho / sqrt(S),
//   dphi   = (x dy - y dx) / rho^2 + a dr / S - a dr / Delta,   rho^2 = x^2 + y^2,
//   dt     = dT - 2 r dr / Delta.
__device__ inline void ks_to_bl(double a, const double s[8], double b[8]) {
  const double X = s[1], Y = s[2], Z = s[3];
  const double R2 = X * X + Y * Y + Z * Z, w = R2 - a * a;
  const double q = sqrt(w * w + 4.0 * a * a * Z * Z);
  const double r2 = (w >= 0.0) ? 0.5 * (w + q) : 2.0 * a * a * Z * Z / (q - w);
  const double r = sqrt(r2);
  const double S = r2 + a * a, D = r2 * r2 + a * a * Z * Z;
  const double rho2 = X * X + Y * Y, rho = sqrt(rho2);
  const double sth = rho / sqrt(S);
  const double Delta = r2 - 2.0 * r + a * a;
  b[0] = s[0] - shift_t(a, r);
  b[1] = r;
  b[2] = atan2(sth, Z / r);
  b[3] = atan2(Y, X) - atan2(a, r) - shift_phi(a, r);
  const double kT = s[4], kx = s[5], ky = s[6], kz = s[7];
  const double dr = r * (r2 * (X * kx + Y * ky) + S * Z * kz) / D;
  b[5] = dr;
  b[6] = (Z * dr / r - kz) / (r * sth);
  b[7] = (X * ky - Y * kx) / rho2 + a * dr / S - a * dr / Delta;
  b[4] = kT - 2.0 * r * dr / Delta;
}

template <int FORM, int LAYOUT, typename T>
__global__ __launch_bounds__(kFixedBlock) void k_pack_fixed(double a, const double* __restrict__ s,
                                                            T* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kFixedBlock + threadIdx.x;
  if (i >= n) return;
  double v[8], out[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) v[c] = s[c * n + i];
  if constexpr (FORM == KH_RHS_BL) {
    ks_to_bl(a, v, out);
  } else {
#pragma unroll
    for (int c = 0; c < 8; ++c) out[c] = v[c];
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) y[comp_index<LAYOUT>(i, c, n)] = static_cast<T>(out[c]);
}

kh_status check_fixed(kh_ctx* ctx, const kh_fixed_params* p, int64_t n, const void* y) {
  if (!p) return fail(ctx, KH_EINVAL, "params must not be NULL");
  if (p->rhs_form != KH_RHS_FACTORED && p->rhs_form != KH_RHS_PAPER && p->rhs_form != KH_RHS_BL)
    return fail(ctx, KH_EINVAL, "rhs_form must be KH_RHS_FACTORED, KH_RHS_PAPER or KH_RHS_BL");
  if (p->layout != KH_SOA && p->layout != KH_AOS) return fail(ctx, KH_EINVAL, "layout must be KH_SOA or KH_AOS");
  if (p->precision != KH_P64 && p->precision != KH_P32)
    return fail(ctx, KH_EINVAL, "precision must be KH_P64 or KH_P32");
  if (!(std::fabs(p->spin) < 1.0)) return fail(ctx, KH_EINVAL, "spin must satisfy |a| < 1");
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(ctx, KH_EINVAL, "n must be in [0, 2^31)");
  const size_t al = p->precision == KH_P64 ? 8 : 4;
  if (n > 0 && (!y || !aligned(y, al) || !device_ok(y)))
    return fail(ctx, KH_EINVAL, "y must be aligned device memory");
  return KH_OK;
}

template <int FORM, int LAYOUT>
void launch_fixed(const kh_fixed_params* p, void* y, int32_t* status, int32_t* steps, int64_t n, dim3 grid,
                  hipStream_t strm) {
  if (p->precision == KH_P64)
    hipLaunchKernelGGL((k_rk4_fixed<FORM, LAYOUT, double>), grid, dim3(kFixedBlock), 0, strm, p->spin, p->h_coeff,
                       p->r_stop, p->r_escape, p->nsteps, static_cast<double*>(y), status, steps, n);
  else
    hipLaunchKernelGGL((k_rk4_fixed<FORM, LAYOUT, float>), grid, dim3(kFixedBlock), 0, strm, (float)p->spin,
                       (float)p->h_coeff, (float)p->r_stop, (float)p->r_escape, p->nsteps, static_cast<float*>(y),
                       status, steps, n);
}

template <int FORM, int LAYOUT>
void launch_pack(const kh_fixed_params* p, const double* s, void* y, int64_t n, dim3 grid, hipStream_t strm) {
  if (p->precision == KH_P64)
    hipLaunchKernelGGL((k_pack_fixed<FORM, LAYOUT, double>), grid, dim3(kFixedBlock), 0, strm, p->spin, s,
                       static_cast<double*>(y), n);
  else
    hipLaunchKernelGGL((k_pack_fixed<FORM, LAYOUT, float>), grid, dim3(kFixedBlock), 0, strm, p->spin, s,
                       static_cast<float*>(y), n);
}

// Dispatch on (rhs_form, layout) to a template taking <FORM, LAYOUT>.
template <template <int, int> class L, typename... A>
void by_form_layout(const kh_fixed_params* p, A... args) {
  const int f = p->rhs_form, l = p->layout;
  if (f == KH_RHS_FACTORED && l == KH_SOA) L<KH_RHS_FACTORED, KH_SOA>::run(p, args...);
  if (f == KH_RHS_FACTORED && l == KH_AOS) L<KH_RHS_FACTORED, KH_AOS>::run(p, args...);
  if (f == KH_RHS_PAPER && l == KH_SOA) L<KH_RHS_PAPER, KH_SOA>::run(p, args...);
  if (f == KH_RHS_PAPER && l == KH_AOS) L<KH_RHS_PAPER, KH_AOS>::run(p, args...);
  if (f == KH_RHS_BL && l == KH_SOA) L<KH_RHS_BL, KH_SOA>::run(p, args...);
  if (f == KH_RHS_BL && l == KH_AOS) L<KH_RHS_BL, KH_AOS>::run(p, args...);
}
template <int F, int L>
struct FixedL {
  static void run(const kh_fixed_params* p, void* y, int32_t* st, int32_t* sp, int64_t n, dim3 g, hipStream_t s) {
    launch_fixed<F, L>(p, y, st, sp, n, g, s);
  }
};
template <int F, int L>
struct PackL {
  static void run(const kh_fixed_params* p, const double* src, void* y, int64_t n, dim3 g, hipStream_t s) {
    launch_pack<F, L>(p, src, y, n, g, s);
  }
};

}  // namespace

extern "C" {

kh_status kh_rk4_fixed(kh_ctx* ctx, const kh_fixed_params* p, void* y, int32_t* status, int32_t* steps, int64_t n,
                       void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = capturing(stream);
  kh_status s = check_fixed(ctx, p, n, y);
  if (s != KH_OK) return s;
  if (p->nsteps < 0) return fail(ctx, KH_EINVAL, "nsteps must be >= 0");
  if (!(p->h_coeff > 0.0) || !std::isfinite(p->h_coeff)) return fail(ctx, KH_EINVAL, "h_coeff must be > 0");
  if (!std::isfinite(p->r_stop) || !std::isfinite(p->r_escape))
    return fail(ctx, KH_EINVAL, "r_stop and r_escape must be finite");
  if (p->precision == KH_P32 && std::fabs(p->r_escape) > 1e38)
    return fail(ctx, KH_EINVAL, "r_escape out of FP32 range");
  if (n == 0) return KH_OK;
  if (!status || !steps || !aligned(status, 4) || !aligned(steps, 4) || !device_ok(status) || !device_ok(steps))
    return fail(ctx, KH_EINVAL, "status and steps must be device int32 arrays");
  if ((s = set_device(ctx)) != KH_OK) return s;
  const dim3 grid((unsigned)((n + kFixedBlock - 1) / kFixedBlock));
  by_form_layout<FixedL>(p, y, status, steps, n, grid, (hipStream_t)stream);
  KH_HIP(ctx, hipGetLastError());
  return KH_OK;
}

kh_status kh_pack_fixed(kh_ctx* ctx, const kh_fixed_params* p, const double* s_ks, void* y, int64_t n,
                        void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = capturing(stream);
  kh_status s = check_fixed(ctx, p, n, y);
  if (s != KH_OK) return s;
  if (n == 0) return KH_OK;
  if (!s_ks || !aligned(s_ks, 8) || !device_ok(s_ks)) return fail(ctx, KH_EINVAL, "s must be device doubles");
  if ((s = set_device(ctx)) != KH_OK) return s;
  const dim3 grid((unsigned)((n + kFixedBlock - 1) / kFixedBlock));
  by_form_layout<PackL>(p, s_ks, y, n, grid, (hipStream_t)stream);
  KH_HIP(ctx, hipGetLastError());
  return KH_OK;
}

}  // extern "C"
