// kerrhip.hip -- MI355X (gfx950) kernels and the C ABI declared in include/kerrhip.h.
//
// One geodesic per lane.  The integrate kernel is persistent: every 64-lane
// wave takes ray ids from a global counter (one atomic per refill, lane
// offsets from mbcnt over the ballot of idle lanes), integrates them with
// register-resident Runge-Kutta stages, writes a ray back the moment it
// terminates and refills the freed lanes, so uneven step counts (tens to
// thousands of steps per ray) do not leave lanes idle until the tail.
// State is structure-of-arrays in HBM (coalesced loads of consecutive ray
// ids); the arithmetic is VALU (no contraction here, so no MFMA).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>

#include "kerrhip.h"
#include "kerrhip_mlp.h"
#include "ks_math.hpp"
#include "steppers.hpp"
#include "internal.hpp"

using namespace kh;
using namespace khi;

// The Python binding mirrors these layouts with ctypes.
static_assert(sizeof(kh_camera) == 64, "kh_camera layout");
static_assert(sizeof(kh_params) == 112, "kh_params layout");
static_assert(sizeof(kh_state) == 160, "kh_state layout");

namespace {

constexpr int kQueueSlots = 16;  // work-queue counters per context
// Status flags that live only between the integrate kernel and its finalize pass.
constexpr int kRetired = 0x100, kPhiPending = 0x200, kStatusMask = 0xff;
// Status of a geodesic that the first pass of the two-queue mixed policy
// paused after max_steps; the second pass loads only KH_ACTIVE and
// KH_MAX_STEPS geodesics, so these wait out that pass and its finalize pass
// turns them into KH_MAX_STEPS.  No call returns with it.
constexpr int kPaused = 6;
// Kernel-template precision of the first pass of the two-queue mixed policy
// (FP64 state and error norm, FP32 right-hand sides and stage sums for every
// geodesic; one inside r_fp64 is written back for the FP64 pass).  Not a
// kh_params.precision value.
constexpr int kPSplit = 3;
constexpr int kParts = 8;        // ray-range partitions = XCDs of an MI355X

__device__ inline double hscale(int kind, double r) { return kind == KH_TIMELIKE ? r * ksqrt(r) : r; }

__device__ inline double r_horizon(double a) { return 1.0 + ksqrt(1.0 - a * a); }

// q^{-1/10} for the step-size controller, where q = err^2 is the mean square
// error norm, so the result is err^{-1/5}.  The controller clamps the factor
// 0.9 err^{-1/5} to [0.2, 5], which only needs q in [3.5e-8, 3.5e6]; q is held
// to [1e-10, 1e8] (a NaN becomes 1e-10: callers test for it first), which
// keeps every clamp decision.  An FP32 estimate from the hardware log2 / exp2
// (relative error below 5e-7 on that range) is refined by one Newton step on
// y^{-10} = q, y <- y + y (1 - q y^10) / 10, which takes the relative error e
// to about 5.5 e^2 < 2e-12: the step factor is then within 2e-12 of the exact
// power, far below anything that moves a step (the accept decision uses q
// itself), in 10 instructions instead of the ~200 of a general FP64 pow.
__device__ inline double kpow_m1_10(double q) {
  q = q > 1e-10 ? q : 1e-10;
  q = q < 1e8 ? q : 1e8;
  const double y = (double)__builtin_amdgcn_exp2f(-0.1f * __builtin_amdgcn_logf((float)q));
  const double y2 = y * y, y5 = y2 * y2 * y;
  const double t = fma(-q, y5 * y5, 1.0);
  return fma(0.1 * y, t, y);
}
__device__ inline float kpow_m1_10(float q) {
  q = q > 1e-10f ? q : 1e-10f;
  q = q < 1e8f ? q : 1e8f;
  return __builtin_amdgcn_exp2f(-0.1f * __builtin_amdgcn_logf(q));
}

// Growth / shrink factors of the step-size controller from err2 = err^2 and
// raw = 0.9 err^{-1/5}, computed once per attempt before the accept / reject
// branch.
template <typename T>
__device__ inline T grow_factor(T err2, T raw, bool after_reject) {
  T fac;
  if (err2 == T(0))
    fac = T(5);
  else {
    fac = raw < T(0.2) ? T(0.2) : raw;
    fac = fac > T(5) ? T(5) : fac;
  }
  if (after_reject && fac > T(1)) fac = T(1);
  return fac;
}
template <typename T>
__device__ inline T shrink_factor(T err2, T raw) {
  if (err2 != err2) return T(0.2);
  return raw < T(0.2) ? T(0.2) : raw;
}

// ---------------------------------------------------------------------------
// Work-queue helpers.
// ---------------------------------------------------------------------------
__global__ void k_reset_counters(unsigned long long* q, int n) {
  if (threadIdx.x < n) q[threadIdx.x] = 0ull;
}

// Work stealing over `parts` partitions of the ray range.  The range is cut
// into chunks of kChunk consecutive ids dealt round-robin to the partitions
// (partition p owns chunks p, p + parts, ...), so every partition advances
// through the images at the same pace and the queue still ends on the last
// rows of the images (the cheap edge rays) instead of several partitions ending
// on expensive rays.  A wave starts on the partition of its XCD (workgroups
// are dispatched round-robin over the XCDs: blockIdx.x % parts), so a refill's
// neighbouring ids stay in one L2, and moves on to the next partition when its
// own is drained.  One atomic per refill; lane offsets from mbcnt over the
// ballot of idle lanes.  Wave-uniform call; `cursor` counts partitions this
// wave has seen drained (== parts: all work handed out).  Returns the lane's
// new id or -1.
constexpr int64_t kChunk = 8192;

__device__ inline int64_t wave_grab(unsigned long long idle, unsigned long long* qctr, int64_t n, int home,
                                    int parts, int& cursor) {
  const int cnt = __popcll(idle);
  const int leader = __ffsll((long long)idle) - 1;
  const int lane = __lane_id();
  const unsigned rank =
      __builtin_amdgcn_mbcnt_hi((unsigned)(idle >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)idle, 0u));
  const int64_t n_chunks = (n + kChunk - 1) / kChunk;
  const int64_t tail = n - (n_chunks - 1) * kChunk;  // length of the last chunk
  while (cursor < parts) {
    const int p = (home + cursor) % parts;
    const int64_t my_chunks = p < n_chunks ? (n_chunks - 1 - p) / parts + 1 : 0;
    const bool owns_last = my_chunks > 0 && (n_chunks - 1) % parts == p;
    const unsigned long long size = (unsigned long long)(my_chunks * kChunk - (owns_last ? kChunk - tail : 0));
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(qctr + p, (unsigned long long)cnt);
    base = __shfl(base, leader);
    if (base < size) {
      if (base + (unsigned long long)cnt >= size) ++cursor;  // this grab drains the partition
      if (!((idle >> lane) & 1ull)) return -1;
      const unsigned long long off = base + rank;
      if (off >= size) return -1;
      return ((int64_t)(off / kChunk) * parts + p) * kChunk + (int64_t)(off % kChunk);
    }
    ++cursor;
  }
  return -1;
}

// Queue position -> ray id: through the per-geodesic schedule or the tile
// order when there is one.  Every index is checked, so a malformed order can
// skip rays but never read or write outside the state.
__device__ inline int64_t queue_id(int64_t pos, const KState& S, int64_t n_tiles) {
  if (pos < 0) return pos;
  if (S.perm) {
    const int64_t id = pos < S.n ? (int64_t)S.perm[pos] : -1;
    return (id >= 0 && id < S.n) ? id : -1;
  }
  if (!S.order) return pos;
  const int64_t t = pos >> 6;
  if (t >= n_tiles) return -1;
  const int64_t tile = S.order[t];
  const int64_t id = tile * 64 + (pos & 63);
  return (tile >= 0 && tile < n_tiles && id < S.n) ? id : -1;
}

// ---------------------------------------------------------------------------
// Equatorial crossings: a lane that sees a sign change of z only queues the
// two nodes of the step in its wave's LDS queue; the wave refines queued
// crossings together, one per lane, once the queue is nearly full and when it
// exits.  This keeps the root find, the two arctangents and the redshift out
// of the divergent per-lane path (a crossing in any lane would otherwise stall
// the other 63).  Field-major layout: field f of record j at f * kQCap + j.
// ---------------------------------------------------------------------------
constexpr int kQCap = 96;
enum { QX0, QY0, QZ0, QKX0, QKY0, QKZ0, QX1, QY1, QZ1, QK01, QKX1, QKY1, QKZ1, QH, QAC, QWIND, QTAG, kQFields };

__device__ inline void refine_crossing(const double* q, int j, const KState& S) {
  const double x0 = q[QX0 * kQCap + j], y0 = q[QY0 * kQCap + j], z0 = q[QZ0 * kQCap + j];
  const double x1 = q[QX1 * kQCap + j], y1 = q[QY1 * kQCap + j], z1 = q[QZ1 * kQCap + j];
  const double h = q[QH * kQCap + j], ac = q[QAC * kQCap + j];
  const int64_t tag = (int64_t)q[QTAG * kQCap + j];  // (ray * 8 + slot) * 2 + kind
  const int kind = (int)(tag & 1);
  const int slot = (int)((tag >> 1) & 7);
  const int64_t ray = tag >> 4;
  const double phi0 = atan2(y0, x0) + (2.0 * M_PI) * q[QWIND * kQCap + j];
  const double th = hermite_zero(z0, q[QKZ0 * kQCap + j], z1, q[QKZ1 * kQCap + j], h);
  const double xc = herm(th, x0, q[QKX0 * kQCap + j], x1, q[QKX1 * kQCap + j], h);
  const double yc = herm(th, y0, q[QKY0 * kQCap + j], y1, q[QKY1 * kQCap + j], h);
  const double qq = xc * xc + yc * yc - ac * ac;
  const double rc = sqrt(qq > 0.0 ? qq : 0.0);
  const double phic = phi0 + atan2(x0 * yc - y0 * xc, x0 * xc + y0 * yc);
  const double xd[4] = {0.0, x1, y1, z1};
  const double kd[4] = {q[QK01 * kQCap + j], q[QKX1 * kQCap + j], q[QKY1 * kQCap + j], q[QKZ1 * kQCap + j]};
  const double xi = photon_xi(ac, xd, kd, kind == KH_NULL);
  const double g = redshift(rc, xi, kind == KH_NULL ? -ac : ac);
  double* out = S.cross + (ray * S.k_cross + slot) * 3;
  out[0] = rc;
  out[1] = phic;
  out[2] = g;
}

// Whole-wave call: refine records [0, count) of this wave's queue.
__device__ inline void flush_crossings(double* q, int* qcnt, int count, const KState& S) {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int lane = __lane_id();
  for (int b = 0; b < count; b += 64)
    if (b + lane < count) refine_crossing(q, b + lane, S);
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) *qcnt = 0;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Persistent integrate kernel.
// METHOD: KH_RK4 / KH_DOPRI5 / KH_DOPRI5_T (coordinate time).  PREC: KH_P64 / KH_P32 / KH_PMIXED / kPSplit.
// FORM: right-hand-side evaluation (KH_RHS_FACTORED / KH_RHS_PAPER).
// ---------------------------------------------------------------------------
// WPE: minimum waves per SIMD the register allocation must allow (1 = no limit).
// DENSE: dense output compiled in (separate variants, so the interpolation code
// adds no registers to the ordinary kernels).
template <int METHOD, int PREC, int FORM, int WPE, bool DENSE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE < 2 ? 2 : WPE)))
k_integrate(KParams P, KState S, unsigned long long* qctr) {
  using TS = typename std::conditional<PREC == KH_P32, float, double>::type;  // state / stages
  using TF = typename std::conditional<PREC == KH_P64, double, float>::type;  // fast right-hand side

  const int64_t n = S.n;
  int ray = -1;  // state.n < 2^31
  // per-wave crossing queue in dynamic LDS (present when crossings are recorded)
  extern __shared__ double kh_lds[];
  const int wave_in_block = threadIdx.x >> 6;
  double* cq = kh_lds + (size_t)wave_in_block * (kQFields * kQCap + 1);
  int* cq_count = reinterpret_cast<int*>(cq + kQFields * kQCap);
  if (P.k_cross > 0) {
    if (__lane_id() == 0) *cq_count = 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  const int parts = P.parts;
  const int home = blockIdx.x % parts;
  // with a tile order the queue runs over whole tiles (ids past n are skipped)
  const int64_t n_tiles = (n + 63) >> 6;
  const int64_t nq = (S.order && !S.perm) ? n_tiles * 64 : n;
  int cursor = 0;  // partitions this wave has seen drained (wave-uniform)
  bool fresh = false;

  // Coordinate-time integration: the state is (t, x^i) and (1, v^i), v = dx/dt;
  // k keeps the slot layout with k[0] = 1, a1[0] = 0.  E0 = -k_t of the entry
  // state restores k^mu = k^0 (1, v) at retirement.
  constexpr bool CT = METHOD == KH_DOPRI5_T;
  TS x[4], k[4], a1[4];
  TS r_cur = TS(0), rdot_cur = TS(0);
  TS a_c = TS(0);
  double h = 0.0, lam = 0.0, rcap = 0.0, E0 = 0.0;
  // dense output: next target index and time (infinite when none is left)
  int j_out = 0;
  double t_next = __builtin_inf();
  int kind = 0, nacc = 0, nrej = 0, ncross = 0, status = KH_ACTIVE;
  // Unwrapped azimuth = atan2(y, x) + 2 pi * wind: wind counts passages across
  // the negative x axis, so no arctangent is needed on ordinary steps.
  int wind = 0;
  int steps = 0, tries = 0;  // bounded by max_steps and max_tries (< 2^31)
  bool after_reject = false;

  // ---- retire: write the ray back and free the lane ----
  auto retire = [&]() {
    if (CT) {
      // k^0 = E0 / E(1, v): the energy of the entry state is kept exactly
      double xd[4], vd[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        xd[c] = (double)x[c];
        vd[c] = (double)k[c];
      }
      const double k0 = E0 / energy((double)a_c, xd, vd);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        S.s[c * n + ray] = xd[c];
        S.s[(4 + c) * n + ray] = k0 * vd[c];
      }
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        S.s[c * n + ray] = (double)x[c];
        S.s[(4 + c) * n + ray] = (double)k[c];
      }
    }
    S.h[ray] = h;
    S.lam[ray] = lam;
    // the finalize pass adds atan2(y, x) to the winding part and clears the
    // flags; without crossings the azimuth is not tracked and phi is left as is
    if (P.k_cross > 0) S.phi[ray] = (2.0 * M_PI) * wind;
    const int st_out = (PREC == kPSplit && status == KH_MAX_STEPS) ? kPaused : status;
    S.status[ray] = st_out | kRetired | (P.k_cross > 0 ? kPhiPending : 0);
    S.n_acc[ray] = nacc;
    S.n_rej[ray] = nrej;
    if (S.n_cross) S.n_cross[ray] = ncross;
    ray = -1;
  };

  while (true) {
    // ---- refine queued crossings with the whole wave (uniform point) ----
    if (P.k_cross > 0) {
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const int qc = *cq_count;
      if (qc > kQCap - 64) flush_crossings(cq, cq_count, qc, S);
    }
    // ---- refill idle lanes (wave-uniform decision) ----
    const unsigned long long idle = __ballot(ray < 0);
    if (cursor < parts && idle != 0ull && (__popcll(idle) >= P.refill_min || idle == ~0ull)) {
      const int64_t id = queue_id(wave_grab(idle, qctr, nq, home, parts, cursor), S, n_tiles);
      if (ray < 0 && id >= 0) {
        const int st = S.status[id];
        if (st == KH_ACTIVE || st == KH_MAX_STEPS) {
          ray = (int)id;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            x[c] = (TS)S.s[c * n + id];
            k[c] = (TS)S.s[(4 + c) * n + id];
          }
          kind = S.kind[id];
          const double a_phys = S.spin[id];
          a_c = (TS)(kind == KH_NULL ? -a_phys : a_phys);
          if (CT) {
            double xd[4], kd[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              xd[c] = S.s[c * n + id];
              kd[c] = S.s[(4 + c) * n + id];
            }
            E0 = energy(kind == KH_NULL ? -a_phys : a_phys, xd, kd);
            const double ik0 = 1.0 / kd[0];
            k[0] = TS(1);
#pragma unroll
            for (int c = 1; c < 4; ++c) k[c] = (TS)(kd[c] * ik0);
          }
          if (DENSE && S.n_out > 0) {
            // first target at or after the entry time; one equal to it takes the entry state
            const double te = S.s[id];
            int lo = 0, hi = S.n_out;
            while (lo < hi) {
              const int mid = (lo + hi) >> 1;
              if (S.t_out[mid] < te)
                lo = mid + 1;
              else
                hi = mid;
            }
            j_out = lo;
            if (j_out < S.n_out && S.t_out[j_out] == te) {
              double* o = S.s_out + ((int64_t)id * S.n_out + j_out) * 8;
#pragma unroll
              for (int c = 0; c < 8; ++c) o[c] = S.s[c * n + id];
              ++j_out;
            }
            t_next = j_out < S.n_out ? S.t_out[j_out] : __builtin_inf();
          }
          h = S.h[id];
          lam = S.lam[id];
          // phi = atan2(y, x) + 2 pi wind on entry; a coarse azimuth recovers wind
          if (P.k_cross > 0) wind = (int)rint((S.phi[id] - atan2_est((double)x[2], (double)x[1])) * (0.5 / M_PI));
          rcap = P.r_h_factor * r_horizon((double)a_c);
          nacc = S.n_acc[id];
          nrej = S.n_rej[id];
          ncross = S.n_cross ? S.n_cross[id] : 0;
          status = KH_ACTIVE;
          steps = 0;
          tries = 0;
          after_reject = false;
          fresh = true;
        }
      }
    }
    if (__ballot(ray >= 0) == 0ull) {
      if (cursor >= parts) break;
      continue;
    }
    // RK4 lanes without a ray skip the rest of this pass.  DOPRI5 keeps the
    // whole wave together: its attempt loop below decides when to leave by
    // ballots that must see every lane, idle ones included.
    if (METHOD == KH_RK4 && ray < 0) continue;

    // ---- first-stage acceleration of a freshly loaded ray (idle lanes have fresh = false) ----
    if (fresh || METHOD == KH_RK4) {
      const Accel<TS> ra = CT ? rhs_ct<FORM, TS>(a_c, x, k) : rhs<FORM, TS>(a_c, x, k);
#pragma unroll
      for (int c = 0; c < 4; ++c) a1[c] = ra.a[c];
      r_cur = ra.r;
      rdot_cur = ra.rdot;
      if (METHOD != KH_RK4 && fresh && !(h > 0.0)) {
        h = P.h_coeff * hscale(kind, (double)r_cur);
        const double hm = P.hmax_coeff * hscale(kind, (double)r_cur);
        h = h < hm ? h : hm;
      }
      fresh = false;
    }

    if (METHOD == KH_RK4) {
      // Termination of the previous step is decided here, with r from a1.
      if (steps > 0) {
        bool bad = false;
#pragma unroll
        for (int c = 0; c < 4; ++c) bad = bad || (x[c] != x[c]) || (k[c] != k[c]);
        if (bad)
          status = KH_FAILED;
        else if ((double)r_cur < rcap)
          status = KH_CAPTURED;
        else if ((double)r_cur > P.r_escape && rdot_cur > TS(0))
          status = KH_ESCAPED;
        else if (steps >= P.max_steps)
          status = KH_MAX_STEPS;
      }
      if (status == KH_ACTIVE) {
        const TS hs = (TS)(P.h_coeff) * r_cur;
        TS xn[4], kn[4];
        if (PREC == KH_PMIXED && __ballot(r_cur < (TS)P.r_fp64) == 0ull)
          rk4_step<FORM, TS, TF>(a_c, x, k, a1, hs, xn, kn);
        else
          rk4_step<FORM, TS, TS>(a_c, x, k, a1, hs, xn, kn);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          x[c] = xn[c];
          k[c] = kn[c];
        }
        lam += (double)hs;
        ++nacc;
        ++steps;
        h = (double)hs;
        continue;
      }
    } else {
      // Attempts until the wave needs service (refill, crossing flush):
      // one entry and one back-edge keep the ray state in fixed registers.
      // Every lane runs this loop (idle lanes skip the attempt), so the exit
      // ballots count all 64 lanes; each ray retires within max_tries
      // attempts, hence all lanes become idle and the loop ends.
      while (true) {
        // two-queue mixed policy, first pass: a geodesic inside r_fp64 is
        // written back as KH_ACTIVE for the FP64 pass, so every attempt of this
        // pass runs in FP32
        if (PREC == kPSplit && ray >= 0 && r_cur < (TS)P.r_fp64) retire();
        if (ray >= 0) {
          TS xn[4], kn[4], a7[4], r_new, rdot_new;
          // coordinate time: a step that would pass t_end is clipped onto it
          const bool landing = CT && P.t_end > 0.0 && (double)x[0] + h >= P.t_end;
          const double hd = landing ? P.t_end - (double)x[0] : h;
          const TS hs = (TS)hd;
          const TS rtol = (TS)P.rtol, atol = (TS)P.atol;
          TS err2;  // squared RMS error norm
          if (PREC == kPSplit || (PREC == KH_PMIXED && __ballot(r_cur < (TS)P.r_fp64) == 0ull))
            err2 = dp5_attempt<FORM, TS, TF, CT, TF>(a_c, x, k, a1, hs, rtol, atol, xn, kn, a7, r_new, rdot_new);
          else
            err2 = dp5_attempt<FORM, TS, TS, CT>(a_c, x, k, a1, hs, rtol, atol, xn, kn, a7, r_new, rdot_new);

          const TS raw = TS(0.9) * kpow_m1_10(err2);
          if (err2 <= TS(1)) {
            ++nacc;
            ++steps;
            bool bad = false;
    #pragma unroll
            for (int c = 0; c < 4; ++c) bad = bad || (xn[c] != xn[c]) || (kn[c] != kn[c]);
            const double lam_old = lam;
            if (CT) {
              if (landing) xn[0] = (TS)P.t_end;  // the clipped step ends on t_end exactly
            } else {
              lam += h;  // the affine parameter is not tracked in coordinate time
            }
            if (bad) {
              status = KH_FAILED;
            } else {
              if (P.k_cross > 0) {
                // Unwrapped azimuth; equatorial crossings are queued for the wave.
                const double x0 = x[1], y0 = x[2], z0 = x[3];
                const double x1 = xn[1], y1 = xn[2], z1 = xn[3];
                const int wind0 = wind;
                const double crs = x0 * y1 - y0 * x1;
                wind += (y0 >= 0.0 && y1 < 0.0 && crs > 0.0) - (y0 < 0.0 && y1 >= 0.0 && crs < 0.0);
                if ((z0 < 0.0 && z1 > 0.0) || (z0 > 0.0 && z1 < 0.0) || (z1 == 0.0 && z0 != 0.0)) {
                  if (ncross < S.k_cross && ncross < P.k_cross) {
                    const int j = atomicAdd(cq_count, 1);  // < kQCap: flushed before 64 more can arrive
                    cq[QX0 * kQCap + j] = x0;
                    cq[QY0 * kQCap + j] = y0;
                    cq[QZ0 * kQCap + j] = z0;
                    cq[QKX0 * kQCap + j] = (double)k[1];
                    cq[QKY0 * kQCap + j] = (double)k[2];
                    cq[QKZ0 * kQCap + j] = (double)k[3];
                    cq[QX1 * kQCap + j] = x1;
                    cq[QY1 * kQCap + j] = y1;
                    cq[QZ1 * kQCap + j] = z1;
                    cq[QK01 * kQCap + j] = (double)kn[0];
                    cq[QKX1 * kQCap + j] = (double)kn[1];
                    cq[QKY1 * kQCap + j] = (double)kn[2];
                    cq[QKZ1 * kQCap + j] = (double)kn[3];
                    cq[QH * kQCap + j] = hd;
                    cq[QAC * kQCap + j] = (double)a_c;
                    cq[QWIND * kQCap + j] = (double)wind0;
                    cq[QTAG * kQCap + j] = (double)((((int64_t)ray * 8 + ncross) << 1) | (kind == KH_NULL ? 0 : 1));
                  }
                  ++ncross;
                }
              }
              // dense output at every target time this step passed (never past t_end)
              while (DENSE && (double)xn[0] >= t_next && !(P.t_end > 0.0 && t_next > P.t_end)) {
                double* o = S.s_out + ((int64_t)ray * S.n_out + j_out) * 8;
                double xo[4], ko[4];
                const double th = CT ? (t_next - (double)x[0]) / hd
                                     : hermite_zero((double)x[0] - t_next, (double)k[0], (double)xn[0] - t_next,
                                                    (double)kn[0], hd);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                  xo[c] = herm(th, (double)x[c], (double)k[c], (double)xn[c], (double)kn[c], hd);
                  ko[c] = herm(th, (double)k[c], (double)a1[c], (double)kn[c], (double)a7[c], hd);
                }
                xo[0] = t_next;
                double ks = 1.0;
                if (CT) {  // k^mu = k^0 (1, v) with k^0 from the entry energy, as on exit
                  ko[0] = 1.0;
                  ks = E0 / energy((double)a_c, xo, ko);
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                  o[c] = xo[c];
                  o[4 + c] = ks * ko[c];
                }
                ++j_out;
                t_next = j_out < S.n_out ? S.t_out[j_out] : __builtin_inf();
              }
              if ((double)r_new < rcap)
                status = KH_CAPTURED;
              else if ((double)r_new > P.r_escape && rdot_new > TS(0))
                status = KH_ESCAPED;
              else if (CT && landing)
                status = KH_T_END;
              else if (!CT && P.t_end > 0.0 && (double)xn[0] >= P.t_end) {
                // Land on t = t_end with the cubic Hermite interpolant of t(lambda);
                // positions use dx/dlambda = k, momenta use dk/dlambda = acc.
                const double th = hermite_zero((double)x[0] - P.t_end, (double)k[0], (double)xn[0] - P.t_end,
                                               (double)kn[0], h);
                TS xl[4], kl[4];
    #pragma unroll
                for (int c = 0; c < 4; ++c) {
                  xl[c] = (TS)herm(th, (double)x[c], (double)k[c], (double)xn[c], (double)kn[c], h);
                  kl[c] = (TS)herm(th, (double)k[c], (double)a1[c], (double)kn[c], (double)a7[c], h);
                }
    #pragma unroll
                for (int c = 0; c < 4; ++c) {
                  xn[c] = xl[c];
                  kn[c] = kl[c];
                }
                lam = lam_old + th * h;
                status = KH_T_END;
              }
            }
    #pragma unroll
            for (int c = 0; c < 4; ++c) {
              x[c] = xn[c];
              k[c] = kn[c];
              a1[c] = a7[c];
            }
            r_cur = r_new;
            rdot_cur = rdot_new;
            if (status == KH_ACTIVE) {
              h = hd * (double)grow_factor<TS>(err2, raw, after_reject);
              const double hm = P.hmax_coeff * hscale(kind, (double)r_cur);
              h = h < hm ? h : hm;
              after_reject = false;
              if (steps >= P.max_steps) status = KH_MAX_STEPS;
            }
          } else {
            ++nrej;
            h = hd * (double)shrink_factor<TS>(err2, raw);
            after_reject = true;
            // written so that a NaN step size also ends the ray
            if (!(h >= 1e-12 * P.h_coeff * hscale(kind, (double)r_cur))) status = KH_FAILED;
          }
          if (status == KH_ACTIVE && ++tries > P.max_tries) status = KH_MAX_STEPS;
          if (status != KH_ACTIVE) retire();
        }
        const unsigned long long idle_now = __ballot(ray < 0);
        bool service = idle_now == ~0ull || (cursor < parts && __popcll(idle_now) >= P.refill_min);
        if (P.k_cross > 0) {
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
          service = service || *cq_count > kQCap - 64;
        }
        if (service) break;
      }
      continue;
    }

    if (status != KH_ACTIVE) retire();
  }
  if (P.k_cross > 0) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int qc = *cq_count;
    if (qc > 0) flush_crossings(cq, cq_count, qc, S);
  }
}

// Finalize the rays an integrate call retired (flagged in their status), fully
// parallel: the unwrapped azimuth's atan2(y, x) term and the constants of
// motion in FP64 are done here rather than in the divergent retire path.
// unpause: the last pass of a two-queue mixed call (kPaused -> KH_MAX_STEPS).
__global__ void k_finalize(KState S, int unpause) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = S.n;
  if (i >= n) return;
  const int st = S.status[i];
  if (unpause && st == kPaused) {
    S.status[i] = KH_MAX_STEPS;
    return;
  }
  if (!(st & kRetired)) return;
  double x[4], k[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    x[c] = S.s[c * n + i];
    k[c] = S.s[(4 + c) * n + i];
  }
  if (st & kPhiPending) S.phi[i] = S.phi[i] + atan2(x[2], x[1]);
  if (S.c1) {
    double cst[4];
    const double a = S.spin[i];
    constants(S.kind[i] == KH_NULL ? -a : a, x, k, cst);
#pragma unroll
    for (int q = 0; q < 4; ++q) S.c1[q * n + i] = cst[q];
  }
  S.status[i] = st & kStatusMask;
}

// ---------------------------------------------------------------------------
// Initial data.
// ---------------------------------------------------------------------------
// cst: the constants of motion (E, L_z, Q, mu^2) in the chart, computed by the
// caller, which also rates the geodesic for scheduling from them.
__device__ inline void finish_init(KState S, int64_t i, const double y[8], double a_phys, int kind, bool ok,
                                   const double cst[4]) {
  const int64_t n = S.n;
#pragma unroll
  for (int c = 0; c < 8; ++c) S.s[c * n + i] = y[c];
  S.spin[i] = a_phys;
  S.kind[i] = kind;
  S.h[i] = 0.0;
  S.lam[i] = 0.0;
  S.phi[i] = atan2(y[2], y[1]);
  S.status[i] = ok ? KH_ACTIVE : KH_FAILED;
  S.n_acc[i] = 0;
  S.n_rej[i] = 0;
  if (S.n_cross) S.n_cross[i] = 0;
  if (S.cross)
    for (int j = 0; j < 3 * S.k_cross; ++j) S.cross[i * 3 * S.k_cross + j] = __builtin_nan("");
  if (S.c0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) S.c0[q * n + i] = cst[q];
  }
}

__device__ inline void camera_ray(double a_phys, double d, double incl, double al, double be, double y[8], bool* ok) {
  double si, ci;
  sincos(incl, &si, &ci);
  y[0] = 0.0;
  y[1] = d * si - be * ci;
  y[2] = al;
  y[3] = d * ci + be * si;
  y[4] = 0.0;
  y[5] = -si;
  y[6] = 0.0;
  y[7] = -ci;
  // traced future-directed in the chart with spin -a
  y[4] = null_k0(-a_phys, y, y + 4, ok);
  *ok = *ok && (y[4] == y[4]);
}

// Scheduling priority of a null ray (0 .. 255, larger = expected to take more
// steps): with xi = L_z / E and eta = Q / E^2 in the chart of spin a, the radial
// potential R(r) = (r^2 + a^2 - a xi)^2 - Delta (eta + (xi - a)^2) has a double
// root on a spherical photon orbit; the closer its minimum between the horizon
// and r = 5 comes to zero, the more times the ray circles the hole.  The
// minimum is bracketed on 17 radii and refined by three Newton steps on R'.
__device__ inline int ray_priority(double a, const double cst[4]) {
  const double E = cst[0];
  if (!(E > 0.0) || !(cst[1] == cst[1]) || !(cst[2] == cst[2])) return 0;
  const double xi = cst[1] / E, eta = cst[2] / (E * E);
  const double a2 = a * a, B = a2 - a * xi, Cc = eta + (xi - a) * (xi - a);
  const double rh = 1.0 + ksqrt(1.0 - a2 > 0.0 ? 1.0 - a2 : 0.0), span = 5.0 - rh;
  double rb = rh, Rb = 1e300;
  for (int j = 0; j <= 16; ++j) {
    const double r = rh + span * (j * (1.0 / 16));
    const double P = r * r + B;
    const double v = P * P - (r * r - 2.0 * r + a2) * Cc;
    if (v < Rb) {
      Rb = v;
      rb = r;
    }
  }
  for (int it = 0; it < 3; ++it) {
    const double P = rb * rb + B;
    const double d1 = 4.0 * rb * P - (2.0 * rb - 2.0) * Cc;
    const double d2 = 4.0 * P + 8.0 * rb * rb - 2.0 * Cc;
    if (d2 > 0.0) {
      const double rn = rb - d1 / d2;
      rb = rn < rh ? rh : (rn > 5.0 ? 5.0 : rn);
    }
  }
  const double P = rb * rb + B;
  const double v = P * P - (rb * rb - 2.0 * rb + a2) * Cc;
  Rb = v < Rb ? v : Rb;
  const double pr = -log2(fabs(Rb) * (1.0 / 30.0) + 1e-12);  // ~ -20 .. 40
  const int key = (int)(4.0 * pr) + 64;
  return key < 0 ? 0 : (key > 255 ? 255 : key);
}

// Scheduling priority of a time-like geodesic (0 .. 255, larger = more steps to
// a common t_end expected): the steps scale with t_end over the orbital period,
// i.e. as A^{-3/2} with A = 1 / (2 (1 - E)) the semi-major axis of a Newtonian
// orbit of the same binding energy.  16 keys per octave of A; unbound or
// undefined energies get 0.
__device__ inline int timelike_priority(const double cst[4]) {
  const double E = cst[0];
  if (!(E > 0.0 && E < 1.0)) return 0;
  const double A = 0.5 / (1.0 - E);
  const double k = 255.0 - 16.0 * log2(A > 1.0 ? A : 1.0);
  return k < 0.0 ? 0 : (int)k;
}

// keys (optional): per-tile scheduling key, the maximum of ray_priority over
// the tile's 64 rays (one wave = one tile: blocks are multiples of 64 threads).
// gkeys (optional): the per-ray key itself.
__global__ void k_init_rays(const kh_camera* cams, const int64_t* offs, int n_cams, KState S, uint8_t* keys,
                            uint8_t* gkeys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int key = 0;
  if (i < S.n) {
    int lo = 0, hi = n_cams - 1;  // last camera with offs[c] <= i
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (offs[mid] <= i)
        lo = mid;
      else
        hi = mid - 1;
    }
    const kh_camera cam = cams[lo];
    const int64_t p = i - offs[lo];
    const int64_t row = p / cam.width, col = p % cam.width;
    const double al = cam.alpha_min + (col + 0.5) * (cam.alpha_max - cam.alpha_min) / cam.width;
    const double be = cam.beta_min + (row + 0.5) * (cam.beta_max - cam.beta_min) / cam.height;
    double y[8];
    bool ok;
    camera_ray(cam.a, cam.r_obs, cam.incl, al, be, y, &ok);
    double cst[4] = {0.0, 0.0, 0.0, 0.0};
    if (S.c0 || keys || gkeys) constants(-cam.a, y, y + 4, cst);
    finish_init(S, i, y, cam.a, KH_NULL, ok, cst);
    if ((keys || gkeys) && ok) key = ray_priority(-cam.a, cst);
    if (gkeys) gkeys[i] = (uint8_t)key;
  }
  if (keys) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const int other = __shfl_xor(key, o);
      key = other > key ? other : key;
    }
    if (__lane_id() == 0 && (i >> 6) < ((S.n + 63) >> 6)) keys[i >> 6] = (uint8_t)key;
  }
}

// Counting sort of the tiles on their keys, largest key first, in one block.
constexpr int kSortThreads = 1024;
__global__ void __launch_bounds__(kSortThreads) k_tile_order(const uint8_t* keys, int64_t n_tiles, int32_t* order) {
  __shared__ unsigned hist[256];
  __shared__ unsigned next[256];
  for (int b = threadIdx.x; b < 256; b += blockDim.x) hist[b] = 0u;
  __syncthreads();
  for (int64_t t = threadIdx.x; t < n_tiles; t += blockDim.x) atomicAdd(&hist[keys[t]], 1u);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned acc = 0;
    for (int b = 255; b >= 0; --b) {
      next[b] = acc;
      acc += hist[b];
    }
  }
  __syncthreads();
  for (int64_t t = threadIdx.x; t < n_tiles; t += blockDim.x) {
    const unsigned pos = atomicAdd(&next[keys[t]], 1u);
    order[pos] = (int32_t)t;
  }
}

__global__ void k_order_identity(int32_t* order, int64_t n_tiles) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_tiles) order[t] = (int32_t)t;
}

// Per-geodesic counting sort of 8-bit keys, largest first, into perm [n]:
// clear the 256 counts, count (one LDS histogram per block of kPermSpan keys),
// scan in one block, then each block reserves its run of every key with one
// global atomic and places its geodesics by LDS atomics (the order within a
// key is unspecified).  cnt [0, 256) holds the counts, cnt [256, 512) the next
// free position of each key.
constexpr int kPermThreads = 256;
constexpr int kPermSpan = 8192;

__global__ void __launch_bounds__(kPermThreads) k_perm_clear(unsigned* cnt) {
  cnt[threadIdx.x] = 0u;
}

__global__ void __launch_bounds__(kPermThreads) k_perm_count(const uint8_t* keys, int64_t n, unsigned* cnt) {
  __shared__ unsigned hist[256];
  hist[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * kPermSpan;
  const int64_t hi = lo + kPermSpan < n ? lo + kPermSpan : n;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kPermThreads) atomicAdd(&hist[keys[i]], 1u);
  __syncthreads();
  if (hist[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], hist[threadIdx.x]);
}

__global__ void __launch_bounds__(kPermThreads) k_perm_scan(unsigned* cnt) {
  __shared__ unsigned v[256];
  const int t = threadIdx.x;  // position t of the descending key order holds key 255 - t
  const unsigned mine = cnt[255 - t];
  v[t] = mine;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const unsigned add = t >= o ? v[t - o] : 0u;
    __syncthreads();
    v[t] += add;
    __syncthreads();
  }
  cnt[256 + 255 - t] = v[t] - mine;
}

__global__ void __launch_bounds__(kPermThreads) k_perm_scatter(const uint8_t* keys, int64_t n, unsigned* cnt,
                                                             int32_t* perm) {
  __shared__ unsigned hist[256];
  __shared__ unsigned base[256];
  hist[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * kPermSpan;
  const int64_t hi = lo + kPermSpan < n ? lo + kPermSpan : n;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kPermThreads) atomicAdd(&hist[keys[i]], 1u);
  __syncthreads();
  const unsigned c = hist[threadIdx.x];
  base[threadIdx.x] = c ? atomicAdd(&cnt[256 + threadIdx.x], c) : 0u;
  hist[threadIdx.x] = 0u;
  __syncthreads();
  for (int64_t i = lo + threadIdx.x; i < hi; i += kPermThreads) {
    const int k = keys[i];
    const unsigned pos = base[k] + atomicAdd(&hist[k], 1u);
    perm[pos] = (int32_t)i;
  }
}

// Rows [count][8] of states first .. first + count - 1 (component-major in the
// state) for one device-to-host copy.
__global__ void k_pack_rows(const double* s, int64_t n, int64_t first, int64_t count, double* rows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
#pragma unroll
  for (int c = 0; c < 8; ++c) rows[i * 8 + c] = s[c * n + first + i];
}

__global__ void k_perm_identity(int32_t* perm, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) perm[i] = (int32_t)i;
}

__global__ void k_init_rays_pixels(kh_camera cam, const int32_t* pix, KState S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  const int64_t p = pix[i];
  const int64_t row = p / cam.width, col = p % cam.width;
  const double al = cam.alpha_min + (col + 0.5) * (cam.alpha_max - cam.alpha_min) / cam.width;
  const double be = cam.beta_min + (row + 0.5) * (cam.beta_max - cam.beta_min) / cam.height;
  double y[8];
  bool ok;
  camera_ray(cam.a, cam.r_obs, cam.incl, al, be, y, &ok);
  double cst[4] = {0.0, 0.0, 0.0, 0.0};
  if (S.c0) constants(-cam.a, y, y + 4, cst);
  finish_init(S, i, y, cam.a, KH_NULL, ok, cst);
}

__global__ void k_init_rays_list(const double* spin, const double* incl, const double* alpha, const double* beta,
                                 double r_obs, KState S, uint8_t* gkeys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  double y[8];
  bool ok;
  camera_ray(spin[i], r_obs, incl[i], alpha[i], beta[i], y, &ok);
  double cst[4] = {0.0, 0.0, 0.0, 0.0};
  if (S.c0 || gkeys) constants(-spin[i], y, y + 4, cst);
  finish_init(S, i, y, spin[i], KH_NULL, ok, cst);
  if (gkeys) gkeys[i] = (uint8_t)(ok ? ray_priority(-spin[i], cst) : 0);
}

__global__ void k_init_geodesics(int kind, const double* spin, const double* x3, const double* v3, KState S,
                                 uint8_t* gkeys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = S.n;
  if (i >= n) return;
  const double a = spin[i];
  double y[8] = {0.0, x3[i], x3[n + i], x3[2 * n + i], 0.0, v3[i], v3[n + i], v3[2 * n + i]};
  bool ok;
  if (kind == KH_TIMELIKE) {
    const double v[3] = {y[5], y[6], y[7]};
    const double u0 = timelike_u0(a, y, v, &ok);
    y[4] = u0;
    y[5] *= u0;
    y[6] *= u0;
    y[7] *= u0;
  } else {
    y[4] = null_k0(-a, y, y + 4, &ok);
  }
  ok = ok && (y[4] == y[4]);
  const double a_c = kind == KH_NULL ? -a : a;
  double cst[4] = {0.0, 0.0, 0.0, 0.0};
  if (S.c0 || gkeys) constants(a_c, y, y + 4, cst);
  finish_init(S, i, y, a, kind, ok, cst);
  if (gkeys) gkeys[i] = (uint8_t)(!ok ? 0 : (kind == KH_TIMELIKE ? timelike_priority(cst) : ray_priority(a_c, cst)));
}

// ---------------------------------------------------------------------------
// Point evaluation of the right-hand side and device-side statistics.
// ---------------------------------------------------------------------------
template <typename T, int FORM>
__global__ void k_rhs(const double* spin_chart, const double* s, double* acc, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T x[4], k[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    x[c] = (T)s[c * n + i];
    k[c] = (T)s[(4 + c) * n + i];
  }
  const Accel<T> ra = rhs<FORM, T>((T)spin_chart[i], x, k);
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c * n + i] = (double)ra.a[c];
}

__global__ void k_stats(const int32_t* status, const int32_t* n_acc, const int32_t* n_rej, int64_t n,
                        unsigned long long* out) {
  __shared__ unsigned long long part[8];
  if (threadIdx.x < 8) part[threadIdx.x] = 0ull;
  __syncthreads();
  unsigned long long loc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int st = status[i];
    if (st >= 0 && st < 6) loc[st] += 1ull;
    loc[6] += (unsigned long long)n_acc[i];
    loc[7] += (unsigned long long)n_rej[i];
  }
  for (int q = 0; q < 8; ++q) {
    unsigned long long v = loc[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    if ((threadIdx.x & 63) == 0) atomicAdd(&part[q], v);
  }
  __syncthreads();
  if (threadIdx.x < 8) atomicAdd(&out[threadIdx.x], part[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// Host-side operation counter for kh_flops.
// ---------------------------------------------------------------------------
struct Tally {
  int64_t add = 0, mul = 0, div = 0, sqrt = 0, trig = 0;
};
thread_local Tally* g_tally = nullptr;

struct Cnt {
  double v;
  Cnt() : v(0) {}
  Cnt(double d) : v(d) {}
};
inline Cnt operator+(Cnt a, Cnt b) {
  ++g_tally->add;
  return Cnt(a.v + b.v);
}
inline Cnt operator-(Cnt a, Cnt b) {
  ++g_tally->add;
  return Cnt(a.v - b.v);
}
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt operator*(Cnt a, Cnt b) {
  ++g_tally->mul;
  return Cnt(a.v * b.v);
}
inline Cnt operator/(Cnt a, Cnt b) {
  ++g_tally->div;
  return Cnt(a.v / b.v);
}
inline bool operator>=(Cnt a, Cnt b) { return a.v >= b.v; }
inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
// found by argument-dependent lookup from the templates in namespace kh
inline Cnt ksqrt(Cnt x) {
  ++g_tally->sqrt;
  return Cnt(std::sqrt(x.v));
}
inline Cnt krsqrt(Cnt x) {
  ++g_tally->sqrt;
  return Cnt(1.0 / std::sqrt(x.v));
}
inline Cnt krcp(Cnt x) {
  ++g_tally->div;
  return Cnt(1.0 / x.v);
}
inline Cnt krcp_est(Cnt x) {
  ++g_tally->div;
  return Cnt(1.0 / x.v);
}
inline void ksincos(Cnt x, Cnt* sn, Cnt* cs) {
  g_tally->trig += 2;
  *sn = Cnt(std::sin(x.v));
  *cs = Cnt(std::cos(x.v));
}
inline Cnt kabs(Cnt x) { return Cnt(std::fabs(x.v)); }
inline Cnt kmax(Cnt x, Cnt y) { return x.v > y.v ? x : y; }

}  // namespace

// ---------------------------------------------------------------------------
// Context and C ABI.
// ---------------------------------------------------------------------------

namespace khi {

kh_status fail(kh_ctx* c, kh_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

kh_status hip_fail(kh_ctx* c, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(c, KH_EHIP, m);
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Device pointer check: a host pointer handed to a kernel would fault the GPU.
bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

// True while `stream` is being captured into a graph: runtime queries such as
// hipPointerGetAttributes are then skipped (the arrays were checked when the
// same state was used eagerly; alignment and NULL checks still apply).
bool capturing(void* stream) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing((hipStream_t)stream, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return cs == hipStreamCaptureStatusActive;
}

thread_local bool g_skip_ptr_query = false;  // set per entry point while its stream is capturing

bool device_ok(const void* p) { return g_skip_ptr_query ? p != nullptr : is_device_ptr(p); }

const char* state_problem(const kh_state* st, bool need_cross) {
  if (!st) return "state is NULL";
  if (st->n < 1 || st->n >= (int64_t(1) << 31)) return "state.n must be in [1, 2^31)";
  if (st->k_cross < 0 || st->k_cross > 8) return "state.k_cross must be in [0, 8]";
  const void* d8[] = {st->s, st->spin, st->h, st->lam, st->phi};
  for (const void* p : d8)
    if (!p || !aligned(p, 8) || !device_ok(p))
      return "state arrays s, spin, h, lam, phi must be 8-byte aligned device memory";
  const void* d4[] = {st->kind, st->status, st->n_acc, st->n_rej};
  for (const void* p : d4)
    if (!p || !aligned(p, 4) || !device_ok(p))
      return "state arrays kind, status, n_acc, n_rej must be 4-byte aligned device memory";
  const void* opt8[] = {st->c0, st->c1, st->cross};
  for (const void* p : opt8)
    if (p && (!aligned(p, 8) || !device_ok(p)))
      return "state arrays c0, c1, cross must be NULL or 8-byte aligned device memory";
  if (st->n_cross && (!aligned(st->n_cross, 4) || !device_ok(st->n_cross)))
    return "state.n_cross must be NULL or 4-byte aligned device memory";
  if (st->order && (!aligned(st->order, 4) || !device_ok(st->order)))
    return "state.order must be NULL or 4-byte aligned device memory";
  if (st->perm && (!aligned(st->perm, 4) || !device_ok(st->perm)))
    return "state.perm must be NULL or 4-byte aligned device memory";
  if (st->n_out < 0) return "state.n_out must be >= 0";
  if (st->n_out > 0 && (!st->t_out || !st->s_out || !aligned(st->t_out, 8) || !aligned(st->s_out, 8) ||
                        !device_ok(st->t_out) || !device_ok(st->s_out)))
    return "state.n_out > 0 needs t_out and s_out in 8-byte aligned device memory";
  if (need_cross && st->k_cross > 0 && (!st->cross || !st->n_cross))
    return "state.k_cross > 0 requires cross and n_cross";
  return nullptr;
}

kh_status check_state(kh_ctx* ctx, const kh_state* st, bool need_cross) {
  const char* m = state_problem(st, need_cross);
  return m ? fail(ctx, KH_EINVAL, m) : KH_OK;
}

kh_status set_device(kh_ctx* ctx) {
  KH_HIP(ctx, hipSetDevice(ctx->device));
  return KH_OK;
}

}  // namespace khi

using namespace khi;

namespace {

template <int M, int P, int F, int W, bool D>
void* kernel_ptr() {
  return reinterpret_cast<void*>(&k_integrate<M, P, F, W, D>);
}

// Kernel variants: every method / precision / form at the default register
// budget, plus DOPRI5 with the factored right-hand side at 2, 3 and 4 waves per
// SIMD for the occupancy choice; dense output in variants of its own for the
// DOPRI5 methods with the factored form at the default budget.
void* pick_kernel(int method, int prec, int form, int wpe, bool dense) {
  if (dense) {
#define KH_PICKD(M, P) \
  if (method == M && prec == P && form == KH_RHS_FACTORED) return kernel_ptr<M, P, KH_RHS_FACTORED, 1, true>();
    KH_PICKD(KH_DOPRI5, KH_P64)
    KH_PICKD(KH_DOPRI5, KH_P32)
    KH_PICKD(KH_DOPRI5, KH_PMIXED)
    KH_PICKD(KH_DOPRI5_T, KH_P64)
    KH_PICKD(KH_DOPRI5_T, KH_P32)
    KH_PICKD(KH_DOPRI5_T, KH_PMIXED)
    KH_PICKD(KH_DOPRI5, kPSplit)
    KH_PICKD(KH_DOPRI5_T, kPSplit)
#undef KH_PICKD
    return nullptr;
  }
#define KH_PICK(M, P, F, W) \
  if (method == M && prec == P && form == F && wpe == W) return kernel_ptr<M, P, F, W, false>();
  KH_PICK(KH_RK4, KH_P64, KH_RHS_FACTORED, 1)
  KH_PICK(KH_RK4, KH_P32, KH_RHS_FACTORED, 1)
  KH_PICK(KH_RK4, KH_PMIXED, KH_RHS_FACTORED, 1)
  KH_PICK(KH_RK4, KH_P64, KH_RHS_PAPER, 1)
  KH_PICK(KH_RK4, KH_P32, KH_RHS_PAPER, 1)
  KH_PICK(KH_DOPRI5, KH_P64, KH_RHS_FACTORED, 1)
  KH_PICK(KH_DOPRI5, KH_P32, KH_RHS_FACTORED, 1)
  KH_PICK(KH_DOPRI5, KH_PMIXED, KH_RHS_FACTORED, 1)
  KH_PICK(KH_DOPRI5, KH_P64, KH_RHS_PAPER, 1)
  KH_PICK(KH_DOPRI5, KH_P32, KH_RHS_PAPER, 1)
  KH_PICK(KH_DOPRI5, KH_P64, KH_RHS_FACTORED, 3)
  KH_PICK(KH_DOPRI5, KH_P64, KH_RHS_FACTORED, 4)
  KH_PICK(KH_DOPRI5, KH_P32, KH_RHS_FACTORED, 4)
  KH_PICK(KH_DOPRI5, KH_P32, KH_RHS_FACTORED, 5)
  KH_PICK(KH_DOPRI5, KH_PMIXED, KH_RHS_FACTORED, 3)
  KH_PICK(KH_DOPRI5, KH_PMIXED, KH_RHS_FACTORED, 4)
  KH_PICK(KH_DOPRI5_T, KH_P64, KH_RHS_FACTORED, 1)
  KH_PICK(KH_DOPRI5_T, KH_P32, KH_RHS_FACTORED, 1)
  KH_PICK(KH_DOPRI5_T, KH_PMIXED, KH_RHS_FACTORED, 1)
  KH_PICK(KH_DOPRI5_T, KH_PMIXED, KH_RHS_FACTORED, 3)
  KH_PICK(KH_DOPRI5, kPSplit, KH_RHS_FACTORED, 1)
  KH_PICK(KH_DOPRI5, kPSplit, KH_RHS_FACTORED, 3)
  KH_PICK(KH_DOPRI5_T, kPSplit, KH_RHS_FACTORED, 1)
  KH_PICK(KH_DOPRI5_T, kPSplit, KH_RHS_FACTORED, 3)
#undef KH_PICK
  return nullptr;
}

}  // namespace

extern "C" {

void kh_default_params(kh_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->method = KH_DOPRI5;
  p->precision = KH_P64;
  p->rhs_form = KH_RHS_FACTORED;
  p->k_cross = 0;
  p->h_coeff = 0.01;
  p->rtol = 1e-8;
  p->atol = 1e-8;
  p->hmax_coeff = 0.1;
  p->r_h_factor = 1.01;
  p->r_escape = 1000.0;
  p->t_end = 0.0;
  p->r_fp64 = 3.0;
  p->max_steps = 1000000;
}

kh_status kh_create(kh_ctx** out, int device) {
  if (!out) return KH_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return KH_EINVAL;
  kh_ctx* c = new kh_ctx();
  c->device = device;
  if (hipSetDevice(device) != hipSuccess ||
      hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      hipMalloc(&c->d_queue, kQueueSlots * sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&c->d_stats, 8 * sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&c->d_perm_cnt, 512 * sizeof(unsigned)) != hipSuccess ||
      hipEventCreateWithFlags(&c->cam_evt, hipEventDisableTiming) != hipSuccess) {
    kh_destroy(c);
    return KH_ENOMEM;
  }
  *out = c;
  return KH_OK;
}

kh_status kh_destroy(kh_ctx* c) {
  if (!c) return KH_OK;
  (void)hipSetDevice(c->device);
  if (c->cam_evt) (void)hipEventSynchronize(c->cam_evt);
  if (c->d_queue) (void)hipFree(c->d_queue);
  if (c->d_stats) (void)hipFree(c->d_stats);
  if (c->d_cams) (void)hipFree(c->d_cams);
  if (c->d_offs) (void)hipFree(c->d_offs);
  if (c->h_cams) (void)hipHostFree(c->h_cams);
  if (c->h_offs) (void)hipHostFree(c->h_offs);
  if (c->cam_evt) (void)hipEventDestroy(c->cam_evt);
  if (c->d_keys) (void)hipFree(c->d_keys);
  if (c->d_gkeys) (void)hipFree(c->d_gkeys);
  if (c->d_perm_cnt) (void)hipFree(c->d_perm_cnt);
  if (c->d_stage) (void)hipFree(c->d_stage);
  delete c;
  return KH_OK;
}

const char* kh_last_error(const kh_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

namespace {
// Per-geodesic key buffer of at least st->n bytes (NULL without st->perm).  It
// grows only outside graph capture.
kh_status geodesic_keys(kh_ctx* ctx, const kh_state* st, uint8_t** out) {
  *out = nullptr;
  if (!st->perm) return KH_OK;
  if (st->n > ctx->gkeys_cap) {
    if (g_skip_ptr_query)
      return fail(ctx, KH_EINVAL, "the geodesic-key buffer must grow: call the init once outside graph capture");
    if (ctx->d_gkeys) KH_HIP(ctx, hipFree(ctx->d_gkeys));
    ctx->d_gkeys = nullptr;
    ctx->gkeys_cap = 0;
    if (hipMalloc(&ctx->d_gkeys, (size_t)st->n) != hipSuccess) return fail(ctx, KH_ENOMEM, "geodesic-key buffer");
    ctx->gkeys_cap = st->n;
  }
  *out = ctx->d_gkeys;
  return KH_OK;
}

// Counting sort of the per-geodesic keys into st->perm (four launches).
kh_status sort_perm(kh_ctx* ctx, const kh_state* st, const uint8_t* gkeys, hipStream_t strm) {
  const unsigned blocks = (unsigned)((st->n + kPermSpan - 1) / kPermSpan);
  hipLaunchKernelGGL(k_perm_clear, dim3(1), dim3(kPermThreads), 0, strm, ctx->d_perm_cnt);
  hipLaunchKernelGGL(k_perm_count, dim3(blocks), dim3(kPermThreads), 0, strm, gkeys, st->n, ctx->d_perm_cnt);
  hipLaunchKernelGGL(k_perm_scan, dim3(1), dim3(kPermThreads), 0, strm, ctx->d_perm_cnt);
  hipLaunchKernelGGL(k_perm_scatter, dim3(blocks), dim3(kPermThreads), 0, strm, gkeys, st->n, ctx->d_perm_cnt,
                     st->perm);
  KH_HIP(ctx, hipGetLastError());
  return KH_OK;
}

// The init kernel over the uploaded camera table, then (with st->order) the
// tile sort and (with st->perm) the per-ray sort.  The key buffers grow only
// outside graph capture.
kh_status launch_init_rays(kh_ctx* ctx, kh_state* st, int n_cams, hipStream_t strm) {
  const int64_t n_tiles = (st->n + 63) / 64;
  uint8_t* keys = nullptr;
  uint8_t* gkeys = nullptr;
  kh_status s = geodesic_keys(ctx, st, &gkeys);
  if (s != KH_OK) return s;
  if (st->order) {
    if (n_tiles > ctx->keys_cap) {
      if (g_skip_ptr_query)
        return fail(ctx, KH_EINVAL, "the tile-key buffer must grow: call kh_init_rays once outside graph capture");
      if (ctx->d_keys) KH_HIP(ctx, hipFree(ctx->d_keys));
      ctx->d_keys = nullptr;
      ctx->keys_cap = 0;
      if (hipMalloc(&ctx->d_keys, (size_t)n_tiles) != hipSuccess) return fail(ctx, KH_ENOMEM, "tile-key buffer");
      ctx->keys_cap = n_tiles;
    }
    keys = ctx->d_keys;
  }
  const KState ks = to_k(st);
  const int block = 256;
  const int64_t grid = (st->n + block - 1) / block;
  hipLaunchKernelGGL(k_init_rays, dim3((unsigned)grid), dim3(block), 0, strm, ctx->d_cams, ctx->d_offs, n_cams, ks,
                     keys, gkeys);
  KH_HIP(ctx, hipGetLastError());
  if (st->order) {
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kSortThreads), 0, strm, (const uint8_t*)keys, n_tiles, st->order);
    KH_HIP(ctx, hipGetLastError());
  }
  return gkeys ? sort_perm(ctx, st, gkeys, strm) : KH_OK;
}

// Natural tile order, and the natural per-geodesic order unless `sorted`
// (the caller then sorts st->perm itself).
kh_status natural_order(kh_ctx* ctx, const kh_state* st, hipStream_t strm, bool sorted = false) {
  if (st->order) {
    const int64_t n_tiles = (st->n + 63) / 64;
    hipLaunchKernelGGL(k_order_identity, dim3((unsigned)((n_tiles + 255) / 256)), dim3(256), 0, strm, st->order,
                       n_tiles);
    KH_HIP(ctx, hipGetLastError());
  }
  if (st->perm && !sorted) {
    hipLaunchKernelGGL(k_perm_identity, dim3((unsigned)((st->n + 255) / 256)), dim3(256), 0, strm, st->perm, st->n);
    KH_HIP(ctx, hipGetLastError());
  }
  return KH_OK;
}
}  // namespace

kh_status kh_init_rays(kh_ctx* ctx, const kh_camera* cams, int32_t n_cams, kh_state* st, void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = capturing(stream);
  if (n_cams < 1) return fail(ctx, KH_EINVAL, "need at least one camera");
  if (!cams) {
    // Reuse the table uploaded by an earlier call: a single kernel launch, so
    // this form can be captured into a graph.
    if (n_cams != ctx->cams_uploaded) return fail(ctx, KH_EINVAL, "cams == NULL needs the same n_cams as the last upload");
    kh_status s = check_state(ctx, st, false);
    if (s != KH_OK) return s;
    if (st->n != ctx->cams_total) return fail(ctx, KH_EINVAL, "state.n must equal the total pixel count of the cameras");
    if ((s = set_device(ctx)) != KH_OK) return s;
    return launch_init_rays(ctx, st, n_cams, (hipStream_t)stream);
  }
  int64_t total = 0;
  for (int i = 0; i < n_cams; ++i) {
    const kh_camera& c = cams[i];
    if (!(std::fabs(c.a) <= 1.0) || !(c.r_obs > 0.0) || c.width < 1 || c.height < 1 || !std::isfinite(c.incl) ||
        !std::isfinite(c.alpha_min) || !std::isfinite(c.alpha_max) || !std::isfinite(c.beta_min) ||
        !std::isfinite(c.beta_max))
      return fail(ctx, KH_EINVAL, "camera " + std::to_string(i) + ": need |a| <= 1, r_obs > 0, width, height >= 1");
    total += int64_t(c.width) * c.height;
  }
  kh_status s = check_state(ctx, st, false);
  if (s != KH_OK) return s;
  if (total != st->n) return fail(ctx, KH_EINVAL, "state.n must equal the total pixel count of the cameras");
  if ((s = set_device(ctx)) != KH_OK) return s;
  hipStream_t strm = (hipStream_t)stream;
  if (n_cams > ctx->cam_cap) {
    KH_HIP(ctx, hipEventSynchronize(ctx->cam_evt));
    if (ctx->d_cams) KH_HIP(ctx, hipFree(ctx->d_cams));
    if (ctx->d_offs) KH_HIP(ctx, hipFree(ctx->d_offs));
    if (ctx->h_cams) KH_HIP(ctx, hipHostFree(ctx->h_cams));
    if (ctx->h_offs) KH_HIP(ctx, hipHostFree(ctx->h_offs));
    ctx->d_cams = nullptr;
    ctx->d_offs = nullptr;
    ctx->h_cams = nullptr;
    ctx->h_offs = nullptr;
    ctx->cam_cap = 0;
    const int cap = std::max(n_cams, 64);
    if (hipMalloc(&ctx->d_cams, cap * sizeof(kh_camera)) != hipSuccess ||
        hipMalloc(&ctx->d_offs, (cap + 1) * sizeof(int64_t)) != hipSuccess ||
        hipHostMalloc(&ctx->h_cams, cap * sizeof(kh_camera), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&ctx->h_offs, (cap + 1) * sizeof(int64_t), hipHostMallocDefault) != hipSuccess)
      return fail(ctx, KH_ENOMEM, "camera table allocation failed");
    ctx->cam_cap = cap;
  }
  // The staging buffers may still feed the previous call's copy.
  KH_HIP(ctx, hipEventSynchronize(ctx->cam_evt));
  int64_t off = 0;
  for (int i = 0; i < n_cams; ++i) {
    ctx->h_cams[i] = cams[i];
    ctx->h_offs[i] = off;
    off += int64_t(cams[i].width) * cams[i].height;
  }
  ctx->h_offs[n_cams] = off;
  KH_HIP(ctx, hipMemcpyAsync(ctx->d_cams, ctx->h_cams, n_cams * sizeof(kh_camera), hipMemcpyHostToDevice, strm));
  KH_HIP(ctx,
         hipMemcpyAsync(ctx->d_offs, ctx->h_offs, (n_cams + 1) * sizeof(int64_t), hipMemcpyHostToDevice, strm));
  KH_HIP(ctx, hipEventRecord(ctx->cam_evt, strm));
  ctx->cams_uploaded = n_cams;
  ctx->cams_total = total;
  return launch_init_rays(ctx, st, n_cams, strm);
}

kh_status kh_init_rays_list(kh_ctx* ctx, const double* spin, const double* incl, const double* alpha,
                            const double* beta, double r_obs, kh_state* st, void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = false;
  kh_status s = check_state(ctx, st, false);
  if (s != KH_OK) return s;
  const double* ins[] = {spin, incl, alpha, beta};
  for (const double* p : ins)
    if (!p || !aligned(p, 8) || !is_device_ptr(p))
      return fail(ctx, KH_EINVAL, "spin, incl, alpha, beta must be 8-byte aligned device arrays of length n");
  if (!(r_obs > 0.0)) return fail(ctx, KH_EINVAL, "r_obs must be > 0");
  if ((s = set_device(ctx)) != KH_OK) return s;
  uint8_t* gkeys = nullptr;
  if ((s = geodesic_keys(ctx, st, &gkeys)) != KH_OK) return s;
  const KState ks = to_k(st);
  const int block = 256;
  const int64_t grid = (st->n + block - 1) / block;
  hipLaunchKernelGGL(k_init_rays_list, dim3((unsigned)grid), dim3(block), 0, (hipStream_t)stream, spin, incl, alpha,
                     beta, r_obs, ks, gkeys);
  KH_HIP(ctx, hipGetLastError());
  if ((s = natural_order(ctx, st, (hipStream_t)stream, gkeys != nullptr)) != KH_OK) return s;
  return gkeys ? sort_perm(ctx, st, gkeys, (hipStream_t)stream) : KH_OK;
}

kh_status kh_init_rays_pixels(kh_ctx* ctx, const kh_camera* cam, const int32_t* pix, kh_state* st, void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = capturing(stream);
  if (!cam || !(std::fabs(cam->a) <= 1.0) || !(cam->r_obs > 0.0) || cam->width < 1 || cam->height < 1)
    return fail(ctx, KH_EINVAL, "camera: need |a| <= 1, r_obs > 0, width, height >= 1");
  kh_status s = check_state(ctx, st, false);
  if (s != KH_OK) return s;
  if (!pix || !aligned(pix, 4) || !device_ok(pix)) return fail(ctx, KH_EINVAL, "pix must be device int32 [n]");
  if ((s = set_device(ctx)) != KH_OK) return s;
  const KState ks = to_k(st);
  const int block = 256;
  hipLaunchKernelGGL(k_init_rays_pixels, dim3((unsigned)((st->n + block - 1) / block)), dim3(block), 0,
                     (hipStream_t)stream, *cam, pix, ks);
  KH_HIP(ctx, hipGetLastError());
  return natural_order(ctx, st, (hipStream_t)stream);
}

kh_status kh_init_geodesics(kh_ctx* ctx, int32_t kind, const double* spin, const double* x3, const double* v3,
                            kh_state* st, void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = false;
  if (kind != KH_NULL && kind != KH_TIMELIKE) return fail(ctx, KH_EINVAL, "kind must be KH_NULL or KH_TIMELIKE");
  kh_status s = check_state(ctx, st, false);
  if (s != KH_OK) return s;
  const double* ins[] = {spin, x3, v3};
  for (const double* p : ins)
    if (!p || !aligned(p, 8) || !is_device_ptr(p))
      return fail(ctx, KH_EINVAL, "spin [n], x3 [3][n], v3 [3][n] must be 8-byte aligned device arrays");
  if ((s = set_device(ctx)) != KH_OK) return s;
  uint8_t* gkeys = nullptr;
  if ((s = geodesic_keys(ctx, st, &gkeys)) != KH_OK) return s;
  const KState ks = to_k(st);
  const int block = 256;
  const int64_t grid = (st->n + block - 1) / block;
  hipLaunchKernelGGL(k_init_geodesics, dim3((unsigned)grid), dim3(block), 0, (hipStream_t)stream, (int)kind, spin,
                     x3, v3, ks, gkeys);
  KH_HIP(ctx, hipGetLastError());
  if ((s = natural_order(ctx, st, (hipStream_t)stream, gkeys != nullptr)) != KH_OK) return s;
  return gkeys ? sort_perm(ctx, st, gkeys, (hipStream_t)stream) : KH_OK;
}

}  // extern "C"

namespace {

// Argument checks of kh_integrate that need no context: nullptr when the
// parameters are usable, else the message (and *code the status).
const char* params_problem(const kh_params* p, const kh_state* st, kh_status* code) {
  *code = KH_EINVAL;
  if (!p) return "params is NULL";
  if (p->method != KH_RK4 && p->method != KH_DOPRI5 && p->method != KH_DOPRI5_T) return "unknown method";
  if (p->precision != KH_P64 && p->precision != KH_P32 && p->precision != KH_PMIXED) return "unknown precision";
  if (p->rhs_form != KH_RHS_FACTORED && p->rhs_form != KH_RHS_PAPER) return "unknown rhs_form";
  if (!(p->h_coeff > 0.0) || !(p->r_h_factor > 0.0) || !(p->r_escape > 0.0) || p->max_steps < 1)
    return "need h_coeff, r_h_factor, r_escape > 0 and max_steps >= 1";
  if (p->method != KH_RK4 && (!(p->rtol > 0.0) || !(p->atol > 0.0) || !(p->hmax_coeff > 0.0)))
    return "DOPRI5 needs rtol, atol, hmax_coeff > 0";
  if (p->k_cross < 0 || p->k_cross > 8) return "k_cross must be in [0, 8]";
  if (p->method == KH_RK4 && (p->k_cross > 0 || p->t_end > 0.0 || (st && st->n_out > 0))) {
    *code = KH_EUNSUPPORTED;
    return "crossings, t_end and dense output need a DOPRI5 method";
  }
  if (p->k_cross > 0 && p->t_end > 0.0) {
    *code = KH_EUNSUPPORTED;
    return "crossing records and t_end landing are not combined";
  }
  if (p->mixed_split != 0 && p->mixed_split != 1) return "mixed_split must be 0 or 1";
  if (p->mixed_split == 1 && p->precision != KH_PMIXED) return "mixed_split applies to KH_PMIXED only";
  if (p->mixed_split == 1 && p->method == KH_RK4) {
    *code = KH_EUNSUPPORTED;
    return "the two-queue mixed policy needs a DOPRI5 method";
  }
  if (p->rhs_form == KH_RHS_PAPER && p->precision == KH_PMIXED) {
    *code = KH_EUNSUPPORTED;
    return "the paper-form right-hand side is built for P64 and P32 only";
  }
  const int block = p->block_size ? p->block_size : 256;
  if (block < 64 || block > 256 || block % 64) return "block_size must be 64, 128, 192 or 256";
  const int refill = p->refill_min ? p->refill_min : 12;
  if (refill < 1 || refill > 64) return "refill_min must be in [1, 64]";
  if (p->grid_blocks < 0) return "grid_blocks must be >= 0";
  if (p->waves_per_eu < 0 || p->waves_per_eu > 8) return "waves_per_eu must be in [0, 8]";
  if (p->queue_parts < 0 || p->queue_parts > kParts) return "queue_parts must be in [0, 8]";
  if (const char* m = state_problem(st, p->k_cross > 0)) return m;
  if (p->k_cross > st->k_cross) return "params.k_cross exceeds state.k_cross";
  *code = KH_OK;
  return nullptr;
}

// Text of the last HIP failure of a launch below (per host thread; no allocation).
thread_local char g_hip_msg[256];

const char* hip_msg(hipError_t e, const char* where) {
  std::snprintf(g_hip_msg, sizeof g_hip_msg, "%s: %s", where, hipGetErrorString(e));
  return g_hip_msg;
}

#define KH_TRY(call)                                          \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) {                                   \
      *msg = hip_msg(e_, #call);                              \
      return KH_EHIP;                                         \
    }                                                         \
  } while (0)

// The launches of an integrate call, after the argument checks, with the
// work-queue counters `q` (at least kParts of them, device memory) on the
// current device of `n_cu` compute units: counter reset, the persistent
// integrate kernel, the finalize pass.  No allocation, no synchronisation.
kh_status launch_integrate(const kh_params* p, const kh_state* st, hipStream_t strm, unsigned long long* q, int n_cu,
                           const char** msg) {
  const int block = p->block_size ? p->block_size : 256;
  KParams kp;
  kp.h_coeff = p->h_coeff;
  kp.rtol = p->rtol;
  kp.atol = p->atol;
  if (p->precision == KH_P32) {  // FP32 cannot honour tolerances near its epsilon
    kp.rtol = std::max(kp.rtol, 1e-6);
    kp.atol = std::max(kp.atol, 1e-6);
  }
  kp.hmax_coeff = p->hmax_coeff;
  kp.r_h_factor = p->r_h_factor;
  kp.r_escape = p->r_escape;
  kp.t_end = p->t_end;
  kp.r_fp64 = p->r_fp64;
  // per-call step counters are 32-bit in the kernel
  kp.max_steps = (int32_t)std::min<int64_t>(p->max_steps, INT32_MAX);
  kp.max_tries = (int32_t)std::min<int64_t>(4 * std::min<int64_t>(p->max_steps, INT32_MAX) + 1000, INT32_MAX);
  kp.k_cross = p->k_cross;
  kp.refill_min = p->refill_min ? p->refill_min : 12;
  kp.parts = p->queue_parts ? p->queue_parts : kParts;
  const bool split = p->precision == KH_PMIXED && p->mixed_split == 1;

  // Default register budget: MIXED DOPRI5 runs faster at three waves per SIMD
  // (spilling a few registers) than at two; FP64 and FP32 do not gain.
  int wpe = p->waves_per_eu;
  if (wpe == 0) wpe = (p->method != KH_RK4 && p->precision == KH_PMIXED && p->rhs_form == KH_RHS_FACTORED) ? 3 : 1;
  void* fn = pick_kernel(p->method, split ? kPSplit : p->precision, p->rhs_form, wpe, st->n_out > 0);
  // the second pass of the two-queue policy: the FP64 kernel of the same method
  void* fn64 = split ? pick_kernel(p->method, KH_P64, p->rhs_form, 1, st->n_out > 0) : nullptr;
  if (!fn || (split && !fn64)) {
    *msg = "no kernel for this method / precision / rhs_form / waves_per_eu";
    return KH_EUNSUPPORTED;
  }
  // dynamic LDS: one crossing queue (kQFields x kQCap doubles + a counter) per wave
  const size_t lds = p->k_cross > 0 ? (size_t)(block / 64) * (kQFields * kQCap + 1) * sizeof(double) : 0;
  const KState ks = to_k(st);
  // one pass: counter reset, the persistent kernel, the finalize pass
  auto pass = [&](void* f, KParams& kpp, int unpause) -> kh_status {
    int grid = p->grid_blocks;
    if (grid == 0) {
      int per_cu = 0;
      KH_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)f, block, lds));
      grid = std::max(1, per_cu) * n_cu;
    }
    const int64_t need = (st->n + block - 1) / block;
    if (grid > need) grid = (int)need;
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, strm, q, kParts);
    KH_TRY(hipGetLastError());
    KState kss = ks;
    void* args[] = {(void*)&kpp, (void*)&kss, (void*)&q};
    KH_TRY(hipLaunchKernel(f, dim3(grid), dim3(block), args, lds, strm));
    const int b = 256;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)((st->n + b - 1) / b)), dim3(b), 0, strm, ks, unpause);
    KH_TRY(hipGetLastError());
    return KH_OK;
  };
  kh_status s = pass(fn, kp, 0);
  if (s != KH_OK || !split) return s;
  // The parked geodesics resume in FP64 from the state the first pass wrote
  // (its finalize pass completed their azimuth, as for a pause).
  return pass(fn64, kp, 1);
}

#undef KH_TRY

// Work-queue counters of kh_integrate_noalloc, for callers that cannot
// allocate: one copy of this array per GPU the library runs on, held until the
// process ends.  On the host the name `scratch` is only a stand-in for the
// symbol, not a device address; host code uses the address that
// hipGetSymbolAddress returns for the current device (noalloc_device below).
constexpr int kNoAllocSlots = kQueueSlots;  // 16 x 8 B; an integrate call uses kParts of them
static_assert(kParts <= kNoAllocSlots, "the static array holds every queue partition's counter");
static __device__ __align__(256) unsigned long long scratch[kNoAllocSlots];

constexpr int kMaxDevices = 64;
struct NoAllocDevice {
  unsigned long long* q = nullptr;  // device address of `scratch` on this device
  int n_cu = 0;
};
NoAllocDevice g_noalloc[kMaxDevices];
std::mutex g_noalloc_mu;

// Set-up of the current device, once per device: the address of its copy of
// `scratch` and its compute-unit count.  Allocates nothing.
const char* noalloc_device(NoAllocDevice* out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return "hipGetDevice failed";
  if (dev < 0 || dev >= kMaxDevices) return "device index beyond the library's table of 64 devices";
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  NoAllocDevice& d = g_noalloc[dev];
  if (!d.q) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_msg(e, "hipGetSymbolAddress(scratch)");
    int n_cu = 0;
    e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_msg(e, "hipDeviceGetAttribute(multiprocessor count)");
    d.n_cu = n_cu;
    d.q = static_cast<unsigned long long*>(ptr);
  }
  *out = d;
  return nullptr;
}

void copy_msg(char* err, int32_t err_len, const char* m) {
  if (err && err_len > 0) std::snprintf(err, (size_t)err_len, "%s", m ? m : "");
}

}  // namespace

extern "C" {

kh_status kh_integrate(kh_ctx* ctx, const kh_params* p, kh_state* st, void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = capturing(stream);
  kh_status code;
  if (const char* m = params_problem(p, st, &code)) return fail(ctx, code, m);
  kh_status s;
  if ((s = set_device(ctx)) != KH_OK) return s;
  const char* msg = nullptr;
  s = launch_integrate(p, st, (hipStream_t)stream, ctx->d_queue, ctx->n_cu, &msg);
  return s == KH_OK ? KH_OK : fail(ctx, s, msg ? msg : "kh_integrate");
}

kh_status kh_integrate_noalloc(const kh_params* p, kh_state* st, void* stream, char* err, int32_t err_len) {
  copy_msg(err, err_len, "");
  g_skip_ptr_query = capturing(stream);
  kh_status code;
  if (const char* m = params_problem(p, st, &code)) {
    copy_msg(err, err_len, m);
    return code;
  }
  NoAllocDevice d;
  if (const char* m = noalloc_device(&d)) {
    copy_msg(err, err_len, m);
    return KH_EHIP;
  }
  const char* msg = nullptr;
  const kh_status s = launch_integrate(p, st, (hipStream_t)stream, d.q, d.n_cu, &msg);
  if (s != KH_OK) copy_msg(err, err_len, msg ? msg : "kh_integrate_noalloc");
  return s;
}

kh_status kh_read_state(kh_ctx* ctx, const kh_state* st, int64_t first, int64_t count, double* host_s,
                        int32_t* host_status, void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = false;
  kh_status s = check_state(ctx, st, false);
  if (s != KH_OK) return s;
  if (first < 0 || count < 0 || first + count > st->n) return fail(ctx, KH_EINVAL, "range outside the state");
  if ((s = set_device(ctx)) != KH_OK) return s;
  hipStream_t strm = (hipStream_t)stream;
  if (host_s && count > 0) {
    // Rows are packed on the device in chunks of at most 2^20 rays (64 MiB
    // of context scratch) and copied straight into host_s.
    const int64_t chunk = std::min<int64_t>(count, int64_t(1) << 20);
    if (chunk > ctx->stage_cap) {
      KH_HIP(ctx, hipStreamSynchronize(strm));
      if (ctx->d_stage) KH_HIP(ctx, hipFree(ctx->d_stage));
      ctx->d_stage = nullptr;
      ctx->stage_cap = 0;
      if (hipMalloc(&ctx->d_stage, (size_t)chunk * 8 * sizeof(double)) != hipSuccess)
        return fail(ctx, KH_ENOMEM, "read-back staging buffer");
      ctx->stage_cap = chunk;
    }
    for (int64_t off = 0; off < count; off += chunk) {
      const int64_t m = std::min<int64_t>(chunk, count - off);
      hipLaunchKernelGGL(k_pack_rows, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, strm, st->s, st->n,
                         first + off, m, ctx->d_stage);
      KH_HIP(ctx, hipGetLastError());
      KH_HIP(ctx, hipMemcpyAsync(host_s + off * 8, ctx->d_stage, (size_t)m * 8 * sizeof(double),
                                 hipMemcpyDeviceToHost, strm));
    }
  }
  if (host_status && count > 0)
    KH_HIP(ctx, hipMemcpyAsync(host_status, st->status + first, count * sizeof(int32_t), hipMemcpyDeviceToHost, strm));
  KH_HIP(ctx, hipStreamSynchronize(strm));
  return KH_OK;
}

kh_status kh_stats(kh_ctx* ctx, const kh_state* st, int64_t out[8], void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = false;
  if (!out) return fail(ctx, KH_EINVAL, "out is NULL");
  kh_status s = check_state(ctx, st, false);
  if (s != KH_OK) return s;
  if ((s = set_device(ctx)) != KH_OK) return s;
  hipStream_t strm = (hipStream_t)stream;
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, strm, ctx->d_stats, 8);
  const int block = 256;
  int64_t grid = std::min<int64_t>((st->n + block - 1) / block, 4 * std::max(ctx->n_cu, 1));
  hipLaunchKernelGGL(k_stats, dim3((unsigned)grid), dim3(block), 0, strm, st->status, st->n_acc, st->n_rej, st->n,
                     ctx->d_stats);
  KH_HIP(ctx, hipGetLastError());
  unsigned long long h[8];
  KH_HIP(ctx, hipMemcpyAsync(h, ctx->d_stats, sizeof h, hipMemcpyDeviceToHost, strm));
  KH_HIP(ctx, hipStreamSynchronize(strm));
  for (int i = 0; i < 8; ++i) out[i] = (int64_t)h[i];
  return KH_OK;
}

kh_status kh_stats_device(kh_ctx* ctx, const kh_state* st, int64_t* d_out, void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = capturing(stream);
  if (!d_out || !aligned(d_out, 8) || !device_ok(d_out))
    return fail(ctx, KH_EINVAL, "d_out must be 8-byte aligned device memory for 8 counts");
  kh_status s = check_state(ctx, st, false);
  if (s != KH_OK) return s;
  if ((s = set_device(ctx)) != KH_OK) return s;
  hipStream_t strm = (hipStream_t)stream;
  unsigned long long* out = reinterpret_cast<unsigned long long*>(d_out);
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, strm, out, 8);
  const int block = 256;
  int64_t grid = std::min<int64_t>((st->n + block - 1) / block, 4 * std::max(ctx->n_cu, 1));
  hipLaunchKernelGGL(k_stats, dim3((unsigned)grid), dim3(block), 0, strm, st->status, st->n_acc, st->n_rej, st->n,
                     out);
  KH_HIP(ctx, hipGetLastError());
  return KH_OK;
}

kh_status kh_rhs(kh_ctx* ctx, int32_t precision, int32_t rhs_form, const double* spin_chart, const double* s,
                 double* acc, int64_t n, void* stream) {
  if (!ctx) return KH_EINVAL;
  if (n < 1 || n >= (int64_t(1) << 31)) return fail(ctx, KH_EINVAL, "n must be in [1, 2^31)");
  const double* ins[] = {spin_chart, s, acc};
  for (const double* p : ins)
    if (!p || !aligned(p, 8) || !is_device_ptr(p)) return fail(ctx, KH_EINVAL, "arrays must be device memory");
  if (precision != KH_P64 && precision != KH_P32) return fail(ctx, KH_EINVAL, "precision must be KH_P64 or KH_P32");
  if (rhs_form != KH_RHS_FACTORED && rhs_form != KH_RHS_PAPER) return fail(ctx, KH_EINVAL, "unknown rhs_form");
  kh_status st = set_device(ctx);
  if (st != KH_OK) return st;
  const int block = 256;
  const dim3 grid((unsigned)((n + block - 1) / block));
  hipStream_t strm = (hipStream_t)stream;
  if (precision == KH_P64 && rhs_form == KH_RHS_FACTORED)
    hipLaunchKernelGGL((k_rhs<double, KH_RHS_FACTORED>), grid, dim3(block), 0, strm, spin_chart, s, acc, n);
  else if (precision == KH_P64)
    hipLaunchKernelGGL((k_rhs<double, KH_RHS_PAPER>), grid, dim3(block), 0, strm, spin_chart, s, acc, n);
  else if (rhs_form == KH_RHS_FACTORED)
    hipLaunchKernelGGL((k_rhs<float, KH_RHS_FACTORED>), grid, dim3(block), 0, strm, spin_chart, s, acc, n);
  else
    hipLaunchKernelGGL((k_rhs<float, KH_RHS_PAPER>), grid, dim3(block), 0, strm, spin_chart, s, acc, n);
  KH_HIP(ctx, hipGetLastError());
  return KH_OK;
}

kh_status kh_flops(int32_t method, int32_t rhs_form, kh_flop_counts* out) {
  if (!out || (method != KH_RK4 && method != KH_DOPRI5 && method != KH_DOPRI5_T) ||
      (rhs_form != KH_RHS_FACTORED && rhs_form != KH_RHS_PAPER && rhs_form != KH_RHS_BL) ||
      (method == KH_DOPRI5_T && rhs_form != KH_RHS_FACTORED) || (rhs_form == KH_RHS_BL && method != KH_RK4))
    return KH_EINVAL;
  if (rhs_form == KH_RHS_BL) {
    // Boyer-Lindquist point (t, r, theta, phi) off the equator and the poles
    Tally tb, ts;
    const Cnt xb[4] = {Cnt(0.0), Cnt(7.0), Cnt(1.1), Cnt(0.3)};
    const Cnt kb[4] = {Cnt(1.2), Cnt(-0.6), Cnt(0.03), Cnt(-0.02)};
    const Cnt a1[4] = {Cnt(0.01), Cnt(0.02), Cnt(-0.01), Cnt(0.005)};
    Cnt xn[4], kn[4];
    g_tally = &tb;
    (void)chart_rhs<KH_RHS_BL, Cnt>(Cnt(0.9), xb, kb);
    g_tally = &ts;
    rk4_step<KH_RHS_BL, Cnt, Cnt>(Cnt(0.9), xb, kb, a1, Cnt(0.1), xn, kn);
    g_tally = nullptr;
    *out = kh_flop_counts{tb.add, tb.mul, tb.div, tb.sqrt, ts.add - 3 * tb.add, ts.mul - 3 * tb.mul,
                          ts.div - 3 * tb.div, ts.sqrt - 3 * tb.sqrt, tb.trig};
    return KH_OK;
  }
  Tally t_rhs, t_step;
  const Cnt x[4] = {Cnt(0.0), Cnt(7.0), Cnt(-3.0), Cnt(2.0)};
  const Cnt k[4] = {Cnt(1.2), Cnt(-0.6), Cnt(0.3), Cnt(-0.2)};
  g_tally = &t_rhs;
  const Cnt v[4] = {Cnt(1.0), Cnt(-0.5), Cnt(0.25), Cnt(-0.15)};
  if (method == KH_DOPRI5_T)
    (void)rhs_ct<KH_RHS_FACTORED, Cnt>(Cnt(0.9), x, v);
  else if (rhs_form == KH_RHS_FACTORED)
    (void)rhs<KH_RHS_FACTORED, Cnt>(Cnt(0.9), x, k);
  else
    (void)rhs<KH_RHS_PAPER, Cnt>(Cnt(0.9), x, k);
  g_tally = &t_step;
  Cnt xn[4], kn[4], a7[4], r, rd;
  const Cnt a1[4] = {Cnt(0.01), Cnt(0.02), Cnt(-0.01), Cnt(0.005)};
  int n_rhs;
  if (method == KH_DOPRI5_T) {
    const Cnt a1t[4] = {Cnt(0.0), Cnt(0.02), Cnt(-0.01), Cnt(0.005)};
    (void)dp5_attempt<KH_RHS_FACTORED, Cnt, Cnt, true>(Cnt(0.9), x, v, a1t, Cnt(0.1), Cnt(1e-8), Cnt(1e-8), xn, kn, a7,
                                                        r, rd);
    n_rhs = 6;
  } else if (method == KH_DOPRI5) {
    if (rhs_form == KH_RHS_FACTORED)
      (void)dp5_attempt<KH_RHS_FACTORED, Cnt, Cnt>(Cnt(0.9), x, k, a1, Cnt(0.1), Cnt(1e-8), Cnt(1e-8), xn, kn, a7, r,
                                                   rd);
    else
      (void)dp5_attempt<KH_RHS_PAPER, Cnt, Cnt>(Cnt(0.9), x, k, a1, Cnt(0.1), Cnt(1e-8), Cnt(1e-8), xn, kn, a7, r, rd);
    n_rhs = 6;
  } else {
    if (rhs_form == KH_RHS_FACTORED)
      rk4_step<KH_RHS_FACTORED, Cnt, Cnt>(Cnt(0.9), x, k, a1, Cnt(0.1), xn, kn);
    else
      rk4_step<KH_RHS_PAPER, Cnt, Cnt>(Cnt(0.9), x, k, a1, Cnt(0.1), xn, kn);
    n_rhs = 3;  // the fourth (first-stage) evaluation is counted by the caller
  }
  g_tally = nullptr;
  out->add = t_rhs.add;
  out->mul = t_rhs.mul;
  out->div = t_rhs.div;
  out->sqrt = t_rhs.sqrt;
  out->step_add = t_step.add - n_rhs * t_rhs.add;
  out->step_mul = t_step.mul - n_rhs * t_rhs.mul;
  out->step_div = t_step.div - n_rhs * t_rhs.div;
  out->step_sqrt = t_step.sqrt - n_rhs * t_rhs.sqrt;
  out->trig = 0;
  return KH_OK;
}

}  // extern "C"
