/*
 * kerrhip.h -- C ABI of the MI355X (gfx950) geodesic integrator.
 *
 * Batched integration of null and time-like geodesics in Cartesian
 * Kerr-Schild coordinates (Chan, Medeiros, Ozel & Psaltis, "GRay2", Sec. 2):
 * one geodesic per GPU lane, state (x^mu, k^mu) with k^mu = dx^mu/dlambda,
 * right-hand side in the regrouped Kerr-Schild form of eq:opt0 / eq:opti
 * (metric def:CKS and its analytic derivatives, no Christoffel table), classic
 * fourth-order Runge-Kutta (Sec. 3) or an adaptive Dormand-Prince 5(4) pair,
 * termination at the horizon or an escape radius (Sec. 4's benchmark
 * workload), equatorial-crossing records, redshift and constants of motion.
 *
 * Units G = c = M = 1.  Every call returns a kh_status (0 = OK).  Per-geodesic
 * numerical failure is a result (status KH_FAILED), not a call error.
 *
 * Memory: every array in kh_state is caller-owned DEVICE memory, contiguous,
 * 8-byte aligned (4-byte for int32), laid out structure-of-arrays as stated.
 * The library never frees or reallocates caller memory.  A kh_ctx owns only
 * its own scratch (work-queue counters, camera table) and is not thread-safe:
 * use one context per concurrently used stream.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).
 * kh_init_*, kh_integrate and kh_rhs are asynchronous with respect to the host;
 * kh_read_state and kh_stats synchronise the stream and report asynchronous
 * faults of earlier work on it.  Argument errors are detected on the host
 * before any launch and return KH_EINVAL with a message in kh_last_error.
 */
#ifndef KERRHIP_H
#define KERRHIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KH_OK = 0,
  KH_EINVAL = -1,       /* bad argument (checked before any launch) */
  KH_EHIP = -2,         /* HIP runtime error; text in kh_last_error */
  KH_EUNSUPPORTED = -3, /* valid but unsupported combination */
  KH_ENOMEM = -4        /* context scratch allocation failed */
} kh_status;

/* Per-geodesic status (kh_state.status). */
enum {
  KH_ACTIVE = 0,    /* still integrating */
  KH_CAPTURED = 1,  /* r < r_h_factor * r_H after an accepted step */
  KH_ESCAPED = 2,   /* r > r_escape and dr/dlambda > 0 after an accepted step */
  KH_T_END = 3,     /* landed on x^0 = t_end (time-like runs) */
  KH_MAX_STEPS = 4, /* paused after max_steps accepted steps; resumable */
  KH_FAILED = 5     /* NaN state, step-size underflow or invalid initial data */
};

/* Geodesic kind (kh_state.kind).  Null rays are traced future-directed in the
 * chart with spin -a (the time reverse of the physical photon, which keeps the
 * Boyer-Lindquist spatial path and stays regular at the future horizon of the
 * ingoing chart); time-like geodesics run forward in the chart with spin +a. */
enum { KH_NULL = 0, KH_TIMELIKE = 1 };

enum { KH_RK4 = 0, KH_DOPRI5 = 1, KH_DOPRI5_T = 2 }; /* kh_params.method */
enum { KH_P64 = 0, KH_P32 = 1, KH_PMIXED = 2 };  /* kh_params.precision */
enum { KH_RHS_FACTORED = 0, KH_RHS_PAPER = 1 };  /* kh_params.rhs_form */
enum { KH_RHS_BL = 2 };  /* Boyer-Lindquist chart: kh_rk4_fixed, kh_pack_fixed and kh_flops only */
enum { KH_SOA = 0, KH_AOS = 1 };                 /* kh_fixed_params.layout */

typedef struct kh_ctx kh_ctx;

/* An image plane (Sec. 4: rays start on an image at large radius and are
 * integrated backwards toward the hole).  Observer direction
 * n = (sin incl, 0, cos incl); screen axes e_alpha = (0, 1, 0),
 * e_beta = (-cos incl, 0, sin incl).  Pixel (row, col) has
 * alpha = alpha_min + (col + 1/2)(alpha_max - alpha_min)/width and
 * beta = beta_min + (row + 1/2)(beta_max - beta_min)/height; the ray starts at
 * r_obs n + alpha e_alpha + beta e_beta with spatial momentum -n and its k^0
 * from the null condition.  Ray id within the image = row * width + col. */
typedef struct {
  double a;      /* physical spin, -1 <= a <= 1 */
  double r_obs;  /* distance of the image plane (Cartesian), > 0 */
  double incl;   /* inclination, radians */
  double alpha_min, alpha_max, beta_min, beta_max;
  int32_t width, height; /* pixels, > 0 */
} kh_camera;

/* Geodesic state: caller-owned device arrays, n geodesics. */
typedef struct {
  int64_t n;        /* number of geodesics, 1 <= n < 2^31 */
  double *s;        /* [8][n]: x^0 (= t), x^1..x^3, k^0..k^3 of the chart */
  double *spin;     /* [n]: physical spin a of each geodesic */
  int32_t *kind;    /* [n]: KH_NULL or KH_TIMELIKE */
  double *h;        /* [n]: next DOPRI5 step (<= 0: choose h0); resume data */
  double *lam;      /* [n]: affine parameter reached */
  double *phi;      /* [n]: unwrapped Cartesian azimuth atan2(y, x) (kept up to date when crossings are recorded) */
  int32_t *status;  /* [n]: KH_ACTIVE ... KH_FAILED */
  int32_t *n_acc;   /* [n]: accepted steps, cumulative over calls */
  int32_t *n_rej;   /* [n]: rejected DOPRI5 attempts, cumulative */
  double *cross;    /* [n][k_cross][3] = (r, phi, g) of equatorial crossings, or NULL.  g = nu_obs / nu_em
                       for an emitter on the Keplerian circular orbit about +z, Omega = 1/(r^{3/2} + a)
                       with the physical spin a (prograde for a >= 0, retrograde for a < 0): g =
                       1 / (u^t (1 - Omega xi)), xi = L_z / E of the photon; NaN where that orbit does
                       not exist (r^{3/2} - 3 r^{1/2} + 2a <= 0) */
  int32_t *n_cross; /* [n]: crossings seen (may exceed k_cross), or NULL */
  int32_t k_cross;  /* 0..8 crossing slots per geodesic */
  double *c0;       /* [4][n] = (E, L_z, Q, mu^2) at initialisation, or NULL */
  double *c1;       /* [4][n] = the same at the end of the last integrate call, or NULL */
  int32_t *order;   /* [ceil(n / 64)] or NULL: tiles of 64 consecutive ray ids (tile t = ids 64t .. 64t + 63)
                       in the order kh_integrate hands them out; NULL = natural order.  kh_init_rays writes
                       it longest-expected-first (see there), the other init calls write the natural order.
                       A caller-written order must be a permutation of the tile numbers; entries out of range
                       are skipped by the integrator (their rays are then not integrated). */
  int32_t n_out;         /* dense output (method (ii) of Sec. 2.2): number of target coordinate times, 0 = none */
  const double *t_out;   /* [n_out] ascending coordinate times, device memory, or NULL when n_out == 0 */
  double *s_out;         /* [n][n_out][8]: (x^mu, k^mu) of each geodesic at t_out[j], taken from the cubic
                            Hermite interpolant of the step that reaches t_out[j] (DOPRI5 methods); in
                            coordinate time k^0 is fixed by the entry energy as on exit.  kh_integrate writes
                            the targets in [t at entry, t at exit] (a target equal to the entry time gets the
                            entry state) and leaves every other entry untouched. */
  int32_t *perm;    /* [n] or NULL: a per-geodesic schedule, which replaces `order` when set: position q of
                       the work queue is geodesic perm[q].  The init calls write it longest-expected-first
                       (see kh_init_geodesics); a caller-written perm must be a permutation of 0 .. n-1
                       (entries out of range are skipped; a repeated entry makes two lanes race on one
                       geodesic, with undefined results but no access outside the state).  Use it for
                       geodesic sets in no particular order (particles); `order` keeps the 64 rays of a
                       wave adjacent in memory, which suits images. */
} kh_state;

/* Integration rules.  Defaults (kh_default_params): DOPRI5, FP64,
 * h_coeff 0.01, rtol = atol = 1e-8, hmax_coeff 0.1, r_h_factor 1.01,
 * r_escape 1000, t_end 0 (off), r_fp64 3, max_steps 1e6, mixed_split 0. */
typedef struct {
  int32_t method;    /* KH_RK4 (fixed step h = h_coeff * r), KH_DOPRI5, or KH_DOPRI5_T: Dormand-Prince in
                        coordinate time (below) */
  int32_t precision; /* KH_P64, KH_P32 (rtol, atol raised to >= 1e-6), KH_PMIXED */
  int32_t rhs_form;  /* KH_RHS_FACTORED (default) or KH_RHS_PAPER */
  int32_t k_cross;   /* crossing slots to fill, 0..state.k_cross */
  double h_coeff;    /* RK4 step / DOPRI5 first step: h = h_coeff * scale(r) */
  double rtol, atol; /* DOPRI5 tolerances, > 0 */
  double hmax_coeff; /* DOPRI5 step cap h <= hmax_coeff * scale(r) */
  double r_h_factor; /* capture radius factor, r_H = 1 + sqrt(1 - a^2) */
  double r_escape;   /* escape radius */
  double t_end;      /* > 0: stop and land on x^0 = t_end (DOPRI5 only) */
  double r_fp64;     /* KH_PMIXED: the radius inside which right-hand sides are evaluated in FP64 (by the whole
                        wave, or by the second pass of the two-queue split; see mixed_split) */
  int64_t max_steps; /* accepted steps per call before KH_MAX_STEPS (> 0) */
  int32_t block_size;   /* threads per block: 64, 128, 192 or 256; 0 = 256 */
  int32_t grid_blocks;  /* persistent grid size; 0 = fill the device from the occupancy query */
  int32_t refill_min;   /* a wave refills once at least this many lanes are idle (1..64); 0 = 12 */
  int32_t waves_per_eu; /* register budget of the kernel variant (minimum waves per SIMD): 1 = two or more
                           waves; DOPRI5 with the factored form also has 3 and 4 (FP64 / mixed; 3 only for the
                           first pass of the two-queue split, whose FP64 pass always uses 1) and 4 and 5 (FP32);
                           coordinate-time mixed has 3; 0 = default (3 for mixed-precision DOPRI5, else 1) */
  int32_t queue_parts;  /* work-queue partitions of the ray range (1..8); 0 = 8, one per XCD: chunks of 8192
                           ids are dealt round-robin to the partitions, a wave starts on its XCD's partition
                           and steals from the others when it is drained */
  int32_t mixed_split;  /* KH_PMIXED with a DOPRI5 method: 0 = per-wave switch (a wave evaluates its right-hand
                           sides and stage sums in FP64 while any of its lanes is inside r_fp64, else in FP32);
                           1 = two-queue split: a first pass integrates every geodesic with FP32 right-hand sides
                           and stage sums until it comes inside r_fp64, where it is parked, and a second pass
                           continues the parked geodesics in FP64 to the end of the call (two launches and two
                           finalize passes on the stream).  With 1 each geodesic's result depends on no other
                           geodesic, as in FP64 and FP32; max_steps and the attempt limit apply to each pass.
                           Must be 0 for other precisions (KH_EINVAL) and for KH_RK4 (KH_EUNSUPPORTED). */
} kh_params;
/* KH_DOPRI5_T (the coordinate-time subsection of Sec. 2.2): the six-variable
 * state (x^i, v^i = dx^i/dt) is integrated in t with dv^i/dt = a^i - a^0 v^i,
 * where a^mu is the affine right-hand side at k = (1, v).  Same tableau and
 * controller; the error norm is the RMS over the six components; h is a
 * coordinate-time step.  With t_end > 0 the step that would pass t_end is
 * clipped onto it (status KH_T_END, x^0 == t_end exactly).  The state is
 * read and written in the affine form: k^mu = k^0 (1, v^i) with k^0 fixed by
 * the energy E = -k_t of the state the call started from (E is kept exactly;
 * L_z, Q and mu^2 in c1 show the drift).  lam is not advanced.  Factored RHS
 * only.
 *
 * scale(r) = r for null geodesics and r^{3/2} for time-like ones.  DOPRI5
 * controller: accept if err <= 1 (err = RMS over the 8 components of
 * (y5 - y4) / (atol + rtol max(|y_n|, |y_n+1|))), next step
 * h min(5, max(0.2, 0.9 err^{-1/5})) with no growth right after a rejection,
 * then capped; a step below 1e-12 h_coeff scale(r) is KH_FAILED. */

/* Algorithmic operation counts, from the right-hand side template instantiated
 * with a counting scalar (an FMA counts as one mul and one add). */
typedef struct {
  int64_t add, mul, div, sqrt; /* per right-hand-side evaluation */
  int64_t step_add, step_mul;  /* per DOPRI5 attempt (or RK4 step) outside the RHS */
  int64_t step_div, step_sqrt;
  int64_t trig;                /* sin and cos evaluations per RHS (Boyer-Lindquist form only) */
} kh_flop_counts;

/* Create a context on `device` (HIP ordinal).  *out receives the handle. */
kh_status kh_create(kh_ctx **out, int device);
/* Free a context and its scratch.  NULL is accepted. */
kh_status kh_destroy(kh_ctx *ctx);
/* Message for the last failed call on ctx (valid until the next call). */
const char *kh_last_error(const kh_ctx *ctx);
/* Fill *p with the defaults listed above. */
void kh_default_params(kh_params *p);

/* Initial states of the rays of n_cams images (host array `cams`), concatenated
 * in camera order: the rays of camera c occupy ids [off_c, off_c + w_c h_c).
 * If st->order is set, the call also orders the 64-ray tiles for integration,
 * longest first: a ray near the critical curve circles the hole many times
 * and takes several times the median number of steps, so it has to start
 * early or the launch waits for it at the end.  Each ray's priority is how
 * close its radial potential R(r) = (r^2 + a^2 - a xi)^2 - Delta (eta + (xi - a)^2)
 * (xi = L_z / E, eta = Q / E^2) comes to a double root between the horizon and
 * r = 5, on a log scale; a tile takes the maximum over its rays and the tiles
 * are counting-sorted on that key (the order within a key is unspecified).  The
 * results of kh_integrate do not depend on the order, only its run time.
 * st->perm, if set, gets the per-ray form of the same key (see
 * kh_init_geodesics) and then takes precedence over the tile order.
 * Requires st->n == sum of width*height.  Writes s, spin, kind (KH_NULL),
 * h = 0, lam = 0, phi = atan2(y, x), status, n_acc = n_rej = 0, n_cross = 0,
 * cross = NaN and c0.  The camera table is copied to the context (one small
 * host-to-device copy on `stream`).  cams == NULL reuses the table of the last
 * call on this context (same n_cams): then the call is one kernel launch and
 * may be captured into a HIP graph (then two launches with st->order set; the
 * context's tile-key buffer must already be large enough, i.e. an earlier call
 * outside capture had at least as many rays); a captured launch reads the
 * context's table when the graph is replayed, so upload no other table on
 * that context while the graph is in use. */
kh_status kh_init_rays(kh_ctx *ctx, const kh_camera *cams, int32_t n_cams, kh_state *st, void *stream);

/* Rays with individual parameters (device arrays [n]): physical spin, inclination,
 * alpha, beta; common image distance r_obs.  Same outputs as kh_init_rays;
 * st->order gets the natural order and st->perm, if set, the ray-by-ray
 * longest-first schedule of kh_init_geodesics. */
kh_status kh_init_rays_list(kh_ctx *ctx, const double *spin, const double *incl, const double *alpha,
                            const double *beta, double r_obs, kh_state *st, void *stream);

/* Geodesics from positions x3 [3][n] and spins [n] (device): the initial data
 * of Sec. 3.2's time-like orbits (a particle given by its position and
 * coordinate velocity) and of null rays started anywhere.  KH_TIMELIKE: v3
 * [3][n] is the coordinate velocity dx^i/dt and u^0 = 1/sqrt(-g_ab v^a v^b) with
 * v^0 = 1, the normalisation of the four-velocity in the metric def:CKS
 * (status KH_FAILED where that norm is not negative).  KH_NULL: v3 is
 * the spatial momentum and k^0 the future root of the null condition.
 * st->order gets the natural order.  If st->perm is set, the call also writes
 * a per-geodesic schedule, longest expected integration first, so that the
 * launch does not end waiting for a few long geodesics started late: each
 * geodesic gets a key (0 .. 255) and perm lists the geodesics by descending
 * key (the order within a key is unspecified; kh_integrate's results do not
 * depend on it).  Time-like key: the orbital time scale, the semi-major axis
 * 1 / (2 (1 - E)) of a Newtonian orbit of the same binding energy (E = -u_t),
 * on a log scale with 16 steps per octave, shorter first (steps to a fixed
 * t_end scale as its power -3/2); unbound geodesics (E >= 1) get key 0.  Null
 * key: the radial-potential priority of kh_init_rays, per ray. */
kh_status kh_init_geodesics(kh_ctx *ctx, int32_t kind, const double *spin, const double *x3, const double *v3,
                            kh_state *st, void *stream);

/* Integrate every geodesic whose status is KH_ACTIVE or KH_MAX_STEPS until it
 * terminates or takes max_steps accepted steps in this call: the geodesic
 * equation eq:geo with its right-hand side in the form of eq:opt0 / eq:opti
 * (Sec. 2.1), stepped by RK4 (Sec. 3) or the Dormand-Prince 5(4) pair, in the
 * affine parameter or (KH_DOPRI5_T) in coordinate time as in eq:geo_t
 * (Sec. 2.2), terminated as in Sec. 4's benchmark (horizon, escape radius).  Asynchronous; no
 * allocation and no host synchronisation.  Re-entrant: a paused state resumes
 * exactly (bitwise) where it stopped.  Persistent kernel: each 64-lane wave
 * takes rays from a global counter and refills retired lanes, in the order of
 * st->perm if set, else of st->order if set, else of the ray ids; the order
 * changes the run time only, never a result (for KH_PMIXED with the per-wave
 * switch, mixed_split = 0, a result can depend on which rays share a wave).
 * With mixed_split = 1 the call enqueues two such launches (see kh_params). */
kh_status kh_integrate(kh_ctx *ctx, const kh_params *p, kh_state *st, void *stream);

/* kh_integrate for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels, launch and results (bitwise), with no context.  It runs on the
 * calling thread's current device and calls no hipMalloc, hipFree or other
 * allocating routine.  Its only scratch is the work-queue counters, kept in a
 * static device array of 16 64-bit counters (128 B) per GPU, held until the
 * process ends; a call uses 8 of them whatever st->n is, so no state is too
 * large for it, and queue_parts above 8 is refused with KH_EINVAL.  The first
 * call on a device looks up that device's copy of the array
 * (hipGetSymbolAddress); make it outside graph capture.  Every call on one
 * GPU shares that array and each launch clears it first, so calls that
 * overlap on one GPU (two streams, two threads) race: serialise them.
 * Errors: the kh_integrate codes; the message (empty on success) is written
 * to err, truncated to err_len bytes (err may be NULL). */
kh_status kh_integrate_noalloc(const kh_params *p, kh_state *st, void *stream, char *err, int32_t err_len);

/* Copy rays [first, first + count) to the host: host_s [count][8] (AoS, may be
 * NULL), host_status [count] (may be NULL).  The rows are packed on the device
 * in chunks of up to 2^20 rays, in context scratch of up to 64 MiB allocated
 * on first use, and copied straight into host_s.  Synchronises the stream. */
kh_status kh_read_state(kh_ctx *ctx, const kh_state *st, int64_t first, int64_t count, double *host_s,
                        int32_t *host_status, void *stream);

/* Reduce the state on the device: out[0..5] = count per status, out[6] = sum of
 * n_acc, out[7] = sum of n_rej.  Synchronises the stream. */
kh_status kh_stats(kh_ctx *ctx, const kh_state *st, int64_t out[8], void *stream);

/* Same reduction as kh_stats, asynchronously into caller device memory
 * d_out [8] (int64); no host synchronisation, so it may be captured in a graph. */
kh_status kh_stats_device(kh_ctx *ctx, const kh_state *st, int64_t *d_out, void *stream);

/* Evaluate the right-hand side (the 4 accelerations d k^mu / d lambda) at n
 * points: spin_chart [n] is the chart spin, s [8][n] the states, acc [4][n]
 * the output (device arrays).  precision KH_P64 or KH_P32; rhs_form as in
 * kh_params. */
kh_status kh_rhs(kh_ctx *ctx, int32_t precision, int32_t rhs_form, const double *spin_chart, const double *s,
                 double *acc, int64_t n, void *stream);

/* Operation counts of the right-hand side and of one step (host only).
 * rhs_form KH_RHS_BL is accepted with method KH_RK4. */
kh_status kh_flops(int32_t method, int32_t rhs_form, kh_flop_counts *out);

/* ---------------------------------------------------------------------------
 * Fixed-step RK4 in either chart: the workload of the comparison of Sec. 4
 * (tab:elapse), which times RK4 steps of fixed rule on the same rays in
 * Cartesian Kerr-Schild and in Boyer-Lindquist coordinates (the line element
 * at the start of Sec. 2.1), with the state stored structure-of-arrays or
 * array-of-structures, in single or double precision.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t rhs_form;  /* KH_RHS_FACTORED or KH_RHS_PAPER: Cartesian Kerr-Schild states
                        (t, x, y, z, k^t, k^x, k^y, k^z); KH_RHS_BL: Boyer-Lindquist states
                        (t, r, theta, phi, k^t, k^r, k^theta, k^phi) */
  int32_t layout;    /* KH_SOA: component c of geodesic i at y[c n + i]; KH_AOS: at y[8 i + c] */
  int32_t precision; /* KH_P64: y holds doubles; KH_P32: floats, and all arithmetic in FP32 */
  int32_t nsteps;    /* steps per geodesic in this call, >= 0 */
  double spin;       /* chart spin a, common to every geodesic; |a| < 1 */
  double h_coeff;    /* step h = h_coeff * r, r at the start of the step; > 0 */
  double r_stop;     /* KH_CAPTURED once r < r_stop after a step */
  double r_escape;   /* KH_ESCAPED once r > r_escape and dr/dlambda > 0 after a step */
} kh_fixed_params;

/* Up to p->nsteps classic RK4 steps (four right-hand-side evaluations each, no
 * error control) for every geodesic i < n with status[i] == KH_ACTIVE.  After
 * each step: a NaN component makes it KH_FAILED, then the r_stop and r_escape
 * tests apply (r is the Boyer-Lindquist radius in both charts); steps[i] is
 * increased by the steps taken.  y: device array of 8 n values in p's
 * precision and layout (8-byte, or 4-byte for FP32, aligned); status, steps:
 * device int32 [n].  One geodesic per lane and no refill, so a wave runs as
 * long as its longest geodesic.  Asynchronous; allocates nothing.  Calls
 * resume exactly where the previous one stopped.  KH_EINVAL for bad
 * arguments (checked before any launch). */
kh_status kh_rk4_fixed(kh_ctx *ctx, const kh_fixed_params *p, void *y, int32_t *status, int32_t *steps,
                       int64_t n, void *stream);

/* Kerr-Schild states s (device double [8][n], as kh_state.s) converted to the
 * chart, precision and layout of p and written to y (device, 8 n values); for
 * the Kerr-Schild forms a copy.  KH_RHS_BL (needs |p->spin| < 1 and every r
 * above the outer horizon): r from eq:CKSr, theta = atan2(sqrt(x^2 + y^2) /
 * sqrt(r^2 + a^2), z / r), phi = atan2(y, x) - atan2(a, r) - G(r),
 * t = T - F(r), with F(r) = int 2r/Delta dr and G(r) = int a/Delta dr (the
 * ingoing Kerr-Schild shifts, integration constants as in
 * 2 (r_+ ln|r - r_+| - r_- ln|r - r_-|) / (r_+ - r_-) and
 * a ln|(r - r_+)/(r - r_-)| / (r_+ - r_-)); the momentum by the inverse
 * Jacobian of that map.  Conversion in FP64, then rounded to p's precision. */
kh_status kh_pack_fixed(kh_ctx *ctx, const kh_fixed_params *p, const double *s, void *y, int64_t n,
                        void *stream);

#ifdef __cplusplus
}
#endif
#endif /* KERRHIP_H */
