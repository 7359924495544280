/*
 * kerrhip_mlp.h -- learned surrogate for the geodesic integrator (C ABI).
 *
 * A multilayer perceptron maps (alpha, beta, a, inclination) of an image ray
 * to its first equatorial crossing (log r, azimuth, redshift) plus a capture
 * logit.  It is trained on rays the integrator of kerrhip.h produces and is
 * evaluated with integrator fallback on the rays it is unsure about.  None of
 * this is in the GRay2 paper; it accelerates the image workload of its Sec. 4.
 *
 * Network: 4 -> 256 -> 256 -> 256 -> 256 -> 4, SiLU on the hidden layers,
 * linear output; 199,684 parameters.  Matrix products run on the BF16 matrix
 * cores (MFMA) with FP32 accumulation; FP32 master weights and Adam moments.
 *
 * Parameter vector (FP32, caller-owned device memory, KH_MLP_NPARAMS floats):
 * W0 [256][4], b0 [256], W1 [256][256], b1, W2 [256][256], b2, W3 [256][256],
 * b3, W4 [4][256], b4 [4]   (W_l[out][in]).
 *
 * Inputs are normalised inside the kernels: (alpha/12, beta/12, (a - 0.5)/0.5,
 * (incl_deg - 45)/40).  Outputs are normalised targets: ((log r - 2)/2,
 * phi/pi, (g - 0.8)/0.3, capture logit).
 *
 * Same conventions as kerrhip.h: kh_status return codes, caller-owned device
 * arrays, `stream` = hipStream_t as void*, asynchronous unless stated.
 */
#ifndef KERRHIP_MLP_H
#define KERRHIP_MLP_H

#include <stdint.h>

#include "kerrhip.h"

#ifdef __cplusplus
extern "C" {
#endif

#define KH_MLP_NPARAMS 199684
#define KH_MLP_WB_ELEMS 208896  /* padded BF16 weights, forward layout */
#define KH_MLP_WBT_ELEMS 204800 /* padded BF16 transposed weights (layers 1..4) */

typedef struct {
  float *params;   /* [KH_MLP_NPARAMS] FP32 master weights */
  float *adam_m;   /* [KH_MLP_NPARAMS] Adam first moment (training only, else NULL) */
  float *adam_v;   /* [KH_MLP_NPARAMS] Adam second moment (training only, else NULL) */
  uint16_t *wb;    /* [KH_MLP_WB_ELEMS] BF16 copies in the forward layout (per layer 16-input
                      blocks [padded rows][16]; written by kh_mlp_sync and the training step) */
  uint16_t *wbt;   /* [KH_MLP_WBT_ELEMS] BF16 transposed copies (training only, else NULL) */
} kh_mlp;

typedef struct {
  float lr, beta1, beta2, eps; /* Adam hyper-parameters */
  int32_t step;                /* 1-based step count for bias correction */
} kh_adam;

typedef struct {
  float r, phi, g, capture; /* weights of the four loss terms (see kh_mlp_grad); all >= 0 */
} kh_mlp_loss_w;

/* Bytes of the training workspace for batches of up to max_batch rays
 * (max_batch a multiple of 256). */
int64_t kh_mlp_work_bytes(int32_t max_batch);

/* Refresh the BF16 copies (wb, and wbt if not NULL) from the FP32 master
 * weights (after the caller initialises or loads params). */
kh_status kh_mlp_sync(kh_ctx *ctx, const kh_mlp *net, void *stream);

/* Raw network outputs y [m][4] (normalised targets, capture logit) for raw
 * features x [m][4] = (alpha, beta, a, incl_radians), FP32 device arrays. */
kh_status kh_mlp_forward(kh_ctx *ctx, const kh_mlp *net, const float *x, float *y, int64_t m, void *stream);

/* Which pixels of a surrogate image go back to the integrator (any rule that
 * holds sends the pixel). */
typedef struct {
  float tau;         /* capture uncertain: tau < p_capture < 1 - tau; tau in [0, 0.5) */
  float shadow_band; /* near the shadow edge: within this distance (M, image plane) of the
                        critical curve of the camera's spin and inclination (Bardeen's closed
                        form for a distant observer; a face-on camera, sin(incl) < 1e-3, sees
                        the circle of the photon orbit with L_z = 0); 0 = off */
  float r_min;       /* strong field: predicted first crossing inside r_min (M) and
                        p_capture <= 1/2, where the crossing radius and the redshift change
                        fastest across the image; 0 = off */
} kh_mlp_fallback;

/* The surrogate image of one camera: out [w*h][4] = (r, phi, g, p_capture)
 * decoded from the network, pixel order as kh_init_rays.  Pixels that a rule
 * of *fb selects are appended (in any order) to fallback_ids (device int32,
 * capacity w*h) and counted in *fallback_count (device int32, zeroed by the
 * call).  fb is a host struct (required). */
kh_status kh_mlp_image(kh_ctx *ctx, const kh_mlp *net, const kh_camera *cam, const kh_mlp_fallback *fb, float *out,
                       int32_t *fallback_ids, int32_t *fallback_count, void *stream);

/* Training data from integrated rays: st (with one crossing slot or more) and
 * the rays' (alpha, beta, a, incl) device arrays [n] -> x [n][4] raw features,
 * t [n][4] normalised targets (capture in t[.][3] as 0/1) and mask [n]:
 * bit 0 = a crossing exists (log r and phi valid), bit 1 = its redshift is finite. */
kh_status kh_mlp_targets(kh_ctx *ctx, const kh_state *st, const double *alpha, const double *beta,
                         const double *spin, const double *incl, float *x, float *t, uint8_t *mask, void *stream);

/* Gradient of the mean loss over a batch of b rays (b a multiple of 256, at
 * most the workspace's max_batch) into grad [KH_MLP_NPARAMS] (FP32 device),
 * and the batch loss into *loss (device float; accumulated, caller zeroes).
 * Loss per ray: mask0 (w.r (y0 - t0)^2 + w.phi (y1 - t1)^2) + mask1 w.g
 * (y2 - t2)^2 + w.capture BCE(sigmoid(y3), t3), with the weights of *lw (a
 * host struct; NULL = all 1; KH_EINVAL unless each is in [0, 1e6)). */
kh_status kh_mlp_grad(kh_ctx *ctx, const kh_mlp *net, void *work, int32_t max_batch, const float *x, const float *t,
                      const uint8_t *mask, int32_t b, const kh_mlp_loss_w *lw, float *grad, float *loss,
                      void *stream);

/* One Adam step on a batch: gradient as kh_mlp_grad, then the update of params,
 * moments and BF16 copies. */
kh_status kh_mlp_train_step(kh_ctx *ctx, const kh_mlp *net, void *work, int32_t max_batch, const float *x,
                            const float *t, const uint8_t *mask, int32_t b, const kh_mlp_loss_w *lw,
                            const kh_adam *opt, float *loss, void *stream);

/* Rays of the listed pixels of one camera: st->n = number of ids in pix
 * (device int32 [st->n]), same outputs as kh_init_rays; st->order and
 * st->perm, where set, get the natural order.  May be captured in a graph. */
kh_status kh_init_rays_pixels(kh_ctx *ctx, const kh_camera *cam, const int32_t *pix, kh_state *st, void *stream);

/* Write integrated rays into an image in the surrogate's format:
 * out[pix[i]] = (r, phi, g of the first crossing (NaN if none), captured 0/1)
 * for i < st->n; pix == NULL means pix[i] = i. */
kh_status kh_image_from_state(kh_ctx *ctx, const kh_state *st, const int32_t *pix, float *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* KERRHIP_MLP_H */
