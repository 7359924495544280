// mlp.hip -- the surrogate network (include/kerrhip_mlp.h) on the BF16 matrix cores.
//
// Every product is written as D^T = W X^T: the weight tile is the MFMA A
// operand (32 output features x 16 inputs, read straight from L2: the BF16
// copy stores each layer in 16-input k-blocks [rows][16], so one k-step's
// fragment is 1 KB of consecutive memory) and the activations are the B operand
// (16 inputs x 32 rays).  The 32x32 accumulator then holds, per lane, four
// consecutive output features of one ray, so bias, SiLU and the BF16 store of
// the next activation row are one 8-byte write.  In every kernel the waves of
// a block split each layer's 256 outputs and share the block's activations in
// LDS rows [ray][feature]: inference (k_mlp_fwd_pp) with 128 rays per group
// of four waves, training (k_mlp_fwd_train, k_mlp_bwd) with 32, because a
// training batch is only a few thousand rays.
//
// MFMA operand layout used (v_mfma_f32_32x32x16_bf16, 64 lanes):
//   A[i][k]: lane l holds i = l % 32, k = 8 (l / 32) + j, j = 0..7
//   B[k][n]: lane l holds n = l % 32, k = 8 (l / 32) + j
//   D[i][n]: lane l, element e holds i = 8 (e / 4) + 4 (l / 32) + e % 4, n = l % 32
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "internal.hpp"
#include "kerrhip_mlp.h"

using namespace khi;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NP = KH_MLP_NPARAMS;
constexpr int HID = 256;
constexpr int RAYS = 32;        // rays per wave
constexpr int LDA = HID + 8;    // LDS row stride (BF16) of the activation tile
constexpr int SPLITS = 16;      // batch splits of the weight-gradient products (a multiple of 8)
static_assert(SPLITS % 8 == 0, "two or more whole splits per XCD");
constexpr int HT0_ROWS = 32;    // input features padded to one 32-row tile

// FP32 parameter offsets: W_l [out][in], then b_l.
__device__ __constant__ int OFF_W[5] = {0, 1280, 67072, 132864, 198656};
__device__ __constant__ int OFF_B[5] = {1024, 66816, 132608, 198400, 199680};
constexpr int h_OFF_W[5] = {0, 1280, 67072, 132864, 198656};
constexpr int h_OFF_B[5] = {1024, 66816, 132608, 198400, 199680};
constexpr int IN_DIM[5] = {4, 256, 256, 256, 256};
constexpr int OUT_DIM[5] = {256, 256, 256, 256, 4};
// BF16 forward copies: layer l is [MPAD_l][KPAD_l] with zero padding.
constexpr int KPAD[5] = {16, 256, 256, 256, 256};
constexpr int MPAD[5] = {256, 256, 256, 256, 32};
constexpr int OFF_WB[5] = {0, 4096, 69632, 135168, 200704};
// BF16 transposed copies W^T of layers 1..4 (rows: the 256 inputs; k: the
// padded outputs) in 16-output k-blocks: element (i, o) at wb_index(256, i, o).
constexpr int OFF_WBT[5] = {0, 0, 65536, 131072, 196608};

// Element (o, i) of the forward copy of a layer with mpad padded rows: the
// inputs are cut into 16-wide k-blocks stored one after another, each
// [mpad][16], so the A fragment of one k-step (32 rows x 16 inputs) is 1 KB of
// consecutive memory and a wave's weight reads use whole cache lines.
__host__ __device__ constexpr int wb_index(int mpad, int o, int i) { return (i >> 4) * (mpad * 16) + o * 16 + (i & 15); }
static_assert(OFF_WB[4] + 32 * 256 == KH_MLP_WB_ELEMS, "forward copy size");
static_assert(OFF_WBT[4] + 256 * 32 == KH_MLP_WBT_ELEMS, "transposed copy size");

// Input and target normalisation.
__device__ inline void norm_features(float alpha, float beta, float a, float incl, float f[4]) {
  f[0] = alpha * (1.0f / 12.0f);
  f[1] = beta * (1.0f / 12.0f);
  f[2] = (a - 0.5f) * 2.0f;
  f[3] = (incl * (180.0f / 3.14159265358979f) - 45.0f) * (1.0f / 40.0f);
}

// 1 / (1 + e^{-z}) with the hardware reciprocal (~1 ulp; the results are
// stored as BF16): an IEEE division would cost ~10 instructions per activation.
// Limits as the division: z -> -inf gives 0, z -> +inf gives 1.
__device__ inline float sigmoidf(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ inline float silu(float z) { return z * sigmoidf(z); }
__device__ inline float dsilu(float z) {
  const float s = sigmoidf(z);
  return s * (1.0f + z * (1.0f - s));
}

// Layer-0 B operand of one ray: the four features in two BF16 terms each,
// hi = bf16(f) in k = 0..3 and lo = bf16(f - hi) in k = 4..7 (the forward
// weight copy repeats W0 in columns 4..7), so the product sees the features
// to ~2^-16 instead of 2^-8: at BF16 alone an image coordinate would be
// quantised to 12 x 2^-8 = 0.047 M over |alpha| in [6, 12], several pixels of
// a 4096^2 image.  Lanes of the upper half hold k = 8..15 (zero).
__device__ inline bf16x8 input_operand(const float f[4], int half) {
  bf16x8 bx;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const __bf16 hi = (__bf16)f[j];
    const __bf16 lo = (__bf16)(f[j] - (float)hi);
    bx[j] = half == 0 ? hi : (__bf16)0.0f;
    bx[4 + j] = half == 0 ? lo : (__bf16)0.0f;
  }
  return bx;
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ inline f32x16 mfma(const bf16x8& a, const bf16x8& b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

constexpr int kCritBins = 256;  // angle bins of the critical-curve table

struct FwdArgs {
  const float* params;
  const __bf16* wb;
  const float* x;  // raw features [m][4] (forward and training)
  int64_t m;
  kh_camera cam;   // mode 1
  float* y;        // raw outputs [m][4], or the decoded image (camera mode)
  float tau;       // camera mode fallback rules (kh_mlp_fallback)
  float crit_band;
  float r_min;
  float crit_ac;                // centre (crit_ac, 0) of the critical-curve table
  float crit_r[kCritBins];      // its radius in equal angle bins over (-pi, pi]
  int32_t* fb_ids;
  int32_t* fb_count;
  float* z;    // training: pre-activations [4][bmax][256]
  __bf16* ht;  // training: HT_0 [32][bmax], then HT_1..HT_4 [256][bmax]
  int64_t bmax;
  // training loss (k_mlp_fwd_train; dz4 NULL = no loss): targets [m][4],
  // mask [m], weights; gradient dz4 [bmax][32] and dz4T [32][bmax]; sum
  const float* t;
  const uint8_t* mask;
  kh_mlp_loss_w wl;
  __bf16* dz4;
  __bf16* dz4T;
  float* loss;
};

__host__ __device__ inline __bf16* ht_layer(__bf16* ht, int l, int64_t bmax) {
  return l == 0 ? ht : ht + (int64_t)HT0_ROWS * bmax + (int64_t)(l - 1) * HID * bmax;
}


// Image-plane coordinates of the centre of pixel `ray` (< 2^31) of a camera.
__device__ inline void pixel_coords(const kh_camera& cam, int64_t ray, float& al, float& be) {
  const uint32_t id = (uint32_t)ray, wdt = (uint32_t)cam.width;
  const uint32_t row = id / wdt, col = id - row * wdt;
  al = (float)(cam.alpha_min + (col + 0.5) * (cam.alpha_max - cam.alpha_min) / cam.width);
  be = (float)(cam.beta_min + (row + 0.5) * (cam.beta_max - cam.beta_min) / cam.height);
}

// Output layer (256 -> 4, padded to 32 rows) of one ray tile whose
// activations are the LDS rows rows[32][LDA] (ray = tile's first ray + r), and
// in camera mode the decode; returns whether the ray goes to the fallback list.
template <int MODE>
__device__ inline bool output_tile(const FwdArgs& A, const __bf16* rows, int64_t ray, int r, int half) {
  const f32x16 zero = {};
  const bool valid = ray < A.m;
  f32x16 o = zero;
  for (int ks = 0; ks < HID / 16; ++ks) {
    const bf16x8 bv = *reinterpret_cast<const bf16x8*>(rows + r * LDA + ks * 16 + 8 * half);
    const bf16x8 aw = *reinterpret_cast<const bf16x8*>(A.wb + OFF_WB[4] + wb_index(32, r, ks * 16 + 8 * half));
    o = mfma(aw, bv, o);
  }
  bool unsure = false;
  if (half == 0 && valid) {
    const float* b4 = A.params + OFF_B[4];
    f32x4 y;
#pragma unroll
    for (int q = 0; q < 4; ++q) y[q] = o[q] + b4[q];
    if (MODE == 1) {
      const float pc = sigmoidf(y[3]);
      f32x4 d;
      d[0] = __expf(2.0f * y[0] + 2.0f);
      d[1] = 3.14159265358979f * y[1];
      d[2] = 0.3f * y[2] + 0.8f;
      d[3] = pc;
      *reinterpret_cast<f32x4*>(A.y + ray * 4) = d;
      // the integrator takes the pixel when the capture is uncertain, when it
      // lies near the critical curve (shadow edge), or when its predicted first
      // crossing is deep in the potential well, where r and g change fastest
      unsure = pc > A.tau && pc < 1.0f - A.tau;
      unsure = unsure || (pc <= 0.5f && d[0] < A.r_min);
      if (A.crit_band > 0.0f) {
        float al, be;
        pixel_coords(A.cam, ray, al, be);
        const float da = al - A.crit_ac;
        const float u = (atan2f(be, da) + 3.14159265358979f) * (kCritBins / (2.0f * 3.14159265358979f)) - 0.5f;
        const float fl = floorf(u);
        const float fr = u - fl;
        const int k0 = ((int)fl + kCritBins) % kCritBins, k1 = (k0 + 1) % kCritBins;
        const float rc = A.crit_r[k0] + fr * (A.crit_r[k1] - A.crit_r[k0]);
        unsure = unsure || fabsf(sqrtf(da * da + be * be) - rc) < A.crit_band;
      }
    } else {
      *reinterpret_cast<f32x4*>(A.y + ray * 4) = y;
    }
  }
  return unsure;
}

// Barrier for LDS hand-offs only: waits for this wave's LDS operations, not
// for its global loads or atomics, which stay in flight across it.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Inference forward, ping-pong: a block of eight waves holds two groups of
// four (waves 0-3 and 4-7; the waves of a block go to the four SIMDs in
// turn, so waves w and w + 4 share a SIMD and each SIMD holds one wave of
// each group).  A group carries 128 rays: its wave w
// computes outputs 64 w .. 64 w + 63 of every hidden layer for all 128 rays
// (2 x 4 accumulator tiles), and the group's activations sit in LDS rows
// [ray][feature], read by its four waves.  A group's work on one batch is eight steps that
// alternate between the VALU (input features, layer 0 and its SiLU epilogue;
// the epilogues of layers 1..3) and the matrix cores (the products of layers
// 1..3; the output layer); group 1 runs one step behind group 0 with a block
// barrier after every step, so on every SIMD one wave feeds the matrix core
// while the other issues transcendentals.  The block is persistent: its k-th
// batch in group g is the 128 rays from 128 (2 (blockIdx + k gridDim) + g).
// A wave that ends an epilogue requests the first PP_AHEAD k-steps of its next
// layer's weights, so its products start without waiting for L2; the biases of
// layers 0..3 sit in LDS and enter as the first k-step's accumulator; in the
// output step each wave also computes the input features of its ray tile of
// the group's next batch (into LDS), and the fallback list entry of a tile is
// written one step after its atomic.
constexpr int PP_AHEAD = 2;  // weight k-steps in flight
template <int MODE>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_mlp_fwd_pp(FwdArgs A, int32_t nb) {
  __shared__ __attribute__((aligned(16))) __bf16 act_all[2 * 4 * RAYS * LDA];
  __shared__ __attribute__((aligned(16))) float bias_s[4 * HID];
  __shared__ __attribute__((aligned(16))) f32x4 feat_s[2][4 * RAYS];  // features of each group's next batch
  const int tid = threadIdx.x, grp = tid >> 8, w = (tid >> 6) & 3, lane = tid & 63, r = lane & 31, half = lane >> 5;
  __bf16* act = act_all + grp * (4 * RAYS * LDA);
  auto batch_base = [&](int64_t k) { return ((int64_t)(blockIdx.x + k * gridDim.x) * 2 + grp) * (4 * RAYS); };
  // the normalised input features of this wave's ray tile of the batch at b0
  auto features = [&](int64_t b0) {
    if (half == 0) {
      const int64_t ray = b0 + 32 * w + r;
      float f[4] = {0.f, 0.f, 0.f, 0.f};
      if (ray < A.m) {
        if (MODE == 1) {
          float al, be;
          pixel_coords(A.cam, ray, al, be);
          norm_features(al, be, (float)A.cam.a, (float)A.cam.incl, f);
        } else {
          const f32x4 xv = *reinterpret_cast<const f32x4*>(A.x + ray * 4);
          norm_features(xv[0], xv[1], xv[2], xv[3], f);
        }
      }
      feat_s[grp][32 * w + r] = f32x4{f[0], f[1], f[2], f[3]};
    }
  };
  for (int i = tid; i < 4 * HID; i += 512) {
    const int l = i / HID;
    bias_s[i] = A.params[(l == 0 ? OFF_B[0] : l == 1 ? OFF_B[1] : l == 2 ? OFF_B[2] : OFF_B[3]) + i % HID];
  }
  features(batch_base(0));
  __syncthreads();

  f32x16 acc[2][4];
  bf16x8 ar[PP_AHEAD + 1][2];  // weight fragments of consecutive k-steps (ring)
  // fallback list entry pending from the last output step
  unsigned long long p_mask = 0;
  int p_slot = 0;
  int64_t p_ray = 0;
  bool p_unsure = false;

  // accumulator tile tt of a layer's bias (per lane: outputs (2 w + tt) 32 +
  // 8 g + 4 half + q of element 4 g + q)
  auto bias_tile = [&](int l, int tt) {
    f32x16 bt;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const f32x4 b = *reinterpret_cast<const f32x4*>(bias_s + l * HID + (2 * w + tt) * 32 + 8 * g + 4 * half);
#pragma unroll
      for (int q = 0; q < 4; ++q) bt[4 * g + q] = b[q];
    }
    return bt;
  };
  auto wrow = [&](int l, int tt) {
    return A.wb + (l == 1 ? OFF_WB[1] : l == 2 ? OFF_WB[2] : OFF_WB[3]) + wb_index(HID, (2 * w + tt) * 32 + r, 8 * half);
  };
  auto prefetch = [&](int l) {
#pragma unroll
    for (int q = 0; q < PP_AHEAD; ++q)
#pragma unroll
      for (int tt = 0; tt < 2; ++tt) ar[q][tt] = *reinterpret_cast<const bf16x8*>(wrow(l, tt) + q * HID * 16);
  };
  auto epilogue = [&]() {
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int m0 = (2 * w + tt) * 32 + 8 * g + 4 * half;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          bf16x4 hv;
#pragma unroll
          for (int q = 0; q < 4; ++q) hv[q] = (__bf16)silu(acc[tt][n][4 * g + q]);
          *reinterpret_cast<bf16x4*>(act + (32 * n + r) * LDA + m0) = hv;
        }
      }
  };
  auto flush_fallback = [&]() {
    if (MODE == 1 && p_mask) {
      const int leader = __ffsll((long long)p_mask) - 1;
      const int slot = __shfl(p_slot, leader);
      if (p_unsure) {
        const unsigned rank =
            __builtin_amdgcn_mbcnt_hi((unsigned)(p_mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)p_mask, 0u));
        A.fb_ids[slot + rank] = (int32_t)p_ray;
      }
      p_mask = 0;
    }
  };

  const int32_t steps = 8 * nb;
  for (int32_t s = 0; s <= steps; ++s) {
    const int32_t t = s - grp;
    const int64_t base = batch_base(t >> 3);
    flush_fallback();
    if (t >= 0 && t < steps && base < A.m) {
      const int j = t & 7;
      if (j == 0) {
        // layer 0 (K = 4 features as two BF16 terms, padded to 16) on the
        // features the group's waves left in LDS during the previous step
        const f32x16 bt0 = bias_tile(0, 0), bt1 = bias_tile(0, 1);
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          const f32x4 fv = feat_s[grp][32 * n + r];
          const float f[4] = {fv[0], fv[1], fv[2], fv[3]};
          const bf16x8 bx = input_operand(f, half);
#pragma unroll
          for (int tt = 0; tt < 2; ++tt) {
            const bf16x8 aw =
                *reinterpret_cast<const bf16x8*>(A.wb + OFF_WB[0] + wb_index(256, (2 * w + tt) * 32 + r, 8 * half));
            acc[tt][n] = mfma(aw, bx, tt == 0 ? bt0 : bt1);
          }
        }
        epilogue();
        prefetch(1);
      } else if (j == 7) {
        const int64_t ray = base + 32 * w + r;
        const bool unsure = output_tile<MODE>(A, act + 32 * w * LDA, ray, r, half);
        features(batch_base((t >> 3) + 1));
        if (MODE == 1) {
          p_mask = __ballot(unsure);
          if (p_mask) {
            const int leader = __ffsll((long long)p_mask) - 1;
            if (lane == leader) p_slot = atomicAdd(A.fb_count, __popcll(p_mask));
          }
          p_unsure = unsure;
          p_ray = ray;
        }
      } else if (j & 1) {
        // products of hidden layer l = 1..3 over the group's 128 rays; the
        // first PP_AHEAD k-steps of weights are in flight since the epilogue
        const int l = (j + 1) >> 1;
        const __bf16* arow0 = wrow(l, 0);
        const __bf16* arow1 = wrow(l, 1);
        bf16x8 bcur[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) bcur[n] = *reinterpret_cast<const bf16x8*>(act + (32 * n + r) * LDA + 8 * half);
        const f32x16 bt0 = bias_tile(l, 0), bt1 = bias_tile(l, 1);
#pragma unroll
        for (int ks = 0; ks < HID / 16; ++ks) {
          if (ks + PP_AHEAD < HID / 16) {
            ar[(ks + PP_AHEAD) % (PP_AHEAD + 1)][0] =
                *reinterpret_cast<const bf16x8*>(arow0 + (ks + PP_AHEAD) * HID * 16);
            ar[(ks + PP_AHEAD) % (PP_AHEAD + 1)][1] =
                *reinterpret_cast<const bf16x8*>(arow1 + (ks + PP_AHEAD) * HID * 16);
          }
          bf16x8 bnext[4];
#pragma unroll
          for (int n = 0; n < 4; ++n)
            bnext[n] = ks + 1 < HID / 16
                           ? *reinterpret_cast<const bf16x8*>(act + (32 * n + r) * LDA + (ks + 1) * 16 + 8 * half)
                           : bcur[n];
          // keep the scheduler from sinking the loads to their uses
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int n = 0; n < 4; ++n) {
            acc[0][n] = mfma(ar[ks % (PP_AHEAD + 1)][0], bcur[n], ks == 0 ? bt0 : acc[0][n]);
            acc[1][n] = mfma(ar[ks % (PP_AHEAD + 1)][1], bcur[n], ks == 0 ? bt1 : acc[1][n]);
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int n = 0; n < 4; ++n) bcur[n] = bnext[n];
        }
      } else {
        epilogue();  // SiLU of layer j / 2 into the group's rows
        if (j < 6) prefetch((j >> 1) + 1);
      }
    }
    lds_barrier();
  }
  flush_fallback();
}

// Loss of one ray and its gradient with respect to the raw outputs, written
// as the BF16 row dz [32] (columns 4..31 zero) and column dzT [32][bmax]:
// mask bit 0: w.r (y0 - t0)^2 + w.phi (y1 - t1)^2; mask bit 1: w.g (y2 - t2)^2;
// always w.capture BCE(sigmoid(y3), t3); the mean over the b rays of the batch.
__device__ inline float ray_loss(const f32x4& yv, const f32x4& tv, int mk, int64_t b, const kh_mlp_loss_w& wl,
                                 __bf16* dz, __bf16* dzT, int64_t bmax, int64_t i) {
  const float inv = 1.0f / (float)b;
  const float e0 = (mk & 1) ? yv[0] - tv[0] : 0.0f;
  const float e1 = (mk & 1) ? yv[1] - tv[1] : 0.0f;
  const float e2 = (mk & 2) ? yv[2] - tv[2] : 0.0f;
  const float s = sigmoidf(yv[3]);
  const float bce = fmaxf(yv[3], 0.0f) - yv[3] * tv[3] + log1pf(__expf(-fabsf(yv[3])));
  const float l = wl.r * (e0 * e0) + wl.phi * (e1 * e1) + wl.g * (e2 * e2) + wl.capture * bce;
  const float d[4] = {2.0f * wl.r * e0 * inv, 2.0f * wl.phi * e1 * inv, 2.0f * wl.g * e2 * inv,
                      wl.capture * (s - tv[3]) * inv};
#pragma unroll
  for (int c = 0; c < 32; ++c) {
    const __bf16 v = (__bf16)(c < 4 ? d[c] : 0.0f);
    dz[i * 32 + c] = v;
    dzT[(int64_t)c * bmax + i] = v;
  }
  return l;
}

// Training forward for batches of a few thousand rays: a block of four waves
// carries one tile of 32 rays and each wave computes 64 of a layer's 256
// outputs (two accumulator tiles), so a batch of b rays keeps b / 8 waves
// busy instead of b / 32.  The tile's activations live in LDS ([ray][feature]
// rows, double-buffered: one barrier per layer).  Saves what the backward
// pass needs: pre-activations z and the transposed BF16 activations.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) k_mlp_fwd_train(FwdArgs A) {
  __shared__ __attribute__((aligned(16))) __bf16 act[2][RAYS * LDA];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, r = lane & 31, half = lane >> 5;
  const int64_t ray = (int64_t)blockIdx.x * RAYS + r;
  const bool valid = ray < A.m;

  float f[4] = {0.f, 0.f, 0.f, 0.f};
  if (valid) {
    const f32x4 xv = *reinterpret_cast<const f32x4*>(A.x + ray * 4);
    norm_features(xv[0], xv[1], xv[2], xv[3], f);
  }
  const bf16x8 bx = input_operand(f, half);
  // the weight gradient of layer 0 uses the leading BF16 term of each feature
  if (w == 0 && valid) {
    __bf16* ht0 = ht_layer(A.ht, 0, A.bmax);
#pragma unroll
    for (int j = 0; j < 16; ++j)
      ht0[(int64_t)(16 * half + j) * A.bmax + ray] = (half == 0 && j < 4) ? (__bf16)f[j & 3] : (__bf16)0.0f;
  }
  // the targets of the loss, requested long before the output layer needs them
  f32x4 tv = {0.f, 0.f, 0.f, 0.f};
  int mk = 0;
  if (A.dz4 && w == 0 && half == 0 && valid) {
    tv = *reinterpret_cast<const f32x4*>(A.t + ray * 4);
    mk = A.mask[ray];
  }
  // A batch keeps one wave per SIMD busy, so nothing hides a load's latency:
  // all 32 weight fragments of a layer are requested together, those of the
  // next layer as soon as this layer's products are issued (they arrive during
  // the epilogue and the barrier).
  bf16x8 aw[HID / 16][2];
  auto load_layer = [&](int l) {
    const __bf16* wl = A.wb + (l == 1 ? OFF_WB[1] : l == 2 ? OFF_WB[2] : OFF_WB[3]);
#pragma unroll
    for (int ks = 0; ks < HID / 16; ++ks)
#pragma unroll
      for (int tt = 0; tt < 2; ++tt)
        aw[ks][tt] = *reinterpret_cast<const bf16x8*>(wl + wb_index(HID, (2 * w + tt) * 32 + r, ks * 16 + 8 * half));
  };
  load_layer(1);
  const f32x16 zero = {};
  f32x16 acc[2];
#pragma unroll
  for (int tt = 0; tt < 2; ++tt) {
    const int t = 2 * w + tt;
    const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(A.wb + OFF_WB[0] + (t * 32 + r) * KPAD[0] + 8 * half);
    acc[tt] = mfma(a0, bx, zero);
  }
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    if (l > 0) {
      const __bf16* in = act[(l - 1) & 1];
#pragma unroll
      for (int tt = 0; tt < 2; ++tt) acc[tt] = zero;
#pragma unroll
      for (int ks = 0; ks < HID / 16; ++ks) {
        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(in + r * LDA + ks * 16 + 8 * half);
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) acc[tt] = mfma(aw[ks][tt], bv, acc[tt]);
      }
      __builtin_amdgcn_sched_barrier(0);
      if (l < 3) {
        load_layer(l + 1);
      } else if (w == 0) {
#pragma unroll
        for (int ks = 0; ks < HID / 16; ++ks)
          aw[ks][0] = *reinterpret_cast<const bf16x8*>(A.wb + OFF_WB[4] + wb_index(32, r, ks * 16 + 8 * half));
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // bias, SiLU, the next activation rows and the saved tensors of this wave's outputs
    const float* bias = A.params + OFF_B[l];
    __bf16* out = act[l & 1];
    __bf16* ht = ht_layer(A.ht, l + 1, A.bmax);
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int m0 = (2 * w + tt) * 32 + 8 * g + 4 * half;
        const f32x4 b = *reinterpret_cast<const f32x4*>(bias + m0);
        f32x4 zz;
        bf16x4 hv;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          zz[q] = acc[tt][4 * g + q] + b[q];
          hv[q] = (__bf16)silu(zz[q]);
        }
        *reinterpret_cast<bf16x4*>(out + r * LDA + m0) = hv;
        if (valid) {
          *reinterpret_cast<f32x4*>(A.z + ((int64_t)l * A.bmax + ray) * HID + m0) = zz;
#pragma unroll
          for (int q = 0; q < 4; ++q) ht[(int64_t)(m0 + q) * A.bmax + ray] = hv[q];
        }
      }
    }
    __syncthreads();  // the layer's activation rows are complete
  }

  // output layer (256 -> 4, padded to 32 rows), one wave; then the loss of
  // the tile's rays and its gradient with respect to the raw outputs
  if (w == 0) {
    const __bf16* in = act[1];
    f32x16 o = zero;
#pragma unroll
    for (int ks = 0; ks < HID / 16; ++ks) {
      const bf16x8 bv = *reinterpret_cast<const bf16x8*>(in + r * LDA + ks * 16 + 8 * half);
      o = mfma(aw[ks][0], bv, o);
    }
    float lsum = 0.0f;
    if (half == 0 && valid) {
      const float* b4 = A.params + OFF_B[4];
      f32x4 y;
#pragma unroll
      for (int q = 0; q < 4; ++q) y[q] = o[q] + b4[q];
      *reinterpret_cast<f32x4*>(A.y + ray * 4) = y;
      if (A.dz4) lsum = ray_loss(y, tv, mk, A.m, A.wl, A.dz4, A.dz4T, A.bmax, ray);
    }
    if (A.dz4) {
      for (int off = 32; off > 0; off >>= 1) lsum += __shfl_down(lsum, off);
      if (lane == 0) atomicAdd(A.loss, lsum / (float)A.m);
    }
  }
}

// Arguments of one layer's backward launch (k_mlp_bwd): its weight-gradient
// tasks and, except for layer 0, its input-gradient ray tiles.
struct BwdLayer {
  // weight and bias gradient: dz^T [opad][bmax] (BF16), h^T [ipad][bmax]
  const __bf16* dzT;
  int opad, nout;
  const __bf16* ht;
  int ipad, nin, tiles;  // tiles = (opad / 32) (ipad / 32)
  int64_t bmax, b;
  float* part;
  int off_w, off_b;
  // input gradient: W^T (k-blocks), dz [bmax][opad], the layer below's z
  const __bf16* wbt;
  const __bf16* dz;
  const float* zprev;
  __bf16* dz_out;
  __bf16* dzT_out;
  int ndx;  // ray tiles (blocks) of the input gradient, a multiple of 8
};

// Gradient with respect to a layer's input, times SiLU' of the layer below,
// dz_out[ray][k] = (sum_o dz[ray][o] W[o][k]) * silu'(zprev[ray][k]), for ray
// tile `blk` (one 32-ray tile per block; wave w computes input features
// 64 w .. 64 w + 63); every fragment is requested before the first product
// (one wave per SIMD).
template <int OPAD>
__device__ inline void bwd_dx_tile(const BwdLayer& L, int blk, int w, int lane) {
  const __bf16* wbt = L.wbt;
  const __bf16* dz = L.dz;
  const float* zprev = L.zprev;
  __bf16* dz_out = L.dz_out;
  __bf16* dzT_out = L.dzT_out;
  const int64_t bmax = L.bmax;
  const int r = lane & 31, half = lane >> 5;
  const int64_t ray = (int64_t)blk * RAYS + r;
  f32x16 acc[2];
  const f32x16 zero = {};
#pragma unroll
  for (int tt = 0; tt < 2; ++tt) acc[tt] = zero;
  bf16x8 aw[OPAD / 16][2], bv[OPAD / 16];
#pragma unroll
  for (int os = 0; os < OPAD / 16; ++os) {
    bv[os] = *reinterpret_cast<const bf16x8*>(dz + ray * OPAD + os * 16 + 8 * half);
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
      aw[os][tt] = *reinterpret_cast<const bf16x8*>(wbt + wb_index(HID, (2 * w + tt) * 32 + r, os * 16 + 8 * half));
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int os = 0; os < OPAD / 16; ++os)
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) acc[tt] = mfma(aw[os][tt], bv[os], acc[tt]);
#pragma unroll
  for (int tt = 0; tt < 2; ++tt) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int k0 = (2 * w + tt) * 32 + 8 * g + 4 * half;
      const f32x4 zz = *reinterpret_cast<const f32x4*>(zprev + ray * HID + k0);
      bf16x4 dv;
#pragma unroll
      for (int q = 0; q < 4; ++q) dv[q] = (__bf16)(acc[tt][4 * g + q] * dsilu(zz[q]));
      *reinterpret_cast<bf16x4*>(dz_out + ray * HID + k0) = dv;
#pragma unroll
      for (int q = 0; q < 4; ++q) dzT_out[(int64_t)(k0 + q) * bmax + ray] = dv[q];
    }
  }
}

// Split-batch partial weight and bias gradients of one layer:
// part[s][W_l + o * nin + i] = sum over split s of dz[b][o] h[b][i],
// part[s][b_l + o] = sum over split s of dz[b][o].
// Task j (0 .. 2 tiles - 1) of XCD xcd: workgroups go to the 8 XCDs
// round-robin by linear id, and each XCD takes two whole batch splits (all
// output tiles of them), so that an XCD's L2 holds only its 1/8 of dz^T and h
// instead of every tile's re-read of all of it.
__device__ inline void bwd_dw_task(const BwdLayer& L, int xcd, int j, int lane) {
  const __bf16* dzT = L.dzT;
  const __bf16* ht = L.ht;
  const int nout = L.nout, ipad = L.ipad, nin = L.nin, tiles = L.tiles, off_w = L.off_w, off_b = L.off_b;
  const int64_t bmax = L.bmax, b = L.b;
  float* part = L.part;
  const int r = lane & 31, half = lane >> 5;
  const int tiles_i = ipad / 32;
  const int s = xcd * (SPLITS / 8) + j / tiles;
  const int tile = j % tiles;
  const int ot = tile / tiles_i, it = tile % tiles_i;
  const int64_t per = b / SPLITS;
  const int64_t b0 = s * per, b1 = b0 + per;
  f32x16 acc = {};
  const __bf16* arow = dzT + (int64_t)(ot * 32 + r) * bmax + 8 * half;
  const __bf16* brow = ht + (int64_t)(it * 32 + r) * bmax + 8 * half;
  int64_t kb = b0;
  // sixteen k-steps' fragments are loaded before their products, so sixteen
  // L2 round trips overlap; the accumulation order is unchanged
  for (; kb + 256 <= b1; kb += 256) {
    bf16x8 aw[16], bv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      aw[u] = *reinterpret_cast<const bf16x8*>(arow + kb + 16 * u);
      bv[u] = *reinterpret_cast<const bf16x8*>(brow + kb + 16 * u);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 16; ++u) acc = mfma(aw[u], bv[u], acc);
  }
  for (; kb < b1; kb += 16) acc = mfma(*reinterpret_cast<const bf16x8*>(arow + kb), *reinterpret_cast<const bf16x8*>(brow + kb), acc);
  float* ps = part + (int64_t)s * NP;
  const int i = it * 32 + r;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int o = ot * 32 + 8 * (e / 4) + 4 * half + (e % 4);
    if (o < nout && i < nin) ps[off_w + o * nin + i] = acc[e];
  }
  if (it == 0) {
    // bias gradient: each half of the wave sums half of the split in order,
    // eight values per 16-byte load (per is a multiple of 16)
    const int o = ot * 32 + r;
    const int64_t mid = b0 + per / 2;
    const __bf16* row = dzT + (int64_t)o * bmax;
    float sb = 0.0f;
    int64_t kb = half ? mid : b0;
    const int64_t ke = half ? b1 : mid;
    for (; kb + 128 <= ke; kb += 128) {
      bf16x8 v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = *reinterpret_cast<const bf16x8*>(row + kb + 8 * u);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < 16; ++u)
#pragma unroll
        for (int j = 0; j < 8; ++j) sb += (float)v[u][j];
    }
    for (; kb < ke; kb += 8) {
      const bf16x8 v = *reinterpret_cast<const bf16x8*>(row + kb);
#pragma unroll
      for (int j = 0; j < 8; ++j) sb += (float)v[j];
    }
    sb += __shfl_down(sb, 32);
    if (half == 0 && o < nout) ps[off_b + o] = sb;
  }
}

// One layer's backward pass in one launch: blocks 0 .. ndx - 1 compute the
// input gradient of a ray tile each, the rest four weight-gradient tasks each
// (the two parts are independent, so their latencies overlap).
template <int OPAD, bool DX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) k_mlp_bwd(BwdLayer L) {
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  int blk = blockIdx.x;
  if (DX) {
    if (blk < L.ndx) {
      bwd_dx_tile<OPAD>(L, blk, w, lane);
      return;
    }
    blk -= L.ndx;  // ndx is a multiple of 8: blk % 8 is still the block's XCD
  }
  bwd_dw_task(L, blk % 8, (blk / 8) * 4 + w, lane);
}

__device__ inline int layer_of(int p) {
  return p < 1280 ? 0 : p < 67072 ? 1 : p < 132864 ? 2 : p < 198656 ? 3 : 4;
}

// BF16 copies of one FP32 weight (biases have none).
__device__ inline void write_bf16(int p, float w, __bf16* wb, __bf16* wbt) {
  const int l = layer_of(p);
  const int rel = p - OFF_W[l];
  const int nin = l == 0 ? 4 : 256;
  const int nw = (l == 0 || l == 4) ? 1024 : 65536;
  if (rel >= nw) return;  // a bias
  const int o = rel / nin, i = rel % nin;
  const int offwb = l == 0 ? 0 : l == 1 ? 4096 : l == 2 ? 69632 : l == 3 ? 135168 : 200704;
  const int mpad = l == 4 ? 32 : 256;
  wb[offwb + wb_index(mpad, o, i)] = (__bf16)w;
  if (l == 0) wb[offwb + wb_index(mpad, o, 4 + i)] = (__bf16)w;  // the lo terms of the split inputs
  if (wbt && l >= 1) {
    // W^T of the layer: rows are the 256 inputs, k the (padded) outputs,
    // stored in 16-output k-blocks [256][16]
    const int offwbt = (l - 1) * 65536;
    wbt[offwbt + wb_index(HID, i, o)] = (__bf16)w;
  }
}

__global__ void k_zero_i32(int32_t* p) {
  if (threadIdx.x == 0) *p = 0;
}

__global__ void k_mlp_fill_bf16(__bf16* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (__bf16)0.0f;
}

__global__ void k_mlp_sync(const float* params, __bf16* wb, __bf16* wbt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NP) write_bf16(p, params[p], wb, wbt);
}

__global__ void k_mlp_reduce(const float* part, float* grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  float g = 0.0f;
  for (int s = 0; s < SPLITS; ++s) g += part[(int64_t)s * NP + p];
  grad[p] = g;
}

__global__ void k_mlp_adam(float* params, float* m, float* v, const float* part, kh_adam opt, __bf16* wb,
                           __bf16* wbt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  float g = 0.0f;
  for (int s = 0; s < SPLITS; ++s) g += part[(int64_t)s * NP + p];
  const float mm = opt.beta1 * m[p] + (1.0f - opt.beta1) * g;
  const float vv = opt.beta2 * v[p] + (1.0f - opt.beta2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float c1 = 1.0f - powf(opt.beta1, (float)opt.step);
  const float c2 = 1.0f - powf(opt.beta2, (float)opt.step);
  const float w = params[p] - opt.lr * (mm / c1) / (sqrtf(vv / c2) + opt.eps);
  params[p] = w;
  write_bf16(p, w, wb, wbt);
}

// Training data from an integrated state.
__global__ void k_mlp_targets(KState S, const double* alpha, const double* beta, const double* spin,
                              const double* incl, float* x, float* t, uint8_t* mask) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  f32x4 xv;
  xv[0] = (float)alpha[i];
  xv[1] = (float)beta[i];
  xv[2] = (float)spin[i];
  xv[3] = (float)incl[i];
  *reinterpret_cast<f32x4*>(x + i * 4) = xv;
  const bool cross = S.n_cross && S.n_cross[i] > 0 && S.k_cross > 0;
  const double r = cross ? S.cross[i * 3 * S.k_cross + 0] : 0.0;
  const double phi = cross ? S.cross[i * 3 * S.k_cross + 1] : 0.0;
  const double g = cross ? S.cross[i * 3 * S.k_cross + 2] : 0.0;
  const bool rok = cross && r > 0.0 && isfinite(r) && isfinite(phi);
  const bool gok = rok && isfinite(g);
  f32x4 tv;
  tv[0] = rok ? (float)((log(r) - 2.0) * 0.5) : 0.0f;
  tv[1] = rok ? (float)(phi / M_PI) : 0.0f;
  tv[2] = gok ? (float)((g - 0.8) / 0.3) : 0.0f;
  tv[3] = S.status[i] == KH_CAPTURED ? 1.0f : 0.0f;
  *reinterpret_cast<f32x4*>(t + i * 4) = tv;
  mask[i] = (uint8_t)((rok ? 1 : 0) | (gok ? 2 : 0));
}

__global__ void k_image_from_state(KState S, const int32_t* pix, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  const int64_t p = pix ? pix[i] : i;
  const bool cross = S.n_cross && S.n_cross[i] > 0 && S.k_cross > 0;
  f32x4 v;
  v[0] = cross ? (float)S.cross[i * 3 * S.k_cross + 0] : __builtin_nanf("");
  v[1] = cross ? (float)S.cross[i * 3 * S.k_cross + 1] : __builtin_nanf("");
  v[2] = cross ? (float)S.cross[i * 3 * S.k_cross + 2] : __builtin_nanf("");
  v[3] = S.status[i] == KH_CAPTURED ? 1.0f : 0.0f;
  *reinterpret_cast<f32x4*>(out + p * 4) = v;
}

// Workspace carving (bytes, 256-aligned pieces).
struct Work {
  float* y;
  float* z;
  __bf16* ht;
  __bf16 *dz_a, *dz_b, *dz4;
  __bf16 *dzT_a, *dzT_b, *dz4T;
  float* part;
};

int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

Work carve(void* base, int64_t bmax, int64_t* total) {
  char* p = static_cast<char*>(base);
  int64_t off = 0;
  Work w{};
  auto take = [&](int64_t bytes) {
    char* q = p ? p + off : nullptr;
    off += align256(bytes);
    return q;
  };
  w.y = reinterpret_cast<float*>(take(bmax * 4 * 4));
  w.z = reinterpret_cast<float*>(take(4 * bmax * HID * 4));
  w.ht = reinterpret_cast<__bf16*>(take((HT0_ROWS + 4 * HID) * bmax * 2));
  w.dz_a = reinterpret_cast<__bf16*>(take(bmax * HID * 2));
  w.dz_b = reinterpret_cast<__bf16*>(take(bmax * HID * 2));
  w.dz4 = reinterpret_cast<__bf16*>(take(bmax * 32 * 2));
  w.dzT_a = reinterpret_cast<__bf16*>(take(bmax * HID * 2));
  w.dzT_b = reinterpret_cast<__bf16*>(take(bmax * HID * 2));
  w.dz4T = reinterpret_cast<__bf16*>(take(bmax * 32 * 2));
  w.part = reinterpret_cast<float*>(take((int64_t)SPLITS * NP * 4));
  if (total) *total = off;
  return w;
}

kh_status check_net(kh_ctx* ctx, const kh_mlp* net, bool train) {
  if (!net || !net->params || !net->wb) return fail(ctx, KH_EINVAL, "network params and wb are required");
  if (!aligned(net->params, 16) || !aligned(net->wb, 16) || !device_ok(net->params) || !device_ok(net->wb))
    return fail(ctx, KH_EINVAL, "network arrays must be 16-byte aligned device memory");
  if (train) {
    const void* ps[] = {net->adam_m, net->adam_v, net->wbt};
    for (const void* q : ps)
      if (!q || !aligned(q, 16) || !device_ok(q))
        return fail(ctx, KH_EINVAL, "training needs adam_m, adam_v and wbt (16-byte aligned device memory)");
  }
  return KH_OK;
}

// Shared body of kh_mlp_grad and kh_mlp_train_step.
kh_status grad_pass(kh_ctx* ctx, const kh_mlp* net, void* work, int32_t max_batch, const float* x, const float* t,
                    const uint8_t* mask, int32_t b, const kh_mlp_loss_w* lw, float* loss, hipStream_t strm,
                    Work* out_w) {
  if (max_batch < 256 || max_batch % 256) return fail(ctx, KH_EINVAL, "max_batch must be a positive multiple of 256");
  if (b < 256 || b % 256 || b > max_batch) return fail(ctx, KH_EINVAL, "b must be a multiple of 256 <= max_batch");
  const void* ins[] = {x, t, mask, loss, work};
  for (const void* q : ins)
    if (!q || !device_ok(q)) return fail(ctx, KH_EINVAL, "x, t, mask, loss and work must be device memory");
  if (!aligned(x, 16) || !aligned(t, 16) || !aligned(work, 256))
    return fail(ctx, KH_EINVAL, "x, t must be 16-byte aligned and work 256-byte aligned");
  kh_mlp_loss_w wl = {1.0f, 1.0f, 1.0f, 1.0f};
  if (lw) {
    wl = *lw;
    const float ws[4] = {wl.r, wl.phi, wl.g, wl.capture};
    for (float v : ws)
      if (!(v >= 0.0f) || !(v < 1e6f)) return fail(ctx, KH_EINVAL, "loss weights must be in [0, 1e6)");
  }
  const int64_t bmax = max_batch;
  Work w = carve(work, bmax, nullptr);
  *out_w = w;
  FwdArgs A{};
  A.params = net->params;
  A.wb = reinterpret_cast<const __bf16*>(net->wb);
  A.x = x;
  A.m = b;
  A.y = w.y;
  A.z = w.z;
  A.ht = w.ht;
  A.bmax = bmax;
  A.t = t;
  A.mask = mask;
  A.wl = wl;
  A.dz4 = w.dz4;
  A.dz4T = w.dz4T;
  A.loss = loss;
  hipLaunchKernelGGL(k_mlp_fwd_train, dim3((unsigned)(b / RAYS)), dim3(256), 0, strm, A);
  const __bf16* wbt = reinterpret_cast<const __bf16*>(net->wbt);
  auto ht = [&](int l) { return ht_layer(w.ht, l, bmax); };
  auto zl = [&](int l) { return w.z + (int64_t)l * bmax * HID; };
  const int ndx = (int)(b / RAYS);
  // one launch per layer: the layer's weight gradient (split over the batch,
  // 4 tiles per block) beside the gradient of its input
  auto layer = [&](int l, const __bf16* dzT, const __bf16* dz, __bf16* dz_out, __bf16* dzT_out) {
    BwdLayer L{};
    L.dzT = dzT;
    L.opad = l == 4 ? 32 : 256;
    L.nout = l == 4 ? 4 : 256;
    L.ht = ht(l);
    L.ipad = l == 0 ? 32 : 256;
    L.nin = l == 0 ? 4 : 256;
    L.tiles = (L.opad / 32) * (L.ipad / 32);
    L.bmax = bmax;
    L.b = b;
    L.part = w.part;
    L.off_w = h_OFF_W[l];
    L.off_b = h_OFF_B[l];
    L.ndx = l == 0 ? 0 : ndx;
    if (l > 0) {
      L.wbt = wbt + OFF_WBT[l];
      L.dz = dz;
      L.zprev = zl(l - 1);
      L.dz_out = dz_out;
      L.dzT_out = dzT_out;
    }
    const dim3 grid((unsigned)(L.ndx + 4 * L.tiles));
    if (l == 4)
      hipLaunchKernelGGL((k_mlp_bwd<32, true>), grid, dim3(256), 0, strm, L);
    else if (l > 0)
      hipLaunchKernelGGL((k_mlp_bwd<256, true>), grid, dim3(256), 0, strm, L);
    else
      hipLaunchKernelGGL((k_mlp_bwd<256, false>), grid, dim3(256), 0, strm, L);
  };
  layer(4, w.dz4T, w.dz4, w.dz_a, w.dzT_a);
  __bf16* cur = w.dz_a;
  __bf16* curT = w.dzT_a;
  __bf16* nxt = w.dz_b;
  __bf16* nxtT = w.dzT_b;
  for (int l = 3; l >= 1; --l) {
    layer(l, curT, cur, nxt, nxtT);
    std::swap(cur, nxt);
    std::swap(curT, nxtT);
  }
  layer(0, curT, nullptr, nullptr, nullptr);  // inputs padded to one 32-row tile
  KH_HIP(ctx, hipGetLastError());
  return KH_OK;
}

}  // namespace

extern "C" {

int64_t kh_mlp_work_bytes(int32_t max_batch) {
  if (max_batch < 256 || max_batch % 256) return -1;
  int64_t total = 0;
  carve(nullptr, max_batch, &total);
  return total;
}

kh_status kh_mlp_sync(kh_ctx* ctx, const kh_mlp* net, void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = false;
  kh_status s = check_net(ctx, net, false);
  if (s != KH_OK) return s;
  if (net->wbt && (!aligned(net->wbt, 16) || !device_ok(net->wbt)))
    return fail(ctx, KH_EINVAL, "wbt must be NULL or 16-byte aligned device memory");
  if ((s = set_device(ctx)) != KH_OK) return s;
  hipStream_t strm = (hipStream_t)stream;
  __bf16* wb = reinterpret_cast<__bf16*>(net->wb);
  __bf16* wbt = reinterpret_cast<__bf16*>(net->wbt);
  hipLaunchKernelGGL(k_mlp_fill_bf16, dim3((KH_MLP_WB_ELEMS + 255) / 256), dim3(256), 0, strm, wb,
                     (int64_t)KH_MLP_WB_ELEMS);
  if (wbt)
    hipLaunchKernelGGL(k_mlp_fill_bf16, dim3((KH_MLP_WBT_ELEMS + 255) / 256), dim3(256), 0, strm, wbt,
                       (int64_t)KH_MLP_WBT_ELEMS);
  hipLaunchKernelGGL(k_mlp_sync, dim3((NP + 255) / 256), dim3(256), 0, strm, net->params, wb, wbt);
  KH_HIP(ctx, hipGetLastError());
  return KH_OK;
}

}  // extern "C"

namespace {
// The persistent inference kernel: one eight-wave block per compute unit (its
// 132 KB of LDS leaves no room for a second), nb batches of 128 rays per group.
template <int MODE>
void launch_fwd(const kh_ctx* ctx, const FwdArgs& A, hipStream_t strm) {
  const int64_t pairs = (A.m + 8 * RAYS - 1) / (8 * RAYS);
  const int64_t grid = std::min<int64_t>(std::max(ctx->n_cu, 1), pairs);
  const int32_t nb = (int32_t)((pairs + grid - 1) / grid);
  hipLaunchKernelGGL(k_mlp_fwd_pp<MODE>, dim3((unsigned)grid), dim3(8 * 64), 0, strm, A, nb);
}
}  // namespace

extern "C" {

kh_status kh_mlp_forward(kh_ctx* ctx, const kh_mlp* net, const float* x, float* y, int64_t m, void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = capturing(stream);
  kh_status s = check_net(ctx, net, false);
  if (s != KH_OK) return s;
  if (m < 1 || m >= (int64_t(1) << 31)) return fail(ctx, KH_EINVAL, "m must be in [1, 2^31)");
  if (!x || !y || !aligned(x, 16) || !aligned(y, 16) || !device_ok(x) || !device_ok(y))
    return fail(ctx, KH_EINVAL, "x and y must be 16-byte aligned device arrays [m][4]");
  if ((s = set_device(ctx)) != KH_OK) return s;
  FwdArgs A{};
  A.params = net->params;
  A.wb = reinterpret_cast<const __bf16*>(net->wb);
  A.x = x;
  A.m = m;
  A.y = y;
  launch_fwd<0>(ctx, A, (hipStream_t)stream);
  KH_HIP(ctx, hipGetLastError());
  return KH_OK;
}

}  // extern "C"

namespace {
// The critical curve of a camera (the shadow boundary seen from infinity,
// Bardeen's closed form): photons on spherical orbits of radius r between the
// prograde and retrograde circular photon orbits have xi = L_z / E and
// eta = Q / E^2 from R(r) = R'(r) = 0,
//   xi = (r^2 (3 - r) - a^2 (r + 1)) / (a (r - 1)),
//   eta = r^3 (4 a^2 - r (r - 3)^2) / (a^2 (r - 1)^2),
// and reach the image at alpha = -xi / sin i, beta = +-sqrt(b2),
// b2 = eta + a^2 cos^2 i - xi^2 cot^2 i.  b2 >= 0 holds on one interval of r
// around the orbit with xi = 0, which narrows as the camera turns face-on;
// the curve is sampled on that interval (its ends found by bisection, the
// samples crowded towards them, where beta -> 0) and tabulated as its radius
// around (ac, 0) in kCritBins equal angle bins (it is star-shaped about that
// centre).  a = 0 gives the circle of radius sqrt(27); a face-on camera
// (sin i < 1e-3), which only the xi = 0 orbit reaches, the circle of radius
// sqrt(eta + a^2) of that orbit.  Returns false if the curve cannot be
// formed.
bool critical_curve(double a, double incl, float* ac, float* rad) {
  const double si = std::sin(incl), ci = std::cos(incl);
  if (std::fabs(a) < 1e-9) {
    *ac = 0.0f;
    for (int k = 0; k < kCritBins; ++k) rad[k] = (float)std::sqrt(27.0);
    return true;
  }
  const double aa = std::fabs(a);
  const double r1 = 2.0 * (1.0 + std::cos(2.0 / 3.0 * std::acos(-aa)));
  const double r2 = 2.0 * (1.0 + std::cos(2.0 / 3.0 * std::acos(aa)));
  auto xi = [&](double r) { return (r * r * (3.0 - r) - a * a * (r + 1.0)) / (a * (r - 1.0)); };
  auto eta = [&](double r) {
    return r * r * r * (4.0 * a * a - r * (r - 3.0) * (r - 3.0)) / (a * a * (r - 1.0) * (r - 1.0));
  };
  auto b2 = [&](double r) { return eta(r) + a * a * ci * ci - xi(r) * xi(r) * ci * ci / (si * si); };
  // bisection for the sign change of f on [lo, hi] (f(lo), f(hi) of opposite signs)
  auto bisect = [](auto f, double lo, double hi) {
    const bool neg_lo = f(lo) < 0.0;
    for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
      const double mid = 0.5 * (lo + hi);
      if ((f(mid) < 0.0) == neg_lo)
        lo = mid;
      else
        hi = mid;
    }
    return 0.5 * (lo + hi);
  };
  // the orbit with xi = 0 (xi changes sign between the two photon orbits)
  const double r0 = bisect([&](double r) { return xi(r); }, r1, r2);
  if (std::fabs(si) < 1e-3) {
    const double e0 = eta(r0);
    if (!(e0 + a * a > 0.0)) return false;
    *ac = 0.0f;
    for (int k = 0; k < kCritBins; ++k) rad[k] = (float)std::sqrt(e0 + a * a);
    return true;
  }
  if (!(b2(r0) > 0.0)) return false;
  const double ra = b2(r1) >= 0.0 ? r1 : bisect(b2, r1, r0);
  const double rb = b2(r2) >= 0.0 ? r2 : bisect(b2, r0, r2);
  constexpr int n = 4096;
  std::vector<std::pair<double, double>> pts;  // (alpha, beta)
  pts.reserve(2 * n + 2);
  for (int j = 0; j <= n; ++j) {
    const double r = ra + (rb - ra) * 0.5 * (1.0 - std::cos(M_PI * j / n));
    const double q = b2(r);
    const double bet = q > 0.0 ? std::sqrt(q) : 0.0;
    pts.emplace_back(-xi(r) / si, bet);
    pts.emplace_back(-xi(r) / si, -bet);
  }
  double amin = pts[0].first, amax = pts[0].first;
  for (const auto& q : pts) {
    amin = std::min(amin, q.first);
    amax = std::max(amax, q.first);
  }
  const double c = 0.5 * (amin + amax);
  std::vector<std::pair<double, double>> pol;  // (angle, radius) about (c, 0)
  pol.reserve(pts.size());
  for (const auto& q : pts) pol.emplace_back(std::atan2(q.second, q.first - c), std::hypot(q.first - c, q.second));
  std::sort(pol.begin(), pol.end());
  const int np = (int)pol.size();
  for (int k = 0; k < kCritBins; ++k) {
    const double th = -M_PI + (k + 0.5) * (2.0 * M_PI / kCritBins);
    // first tabulated angle at or after th, and its predecessor (periodic)
    int hi = (int)(std::lower_bound(pol.begin(), pol.end(), std::make_pair(th, -1.0)) - pol.begin());
    const int lo = (hi + np - 1) % np;
    hi %= np;
    double t0 = pol[lo].first, t1 = pol[hi].first;
    if (t0 > th) t0 -= 2.0 * M_PI;
    if (t1 < th) t1 += 2.0 * M_PI;
    const double f = t1 > t0 ? (th - t0) / (t1 - t0) : 0.0;
    rad[k] = (float)(pol[lo].second + f * (pol[hi].second - pol[lo].second));
  }
  *ac = (float)c;
  return true;
}
}  // namespace

extern "C" {

kh_status kh_mlp_image(kh_ctx* ctx, const kh_mlp* net, const kh_camera* cam, const kh_mlp_fallback* fb, float* out,
                       int32_t* fallback_ids, int32_t* fallback_count, void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = capturing(stream);
  kh_status s = check_net(ctx, net, false);
  if (s != KH_OK) return s;
  if (!cam || cam->width < 1 || cam->height < 1 || !(std::fabs(cam->a) <= 1.0))
    return fail(ctx, KH_EINVAL, "camera: need width, height >= 1 and |a| <= 1");
  const int64_t m = int64_t(cam->width) * cam->height;
  if (m >= (int64_t(1) << 31)) return fail(ctx, KH_EINVAL, "image too large");
  if (!fb) return fail(ctx, KH_EINVAL, "fallback rules are required");
  if (!(fb->tau >= 0.0f && fb->tau < 0.5f)) return fail(ctx, KH_EINVAL, "tau must be in [0, 0.5)");
  if (!(fb->shadow_band >= 0.0f && fb->shadow_band < 1e3f) || !(fb->r_min >= 0.0f && fb->r_min < 1e6f))
    return fail(ctx, KH_EINVAL, "shadow_band and r_min must be finite and >= 0");
  const void* ps[] = {out, fallback_ids, fallback_count};
  for (const void* q : ps)
    if (!q || !device_ok(q)) return fail(ctx, KH_EINVAL, "out, fallback_ids, fallback_count must be device memory");
  if (!aligned(out, 16)) return fail(ctx, KH_EINVAL, "out must be 16-byte aligned");
  if ((s = set_device(ctx)) != KH_OK) return s;
  hipStream_t strm = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, strm, fallback_count);
  FwdArgs A{};
  A.params = net->params;
  A.wb = reinterpret_cast<const __bf16*>(net->wb);
  A.m = m;
  A.cam = *cam;
  A.y = out;
  A.tau = fb->tau;
  A.r_min = fb->r_min;
  A.crit_band = 0.0f;
  if (fb->shadow_band > 0.0f && critical_curve(cam->a, cam->incl, &A.crit_ac, A.crit_r)) A.crit_band = fb->shadow_band;
  A.fb_ids = fallback_ids;
  A.fb_count = fallback_count;
  launch_fwd<1>(ctx, A, strm);
  KH_HIP(ctx, hipGetLastError());
  return KH_OK;
}

kh_status kh_mlp_targets(kh_ctx* ctx, const kh_state* st, const double* alpha, const double* beta,
                         const double* spin, const double* incl, float* x, float* t, uint8_t* mask, void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = false;
  kh_status s = check_state(ctx, st, false);
  if (s != KH_OK) return s;
  const void* ps[] = {alpha, beta, spin, incl, x, t, mask};
  for (const void* q : ps)
    if (!q || !device_ok(q)) return fail(ctx, KH_EINVAL, "alpha, beta, spin, incl, x, t, mask must be device memory");
  if (!aligned(x, 16) || !aligned(t, 16)) return fail(ctx, KH_EINVAL, "x and t must be 16-byte aligned");
  if ((s = set_device(ctx)) != KH_OK) return s;
  const KState ks = to_k(st);
  hipLaunchKernelGGL(k_mlp_targets, dim3((unsigned)((st->n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, ks,
                     alpha, beta, spin, incl, x, t, mask);
  KH_HIP(ctx, hipGetLastError());
  return KH_OK;
}

kh_status kh_mlp_grad(kh_ctx* ctx, const kh_mlp* net, void* work, int32_t max_batch, const float* x, const float* t,
                      const uint8_t* mask, int32_t b, const kh_mlp_loss_w* lw, float* grad, float* loss,
                      void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = capturing(stream);
  kh_status s = check_net(ctx, net, false);
  if (s != KH_OK) return s;
  if (!net->wbt || !device_ok(net->wbt)) return fail(ctx, KH_EINVAL, "gradients need wbt");
  if (!grad || !aligned(grad, 16) || !device_ok(grad)) return fail(ctx, KH_EINVAL, "grad must be device memory");
  if ((s = set_device(ctx)) != KH_OK) return s;
  hipStream_t strm = (hipStream_t)stream;
  Work w;
  if ((s = grad_pass(ctx, net, work, max_batch, x, t, mask, b, lw, loss, strm, &w)) != KH_OK) return s;
  hipLaunchKernelGGL(k_mlp_reduce, dim3((NP + 255) / 256), dim3(256), 0, strm, w.part, grad);
  KH_HIP(ctx, hipGetLastError());
  return KH_OK;
}

kh_status kh_mlp_train_step(kh_ctx* ctx, const kh_mlp* net, void* work, int32_t max_batch, const float* x,
                            const float* t, const uint8_t* mask, int32_t b, const kh_mlp_loss_w* lw,
                            const kh_adam* opt, float* loss, void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = capturing(stream);
  kh_status s = check_net(ctx, net, true);
  if (s != KH_OK) return s;
  if (!opt || !(opt->lr > 0.0f) || opt->step < 1) return fail(ctx, KH_EINVAL, "need lr > 0 and step >= 1");
  if ((s = set_device(ctx)) != KH_OK) return s;
  hipStream_t strm = (hipStream_t)stream;
  Work w;
  if ((s = grad_pass(ctx, net, work, max_batch, x, t, mask, b, lw, loss, strm, &w)) != KH_OK) return s;
  hipLaunchKernelGGL(k_mlp_adam, dim3((NP + 255) / 256), dim3(256), 0, strm, net->params, net->adam_m, net->adam_v,
                     w.part, *opt, reinterpret_cast<__bf16*>(net->wb), reinterpret_cast<__bf16*>(net->wbt));
  KH_HIP(ctx, hipGetLastError());
  return KH_OK;
}

kh_status kh_image_from_state(kh_ctx* ctx, const kh_state* st, const int32_t* pix, float* out, void* stream) {
  if (!ctx) return KH_EINVAL;
  g_skip_ptr_query = capturing(stream);
  kh_status s = check_state(ctx, st, false);
  if (s != KH_OK) return s;
  if (!out || !aligned(out, 16) || !device_ok(out)) return fail(ctx, KH_EINVAL, "out must be device memory");
  if (pix && !device_ok(pix)) return fail(ctx, KH_EINVAL, "pix must be NULL or device memory");
  if ((s = set_device(ctx)) != KH_OK) return s;
  const KState ks = to_k(st);
  hipLaunchKernelGGL(k_image_from_state, dim3((unsigned)((st->n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     ks, pix, out);
  KH_HIP(ctx, hipGetLastError());
  return KH_OK;
}

}  // extern "C"
