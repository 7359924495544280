// internal.hpp -- pieces shared by the library's translation units (not part
// of the C ABI): the context, the device view of a state, host-side checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "kerrhip.h"

struct kh_ctx {
  int device = 0;
  int n_cu = 0;
  unsigned long long* d_queue = nullptr;  // kQueueSlots counters
  unsigned long long* d_stats = nullptr;  // 8 counters
  kh_camera* d_cams = nullptr;
  int64_t* d_offs = nullptr;
  int cam_cap = 0;
  int cams_uploaded = 0;        // cameras currently in d_cams / d_offs
  int64_t cams_total = 0;       // their total pixel count
  kh_camera* h_cams = nullptr;  // pinned staging
  int64_t* h_offs = nullptr;
  hipEvent_t cam_evt = nullptr;
  uint8_t* d_keys = nullptr;  // per-tile scheduling keys of kh_init_rays
  int64_t keys_cap = 0;
  uint8_t* d_gkeys = nullptr;  // per-geodesic scheduling keys (state.perm)
  int64_t gkeys_cap = 0;
  unsigned* d_perm_cnt = nullptr;  // 512 counters of the per-geodesic sort: counts, then next free position
  double* d_stage = nullptr;       // kh_read_state: rows [chunk][8] packed on the device
  int64_t stage_cap = 0;           // rows
  std::string err;
};

namespace khi {

struct KState {
  int64_t n;
  double* s;
  double* spin;
  int32_t* kind;
  double* h;
  double* lam;
  double* phi;
  int32_t* status;
  int32_t* n_acc;
  int32_t* n_rej;
  double* cross;
  int32_t* n_cross;
  int32_t k_cross;
  double* c0;
  double* c1;
  int32_t* order;  // tile permutation or nullptr
  int32_t* perm;   // per-geodesic queue order or nullptr (replaces order)
  int32_t n_out;   // dense-output targets
  const double* t_out;
  double* s_out;
};

struct KParams {
  double h_coeff, rtol, atol, hmax_coeff, r_h_factor, r_escape, t_end, r_fp64;
  int32_t max_steps;  // accepted steps per call (clamped to 2^31 - 1)
  int32_t max_tries;  // attempts per call before KH_MAX_STEPS (4 max_steps + 1000, clamped)
  int32_t k_cross;
  int32_t refill_min;  // a wave refills once this many of its lanes are idle
  int32_t parts;  // ray-range partitions of the work queue (1 .. kParts)
};

inline KState to_k(const kh_state* st) {
  KState k;
  k.n = st->n;
  k.s = st->s;
  k.spin = st->spin;
  k.kind = st->kind;
  k.h = st->h;
  k.lam = st->lam;
  k.phi = st->phi;
  k.status = st->status;
  k.n_acc = st->n_acc;
  k.n_rej = st->n_rej;
  k.cross = st->cross;
  k.n_cross = st->n_cross;
  k.k_cross = st->k_cross;
  k.c0 = st->c0;
  k.c1 = st->c1;
  k.order = st->order;
  k.perm = st->perm;
  k.n_out = st->n_out;
  k.t_out = st->t_out;
  k.s_out = st->s_out;
  return k;
}


kh_status fail(kh_ctx* c, kh_status s, const std::string& msg);
kh_status hip_fail(kh_ctx* c, hipError_t e, const char* where);
bool aligned(const void* p, size_t a);
bool is_device_ptr(const void* p);
bool capturing(void* stream);
extern thread_local bool g_skip_ptr_query;
bool device_ok(const void* p);
kh_status check_state(kh_ctx* ctx, const kh_state* st, bool need_cross);
kh_status set_device(kh_ctx* ctx);

}  // namespace khi

#define KH_HIP(ctx, call)                                        \
  do {                                                           \
    hipError_t e_ = (call);                                      \
    if (e_ != hipSuccess) return khi::hip_fail(ctx, e_, #call); \
  } while (0)
