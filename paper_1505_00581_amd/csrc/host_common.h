// Host-side helpers shared by the C-ABI sources of libstm.so: error state,
// the context, device scratch buffers, argument and data validation, and the
// preparation of one (model, scene) pair on the device.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "stm.h"
#include "stm_internal.h"

namespace stmh {

// Message of the last failure on this thread.
std::string& err();

inline int fail(int code, const std::string& msg) {
  err() = msg;
  return code;
}

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

}  // namespace stmh

#define STM_HIP(expr)                                                                               \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) return stmh::fail(STM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct stm_ctx {
  int device = 0;
  // scratch
  stmh::DevBuf fstart, theta, U, vt, last2, degen, val, counts;
  // staging for host-pointer calls
  stmh::DevBuf mxy, mt, mdesc, sxy, st, sdesc;
  stmh::DevBuf o_e32, o_e64, o_eu, o_assign, o_cand, o_cnt;
  stmh::DevBuf fb, fn, gb, gn;  // BF16 descriptors and squared norms
  // multiple-points chains: gathered chain points and per-chain results
  stmh::DevBuf ch_xy, ch_t, ch_desc, ch_idx, ch_off, ch_e32, ch_e64, ch_eu, ch_as;
  size_t vt_chunk_bytes = size_t(4) << 30;  // value-table scratch per chunk of offsets
  // kernel timing
  bool prof = false;
  std::vector<hipEvent_t> prof_ev;  // pairs (start, stop)
  size_t prof_used = 0;             // events in use
  int64_t prof_matchings = 0;
  double prof_plan_ms = 0.0;      // recursion launches of plan runs (events inside the graph)
  int64_t prof_plan_launches = 0;
  int dp_waves = 8;
};

// The learned candidate pruner: FP32 parameters packed as
// [W1 (128 x (2 dim + 8)), b1, W2 (128 x 128), b2, w3, b3], Adam moments, and
// per-call scratch.
struct stm_pruner {
  stm_ctx* ctx = nullptr;
  int dim = 0;
  long long n = 0;
  long long step = 0;  // Adam steps taken since the parameters were set
  int rule = STM_PRUNE_TIME_NEAREST;
  stmh::DevBuf theta, grad, am, av;
  // per-call scratch
  stmh::DevBuf groups, labels, node, phi, q, h1, h2, dz1, dz2, ds, loss, scores, part;
  stmh::DevBuf wa, wb, A, B, xm, xs, norms, cand, count;
  stmh::DevBuf taus, f32, f64, fu, fas, fell;
};

namespace stmh {

// Grows `b` to at least `bytes` (waiting for `st` before freeing); the old
// contents are not kept.
int grow(stm_ctx* ctx, DevBuf& b, size_t bytes, hipStream_t st);
void release(DevBuf& b);

// Checks that do not need the data.
int check_shapes(const stm_points* m, const stm_points* s, const stm_params* p);
// Bits of invalid host data (see bit_message).
int host_validate(const stm_points* m, const stm_points* s);
const char* bit_message(int bits);

// Inputs on the device, validated, with the frame index built.
struct Prepared {
  stm::ModelView m;
  stm::SceneView s;
  stm::SearchParams sp;
  int32_t span = 0;
  hipStream_t st = nullptr;
  bool device = false;
  bool bf16 = false;
};

// Fixed device buffers for prepare() instead of the context's: the
// validation words (2 int32, cleared here by a fill kernel) and the frame
// index (n_frames + 1 int32).
struct FixedPrep {
  int32_t* val = nullptr;
  int32_t* fstart = nullptr;
};

int prepare(stm_ctx* ctx, const stm_points* m, const stm_points* s, const stm_params* p,
            void* hip_stream, Prepared& out, const FixedPrep* fixed = nullptr);

// Buffers of the split-precision unary table: BF16 descriptors (rows padded to
// the MFMA tile) and their squared norms.  All null: the context's, grown on
// demand.
struct Bf16Bufs {
  uint16_t* fb = nullptr;
  float* fn = nullptr;
  uint16_t* gb = nullptr;
  float* gn = nullptr;
};
// Rows and padded dimension of the BF16 copies of M model and S scene rows.
inline int bf16_rows_model(int M) { return (M + 15) / 16 * 16; }
inline int bf16_rows_scene(int S) { return (S + 255) / 256 * 256; }

// The unary table U [M][S] (Section 3.3), FP32 direct or BF16 on MFMA.
int unary_table(stm_ctx* ctx, const Prepared& pr, float* U, const Bf16Bufs* fixed = nullptr);
int check_range(const Prepared& pr, int32_t tau_begin, int32_t tau_end);

// Device scratch of one exact matching call: the model angles [M], the unary
// table [M][S], the BF16 buffers (split precision), and for `chunk` offsets
// at a time the value tables (per offset (M - 2) x side^2 floats), the last
// state pairs and the degenerate flags.
struct MatchScratch {
  float2* theta = nullptr;
  float* U = nullptr;
  Bf16Bufs bf;
  float* vt = nullptr;
  int2* last2 = nullptr;
  int32_t* degen = nullptr;
  int chunk = 0;
};

// The kernels of stm_match over offsets [tau_begin, tau_begin + n_tau) on
// prepared inputs and device outputs: model angles, unary table, then per
// chunk of offsets the recursion (fast and degenerate variants),
// backtracking and the FP64 re-score.  `timed`: HIP events around the fast
// recursion launches when the context's profiling is on.
int match_kernels(stm_ctx* ctx, const Prepared& pr, const stm_params* p, int32_t tau_begin, int n_tau,
                  float* e32, double* e64, double* eu, int32_t* assign, const MatchScratch& sc, bool timed);


// Looks up the device address of stm_match_noalloc's fixed array on the
// current device `device`, once per device (at context creation).
int noalloc_init(int device);

// Dummy assignments (STM_DUMMY): W^d for the FP64 re-score (0 when off), and
// the value-table side K (+1 for the dummy state).
inline bool dummy_on(const stm_params* p) { return (p->flags & STM_DUMMY) != 0; }
inline double w_dummy_of(const stm_params* p) { return dummy_on(p) ? p->w_dummy : 0.0; }
inline long long vt_side(const stm_params* p) { return (long long)p->k_max + (dummy_on(p) ? 1 : 0); }
inline size_t vt_bytes_per_offset(int M, const stm_params* p) {
  return (size_t)(M - 2) * vt_side(p) * vt_side(p) * sizeof(float);
}
// Packed schedules for sparse scenes (at most 3 points per frame on average,
// as interest points usually are), where a frame group holds a few cells.
inline bool sparse_scene(int32_t S, int32_t F) { return (long long)S <= 3LL * F; }
// The kernels' search parameters of a call: closeness, window, cap, density
// rule and the span reading of closeness.
inline stm::SearchParams search_params(const stm_params* p, int32_t window) {
  return stm::SearchParams{p->T, window, p->k_max, (p->flags & STM_K_DENSITY) ? 1 : 0,
                           (p->flags & STM_CLOSENESS_SPAN) ? 1 : 0, (p->flags & STM_ANGLE_UNSIGNED) ? 1 : 0,
                           (p->flags & STM_CAUSAL_NODE) ? 1 : 0};
}
// lambda1 * W^d in FP32, the dummy's unary term in the recursion.
inline float dummy_cost32(const stm_params* p) {
  return dummy_on(p) ? static_cast<float>(p->lambda1 * p->w_dummy) : 0.f;
}

}  // namespace stmh
