// Host side of libstm.so: argument and data validation, the context and its
// device scratch, and the order of the kernels on the stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "host_common.h"

namespace stmh {

std::string& err() {
  thread_local std::string e;
  return e;
}

// Grows `b` to at least `bytes`; the old contents are not kept.
int grow(stm_ctx* ctx, DevBuf& b, size_t bytes, hipStream_t st) {
  if (bytes <= b.cap) return STM_OK;
  if (b.p) {
    STM_HIP(hipStreamSynchronize(st));
    STM_HIP(hipFree(b.p));
    b.p = nullptr;
    b.cap = 0;
  }
  size_t want = bytes + bytes / 8 + 256;
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(STM_ENOMEM, "device allocation of " + std::to_string(want) + " bytes failed");
  }
  b.cap = want;
  return STM_OK;
}

void release(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}

bool finite_lambda(double v) { return std::isfinite(v) && v >= 0.0; }

int check_shapes(const stm_points* m, const stm_points* s, const stm_params* p) {
  if (!m || !s || !p) return fail(STM_EINVAL, "null model, scene or params");
  if (m->n < 3) return fail(STM_EINVAL, "model needs at least 3 points");
  if (s->n < 1) return fail(STM_EINVAL, "scene needs at least 1 point");
  if (m->dim < 1 || m->dim != s->dim) return fail(STM_EINVAL, "descriptor dims differ or are < 1");
  if (m->dim > 256) return fail(STM_EUNSUPPORTED, "descriptor dim above 256");
  if (s->n_frames < 1) return fail(STM_EINVAL, "scene needs n_frames >= 1");
  if (m->reserved != 0 || s->reserved != 0) return fail(STM_EINVAL, "reserved field must be 0");
  if (!m->xy || !m->t || !m->desc || !s->xy || !s->t || !s->desc)
    return fail(STM_EINVAL, "null point array");
  if (p->k_max < 1) return fail(STM_EINVAL, "k_max below 1");
  if (p->k_max > STM_K_LIMIT)
    return fail(STM_EUNSUPPORTED, "k_max above 64: per-offset lists hold at most 64 candidates (one wavefront); "
                                  "the trellis over a scene block (stm_trellis_*) searches every node");
  if (p->window < 0) return fail(STM_EINVAL, "window < 0");
  if (!finite_lambda(p->lambda1) || !finite_lambda(p->lambda2) || !finite_lambda(p->lambda3))
    return fail(STM_EINVAL, "lambdas must be finite and >= 0");
  if (p->flags & ~(STM_DEVICE_PTRS | STM_UNARY_BF16 | STM_K_DENSITY | STM_DUMMY | STM_CLOSENESS_SPAN |
                   STM_ANGLE_UNSIGNED | STM_CAUSAL_NODE))
    return fail(STM_EUNSUPPORTED, "unknown flag");
  if ((p->flags & STM_CAUSAL_NODE) && (p->flags & (STM_DUMMY | STM_CLOSENESS_SPAN)))
    return fail(STM_EUNSUPPORTED, "node-order causality is built for the pairwise reading without dummies only");
  if ((p->flags & STM_DUMMY) && (p->flags & STM_CLOSENESS_SPAN))
    return fail(STM_EUNSUPPORTED, "the span reading of closeness is not defined with dummies");
  if ((p->flags & STM_DUMMY) && (p->flags & STM_ANGLE_UNSIGNED))
    return fail(STM_EUNSUPPORTED, "unsigned angles with dummy assignments are not built");
  if ((p->flags & STM_DUMMY) && !finite_lambda(p->w_dummy))
    return fail(STM_EINVAL, "w_dummy must be finite and >= 0");
  return STM_OK;
}

const char* bit_message(int bits) {
  if (bits & 1) return "model frames not strictly increasing";
  if (bits & 2) return "scene frames not sorted (non-decreasing)";
  if (bits & 4) return "scene frame outside [0, n_frames)";
  if (bits & 8) return "non-finite model coordinate or descriptor";
  if (bits & 16) return "non-finite scene coordinate or descriptor";
  return "invalid input";
}

int host_validate(const stm_points* m, const stm_points* s) {
  int bits = 0;
  for (int i = 0; i < m->n; ++i) {
    if (i > 0 && m->t[i] <= m->t[i - 1]) bits |= 1;
    if (!std::isfinite(m->xy[2 * i]) || !std::isfinite(m->xy[2 * i + 1])) bits |= 8;
  }
  for (size_t i = 0; i < (size_t)m->n * m->dim; ++i)
    if (!std::isfinite(m->desc[i])) bits |= 8;
  for (int i = 0; i < s->n; ++i) {
    if (i > 0 && s->t[i] < s->t[i - 1]) bits |= 2;
    if (s->t[i] < 0 || s->t[i] >= s->n_frames) bits |= 4;
    if (!std::isfinite(s->xy[2 * i]) || !std::isfinite(s->xy[2 * i + 1])) bits |= 16;
  }
  for (size_t i = 0; i < (size_t)s->n * s->dim; ++i)
    if (!std::isfinite(s->desc[i])) bits |= 16;
  return bits;
}

template <class T>
int stage(stm_ctx* ctx, DevBuf& b, const T* host, size_t count, hipStream_t st) {
  int rc = grow(ctx, b, count * sizeof(T), st);
  if (rc) return rc;
  STM_HIP(hipMemcpyAsync(b.p, host, count * sizeof(T), hipMemcpyHostToDevice, st));
  return STM_OK;
}

int prepare(stm_ctx* ctx, const stm_points* m, const stm_points* s, const stm_params* p,
            void* hip_stream, Prepared& out, const FixedPrep* fixed) {
  int rc = check_shapes(m, s, p);
  if (rc) return rc;
  if (!(p->flags & STM_DEVICE_PTRS)) {
    const int bits = host_validate(m, s);
    if (bits) return fail(STM_EINVAL, bit_message(bits));
  }
  if (!ctx) return fail(STM_EINVAL, "null context");
  STM_HIP(hipSetDevice(ctx->device));
  out.st = static_cast<hipStream_t>(hip_stream);
  out.device = (p->flags & STM_DEVICE_PTRS) != 0;
  out.bf16 = (p->flags & STM_UNARY_BF16) != 0;
  const int M = m->n, S = s->n, D = m->dim, F = s->n_frames;
  if (out.device) {
    out.m = {reinterpret_cast<const float2*>(m->xy), m->t, m->desc, M};
    out.s = {reinterpret_cast<const float2*>(s->xy), s->t, s->desc, nullptr, S, F, D};
    int32_t* val = nullptr;
    if (fixed) {
      val = fixed->val;
      STM_HIP(stm::launch_fill_i32(val, 2, 0, out.st));
    } else {
      if ((rc = grow(ctx, ctx->val, 2 * sizeof(int32_t), out.st))) return rc;
      val = static_cast<int32_t*>(ctx->val.p);
      STM_HIP(hipMemsetAsync(val, 0, 2 * sizeof(int32_t), out.st));
    }
    STM_HIP(stm::launch_validate(out.m, out.s, val, out.st));
    int32_t hv[2] = {0, 0};
    STM_HIP(hipMemcpyAsync(hv, val, sizeof(hv), hipMemcpyDeviceToHost, out.st));
    STM_HIP(hipStreamSynchronize(out.st));
    if (hv[0]) return fail(STM_EINVAL, bit_message(hv[0]));
    out.span = hv[1];
  } else {
    out.span = m->t[M - 1] - m->t[0];
    if ((rc = stage(ctx, ctx->mxy, m->xy, (size_t)M * 2, out.st))) return rc;
    if ((rc = stage(ctx, ctx->mt, m->t, (size_t)M, out.st))) return rc;
    if ((rc = stage(ctx, ctx->mdesc, m->desc, (size_t)M * D, out.st))) return rc;
    if ((rc = stage(ctx, ctx->sxy, s->xy, (size_t)S * 2, out.st))) return rc;
    if ((rc = stage(ctx, ctx->st, s->t, (size_t)S, out.st))) return rc;
    if ((rc = stage(ctx, ctx->sdesc, s->desc, (size_t)S * D, out.st))) return rc;
    out.m = {static_cast<const float2*>(ctx->mxy.p), static_cast<const int32_t*>(ctx->mt.p),
             static_cast<const float*>(ctx->mdesc.p), M};
    out.s = {static_cast<const float2*>(ctx->sxy.p), static_cast<const int32_t*>(ctx->st.p),
             static_cast<const float*>(ctx->sdesc.p), nullptr, S, F, D};
  }
  int32_t* fst = nullptr;
  if (fixed) {
    fst = fixed->fstart;
  } else {
    if ((rc = grow(ctx, ctx->fstart, ((size_t)F + 1) * sizeof(int32_t), out.st))) return rc;
    fst = static_cast<int32_t*>(ctx->fstart.p);
  }
  STM_HIP(stm::launch_fstart(out.s.t, S, F, fst, out.st));
  out.s.fstart = fst;
  // a window wider than the scene adds only empty frames
  out.sp = search_params(p, std::min(p->window, F));
  return STM_OK;
}

int unary_table(stm_ctx* ctx, const Prepared& pr, float* U, const Bf16Bufs* fixed) {
  if (!pr.bf16) {
    STM_HIP(stm::launch_unary_f32(pr.m, pr.s, U, pr.st));
    return STM_OK;
  }
  const int M = pr.m.M, S = pr.s.S, dim = pr.s.dim;
  const int Mp = bf16_rows_model(M), Sp = bf16_rows_scene(S), dp = stm::bf16_padded_dim(dim);
  uint16_t *fb, *gb;
  float *fn, *gn;
  if (fixed && fixed->fb) {
    fb = fixed->fb;
    fn = fixed->fn;
    gb = fixed->gb;
    gn = fixed->gn;
  } else {
    int rc;
    if ((rc = grow(ctx, ctx->fb, (size_t)Mp * dp * 2, pr.st))) return rc;
    if ((rc = grow(ctx, ctx->fn, (size_t)Mp * sizeof(float), pr.st))) return rc;
    if ((rc = grow(ctx, ctx->gb, (size_t)Sp * dp * 2, pr.st))) return rc;
    if ((rc = grow(ctx, ctx->gn, (size_t)Sp * sizeof(float), pr.st))) return rc;
    fb = static_cast<uint16_t*>(ctx->fb.p);
    gb = static_cast<uint16_t*>(ctx->gb.p);
    fn = static_cast<float*>(ctx->fn.p);
    gn = static_cast<float*>(ctx->gn.p);
  }
  STM_HIP(stm::launch_to_bf16(pr.m.desc, M, dim, Mp, fb, fn, pr.st));
  STM_HIP(stm::launch_to_bf16(pr.s.desc, S, dim, Sp, gb, gn, pr.st));
  STM_HIP(stm::launch_unary_bf16(fb, fn, M, gb, gn, S, dim, U, pr.st));
  return STM_OK;
}

int check_range(const Prepared& pr, int32_t tau_begin, int32_t tau_end) {
  const long long n_off = std::max(0LL, (long long)pr.s.F - pr.span);
  if (tau_begin < 0 || tau_end < tau_begin || tau_end > n_off)
    return fail(STM_EINVAL, "offset range [" + std::to_string(tau_begin) + ", " +
                                std::to_string(tau_end) + ") outside [0, " + std::to_string(n_off) + ")");
  return STM_OK;
}

int match_kernels(stm_ctx* ctx, const Prepared& pr, const stm_params* params, int32_t tau_begin, int n_tau,
                  float* d_e32, double* d_e64, double* d_eu, int32_t* d_as, const MatchScratch& sc, bool timed) {
  const int M = pr.m.M;
  const hipStream_t st = pr.st;
  int rc;
  STM_HIP(stm::launch_model_angles(pr.m, sc.theta, st));
  if ((rc = unary_table(ctx, pr, sc.U, &sc.bf))) return rc;
  for (int c0 = 0; c0 < n_tau; c0 += sc.chunk) {
    const int nc = std::min(sc.chunk, n_tau - c0);
    stm::DPLaunch a;
    a.m = pr.m;
    a.s = pr.s;
    a.sp = pr.sp;
    a.U = sc.U;
    a.theta = sc.theta;
    a.lambda1 = static_cast<float>(params->lambda1);
    a.lambda2 = static_cast<float>(params->lambda2);
    a.w = static_cast<float>(params->lambda2 * params->lambda3);
    a.dummy = dummy_on(params) ? 1 : 0;
    a.cw = dummy_cost32(params);
    a.packed = !a.dummy && sparse_scene(pr.s.S, pr.s.F) ? 1 : 0;
    a.tau0 = tau_begin + c0;
    a.n_tau = nc;
    a.vt = sc.vt;
    a.e32 = d_e32 + c0;
    a.last2 = sc.last2;
    a.degen = sc.degen;
    a.waves = ctx->dp_waves;
    if (timed && ctx->prof) {
      if (ctx->prof_used + 2 > ctx->prof_ev.size()) {
        for (int q = 0; q < 2; ++q) {
          hipEvent_t ev;
          STM_HIP(hipEventCreate(&ev));
          ctx->prof_ev.push_back(ev);
        }
      }
      STM_HIP(hipEventRecord(ctx->prof_ev[ctx->prof_used], st));
      STM_HIP(stm::launch_dp_fast(a, st));
      STM_HIP(hipEventRecord(ctx->prof_ev[ctx->prof_used + 1], st));
      ctx->prof_used += 2;
      ctx->prof_matchings += nc;
    } else {
      STM_HIP(stm::launch_dp_fast(a, st));
    }
    STM_HIP(stm::launch_dp_degenerate(a, st));
    STM_HIP(stm::launch_backtrack(a, d_as + (size_t)c0 * M, st));
    STM_HIP(stm::launch_rescore(pr.m, pr.s, pr.sp, params->lambda1, params->lambda2,
                                params->lambda3, w_dummy_of(params), d_as + (size_t)c0 * M, nc,
                                d_e64 ? d_e64 + c0 : nullptr, d_eu ? d_eu + c0 : nullptr, st));
  }
  return STM_OK;
}

}  // namespace stmh

using namespace stmh;

extern "C" {

int stm_create(stm_ctx** out, int hip_device) {
  err().clear();
  if (!out) return fail(STM_EINVAL, "null output pointer");
  *out = nullptr;
  int n = 0;
  STM_HIP(hipGetDeviceCount(&n));
  if (hip_device < 0 || hip_device >= n) return fail(STM_EINVAL, "no such HIP device");
  STM_HIP(hipSetDevice(hip_device));
  stm_ctx* c = new (std::nothrow) stm_ctx();
  if (!c) return fail(STM_ENOMEM, "host allocation failed");
  c->device = hip_device;
  // the fixed scratch of stm_match_noalloc on this device; a failed lookup is
  // reported by that entry point only
  (void)noalloc_init(hip_device);
  *out = c;
  return STM_OK;
}

void stm_destroy(stm_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  DevBuf* bufs[] = {&ctx->fstart, &ctx->theta, &ctx->U,     &ctx->vt,    &ctx->last2, &ctx->degen,
                    &ctx->val,    &ctx->counts, &ctx->mxy,  &ctx->mt,    &ctx->mdesc, &ctx->sxy,
                    &ctx->st,     &ctx->sdesc,  &ctx->o_e32, &ctx->o_e64, &ctx->o_eu, &ctx->o_assign,
                    &ctx->o_cand, &ctx->o_cnt, &ctx->fb,   &ctx->fn,    &ctx->gb,    &ctx->gn,
                    &ctx->ch_xy,  &ctx->ch_t,  &ctx->ch_desc, &ctx->ch_idx, &ctx->ch_off, &ctx->ch_e32, &ctx->ch_e64,
                    &ctx->ch_eu,  &ctx->ch_as};
  for (DevBuf* b : bufs) release(*b);
  for (hipEvent_t ev : ctx->prof_ev) (void)hipEventDestroy(ev);
  delete ctx;
}

const char* stm_last_error(void) { return err().c_str(); }

int stm_offsets(stm_ctx* ctx, const stm_points* model, const stm_points* scene, uint32_t flags,
                int32_t* begin, int32_t* end) {
  err().clear();
  if (!model || !scene || !begin || !end || !model->t) return fail(STM_EINVAL, "null argument");
  if (model->n < 1) return fail(STM_EINVAL, "empty model");
  int32_t t0 = 0, t1 = 0;
  if (flags & STM_DEVICE_PTRS) {
    if (!ctx) return fail(STM_EINVAL, "device pointers need a context");
    STM_HIP(hipSetDevice(ctx->device));
    STM_HIP(hipMemcpy(&t0, model->t, sizeof(int32_t), hipMemcpyDeviceToHost));
    STM_HIP(hipMemcpy(&t1, model->t + model->n - 1, sizeof(int32_t), hipMemcpyDeviceToHost));
  } else {
    t0 = model->t[0];
    t1 = model->t[model->n - 1];
  }
  *begin = 0;
  const long long e = (long long)scene->n_frames - ((long long)t1 - t0);
  *end = static_cast<int32_t>(e > 0 ? e : 0);
  return STM_OK;
}

int stm_match(stm_ctx* ctx, const stm_points* model, const stm_points* scene,
              const stm_params* params, int32_t tau_begin, int32_t tau_end, float* energy32,
              double* energy64, double* energy_u64, int32_t* assign, void* hip_stream) {
  err().clear();
  Prepared pr;
  int rc = prepare(ctx, model, scene, params, hip_stream, pr);
  if (rc) return rc;
  if ((rc = check_range(pr, tau_begin, tau_end))) return rc;
  const int n_tau = tau_end - tau_begin;
  if (n_tau == 0) return STM_OK;
  if (!energy32 || !assign) return fail(STM_EINVAL, "energy32 and assign are required");
  const int M = pr.m.M, S = pr.s.S;
  const hipStream_t st = pr.st;

  // outputs: caller's device buffers, or staging for host pointers
  float* d_e32 = energy32;
  double* d_e64 = energy64;
  double* d_eu = energy_u64;
  int32_t* d_as = assign;
  if (!pr.device) {
    if ((rc = grow(ctx, ctx->o_e32, (size_t)n_tau * sizeof(float), st))) return rc;
    if ((rc = grow(ctx, ctx->o_assign, (size_t)n_tau * M * sizeof(int32_t), st))) return rc;
    d_e32 = static_cast<float*>(ctx->o_e32.p);
    d_as = static_cast<int32_t*>(ctx->o_assign.p);
    if (energy64) {
      if ((rc = grow(ctx, ctx->o_e64, (size_t)n_tau * sizeof(double), st))) return rc;
      d_e64 = static_cast<double*>(ctx->o_e64.p);
    }
    if (energy_u64) {
      if ((rc = grow(ctx, ctx->o_eu, (size_t)n_tau * sizeof(double), st))) return rc;
      d_eu = static_cast<double*>(ctx->o_eu.p);
    }
  }

  // model angles, the unary table (Section 3.3) and the recursion's scratch,
  // the value tables in chunks of offsets bounded by vt_chunk_bytes
  MatchScratch sc;
  if ((rc = grow(ctx, ctx->theta, (size_t)M * sizeof(float2), st))) return rc;
  if ((rc = grow(ctx, ctx->U, (size_t)M * S * sizeof(float), st))) return rc;
  const size_t per_tau = vt_bytes_per_offset(M, params);
  sc.chunk = static_cast<int>(std::min<size_t>(n_tau, std::max<size_t>(1, ctx->vt_chunk_bytes / per_tau)));
  if ((rc = grow(ctx, ctx->vt, per_tau * sc.chunk, st))) return rc;
  if ((rc = grow(ctx, ctx->last2, (size_t)sc.chunk * sizeof(int2), st))) return rc;
  if ((rc = grow(ctx, ctx->degen, (size_t)sc.chunk * sizeof(int32_t), st))) return rc;
  sc.theta = static_cast<float2*>(ctx->theta.p);
  sc.U = static_cast<float*>(ctx->U.p);
  sc.vt = static_cast<float*>(ctx->vt.p);
  sc.last2 = static_cast<int2*>(ctx->last2.p);
  sc.degen = static_cast<int32_t*>(ctx->degen.p);
  if ((rc = match_kernels(ctx, pr, params, tau_begin, n_tau, d_e32, d_e64, d_eu, d_as, sc, true))) return rc;

  if (!pr.device) {
    STM_HIP(hipMemcpyAsync(energy32, d_e32, (size_t)n_tau * sizeof(float), hipMemcpyDeviceToHost, st));
    STM_HIP(hipMemcpyAsync(assign, d_as, (size_t)n_tau * M * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (energy64)
      STM_HIP(hipMemcpyAsync(energy64, d_e64, (size_t)n_tau * sizeof(double), hipMemcpyDeviceToHost, st));
    if (energy_u64)
      STM_HIP(hipMemcpyAsync(energy_u64, d_eu, (size_t)n_tau * sizeof(double), hipMemcpyDeviceToHost, st));
    STM_HIP(hipStreamSynchronize(st));
  }
  return STM_OK;
}

int stm_candidates(stm_ctx* ctx, const stm_points* model, const stm_points* scene,
                   const stm_params* params, int32_t tau_begin, int32_t tau_end, int32_t* cand,
                   int32_t* count, void* hip_stream) {
  err().clear();
  Prepared pr;
  int rc = prepare(ctx, model, scene, params, hip_stream, pr);
  if (rc) return rc;
  if ((rc = check_range(pr, tau_begin, tau_end))) return rc;
  const int n_tau = tau_end - tau_begin;
  if (n_tau == 0) return STM_OK;
  if (!cand || !count) return fail(STM_EINVAL, "null output");
  const size_t nc = (size_t)n_tau * pr.m.M * pr.sp.K, nn = (size_t)n_tau * pr.m.M;
  int32_t* d_c = cand;
  int32_t* d_n = count;
  if (!pr.device) {
    if ((rc = grow(ctx, ctx->o_cand, nc * sizeof(int32_t), pr.st))) return rc;
    if ((rc = grow(ctx, ctx->o_cnt, nn * sizeof(int32_t), pr.st))) return rc;
    d_c = static_cast<int32_t*>(ctx->o_cand.p);
    d_n = static_cast<int32_t*>(ctx->o_cnt.p);
  }
  STM_HIP(stm::launch_candidates(pr.m, pr.s, pr.sp, tau_begin, n_tau, d_c, d_n, pr.st));
  if (!pr.device) {
    STM_HIP(hipMemcpyAsync(cand, d_c, nc * sizeof(int32_t), hipMemcpyDeviceToHost, pr.st));
    STM_HIP(hipMemcpyAsync(count, d_n, nn * sizeof(int32_t), hipMemcpyDeviceToHost, pr.st));
    STM_HIP(hipStreamSynchronize(pr.st));
  }
  return STM_OK;
}

int stm_unary(stm_ctx* ctx, const stm_points* model, const stm_points* scene,
              const stm_params* params, float* U, void* hip_stream) {
  err().clear();
  Prepared pr;
  int rc = prepare(ctx, model, scene, params, hip_stream, pr);
  if (rc) return rc;
  if (!U) return fail(STM_EINVAL, "null output");
  const size_t n = (size_t)pr.m.M * pr.s.S;
  float* d_u = U;
  if (!pr.device) {
    if ((rc = grow(ctx, ctx->U, n * sizeof(float), pr.st))) return rc;
    d_u = static_cast<float*>(ctx->U.p);
  }
  if ((rc = unary_table(ctx, pr, d_u))) return rc;
  if (!pr.device) {
    STM_HIP(hipMemcpyAsync(U, d_u, n * sizeof(float), hipMemcpyDeviceToHost, pr.st));
    STM_HIP(hipStreamSynchronize(pr.st));
  }
  return STM_OK;
}

int stm_count_work(stm_ctx* ctx, const stm_points* model, const stm_points* scene,
                   const stm_params* params, int32_t tau_begin, int32_t tau_end, int64_t* counts,
                   void* hip_stream) {
  err().clear();
  Prepared pr;
  int rc = prepare(ctx, model, scene, params, hip_stream, pr);
  if (rc) return rc;
  if ((rc = check_range(pr, tau_begin, tau_end))) return rc;
  if (!counts) return fail(STM_EINVAL, "null output");
  if ((rc = grow(ctx, ctx->counts, 4 * sizeof(unsigned long long), pr.st))) return rc;
  STM_HIP(hipMemsetAsync(ctx->counts.p, 0, 4 * sizeof(unsigned long long), pr.st));
  STM_HIP(stm::launch_count(pr.m, pr.s, pr.sp, tau_begin, tau_end - tau_begin,
                            static_cast<unsigned long long*>(ctx->counts.p), pr.st));
  unsigned long long h[4];
  STM_HIP(hipMemcpyAsync(h, ctx->counts.p, sizeof(h), hipMemcpyDeviceToHost, pr.st));
  STM_HIP(hipStreamSynchronize(pr.st));
  for (int i = 0; i < 4; ++i) counts[i] = static_cast<int64_t>(h[i]);
  return STM_OK;
}

int stm_set_dp_waves(stm_ctx* ctx, int waves) {
  err().clear();
  if (!ctx) return fail(STM_EINVAL, "null context");
  if (waves == 0) waves = 8;
  if (waves != 4 && waves != 8 && waves != 16) return fail(STM_EINVAL, "waves must be 4, 8 or 16");
  ctx->dp_waves = waves;
  return STM_OK;
}

int stm_profile_enable(stm_ctx* ctx, int enable) {
  err().clear();
  if (!ctx) return fail(STM_EINVAL, "null context");
  STM_HIP(hipSetDevice(ctx->device));
  ctx->prof = enable != 0;
  ctx->prof_used = 0;
  ctx->prof_matchings = 0;
  ctx->prof_plan_ms = 0.0;
  ctx->prof_plan_launches = 0;
  return STM_OK;
}

int stm_profile_read(stm_ctx* ctx, double* dp_ms, int64_t* dp_launches, int64_t* dp_matchings) {
  err().clear();
  if (!ctx) return fail(STM_EINVAL, "null context");
  STM_HIP(hipSetDevice(ctx->device));
  double total = 0.0;
  for (size_t q = 0; q + 1 < ctx->prof_used; q += 2) {
    STM_HIP(hipEventSynchronize(ctx->prof_ev[q + 1]));
    float ms = 0.f;
    STM_HIP(hipEventElapsedTime(&ms, ctx->prof_ev[q], ctx->prof_ev[q + 1]));
    total += ms;
  }
  if (dp_ms) *dp_ms = total + ctx->prof_plan_ms;
  if (dp_launches) *dp_launches = static_cast<int64_t>(ctx->prof_used / 2) + ctx->prof_plan_launches;
  if (dp_matchings) *dp_matchings = ctx->prof_matchings;
  return STM_OK;
}

}  // extern "C"
