// C ABI of the learned candidate pruner: parameters, FP32 training on the
// device, BF16 inference, and the matching on pruned candidate lists with the
// exact recursion (Section 2.2) as fallback for offsets the pruned lists make
// infeasible.
#include <cstdint>
#include <cstdio>
#include <limits>

#include "host_common.h"

using namespace stmh;

namespace {

constexpr int H = stm::kPrunerHidden;
constexpr int kSlots = 64;  // slots per group

long long n_params(int dim) {
  const long long ni = 2LL * dim + 8;
  return H * ni + H + (long long)H * H + H + H + 1;
}

}  // namespace

namespace {

template <class T>
T* as(DevBuf& b) {
  return static_cast<T*>(b.p);
}

int check_pruner(stm_pruner* P) {
  if (!P || !P->ctx) return fail(STM_EINVAL, "null pruner");
  STM_HIP(hipSetDevice(P->ctx->device));
  return STM_OK;
}

// Inputs of one pair on the device with the unary table in ctx->U.
int pair_inputs(stm_pruner* P, const stm_points* m, const stm_points* s, const stm_params* prm, void* stream,
                Prepared& pr) {
  int rc = prepare(P->ctx, m, s, prm, stream, pr);
  if (rc) return rc;
  if (m->dim != P->dim) return fail(STM_EINVAL, "descriptor dimension differs from the pruner's");
  stm_ctx* ctx = P->ctx;
  if ((rc = grow(ctx, ctx->U, (size_t)pr.m.M * pr.s.S * sizeof(float), pr.st))) return rc;
  return unary_table(ctx, pr, static_cast<float*>(ctx->U.p));
}

// Host group list (tau, i) checked against the pair and staged on the device.
int stage_groups(stm_pruner* P, const Prepared& pr, const int32_t* groups, int G) {
  if (G < 0) return fail(STM_EINVAL, "negative group count");
  if (G > 0 && !groups) return fail(STM_EINVAL, "null group list");
  const long long n_off = std::max(0LL, (long long)pr.s.F - pr.span);
  for (int g = 0; g < G; ++g) {
    const int tau = groups[2 * g], i = groups[2 * g + 1];
    if (tau < 0 || tau >= n_off || i < 0 || i >= pr.m.M)
      return fail(STM_EINVAL, "group " + std::to_string(g) + " (tau " + std::to_string(tau) + ", i " +
                                  std::to_string(i) + ") is outside the pair");
  }
  int rc = grow(P->ctx, P->groups, (size_t)std::max(G, 1) * sizeof(int2), pr.st);
  if (rc) return rc;
  if (G > 0) STM_HIP(hipMemcpyAsync(P->groups.p, groups, (size_t)G * sizeof(int2), hipMemcpyHostToDevice, pr.st));
  return STM_OK;
}

int group_rows(stm_pruner* P, const Prepared& pr, int G) {
  const size_t R = (size_t)G * kSlots;
  int rc;
  if ((rc = grow(P->ctx, P->node, R * sizeof(int32_t), pr.st))) return rc;
  if ((rc = grow(P->ctx, P->phi, R * 8 * sizeof(float), pr.st))) return rc;
  if ((rc = grow(P->ctx, P->q, (size_t)G * 2 * sizeof(int32_t), pr.st))) return rc;
  STM_HIP(stm::launch_group_rows(pr.m, pr.s, static_cast<const float*>(P->ctx->U.p), pr.s.S, pr.sp,
                                 as<const int2>(P->groups), 0, G, as<int32_t>(P->node), as<float>(P->phi),
                                 as<int32_t>(P->q), pr.st));
  return STM_OK;
}

// FP32 forward (and backward with labels) over the staged groups.
int train_pass(stm_pruner* P, const Prepared& pr, int G, bool backward) {
  const size_t R = (size_t)G * kSlots;
  stm_ctx* ctx = P->ctx;
  int rc;
  DevBuf* rows[] = {&P->h1, &P->h2, &P->dz1, &P->dz2};
  for (DevBuf* b : rows)
    if ((rc = grow(ctx, *b, R * H * sizeof(float), pr.st))) return rc;
  if ((rc = grow(ctx, P->ds, R * sizeof(float), pr.st))) return rc;
  if ((rc = grow(ctx, P->scores, R * sizeof(float), pr.st))) return rc;
  if ((rc = grow(ctx, P->loss, (size_t)G * sizeof(float), pr.st))) return rc;
  if ((rc = grow(ctx, P->part, (size_t)stm::pruner_part_floats(G, P->dim) * sizeof(float), pr.st))) return rc;
  stm::PrunerTrain t;
  t.mdesc = pr.m.desc;
  t.sdesc = pr.s.desc;
  t.groups = as<const int2>(P->groups);
  t.node = as<const int32_t>(P->node);
  t.phi = as<const float>(P->phi);
  t.labels = backward ? as<const int32_t>(P->labels) : nullptr;
  t.D = P->dim;
  t.G = G;
  t.theta = as<const float>(P->theta);
  t.grad = as<float>(P->grad);
  t.h1 = as<float>(P->h1);
  t.h2 = as<float>(P->h2);
  t.dz1 = as<float>(P->dz1);
  t.dz2 = as<float>(P->dz2);
  t.ds = as<float>(P->ds);
  t.loss = as<float>(P->loss);
  t.scores = as<float>(P->scores);
  t.part = as<float>(P->part);
  STM_HIP(stm::launch_pruner_train(t, pr.st));
  return STM_OK;
}

// Loss and gradient of G labelled groups; the mean loss into *loss.
int gradient(stm_pruner* P, const stm_points* m, const stm_points* s, const stm_params* prm,
             const int32_t* groups, const int32_t* labels, int G, float* loss, float* scores, void* stream,
             Prepared& pr) {
  int rc = check_pruner(P);
  if (rc) return rc;
  if (!loss) return fail(STM_EINVAL, "null loss pointer");
  if (G < 1) return fail(STM_EINVAL, "a training pass needs at least one group");
  if (!labels) return fail(STM_EINVAL, "null labels");
  if ((rc = pair_inputs(P, m, s, prm, stream, pr))) return rc;
  for (int g = 0; g < G; ++g)
    if (labels[g] < 0 || labels[g] >= pr.s.S)
      return fail(STM_EINVAL, "label of group " + std::to_string(g) + " is not a scene node");
  if ((rc = stage_groups(P, pr, groups, G))) return rc;
  if ((rc = grow(P->ctx, P->labels, (size_t)G * sizeof(int32_t), pr.st))) return rc;
  STM_HIP(hipMemcpyAsync(P->labels.p, labels, (size_t)G * sizeof(int32_t), hipMemcpyHostToDevice, pr.st));
  if ((rc = group_rows(P, pr, G))) return rc;
  if ((rc = train_pass(P, pr, G, true))) return rc;
  std::vector<float> lv(G);
  STM_HIP(hipMemcpyAsync(lv.data(), P->loss.p, (size_t)G * sizeof(float), hipMemcpyDeviceToHost, pr.st));
  if (scores)
    STM_HIP(hipMemcpyAsync(scores, P->scores.p, (size_t)G * kSlots * sizeof(float), hipMemcpyDeviceToHost, pr.st));
  STM_HIP(hipStreamSynchronize(pr.st));
  double sum = 0.0;
  for (int g = 0; g < G; ++g) {
    if (std::isnan(lv[g]))
      return fail(STM_EINVAL, "label of group " + std::to_string(g) + " is not among its candidates");
    sum += lv[g];
  }
  *loss = static_cast<float>(sum / G);
  return STM_OK;
}

// BF16 first-layer projections A = W1[:, :D] (D f) + b1 (model) and
// B = W1[:, D:2D] (D g) (scene).
int project(stm_pruner* P, const Prepared& pr) {
  stm_ctx* ctx = P->ctx;
  const int D = P->dim, M = pr.m.M, S = pr.s.S, NI = 2 * D + 8;
  const int dp = stm::bf16_padded_dim(D), Mp = (M + 15) / 16 * 16, Sp = (S + 15) / 16 * 16;
  int rc;
  if ((rc = grow(ctx, P->wa, (size_t)H * dp * 2, pr.st))) return rc;
  if ((rc = grow(ctx, P->wb, (size_t)H * dp * 2, pr.st))) return rc;
  if ((rc = grow(ctx, P->xm, (size_t)Mp * dp * 2, pr.st))) return rc;
  if ((rc = grow(ctx, P->xs, (size_t)Sp * dp * 2, pr.st))) return rc;
  if ((rc = grow(ctx, P->norms, (size_t)std::max(Mp, Sp) * sizeof(float), pr.st))) return rc;
  if ((rc = grow(ctx, P->A, (size_t)M * H * sizeof(float), pr.st))) return rc;
  if ((rc = grow(ctx, P->B, (size_t)S * H * sizeof(float), pr.st))) return rc;
  const float* W1 = as<const float>(P->theta);
  STM_HIP(stm::launch_cast_rows_bf16(W1, H, NI, 0, D, dp, as<uint16_t>(P->wa), pr.st));
  STM_HIP(stm::launch_cast_rows_bf16(W1, H, NI, D, D, dp, as<uint16_t>(P->wb), pr.st));
  STM_HIP(stm::launch_to_bf16(pr.m.desc, M, D, Mp, as<uint16_t>(P->xm), as<float>(P->norms), pr.st));
  STM_HIP(stm::launch_project_bf16(as<const uint16_t>(P->xm), M, dp, as<const uint16_t>(P->wa),
                                   static_cast<float>(D), W1 + (long long)H * NI, as<float>(P->A), pr.st));
  STM_HIP(stm::launch_to_bf16(pr.s.desc, S, D, Sp, as<uint16_t>(P->xs), as<float>(P->norms), pr.st));
  STM_HIP(stm::launch_project_bf16(as<const uint16_t>(P->xs), S, dp, as<const uint16_t>(P->wb),
                                   static_cast<float>(D), nullptr, as<float>(P->B), pr.st));
  return STM_OK;
}

stm::PrunerInfer infer_args(stm_pruner* P, const Prepared& pr, int topk) {
  stm::PrunerInfer q;
  q.m = pr.m;
  q.s = pr.s;
  q.U = static_cast<const float*>(P->ctx->U.p);
  q.us = pr.s.S;
  q.sp = pr.sp;
  q.groups = nullptr;
  q.n_groups = 0;
  q.tau0 = 0;
  q.node = nullptr;
  q.phi = nullptr;
  q.theta = as<const float>(P->theta);
  q.D = P->dim;
  q.A = as<const float>(P->A);
  q.B = as<const float>(P->B);
  q.topk = topk;
  q.rule = P->rule;
  q.cand = nullptr;
  q.count = nullptr;
  q.scores = nullptr;
  return q;
}

}  // namespace

namespace {
struct FallbackBufs {
  DevBuf *taus, *f32, *f64, *fu, *fas;
};

// Output pointers of a matching call: the caller's device buffers, or staging
// for host pointers.
struct Outs {
  float* e32;
  double* e64;
  double* eu;
  int32_t* as;
  int32_t* fell;
};

int outputs(stm_ctx* ctx, DevBuf* fell_buf, const Prepared& pr, int n_tau, float* energy32, double* energy64,
            double* energy_u64, int32_t* assign, int32_t* fell_back, Outs& o) {
  o = {energy32, energy64, energy_u64, assign, fell_back};
  if (pr.device) return STM_OK;
  const int M = pr.m.M;
  const hipStream_t st = pr.st;
  int rc;
  if ((rc = grow(ctx, ctx->o_e32, (size_t)n_tau * sizeof(float), st))) return rc;
  if ((rc = grow(ctx, ctx->o_assign, (size_t)n_tau * M * sizeof(int32_t), st))) return rc;
  o.e32 = static_cast<float*>(ctx->o_e32.p);
  o.as = static_cast<int32_t*>(ctx->o_assign.p);
  if (energy64) {
    if ((rc = grow(ctx, ctx->o_e64, (size_t)n_tau * sizeof(double), st))) return rc;
    o.e64 = static_cast<double*>(ctx->o_e64.p);
  }
  if (energy_u64) {
    if ((rc = grow(ctx, ctx->o_eu, (size_t)n_tau * sizeof(double), st))) return rc;
    o.eu = static_cast<double*>(ctx->o_eu.p);
  }
  if (fell_back) {
    if ((rc = grow(ctx, *fell_buf, (size_t)n_tau * sizeof(int32_t), st))) return rc;
    o.fell = as<int32_t>(*fell_buf);
  }
  return STM_OK;
}

int copy_back(const Prepared& pr, int n_tau, const Outs& o, float* energy32, double* energy64, double* energy_u64,
              int32_t* assign, int32_t* fell_back) {
  const hipStream_t st = pr.st;
  if (!pr.device) {
    const int M = pr.m.M;
    STM_HIP(hipMemcpyAsync(energy32, o.e32, (size_t)n_tau * sizeof(float), hipMemcpyDeviceToHost, st));
    STM_HIP(hipMemcpyAsync(assign, o.as, (size_t)n_tau * M * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (energy64) STM_HIP(hipMemcpyAsync(energy64, o.e64, (size_t)n_tau * sizeof(double), hipMemcpyDeviceToHost, st));
    if (energy_u64)
      STM_HIP(hipMemcpyAsync(energy_u64, o.eu, (size_t)n_tau * sizeof(double), hipMemcpyDeviceToHost, st));
    if (fell_back)
      STM_HIP(hipMemcpyAsync(fell_back, o.fell, (size_t)n_tau * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  }
  STM_HIP(hipStreamSynchronize(st));
  return STM_OK;
}

stm::DPLaunch dp_base(stm_ctx* ctx, const Prepared& pr, const stm_params* params) {
  stm::DPLaunch a;
  a.m = pr.m;
  a.s = pr.s;
  a.sp = pr.sp;
  a.U = static_cast<const float*>(ctx->U.p);
  a.theta = static_cast<const float2*>(ctx->theta.p);
  a.lambda1 = static_cast<float>(params->lambda1);
  a.lambda2 = static_cast<float>(params->lambda2);
  a.w = static_cast<float>(params->lambda2 * params->lambda3);
  a.dummy = dummy_on(params) ? 1 : 0;
  a.cw = dummy_cost32(params);
  a.packed = !a.dummy && sparse_scene(pr.s.S, pr.s.F) ? 1 : 0;
  a.waves = ctx->dp_waves;
  a.vt = static_cast<float*>(ctx->vt.p);
  a.last2 = static_cast<int2*>(ctx->last2.p);
  a.degen = static_cast<int32_t*>(ctx->degen.p);
  return a;
}

// Largest number of offsets whose value tables (K x K per step, (K + 1)^2 with
// dummies) fit the scratch budget.
int dp_chunk(stm_ctx* ctx, const Prepared& pr, const stm_params* params, int n, int K, size_t cap_rows) {
  const size_t side = (size_t)K + (dummy_on(params) ? 1 : 0);
  const size_t per_tau = (size_t)std::max(pr.m.M - 2, 1) * side * side * sizeof(float);
  return static_cast<int>(std::min<size_t>({(size_t)n, cap_rows, std::max<size_t>(1, ctx->vt_chunk_bytes / per_tau)}));
}

int dp_scratch(stm_ctx* ctx, const Prepared& pr, const stm_params* params, int chunk, int K) {
  const size_t side = (size_t)K + (dummy_on(params) ? 1 : 0);
  const size_t per_tau = (size_t)std::max(pr.m.M - 2, 1) * side * side * sizeof(float);
  int rc;
  if ((rc = grow(ctx, ctx->vt, per_tau * chunk, pr.st))) return rc;
  if ((rc = grow(ctx, ctx->last2, (size_t)chunk * sizeof(int2), pr.st))) return rc;
  return grow(ctx, ctx->degen, (size_t)chunk * sizeof(int32_t), pr.st);
}

// Forward pass (both variants), backtracking and FP64 re-score of the
// matchings of launch b, rows written from e32 / e64 / eu / as.
int dp_rows(const Prepared& pr, const stm_params* params, stm::DPLaunch b, float* e32, double* e64, double* eu,
            int32_t* as) {
  b.e32 = e32;
  STM_HIP(stm::launch_dp_fast(b, pr.st));
  STM_HIP(stm::launch_dp_degenerate(b, pr.st));
  STM_HIP(stm::launch_backtrack(b, as, pr.st));
  STM_HIP(stm::launch_rescore(pr.m, pr.s, pr.sp, params->lambda1, params->lambda2, params->lambda3,
                              w_dummy_of(params), as, b.n_tau,
                              e64, eu, pr.st));
  return STM_OK;
}

// Offsets of [tau_begin, tau_begin + n_tau) left infeasible: solved again on
// the full windowed lists, their rows replaced and fell_back set.
int exact_fallback(stm_ctx* ctx, const FallbackBufs& fb, const Prepared& pr, const stm_params* params, int tau_begin,
                   int n_tau, const Outs& o) {
  std::vector<float> e(n_tau);
  STM_HIP(hipMemcpyAsync(e.data(), o.e32, (size_t)n_tau * sizeof(float), hipMemcpyDeviceToHost, pr.st));
  STM_HIP(hipStreamSynchronize(pr.st));
  std::vector<int32_t> redo;
  for (int j = 0; j < n_tau; ++j)
    if (!(e[j] < std::numeric_limits<float>::infinity())) redo.push_back(tau_begin + j);
  if (redo.empty()) return STM_OK;
  const int nr = static_cast<int>(redo.size()), M = pr.m.M;
  const int chunk = dp_chunk(ctx, pr, params, nr, pr.sp.K, (size_t)nr);
  int rc;
  if ((rc = dp_scratch(ctx, pr, params, chunk, pr.sp.K))) return rc;
  if ((rc = grow(ctx, *fb.taus, (size_t)nr * sizeof(int32_t), pr.st))) return rc;
  if ((rc = grow(ctx, *fb.f32, (size_t)chunk * sizeof(float), pr.st))) return rc;
  if ((rc = grow(ctx, *fb.f64, (size_t)chunk * sizeof(double), pr.st))) return rc;
  if ((rc = grow(ctx, *fb.fu, (size_t)chunk * sizeof(double), pr.st))) return rc;
  if ((rc = grow(ctx, *fb.fas, (size_t)chunk * M * sizeof(int32_t), pr.st))) return rc;
  STM_HIP(hipMemcpyAsync(fb.taus->p, redo.data(), (size_t)nr * sizeof(int32_t), hipMemcpyHostToDevice, pr.st));
  for (int c0 = 0; c0 < nr; c0 += chunk) {
    const int nc = std::min(chunk, nr - c0);
    stm::DPLaunch b = dp_base(ctx, pr, params);
    b.taus = as<const int32_t>(*fb.taus) + c0;
    b.tau0 = 0;
    b.n_tau = nc;
    if ((rc = dp_rows(pr, params, b, as<float>(*fb.f32), as<double>(*fb.f64), as<double>(*fb.fu),
                      as<int32_t>(*fb.fas))))
      return rc;
    STM_HIP(stm::launch_scatter_fallback(as<const int32_t>(*fb.taus) + c0, nc, tau_begin, M, as<const float>(*fb.f32),
                                         as<const double>(*fb.f64), as<const double>(*fb.fu),
                                         as<const int32_t>(*fb.fas), o.e32, o.e64, o.eu, o.as, o.fell, pr.st));
  }
  return STM_OK;
}

}  // namespace

extern "C" {

int64_t stm_pruner_num_params(int32_t dim) { return dim >= 1 ? n_params(dim) : -1; }

int stm_pruner_create(stm_ctx* ctx, int32_t dim, stm_pruner** out) {
  err().clear();
  if (!out) return fail(STM_EINVAL, "null output pointer");
  *out = nullptr;
  if (!ctx) return fail(STM_EINVAL, "null context");
  if (dim < 1 || dim > 4096) return fail(STM_EINVAL, "descriptor dimension must be in [1, 4096]");
  STM_HIP(hipSetDevice(ctx->device));
  stm_pruner* P = new (std::nothrow) stm_pruner();
  if (!P) return fail(STM_ENOMEM, "host allocation failed");
  P->ctx = ctx;
  P->dim = dim;
  P->n = n_params(dim);
  const size_t bytes = (size_t)P->n * sizeof(float);
  int rc = STM_OK;
  DevBuf* bufs[] = {&P->theta, &P->grad, &P->am, &P->av};
  for (DevBuf* b : bufs) {
    if ((rc = grow(ctx, *b, bytes, nullptr))) break;
    if (hipMemset(b->p, 0, bytes) != hipSuccess) {
      rc = fail(STM_EHIP, "hipMemset failed");
      break;
    }
  }
  if (rc) {
    stm_pruner_destroy(P);
    return rc;
  }
  *out = P;
  return STM_OK;
}

void stm_pruner_destroy(stm_pruner* P) {
  if (!P) return;
  if (P->ctx) {
    (void)hipSetDevice(P->ctx->device);
    (void)hipDeviceSynchronize();
  }
  DevBuf* bufs[] = {&P->theta, &P->grad, &P->am,  &P->av,    &P->groups, &P->labels, &P->node,  &P->phi,
                    &P->q,     &P->h1,   &P->h2,  &P->dz1,   &P->dz2,    &P->ds,     &P->loss,  &P->scores,
                    &P->part,  &P->wa,   &P->wb,  &P->A,      &P->B,      &P->xm,    &P->xs,
                    &P->norms, &P->cand, &P->count, &P->taus, &P->f32,   &P->f64,    &P->fu,    &P->fas,
                    &P->fell};
  for (DevBuf* b : bufs) release(*b);
  delete P;
}

int stm_pruner_set_rule(stm_pruner* P, int32_t rule) {
  err().clear();
  int rc = check_pruner(P);
  if (rc) return rc;
  if (rule != STM_PRUNE_SCORE && rule != STM_PRUNE_FRAMES_FIRST && rule != STM_PRUNE_TIME_NEAREST)
    return fail(STM_EINVAL, "unknown selection rule");
  P->rule = rule;
  return STM_OK;
}

int stm_pruner_set_params(stm_pruner* P, const float* theta, int64_t n) {
  err().clear();
  int rc = check_pruner(P);
  if (rc) return rc;
  if (!theta || n != P->n) return fail(STM_EINVAL, "expected " + std::to_string(P->n) + " parameters");
  for (int64_t j = 0; j < n; ++j)
    if (!std::isfinite(theta[j])) return fail(STM_EINVAL, "non-finite parameter " + std::to_string(j));
  const size_t bytes = (size_t)n * sizeof(float);
  STM_HIP(hipMemcpy(P->theta.p, theta, bytes, hipMemcpyHostToDevice));
  STM_HIP(hipMemset(P->am.p, 0, bytes));
  STM_HIP(hipMemset(P->av.p, 0, bytes));
  P->step = 0;
  return STM_OK;
}

int stm_pruner_get_params(stm_pruner* P, float* theta, int64_t n) {
  err().clear();
  int rc = check_pruner(P);
  if (rc) return rc;
  if (!theta || n != P->n) return fail(STM_EINVAL, "expected " + std::to_string(P->n) + " parameters");
  STM_HIP(hipDeviceSynchronize());
  STM_HIP(hipMemcpy(theta, P->theta.p, (size_t)n * sizeof(float), hipMemcpyDeviceToHost));
  return STM_OK;
}

int stm_pruner_save(stm_pruner* P, const char* path) {
  err().clear();
  int rc = check_pruner(P);
  if (rc) return rc;
  if (!path) return fail(STM_EINVAL, "null path");
  std::vector<float> th(P->n);
  if ((rc = stm_pruner_get_params(P, th.data(), P->n))) return rc;
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(STM_EINVAL, std::string("cannot open ") + path);
  const int32_t hdr[2] = {P->dim, 0};
  const int64_t n = P->n;
  bool ok = std::fwrite("STMPRUN1", 1, 8, f) == 8 && std::fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
            std::fwrite(&n, sizeof(n), 1, f) == 1 && std::fwrite(th.data(), sizeof(float), th.size(), f) == th.size();
  ok = (std::fclose(f) == 0) && ok;
  return ok ? STM_OK : fail(STM_EINVAL, std::string("write to ") + path + " failed");
}

int stm_pruner_load(stm_pruner* P, const char* path) {
  err().clear();
  int rc = check_pruner(P);
  if (rc) return rc;
  if (!path) return fail(STM_EINVAL, "null path");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(STM_EINVAL, std::string("cannot open ") + path);
  char tag[8];
  int32_t hdr[2];
  int64_t n = 0;
  bool ok = std::fread(tag, 1, 8, f) == 8 && std::memcmp(tag, "STMPRUN1", 8) == 0 &&
            std::fread(hdr, sizeof(hdr), 1, f) == 1 && std::fread(&n, sizeof(n), 1, f) == 1 && hdr[0] == P->dim &&
            n == P->n;
  std::vector<float> th(ok ? n : 0);
  ok = ok && std::fread(th.data(), sizeof(float), th.size(), f) == th.size();
  std::fclose(f);
  if (!ok) return fail(STM_EINVAL, std::string(path) + " is not a pruner of this dimension");
  return stm_pruner_set_params(P, th.data(), n);
}

int stm_pruner_features(stm_pruner* P, const stm_points* model, const stm_points* scene, const stm_params* params,
                        const int32_t* groups, int32_t G, int32_t* node, float* phi, int32_t* q, void* hip_stream) {
  err().clear();
  int rc = check_pruner(P);
  if (rc) return rc;
  Prepared pr;
  if ((rc = pair_inputs(P, model, scene, params, hip_stream, pr))) return rc;
  if ((rc = stage_groups(P, pr, groups, G))) return rc;
  if (G == 0) return STM_OK;
  if ((rc = group_rows(P, pr, G))) return rc;
  const size_t R = (size_t)G * kSlots;
  if (node) STM_HIP(hipMemcpyAsync(node, P->node.p, R * sizeof(int32_t), hipMemcpyDeviceToHost, pr.st));
  if (phi) STM_HIP(hipMemcpyAsync(phi, P->phi.p, R * 8 * sizeof(float), hipMemcpyDeviceToHost, pr.st));
  if (q) STM_HIP(hipMemcpyAsync(q, P->q.p, (size_t)G * 2 * sizeof(int32_t), hipMemcpyDeviceToHost, pr.st));
  STM_HIP(hipStreamSynchronize(pr.st));
  return STM_OK;
}

int stm_pruner_gradient(stm_pruner* P, const stm_points* model, const stm_points* scene, const stm_params* params,
                        const int32_t* groups, const int32_t* labels, int32_t G, float* loss, float* grad,
                        float* scores, void* hip_stream) {
  err().clear();
  Prepared pr;
  int rc = gradient(P, model, scene, params, groups, labels, G, loss, scores, hip_stream, pr);
  if (rc) return rc;
  if (grad) {
    STM_HIP(hipMemcpyAsync(grad, P->grad.p, (size_t)P->n * sizeof(float), hipMemcpyDeviceToHost, pr.st));
    STM_HIP(hipStreamSynchronize(pr.st));
  }
  return STM_OK;
}

int stm_pruner_train_step(stm_pruner* P, const stm_points* model, const stm_points* scene, const stm_params* params,
                          const int32_t* groups, const int32_t* labels, int32_t G, float lr, float* loss,
                          void* hip_stream) {
  err().clear();
  if (!(lr >= 0.f) || !std::isfinite(lr)) return fail(STM_EINVAL, "learning rate must be finite and >= 0");
  Prepared pr;
  int rc = gradient(P, model, scene, params, groups, labels, G, loss, nullptr, hip_stream, pr);
  if (rc) return rc;
  const long long t = ++P->step;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = static_cast<float>(1.0 - std::pow(b1, (double)t));
  const float c2 = static_cast<float>(1.0 - std::pow(b2, (double)t));
  STM_HIP(stm::launch_adam(as<float>(P->theta), as<const float>(P->grad), as<float>(P->am), as<float>(P->av), P->n,
                           lr, static_cast<float>(b1), static_cast<float>(b2), 1e-8f, c1, c2, pr.st));
  STM_HIP(hipStreamSynchronize(pr.st));
  return STM_OK;
}

int stm_pruner_infer(stm_pruner* P, const stm_points* model, const stm_points* scene, const stm_params* params,
                     const int32_t* groups, int32_t G, int32_t topk, float* scores, int32_t* cand, int32_t* count,
                     void* hip_stream) {
  err().clear();
  int rc = check_pruner(P);
  if (rc) return rc;
  if (topk < 1 || topk > kSlots) return fail(STM_EINVAL, "topk must be in [1, 64]");
  Prepared pr;
  if ((rc = pair_inputs(P, model, scene, params, hip_stream, pr))) return rc;
  if ((rc = stage_groups(P, pr, groups, G))) return rc;
  if (G == 0) return STM_OK;
  if ((rc = project(P, pr))) return rc;
  if ((rc = grow(P->ctx, P->cand, (size_t)G * topk * sizeof(int32_t), pr.st))) return rc;
  if ((rc = grow(P->ctx, P->count, (size_t)G * sizeof(int32_t), pr.st))) return rc;
  if ((rc = grow(P->ctx, P->scores, (size_t)G * kSlots * sizeof(float), pr.st))) return rc;
  if ((rc = grow(P->ctx, P->node, (size_t)G * kSlots * sizeof(int32_t), pr.st))) return rc;
  if ((rc = grow(P->ctx, P->phi, (size_t)G * kSlots * 8 * sizeof(float), pr.st))) return rc;
  stm::PrunerInfer q = infer_args(P, pr, topk);
  q.groups = as<const int2>(P->groups);
  q.n_groups = G;
  q.node = as<int32_t>(P->node);
  q.phi = as<float>(P->phi);
  q.cand = as<int32_t>(P->cand);
  q.count = as<int32_t>(P->count);
  q.scores = as<float>(P->scores);
  STM_HIP(stm::launch_pruner_infer(q, pr.st));
  if (scores)
    STM_HIP(hipMemcpyAsync(scores, P->scores.p, (size_t)G * kSlots * sizeof(float), hipMemcpyDeviceToHost, pr.st));
  if (cand) STM_HIP(hipMemcpyAsync(cand, P->cand.p, (size_t)G * topk * sizeof(int32_t), hipMemcpyDeviceToHost, pr.st));
  if (count) STM_HIP(hipMemcpyAsync(count, P->count.p, (size_t)G * sizeof(int32_t), hipMemcpyDeviceToHost, pr.st));
  STM_HIP(hipStreamSynchronize(pr.st));
  return STM_OK;
}

int stm_match_pruned(stm_ctx* ctx, stm_pruner* P, const stm_points* model, const stm_points* scene,
                     const stm_params* params, int32_t topk, int32_t tau_begin, int32_t tau_end, float* energy32,
                     double* energy64, double* energy_u64, int32_t* assign, int32_t* fell_back, void* hip_stream) {
  err().clear();
  int rc = check_pruner(P);
  if (rc) return rc;
  if (P->ctx != ctx) return fail(STM_EINVAL, "the pruner belongs to another context");
  if (topk < 1 || topk > kSlots) return fail(STM_EINVAL, "topk must be in [1, 64]");
  if (params && dummy_on(params)) return fail(STM_EUNSUPPORTED, "pruned matching with dummy assignments is not built");
  if (params && (params->flags & (STM_ANGLE_UNSIGNED | STM_CAUSAL_NODE)))
    return fail(STM_EUNSUPPORTED, "pruned matching with unsigned angles or node-order causality is not built");
  Prepared pr;
  if ((rc = pair_inputs(P, model, scene, params, hip_stream, pr))) return rc;
  if ((rc = check_range(pr, tau_begin, tau_end))) return rc;
  const int n_tau = tau_end - tau_begin;
  if (n_tau == 0) return STM_OK;
  if (!energy32 || !assign) return fail(STM_EINVAL, "energy32 and assign are required");
  const int M = pr.m.M;
  Outs o;
  if ((rc = outputs(ctx, &P->fell, pr, n_tau, energy32, energy64, energy_u64, assign, fell_back, o))) return rc;
  if (o.fell) STM_HIP(stm::launch_fill_i32(o.fell, n_tau, 0, pr.st));
  if ((rc = grow(ctx, ctx->theta, (size_t)M * sizeof(float2), pr.st))) return rc;
  STM_HIP(stm::launch_model_angles(pr.m, static_cast<float2*>(ctx->theta.p), pr.st));
  // the time-nearest rule keeps the windowed rule's first topk candidates: the
  // recursion builds them itself (K = topk) and the network is not evaluated
  const bool scored = P->rule != STM_PRUNE_TIME_NEAREST;
  if (scored && (rc = project(P, pr))) return rc;

  // pruned lists and the recursion on them, in chunks of offsets
  const int kp = std::min(topk, pr.sp.K);
  const int chunk = dp_chunk(ctx, pr, params, n_tau, kp, (size_t)std::max(1, (1 << 20) / M));
  if ((rc = dp_scratch(ctx, pr, params, chunk, kp))) return rc;
  stm::PrunerInfer q = infer_args(P, pr, kp);
  stm::DPLaunch b = dp_base(ctx, pr, params);
  b.sp.K = kp;
  if (scored) {
    if ((rc = grow(ctx, P->cand, (size_t)chunk * M * kp * sizeof(int32_t), pr.st))) return rc;
    if ((rc = grow(ctx, P->count, (size_t)chunk * M * sizeof(int32_t), pr.st))) return rc;
    if ((rc = grow(ctx, P->node, (size_t)chunk * M * kSlots * sizeof(int32_t), pr.st))) return rc;
    if ((rc = grow(ctx, P->phi, (size_t)chunk * M * kSlots * 8 * sizeof(float), pr.st))) return rc;
    q.cand = as<int32_t>(P->cand);
    q.count = as<int32_t>(P->count);
    q.node = as<int32_t>(P->node);
    q.phi = as<float>(P->phi);
    b.cand = q.cand;
    b.ccount = q.count;
    b.cstride = kp;
  }
  for (int c0 = 0; c0 < n_tau; c0 += chunk) {
    const int nc = std::min(chunk, n_tau - c0);
    q.tau0 = tau_begin + c0;
    q.n_groups = (long long)nc * M;
    if (scored) STM_HIP(stm::launch_pruner_infer(q, pr.st));
    b.tau0 = tau_begin + c0;
    b.n_tau = nc;
    if ((rc = dp_rows(pr, params, b, o.e32 + c0, o.e64 ? o.e64 + c0 : nullptr, o.eu ? o.eu + c0 : nullptr,
                      o.as + (size_t)c0 * M)))
      return rc;
  }
  const FallbackBufs fb{&P->taus, &P->f32, &P->f64, &P->fu, &P->fas};
  if ((rc = exact_fallback(ctx, fb, pr, params, tau_begin, n_tau, o))) return rc;
  return copy_back(pr, n_tau, o, energy32, energy64, energy_u64, assign, fell_back);
}

int stm_match_lists(stm_ctx* ctx, const stm_points* model, const stm_points* scene, const stm_params* params,
                    int32_t tau_begin, int32_t tau_end, const int32_t* cand, const int32_t* count, int32_t kc,
                    float* energy32, double* energy64, double* energy_u64, int32_t* assign, void* hip_stream) {
  err().clear();
  if (params && (params->flags & STM_CAUSAL_NODE))
    return fail(STM_EUNSUPPORTED, "node-order causality on given lists is not built");
  Prepared pr;
  int rc = prepare(ctx, model, scene, params, hip_stream, pr);
  if (rc) return rc;
  if ((rc = check_range(pr, tau_begin, tau_end))) return rc;
  const int n_tau = tau_end - tau_begin;
  if (n_tau == 0) return STM_OK;
  if (!energy32 || !assign || !cand || !count) return fail(STM_EINVAL, "cand, count, energy32 and assign are required");
  if (kc < 1 || kc > kSlots) return fail(STM_EINVAL, "list stride kc must be in [1, 64]");
  const int M = pr.m.M, S = pr.s.S;
  const long long rows = (long long)n_tau * M;
  const int32_t* d_cand = cand;
  const int32_t* d_cnt = count;
  if (pr.device) {
    if ((rc = grow(ctx, ctx->val, sizeof(int32_t), pr.st))) return rc;
    STM_HIP(stm::launch_fill_i32(static_cast<int32_t*>(ctx->val.p), 1, 0, pr.st));
    STM_HIP(stm::launch_check_lists(cand, count, rows, kc, S, static_cast<int32_t*>(ctx->val.p), pr.st));
    int32_t bad = 0;
    STM_HIP(hipMemcpyAsync(&bad, ctx->val.p, sizeof(bad), hipMemcpyDeviceToHost, pr.st));
    STM_HIP(hipStreamSynchronize(pr.st));
    if (bad) return fail(STM_EINVAL, "candidate lists: count outside [0, kc], node outside the scene or not ascending");
  } else {
    for (long long r = 0; r < rows; ++r) {
      const int n = count[r];
      if (n < 0 || n > kc) return fail(STM_EINVAL, "candidate count outside [0, kc]");
      for (int a = 0; a < n; ++a) {
        const int v = cand[r * kc + a];
        if (v < 0 || v >= S || (a > 0 && v <= cand[r * kc + a - 1]))
          return fail(STM_EINVAL, "candidate lists must hold ascending scene nodes");
      }
    }
    if ((rc = grow(ctx, ctx->o_cand, (size_t)rows * kc * sizeof(int32_t), pr.st))) return rc;
    if ((rc = grow(ctx, ctx->o_cnt, (size_t)rows * sizeof(int32_t), pr.st))) return rc;
    STM_HIP(hipMemcpyAsync(ctx->o_cand.p, cand, (size_t)rows * kc * sizeof(int32_t), hipMemcpyHostToDevice, pr.st));
    STM_HIP(hipMemcpyAsync(ctx->o_cnt.p, count, (size_t)rows * sizeof(int32_t), hipMemcpyHostToDevice, pr.st));
    d_cand = static_cast<const int32_t*>(ctx->o_cand.p);
    d_cnt = static_cast<const int32_t*>(ctx->o_cnt.p);
  }
  Outs o;
  if ((rc = outputs(ctx, nullptr, pr, n_tau, energy32, energy64, energy_u64, assign, nullptr, o))) return rc;
  if ((rc = grow(ctx, ctx->theta, (size_t)M * sizeof(float2), pr.st))) return rc;
  STM_HIP(stm::launch_model_angles(pr.m, static_cast<float2*>(ctx->theta.p), pr.st));
  if ((rc = grow(ctx, ctx->U, (size_t)M * S * sizeof(float), pr.st))) return rc;
  if ((rc = unary_table(ctx, pr, static_cast<float*>(ctx->U.p)))) return rc;
  const int chunk = dp_chunk(ctx, pr, params, n_tau, kc, (size_t)n_tau);
  if ((rc = dp_scratch(ctx, pr, params, chunk, kc))) return rc;
  stm::DPLaunch b = dp_base(ctx, pr, params);
  b.sp.K = kc;
  b.cstride = kc;
  for (int c0 = 0; c0 < n_tau; c0 += chunk) {
    const int nc = std::min(chunk, n_tau - c0);
    b.cand = d_cand + (size_t)c0 * M * kc;
    b.ccount = d_cnt + (size_t)c0 * M;
    b.tau0 = tau_begin + c0;
    b.n_tau = nc;
    if ((rc = dp_rows(pr, params, b, o.e32 + c0, o.e64 ? o.e64 + c0 : nullptr, o.eu ? o.eu + c0 : nullptr,
                      o.as + (size_t)c0 * M)))
      return rc;
  }
  if (pr.device) return STM_OK;
  return copy_back(pr, n_tau, o, energy32, energy64, energy_u64, assign, nullptr);
}

}  // extern "C"
