// Host side of batched plans: many (model, scene) pairs, every offset, one
// persistent recursion launch replayed as a HIP graph, and its autotuner.
#include <cstdlib>

#include "host_common.h"

using namespace stmh;

// ---- batched plans -------------------------------------------------------------

struct stm_plan {
  stm_ctx* ctx = nullptr;
  stm_params params{};
  int n_models = 0, n_scenes = 0, n_pairs = 0;
  bool device = false, bf16 = false;
  int dim = 0;
  std::vector<stm::ModelView> mv;
  std::vector<stm::SceneView> sv;
  std::vector<int32_t> msize, mspan;
  std::vector<long long> mrow;          // first row of each model in the concatenated arrays
  long long m_total = 0;                // sum of model sizes
  int m_max = 0;
  std::vector<void*> owned;             // every device allocation of the plan
  float* mdesc_all = nullptr;           // [m_total][dim]
  float2* theta_all = nullptr;          // [m_total]
  std::vector<float*> U;                // per scene: [m_total][S]
  std::vector<int32_t*> fstart;         // per scene: [F + 1]
  uint16_t* fb_all = nullptr;           // BF16 models [mp_total][dp]
  float* fn_all = nullptr;
  long long mp_total = 0;
  std::vector<uint16_t*> gb;            // BF16 scenes [Sp][dp]
  std::vector<float*> gn;
  stm::PairDev* pairs_dev = nullptr;
  int2* items_dev = nullptr;
  int32_t n_items = 0;
  int32_t* counters = nullptr;          // [0..1] work counters, [2] degenerate count
  int32_t* degen_items = nullptr;
  float* vt = nullptr;
  long long vt_stride = 0;
  size_t vt_cap = 0;                    // floats allocated in vt
  int batch = 1;                        // items a workgroup takes at a time
  std::vector<int64_t> row_off, asg_off;
  int n_cu = 0;
  int waves = 8, wgs_per_cu = 2;
  int batch_req = 0;                    // requested batch (0: the largest that fits)
  int sched = -1;                       // schedule: -1 the rule, 0 dense, 1 packed
  // graph of the last run
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipEvent_t ev_k0 = nullptr, ev_k1 = nullptr;  // around the recursion launch, when profiled
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* cap_out[4] = {nullptr, nullptr, nullptr, nullptr};
  // staging for host-pointer runs
  float* o_e32 = nullptr;
  double* o_e64 = nullptr;
  double* o_eu = nullptr;
  int32_t* o_asg = nullptr;
  int32_t* o_fell = nullptr;
  // pruned runs: projections, per-pair lists, the exact fallback's item list
  std::vector<stm::PairDev> pairs_host;
  std::vector<int2> pair_ms;            // (model, scene) of each pair
  int pr_dim = 0, pr_k = 0;             // buffers sized for this dim / list length
  uint16_t *pr_wa = nullptr, *pr_wb = nullptr, *pr_xm = nullptr;
  float *pr_A = nullptr, *pr_norm = nullptr;
  std::vector<uint16_t*> pr_xs;
  std::vector<float*> pr_B;
  int32_t *pr_cand = nullptr, *pr_cnt = nullptr, *pr_node = nullptr, *pr_list = nullptr;
  float* pr_phi = nullptr;
  stm::PairDev* pr_pairs_dev = nullptr;
  hipGraph_t graph_pr = nullptr;
  hipGraphExec_t exec_pr = nullptr;
  const void* cap_pr[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  // runs on caller-given lists: the pair table with the lists, a check flag
  stm::PairDev* ls_pairs_dev = nullptr;
  int32_t* ls_bad = nullptr;
};

namespace {

// Allocation failure injection for tests of the error paths: while the
// environment variable STM_FAILPOINT_PLAN_ALLOC is set, every plan allocation
// larger than its value in bytes fails as if the device were out of memory.
bool plan_alloc_refused(size_t bytes) {
  const char* v = std::getenv("STM_FAILPOINT_PLAN_ALLOC");
  if (!v || !*v) return false;
  return bytes > std::strtoull(v, nullptr, 10);
}

void* plan_alloc(stm_plan* p, size_t bytes, int* rc) {
  void* q = nullptr;
  if (plan_alloc_refused(bytes) || hipMalloc(&q, bytes ? bytes : 1) != hipSuccess) {
    (void)hipGetLastError();
    *rc = fail(STM_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    return nullptr;
  }
  p->owned.push_back(q);
  return q;
}

void plan_drop_graph(stm_plan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
}

void plan_drop_pruned_graph(stm_plan* p) {
  if (p->exec_pr) (void)hipGraphExecDestroy(p->exec_pr);
  if (p->graph_pr) (void)hipGraphDestroy(p->graph_pr);
  p->exec_pr = nullptr;
  p->graph_pr = nullptr;
}

void plan_free(stm_plan* p) {
  if (!p) return;
  (void)hipSetDevice(p->ctx->device);
  (void)hipDeviceSynchronize();
  plan_drop_graph(p);
  plan_drop_pruned_graph(p);
  for (void* q : p->owned) (void)hipFree(q);
  if (p->ev_in) (void)hipEventDestroy(p->ev_in);
  if (p->ev_out) (void)hipEventDestroy(p->ev_out);
  if (p->ev_k0) (void)hipEventDestroy(p->ev_k0);
  if (p->ev_k1) (void)hipEventDestroy(p->ev_k1);
  if (p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

// Launch-shape limits: 4, 8 or 16 waves per workgroup, 1..3 resident
// workgroups per CU (16-wave workgroups at most 2), 1..kMaxBatch items per
// workgroup batch, schedule -1 (the rule), 0 (dense) or 1 (packed).
const char* shape_error(int waves, int wgs, int batch, int sched) {
  if (waves != 4 && waves != 8 && waves != 16) return "waves must be 4, 8 or 16";
  if (wgs < 1 || wgs > 3 || (waves == 16 && wgs > 2)) return "workgroups per CU must be 1..3 (1..2 with 16 waves)";
  if (batch < 0 || batch > stm::kMaxBatch) return "batch must be 0 (automatic) or 1..8";
  if (sched < -1 || sched > 1) return "schedule must be -1 (rule), 0 (dense) or 1 (packed)";
  return nullptr;
}

// The schedule variant a run uses: dummies always take the dense one; packed
// by the plan's request, or by the rule (every scene sparse).
int plan_packed(const stm_plan* p, int sched) {
  if (dummy_on(&p->params)) return 0;
  if (sched >= 0) return sched;
  int packed = 1;
  for (const auto& sv : p->sv) packed &= sparse_scene(sv.S, sv.F) ? 1 : 0;
  return packed;
}

// Waves per workgroup of the kernel a shape launches (the dummy and packed
// variants run 8 whatever the request).
int plan_eff_waves(const stm_plan* p, int waves, int sched) {
  return dummy_on(&p->params) || plan_packed(p, sched) ? 8 : waves;
}

// Makes (waves, wgs, batch_req, sched) the plan's launch shape, with the
// value-table scratch it needs: batch items per workgroup, each item's tables
// vt_stride floats.  batch_req 0 takes the largest batch (at most kMaxBatch
// and the workgroup's waves) whose tables fit an eighth of the free device
// memory and 16 GiB, halved while the allocation fails, down to one; a given
// batch must fit as it is.  The shape is committed only once its scratch is
// in place: on failure the plan keeps its previous shape, batch and scratch,
// so a later run never indexes past the buffer it has.  Graphs captured with
// the previous shape are dropped.
int plan_set_shape(stm_plan* p, int waves, int wgs, int batch_req, int sched) {
  const int nw = plan_eff_waves(p, waves, sched);
  const size_t per_batch = (size_t)p->n_cu * wgs * (size_t)p->vt_stride;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    (void)hipGetLastError();
    free_b = 0;
  }
  const size_t budget = std::min<size_t>(size_t(16) << 30, free_b / 8);
  int batch = batch_req > 0 ? batch_req : std::min(stm::kMaxBatch, nw);
  if (batch_req <= 0)
    while (batch > 1 && per_batch * batch * sizeof(float) > budget) --batch;
  for (;;) {
    const size_t need = per_batch * batch;
    if (need > p->vt_cap) {
      int rc = STM_OK;
      float* q = static_cast<float*>(plan_alloc(p, need * sizeof(float), &rc));
      if (!q) {
        if (batch_req > 0 || batch == 1) return rc;
        batch = batch / 2;
        continue;
      }
      p->vt = q;  // an older, smaller buffer stays owned until the plan is freed
      p->vt_cap = need;
      err().clear();
    }
    break;
  }
  if (p->waves != waves || p->wgs_per_cu != wgs || p->batch != batch || p->sched != sched) {
    plan_drop_graph(p);
    plan_drop_pruned_graph(p);
  }
  p->waves = waves;
  p->wgs_per_cu = wgs;
  p->batch = batch;
  p->batch_req = batch_req;
  p->sched = sched;
  return STM_OK;
}

stm::BatchLaunch plan_launch(stm_plan* p, const stm::PairDev* pairs, const int2* items, int n_items,
                             float* e32, int32_t* assign) {
  stm::BatchLaunch b;
  b.pairs = pairs;
  b.items = items;
  b.n_items = n_items;
  b.counter = p->counters;
  b.degen_count = p->counters + 2;
  b.degen_items = p->degen_items;
  b.sp = stmh::search_params(&p->params, p->params.window);
  b.lambda1 = static_cast<float>(p->params.lambda1);
  b.lambda2 = static_cast<float>(p->params.lambda2);
  b.w = static_cast<float>(p->params.lambda2 * p->params.lambda3);
  b.vt = p->vt;
  b.vt_stride = p->vt_stride;
  b.batch = p->batch;
  b.dummy = dummy_on(&p->params) ? 1 : 0;
  b.cw = dummy_cost32(&p->params);
  b.packed = plan_packed(p, p->sched);
  b.e32 = e32;
  b.assign = assign;
  b.waves = p->waves;
  return b;
}

// Queues the frame indices, model angles and unary tables of every scene.
int plan_enqueue_tables(stm_plan* p, hipStream_t st) {
  for (int j = 0; j < p->n_scenes; ++j)
    STM_HIP(stm::launch_fstart(p->sv[j].t, p->sv[j].S, p->sv[j].F, p->fstart[j], st));
  for (int i = 0; i < p->n_models; ++i)
    STM_HIP(stm::launch_model_angles(p->mv[i], p->theta_all + p->mrow[i], st));
  stm::ModelView all{nullptr, nullptr, p->mdesc_all, static_cast<int32_t>(p->m_total)};
  if (p->bf16)
    STM_HIP(stm::launch_to_bf16(p->mdesc_all, static_cast<int32_t>(p->m_total), p->dim,
                                static_cast<int32_t>(p->mp_total), p->fb_all, p->fn_all, st));
  for (int j = 0; j < p->n_scenes; ++j) {
    if (p->bf16) {
      const int32_t sp = (p->sv[j].S + 255) / 256 * 256;
      STM_HIP(stm::launch_to_bf16(p->sv[j].desc, p->sv[j].S, p->dim, sp, p->gb[j], p->gn[j], st));
      STM_HIP(stm::launch_unary_bf16(p->fb_all, p->fn_all, static_cast<int32_t>(p->m_total), p->gb[j],
                                     p->gn[j], p->sv[j].S, p->dim, p->U[j], st));
    } else {
      STM_HIP(stm::launch_unary_f32(all, p->sv[j], p->U[j], st));
    }
  }
  return STM_OK;
}

int plan_enqueue_run(stm_plan* p, float* e32, double* e64, double* eu, int32_t* assign, hipStream_t st,
                     bool timed) {
  int rc;
  if ((rc = plan_enqueue_tables(p, st))) return rc;
  STM_HIP(stm::launch_fill_i32(p->counters, 3, 0, st));
  const stm::BatchLaunch b = plan_launch(p, p->pairs_dev, p->items_dev, p->n_items, e32, assign);
  // timed: the two events bracket the recursion launches (the fast persistent
  // kernel and the re-run of flagged degenerate matchings)
  if (timed) STM_HIP(hipEventRecord(p->ev_k0, st));
  STM_HIP(stm::launch_dp_persistent(b, p->n_cu * p->wgs_per_cu, st));
  if (timed) STM_HIP(hipEventRecord(p->ev_k1, st));
  STM_HIP(stm::launch_rescore_batch(p->pairs_dev, p->items_dev, p->n_items, stmh::search_params(&p->params, p->params.window),
                                    p->params.lambda1, p->params.lambda2, p->params.lambda3,
                                    w_dummy_of(&p->params), assign, e64, eu, st));
  return STM_OK;
}

std::string plan_key(const stm_plan* p) {
  int k = 1;
  while (k < p->params.k_max) k <<= 1;
  const int mb = (p->m_max + 31) / 32 * 32;
  return std::string("gfx950/K") + std::to_string(k) + "/M" + std::to_string(mb) + "/dens" +
         ((p->params.flags & STM_K_DENSITY) ? "1" : "0") + (p->bf16 ? "/bf16" : "/f32") +
         (dummy_on(&p->params) ? "/dummy" : "") + (plan_packed(p, -1) ? "/sparse" : "/dense");
}

}  // namespace

extern "C" {

int stm_plan_create(stm_ctx* ctx, const stm_points* models, int32_t n_models, const stm_points* scenes,
                    int32_t n_scenes, const int32_t* pairs, int32_t n_pairs, const stm_params* params,
                    stm_plan** out) {
  err().clear();
  if (!out) return fail(STM_EINVAL, "null output pointer");
  *out = nullptr;
  if (!ctx || !models || !scenes || !params || (n_pairs > 0 && !pairs))
    return fail(STM_EINVAL, "null argument");
  if (n_models < 1 || n_scenes < 1 || n_pairs < 0) return fail(STM_EINVAL, "empty batch");
  int rc;
  for (int i = 0; i < n_models; ++i)
    for (int j = 0; j < n_scenes; ++j)
      if ((i == 0 || j == 0) && (rc = check_shapes(&models[i], &scenes[j], params))) return rc;
  for (int q = 0; q < n_pairs; ++q)
    if (pairs[2 * q] < 0 || pairs[2 * q] >= n_models || pairs[2 * q + 1] < 0 || pairs[2 * q + 1] >= n_scenes)
      return fail(STM_EINVAL, "pair index out of range");
  STM_HIP(hipSetDevice(ctx->device));
  stm_plan* p = new (std::nothrow) stm_plan();
  if (!p) return fail(STM_ENOMEM, "host allocation failed");
  p->ctx = ctx;
  p->params = *params;
  p->n_models = n_models;
  p->n_scenes = n_scenes;
  p->n_pairs = n_pairs;
  p->device = (params->flags & STM_DEVICE_PTRS) != 0;
  p->bf16 = (params->flags & STM_UNARY_BF16) != 0;
  p->dim = models[0].dim;
  {  // a window wider than every scene adds only empty frames
    int32_t fmax = 1;
    for (int j = 0; j < n_scenes; ++j) fmax = std::max(fmax, scenes[j].n_frames);
    p->params.window = std::min(params->window, fmax);
  }
  rc = [&]() -> int {
    int rc2 = STM_OK;
    hipDeviceProp_t prop;
    STM_HIP(hipGetDeviceProperties(&prop, ctx->device));
    p->n_cu = prop.multiProcessorCount;
    STM_HIP(hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking));
    STM_HIP(hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming));
    STM_HIP(hipEventCreateWithFlags(&p->ev_out, hipEventDisableTiming));
    STM_HIP(hipEventCreate(&p->ev_k0));
    STM_HIP(hipEventCreate(&p->ev_k1));
    const hipStream_t st = p->stream;
    // point sets on the device, validated
    p->mv.resize(n_models);
    p->sv.resize(n_scenes);
    p->msize.resize(n_models);
    p->mspan.resize(n_models);
    p->mrow.resize(n_models);
    if (!p->device) {
      for (int i = 0; i < n_models; ++i)
        if (int bits = host_validate(&models[i], &scenes[0]) & 9) return fail(STM_EINVAL, bit_message(bits));
      for (int j = 0; j < n_scenes; ++j)
        if (int bits = host_validate(&models[0], &scenes[j]) & 22) return fail(STM_EINVAL, bit_message(bits));
      auto up = [&](const void* h, size_t bytes) -> void* {
        void* d = plan_alloc(p, bytes, &rc2);
        if (d && hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st) != hipSuccess) {
          rc2 = fail(STM_EHIP, "host-to-device copy failed");
          return nullptr;
        }
        return d;
      };
      for (int i = 0; i < n_models; ++i) {
        const stm_points& m = models[i];
        void* xy = up(m.xy, (size_t)m.n * 2 * sizeof(float));
        void* t = up(m.t, (size_t)m.n * sizeof(int32_t));
        void* d = up(m.desc, (size_t)m.n * m.dim * sizeof(float));
        if (!xy || !t || !d) return rc2;
        p->mv[i] = {static_cast<const float2*>(xy), static_cast<const int32_t*>(t),
                    static_cast<const float*>(d), m.n};
        p->mspan[i] = m.t[m.n - 1] - m.t[0];
      }
      for (int j = 0; j < n_scenes; ++j) {
        const stm_points& s = scenes[j];
        void* xy = up(s.xy, (size_t)s.n * 2 * sizeof(float));
        void* t = up(s.t, (size_t)s.n * sizeof(int32_t));
        void* d = up(s.desc, (size_t)s.n * s.dim * sizeof(float));
        if (!xy || !t || !d) return rc2;
        p->sv[j] = {static_cast<const float2*>(xy), static_cast<const int32_t*>(t),
                    static_cast<const float*>(d), nullptr, s.n, s.n_frames, s.dim};
      }
    } else {
      for (int i = 0; i < n_models; ++i)
        p->mv[i] = {reinterpret_cast<const float2*>(models[i].xy), models[i].t, models[i].desc, models[i].n};
      for (int j = 0; j < n_scenes; ++j)
        p->sv[j] = {reinterpret_cast<const float2*>(scenes[j].xy), scenes[j].t, scenes[j].desc, nullptr,
                    scenes[j].n, scenes[j].n_frames, scenes[j].dim};
      const int nv = n_models + n_scenes;
      int32_t* val = static_cast<int32_t*>(plan_alloc(p, (size_t)nv * 2 * sizeof(int32_t), &rc2));
      if (!val) return rc2;
      STM_HIP(hipMemsetAsync(val, 0, (size_t)nv * 2 * sizeof(int32_t), st));
      for (int i = 0; i < n_models; ++i) STM_HIP(stm::launch_validate(p->mv[i], p->sv[0], val + 2 * i, st));
      for (int j = 0; j < n_scenes; ++j)
        STM_HIP(stm::launch_validate(p->mv[0], p->sv[j], val + 2 * (n_models + j), st));
      std::vector<int32_t> hv((size_t)nv * 2);
      STM_HIP(hipMemcpyAsync(hv.data(), val, hv.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
      STM_HIP(hipStreamSynchronize(st));
      for (int i = 0; i < n_models; ++i) {
        if (hv[2 * i] & 9) return fail(STM_EINVAL, bit_message(hv[2 * i] & 9));
        p->mspan[i] = hv[2 * i + 1];
      }
      for (int j = 0; j < n_scenes; ++j)
        if (hv[2 * (n_models + j)] & 22) return fail(STM_EINVAL, bit_message(hv[2 * (n_models + j)] & 22));
    }
    // concatenated model arrays
    for (int i = 0; i < n_models; ++i) {
      p->msize[i] = p->mv[i].M;
      p->mrow[i] = p->m_total;
      p->m_total += p->mv[i].M;
      p->m_max = std::max(p->m_max, p->mv[i].M);
    }
    p->mdesc_all = static_cast<float*>(plan_alloc(p, (size_t)p->m_total * p->dim * sizeof(float), &rc2));
    p->theta_all = static_cast<float2*>(plan_alloc(p, (size_t)p->m_total * sizeof(float2), &rc2));
    if (!p->mdesc_all || !p->theta_all) return rc2;
    for (int i = 0; i < n_models; ++i)
      STM_HIP(hipMemcpyAsync(p->mdesc_all + p->mrow[i] * p->dim, p->mv[i].desc,
                             (size_t)p->mv[i].M * p->dim * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (p->bf16) {
      p->mp_total = (p->m_total + 15) / 16 * 16;
      const int dp = stm::bf16_padded_dim(p->dim);
      p->fb_all = static_cast<uint16_t*>(plan_alloc(p, (size_t)p->mp_total * dp * 2, &rc2));
      p->fn_all = static_cast<float*>(plan_alloc(p, (size_t)p->mp_total * sizeof(float), &rc2));
      if (!p->fb_all || !p->fn_all) return rc2;
    }
    // per scene: frame index, unary table (and BF16 copies)
    p->U.resize(n_scenes);
    p->fstart.resize(n_scenes);
    p->gb.resize(n_scenes);
    p->gn.resize(n_scenes);
    for (int j = 0; j < n_scenes; ++j) {
      p->fstart[j] = static_cast<int32_t*>(plan_alloc(p, ((size_t)p->sv[j].F + 1) * sizeof(int32_t), &rc2));
      p->U[j] = static_cast<float*>(plan_alloc(p, (size_t)p->m_total * p->sv[j].S * sizeof(float), &rc2));
      if (!p->fstart[j] || !p->U[j]) return rc2;
      p->sv[j].fstart = p->fstart[j];
      if (p->bf16) {
        const size_t sp = (size_t)(p->sv[j].S + 255) / 256 * 256;
        p->gb[j] = static_cast<uint16_t*>(plan_alloc(p, sp * stm::bf16_padded_dim(p->dim) * 2, &rc2));
        p->gn[j] = static_cast<float*>(plan_alloc(p, sp * sizeof(float), &rc2));
        if (!p->gb[j] || !p->gn[j]) return rc2;
      }
      STM_HIP(stm::launch_fstart(p->sv[j].t, p->sv[j].S, p->sv[j].F, p->fstart[j], st));
    }
    // pair table, output layout, work items
    std::vector<stm::PairDev> ph((size_t)n_pairs);
    p->row_off.assign((size_t)n_pairs + 1, 0);
    p->asg_off.assign((size_t)n_pairs + 1, 0);
    std::vector<int2> items;
    for (int q = 0; q < n_pairs; ++q) {
      const int i = pairs[2 * q], j = pairs[2 * q + 1];
      const long long n_tau = std::max(0LL, (long long)p->sv[j].F - p->mspan[i]);
      stm::PairDev& d = ph[q];
      d.m = p->mv[i];
      d.s = p->sv[j];
      d.us = p->sv[j].S;
      d.U = p->U[j] + p->mrow[i] * d.us;
      d.theta = p->theta_all + p->mrow[i];
      d.row0 = p->row_off[q];
      d.assign0 = p->asg_off[q];
      d.n_tau = static_cast<int32_t>(n_tau);
      p->row_off[q + 1] = p->row_off[q] + n_tau;
      p->asg_off[q + 1] = p->asg_off[q] + n_tau * p->mv[i].M;
      for (int t = 0; t < n_tau; ++t) items.push_back(make_int2(q, t));
    }
    if (items.size() > 0x7fffffffULL) return fail(STM_EUNSUPPORTED, "more than 2^31 matchings in one plan");
    p->n_items = static_cast<int32_t>(items.size());
    p->pairs_dev = static_cast<stm::PairDev*>(plan_alloc(p, ph.size() * sizeof(stm::PairDev), &rc2));
    p->items_dev = static_cast<int2*>(plan_alloc(p, items.size() * sizeof(int2), &rc2));
    p->counters = static_cast<int32_t*>(plan_alloc(p, 4 * sizeof(int32_t), &rc2));
    p->degen_items = static_cast<int32_t*>(plan_alloc(p, items.size() * sizeof(int32_t), &rc2));
    long long* cost = static_cast<long long*>(plan_alloc(p, items.size() * sizeof(long long), &rc2));
    if (!p->pairs_dev || !p->items_dev || !p->counters || !p->degen_items || !cost) return rc2;
    if (!ph.empty())
      STM_HIP(hipMemcpyAsync(p->pairs_dev, ph.data(), ph.size() * sizeof(stm::PairDev), hipMemcpyHostToDevice, st));
    p->pairs_host = ph;
    p->pair_ms.resize(n_pairs);
    for (int q = 0; q < n_pairs; ++q) p->pair_ms[q] = make_int2(pairs[2 * q], pairs[2 * q + 1]);
    if (!items.empty()) {
      STM_HIP(hipMemcpyAsync(p->items_dev, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice, st));
      const stm::SearchParams sp = stmh::search_params(&p->params, p->params.window);
      STM_HIP(stm::launch_item_cost(p->pairs_dev, p->items_dev, p->n_items, sp, cost, st));
      std::vector<long long> hc(items.size());
      STM_HIP(hipMemcpyAsync(hc.data(), cost, hc.size() * sizeof(long long), hipMemcpyDeviceToHost, st));
      STM_HIP(hipStreamSynchronize(st));
      std::vector<int32_t> order(items.size());
      for (size_t k = 0; k < order.size(); ++k) order[k] = static_cast<int32_t>(k);
      std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return hc[a] > hc[b]; });
      std::vector<int2> sorted(items.size());
      for (size_t k = 0; k < order.size(); ++k) sorted[k] = items[order[k]];
      STM_HIP(hipMemcpyAsync(p->items_dev, sorted.data(), sorted.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    }
    p->vt_stride = (long long)std::max(1, p->m_max - 2) * vt_side(params) * vt_side(params);
    if ((rc2 = plan_set_shape(p, p->waves, p->wgs_per_cu, 0, -1))) return rc2;
    if (!p->device) {
      const int64_t nr = p->row_off.back(), na = p->asg_off.back();
      p->o_e32 = static_cast<float*>(plan_alloc(p, (size_t)nr * sizeof(float), &rc2));
      p->o_e64 = static_cast<double*>(plan_alloc(p, (size_t)nr * sizeof(double), &rc2));
      p->o_eu = static_cast<double*>(plan_alloc(p, (size_t)nr * sizeof(double), &rc2));
      p->o_asg = static_cast<int32_t*>(plan_alloc(p, (size_t)na * sizeof(int32_t), &rc2));
      if (!p->o_e32 || !p->o_e64 || !p->o_eu || !p->o_asg) return rc2;
    }
    STM_HIP(hipStreamSynchronize(st));
    return STM_OK;
  }();
  if (rc) {
    std::string msg = err();
    plan_free(p);
    err() = msg;
    return rc;
  }
  *out = p;
  return STM_OK;
}

void stm_plan_destroy(stm_plan* plan) { plan_free(plan); }

int stm_plan_rows(const stm_plan* p, int64_t* row_offsets, int64_t* assign_offsets, int64_t* n_rows,
                  int64_t* n_assign) {
  err().clear();
  if (!p) return fail(STM_EINVAL, "null plan");
  if (row_offsets) std::copy(p->row_off.begin(), p->row_off.end(), row_offsets);
  if (assign_offsets) std::copy(p->asg_off.begin(), p->asg_off.end(), assign_offsets);
  if (n_rows) *n_rows = p->row_off.back();
  if (n_assign) *n_assign = p->asg_off.back();
  return STM_OK;
}

int stm_plan_set_tuning(stm_plan* p, int32_t waves, int32_t wgs_per_cu) {
  err().clear();
  if (!p) return fail(STM_EINVAL, "null plan");
  if (const char* e = shape_error(waves, wgs_per_cu, 0, -1)) return fail(STM_EINVAL, e);
  STM_HIP(hipSetDevice(p->ctx->device));
  STM_HIP(hipStreamSynchronize(p->stream));
  return plan_set_shape(p, waves, wgs_per_cu, p->batch_req, p->sched);
}

int stm_plan_set_shape(stm_plan* p, const int32_t* shape) {
  err().clear();
  if (!p || !shape) return fail(STM_EINVAL, "null plan or shape");
  if (const char* e = shape_error(shape[0], shape[1], shape[2], shape[3])) return fail(STM_EINVAL, e);
  STM_HIP(hipSetDevice(p->ctx->device));
  STM_HIP(hipStreamSynchronize(p->stream));
  return plan_set_shape(p, shape[0], shape[1], shape[2], shape[3]);
}

int stm_plan_get_shape(const stm_plan* p, int32_t* shape) {
  err().clear();
  if (!p || !shape) return fail(STM_EINVAL, "null plan or shape");
  shape[0] = plan_eff_waves(p, p->waves, p->sched);
  shape[1] = p->wgs_per_cu;
  shape[2] = std::min(p->batch, shape[0]);
  shape[3] = plan_packed(p, p->sched);
  return STM_OK;
}

int stm_plan_run(stm_plan* p, float* energy32, double* energy64, double* energy_u64, int32_t* assign,
                 void* hip_stream) {
  err().clear();
  if (!p) return fail(STM_EINVAL, "null plan");
  if (p->row_off.back() > 0 && (!energy32 || !assign)) return fail(STM_EINVAL, "energy32 and assign are required");
  STM_HIP(hipSetDevice(p->ctx->device));
  const hipStream_t user = static_cast<hipStream_t>(hip_stream);
  float* e32 = p->device ? energy32 : p->o_e32;
  double* e64 = p->device ? energy64 : (energy64 ? p->o_e64 : nullptr);
  double* eu = p->device ? energy_u64 : (energy_u64 ? p->o_eu : nullptr);
  int32_t* asg = p->device ? assign : p->o_asg;
  const void* outs[4] = {e32, e64, eu, asg};
  // timed runs launch the same kernels directly on the plan stream, with two
  // events around the recursion launches (HIP cannot time events recorded
  // inside a graph); other runs replay the captured graph
  const bool timed = p->ctx->prof;
  if (!timed && (!p->exec || !std::equal(outs, outs + 4, p->cap_out))) {
    plan_drop_graph(p);
    STM_HIP(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
    int rc = plan_enqueue_run(p, e32, e64, eu, asg, p->stream, false);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(p->stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess) return fail(STM_EHIP, std::string("graph capture: ") + hipGetErrorString(ec));
    p->graph = g;
    STM_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    std::copy(outs, outs + 4, p->cap_out);
  }
  // order: caller's stream -> plan stream (graph) -> caller's stream
  STM_HIP(hipEventRecord(p->ev_in, user));
  STM_HIP(hipStreamWaitEvent(p->stream, p->ev_in, 0));
  if (timed) {
    int rc = plan_enqueue_run(p, e32, e64, eu, asg, p->stream, true);
    if (rc) return rc;
  } else {
    STM_HIP(hipGraphLaunch(p->exec, p->stream));
  }
  STM_HIP(hipEventRecord(p->ev_out, p->stream));
  STM_HIP(hipStreamWaitEvent(user, p->ev_out, 0));
  if (timed) {  // the events are re-recorded by every timed run: read this one's now
    STM_HIP(hipEventSynchronize(p->ev_k1));
    float ms = 0.f;
    STM_HIP(hipEventElapsedTime(&ms, p->ev_k0, p->ev_k1));
    p->ctx->prof_plan_ms += ms;
    p->ctx->prof_plan_launches += 1;
    p->ctx->prof_matchings += p->row_off.back();
  }
  if (!p->device) {
    const int64_t nr = p->row_off.back(), na = p->asg_off.back();
    STM_HIP(hipMemcpyAsync(energy32, e32, (size_t)nr * sizeof(float), hipMemcpyDeviceToHost, p->stream));
    STM_HIP(hipMemcpyAsync(assign, asg, (size_t)na * sizeof(int32_t), hipMemcpyDeviceToHost, p->stream));
    if (energy64)
      STM_HIP(hipMemcpyAsync(energy64, e64, (size_t)nr * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    if (energy_u64)
      STM_HIP(hipMemcpyAsync(energy_u64, eu, (size_t)nr * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    STM_HIP(hipStreamSynchronize(p->stream));
  }
  return STM_OK;
}

}  // extern "C"

// ---- pruned plan runs ------------------------------------------------------------

namespace {

constexpr int kHid = stm::kPrunerHidden;

// Buffers of pruned runs for pruner dimension `dim` and lists of `kp` nodes.
int plan_pruned_buffers(stm_plan* p, int dim, int kp) {
  int rc = STM_OK;
  if (p->pr_dim != dim) {
    const int dp = stm::bf16_padded_dim(dim);
    const long long mp = (p->m_total + 15) / 16 * 16;
    p->pr_wa = static_cast<uint16_t*>(plan_alloc(p, (size_t)kHid * dp * 2, &rc));
    p->pr_wb = static_cast<uint16_t*>(plan_alloc(p, (size_t)kHid * dp * 2, &rc));
    p->pr_xm = static_cast<uint16_t*>(plan_alloc(p, (size_t)mp * dp * 2, &rc));
    p->pr_A = static_cast<float*>(plan_alloc(p, (size_t)std::max(1LL, p->m_total) * kHid * sizeof(float), &rc));
    long long smax = 16;
    for (const auto& sv : p->sv) smax = std::max<long long>(smax, (sv.S + 15) / 16 * 16);
    p->pr_norm = static_cast<float*>(plan_alloc(p, (size_t)std::max(mp, smax) * sizeof(float), &rc));
    p->pr_xs.assign(p->n_scenes, nullptr);
    p->pr_B.assign(p->n_scenes, nullptr);
    for (int j = 0; j < p->n_scenes; ++j) {
      const size_t sp = (size_t)(p->sv[j].S + 15) / 16 * 16;
      p->pr_xs[j] = static_cast<uint16_t*>(plan_alloc(p, sp * dp * 2, &rc));
      p->pr_B[j] = static_cast<float*>(plan_alloc(p, (size_t)std::max(1, p->sv[j].S) * kHid * sizeof(float), &rc));
    }
    if (rc) return rc;
    p->pr_dim = dim;
  }
  if (p->pr_k < kp) {
    long long groups = 0, gmax = 1;
    for (const auto& d : p->pairs_host) {
      groups += (long long)d.n_tau * d.m.M;
      gmax = std::max(gmax, (long long)d.n_tau * d.m.M);
    }
    p->pr_cand = static_cast<int32_t*>(plan_alloc(p, (size_t)std::max(1LL, groups) * kp * sizeof(int32_t), &rc));
    p->pr_cnt = static_cast<int32_t*>(plan_alloc(p, (size_t)std::max(1LL, groups) * sizeof(int32_t), &rc));
    if (!p->pr_node) {
      p->pr_node = static_cast<int32_t*>(plan_alloc(p, (size_t)gmax * 64 * sizeof(int32_t), &rc));
      p->pr_phi = static_cast<float*>(plan_alloc(p, (size_t)gmax * 64 * 8 * sizeof(float), &rc));
      p->pr_list = static_cast<int32_t*>(plan_alloc(p, (size_t)std::max(1, p->n_items) * sizeof(int32_t), &rc));
      p->pr_pairs_dev = static_cast<stm::PairDev*>(
          plan_alloc(p, (size_t)std::max(1, p->n_pairs) * sizeof(stm::PairDev), &rc));
    }
    if (rc) return rc;
    // the pair table of pruned runs: each pair's lists inside pr_cand / pr_cnt
    std::vector<stm::PairDev> ph = p->pairs_host;
    long long off = 0;
    for (auto& d : ph) {
      d.cand = p->pr_cand + off * kp;
      d.ccount = p->pr_cnt + off;
      d.cstride = kp;
      off += (long long)d.n_tau * d.m.M;
    }
    if (!ph.empty())
      STM_HIP(hipMemcpy(p->pr_pairs_dev, ph.data(), ph.size() * sizeof(stm::PairDev), hipMemcpyHostToDevice));
    p->pr_k = kp;
  }
  return STM_OK;
}

// The pruner's lists of every (pair, offset, point): first-layer projections,
// then one inference launch per pair.
int plan_enqueue_lists(stm_plan* p, stm_pruner* P, int kp, hipStream_t st) {
  const int D = P->dim, NI = 2 * D + 8, dp = stm::bf16_padded_dim(D);
  const float* W1 = static_cast<const float*>(P->theta.p);
  const int mp = static_cast<int>((p->m_total + 15) / 16 * 16);
  // first-layer projections: models (with b1) and scenes
  STM_HIP(stm::launch_cast_rows_bf16(W1, kHid, NI, 0, D, dp, p->pr_wa, st));
  STM_HIP(stm::launch_cast_rows_bf16(W1, kHid, NI, D, D, dp, p->pr_wb, st));
  STM_HIP(stm::launch_to_bf16(p->mdesc_all, static_cast<int32_t>(p->m_total), D, mp, p->pr_xm, p->pr_norm, st));
  STM_HIP(stm::launch_project_bf16(p->pr_xm, static_cast<int>(p->m_total), dp, p->pr_wa, static_cast<float>(D),
                                   W1 + (long long)kHid * NI, p->pr_A, st));
  for (int j = 0; j < p->n_scenes; ++j) {
    const int S = p->sv[j].S, sp = (S + 15) / 16 * 16;
    STM_HIP(stm::launch_to_bf16(p->sv[j].desc, S, D, sp, p->pr_xs[j], p->pr_norm, st));
    STM_HIP(stm::launch_project_bf16(p->pr_xs[j], S, dp, p->pr_wb, static_cast<float>(D), nullptr, p->pr_B[j], st));
  }
  // the pruned lists of every pair
  const stm::SearchParams sp = stmh::search_params(&p->params, std::min(p->params.window, 0x3fffffff));
  long long off = 0;
  for (int q = 0; q < p->n_pairs; ++q) {
    const stm::PairDev& d = p->pairs_host[q];
    const int i = p->pair_ms[q].x, js = p->pair_ms[q].y;
    const long long G = (long long)d.n_tau * d.m.M;
    stm::PrunerInfer q_;
    q_.m = d.m;
    q_.s = d.s;
    q_.U = d.U;
    q_.us = d.us;
    q_.sp = sp;
    q_.sp.W = std::min(q_.sp.W, d.s.F);
    q_.groups = nullptr;
    q_.n_groups = G;
    q_.tau0 = 0;
    q_.node = p->pr_node;
    q_.phi = p->pr_phi;
    q_.theta = W1;
    q_.D = D;
    q_.A = p->pr_A + p->mrow[i] * kHid;
    q_.B = p->pr_B[js];
    q_.topk = kp;
    q_.rule = P->rule;
    q_.cand = p->pr_cand + off * kp;
    q_.count = p->pr_cnt + off;
    q_.scores = nullptr;
    STM_HIP(stm::launch_pruner_infer(q_, st));
    off += G;
  }
  return STM_OK;
}

int plan_enqueue_pruned(stm_plan* p, stm_pruner* P, int kp, float* e32, double* e64, double* eu, int32_t* asg,
                        int32_t* fell, hipStream_t st) {
  int rc;
  if ((rc = plan_enqueue_tables(p, st))) return rc;
  // the time-nearest rule keeps the windowed rule's first kp candidates: the
  // recursion builds them itself (K = kp) and the network is not evaluated
  const bool scored = P->rule != STM_PRUNE_TIME_NEAREST;
  if (scored && (rc = plan_enqueue_lists(p, P, kp, st))) return rc;
  // the recursion on the pruned lists, then the exact one on the items they left infeasible
  int32_t* inf_count = p->counters + 3;
  STM_HIP(stm::launch_fill_i32(p->counters, 4, 0, st));
  if (fell) STM_HIP(stm::launch_fill_i32(fell, static_cast<int>(p->row_off.back()), 0, st));
  stm::BatchLaunch b = plan_launch(p, scored ? p->pr_pairs_dev : p->pairs_dev, p->items_dev, p->n_items, e32, asg);
  b.sp.K = kp;
  STM_HIP(stm::launch_dp_persistent(b, p->n_cu * p->wgs_per_cu, st));
  STM_HIP(stm::launch_collect_infeasible(p->pairs_dev, p->items_dev, p->n_items, e32, p->pr_list, inf_count, fell,
                                         st));
  STM_HIP(stm::launch_fill_i32(p->counters, 3, 0, st));
  stm::BatchLaunch x = plan_launch(p, p->pairs_dev, p->items_dev, p->n_items, e32, asg);
  x.list = p->pr_list;
  x.list_count = inf_count;
  STM_HIP(stm::launch_dp_persistent(x, p->n_cu * p->wgs_per_cu, st));
  STM_HIP(stm::launch_rescore_batch(p->pairs_dev, p->items_dev, p->n_items, stmh::search_params(&p->params, p->params.window), p->params.lambda1,
                                    p->params.lambda2, p->params.lambda3, w_dummy_of(&p->params), asg, e64,
                                    eu, st));
  return STM_OK;
}

}  // namespace

extern "C" {

int stm_plan_run_pruned(stm_plan* p, stm_pruner* P, int32_t topk, float* energy32, double* energy64,
                        double* energy_u64, int32_t* assign, int32_t* fell_back, void* hip_stream) {
  err().clear();
  if (!p || !P) return fail(STM_EINVAL, "null plan or pruner");
  if (P->ctx != p->ctx) return fail(STM_EINVAL, "the pruner belongs to another context");
  if (P->dim != p->dim) return fail(STM_EINVAL, "descriptor dimension differs from the pruner's");
  if (topk < 1 || topk > 64) return fail(STM_EINVAL, "topk must be in [1, 64]");
  if (p->bf16) return fail(STM_EUNSUPPORTED, "pruned runs of plans with the BF16 unary table are not built");
  if (dummy_on(&p->params)) return fail(STM_EUNSUPPORTED, "pruned runs of plans with dummy assignments are not built");
  if (p->params.flags & (STM_ANGLE_UNSIGNED | STM_CAUSAL_NODE))
    return fail(STM_EUNSUPPORTED, "pruned runs of plans with unsigned angles or node-order causality are not built");
  if (p->row_off.back() > 0 && (!energy32 || !assign)) return fail(STM_EINVAL, "energy32 and assign are required");
  STM_HIP(hipSetDevice(p->ctx->device));
  const int kp = std::min<int>(topk, p->params.k_max);
  int rc;
  if ((rc = plan_pruned_buffers(p, P->dim, kp))) return rc;
  const hipStream_t user = static_cast<hipStream_t>(hip_stream);
  if (!p->device && fell_back && !p->o_fell) {
    p->o_fell = static_cast<int32_t*>(plan_alloc(p, (size_t)std::max<int64_t>(1, p->row_off.back()) * 4, &rc));
    if (rc) return rc;
  }
  float* e32 = p->device ? energy32 : p->o_e32;
  double* e64 = p->device ? energy64 : (energy64 ? p->o_e64 : nullptr);
  double* eu = p->device ? energy_u64 : (energy_u64 ? p->o_eu : nullptr);
  int32_t* asg = p->device ? assign : p->o_asg;
  int32_t* fell = p->device ? fell_back : (fell_back ? p->o_fell : nullptr);
  const void* key[7] = {e32, e64, eu, asg, fell, P, reinterpret_cast<const void*>((intptr_t)(kp * 4 + P->rule))};
  if (!p->exec_pr || !std::equal(key, key + 7, p->cap_pr)) {
    plan_drop_pruned_graph(p);
    STM_HIP(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
    rc = plan_enqueue_pruned(p, P, kp, e32, e64, eu, asg, fell, p->stream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(p->stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess) return fail(STM_EHIP, std::string("graph capture: ") + hipGetErrorString(ec));
    p->graph_pr = g;
    STM_HIP(hipGraphInstantiate(&p->exec_pr, p->graph_pr, nullptr, nullptr, 0));
    std::copy(key, key + 7, p->cap_pr);
  }
  STM_HIP(hipEventRecord(p->ev_in, user));
  STM_HIP(hipStreamWaitEvent(p->stream, p->ev_in, 0));
  STM_HIP(hipGraphLaunch(p->exec_pr, p->stream));
  STM_HIP(hipEventRecord(p->ev_out, p->stream));
  STM_HIP(hipStreamWaitEvent(user, p->ev_out, 0));
  if (!p->device) {
    const int64_t nr = p->row_off.back(), na = p->asg_off.back();
    STM_HIP(hipMemcpyAsync(energy32, e32, (size_t)nr * sizeof(float), hipMemcpyDeviceToHost, p->stream));
    STM_HIP(hipMemcpyAsync(assign, asg, (size_t)na * sizeof(int32_t), hipMemcpyDeviceToHost, p->stream));
    if (energy64)
      STM_HIP(hipMemcpyAsync(energy64, e64, (size_t)nr * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    if (energy_u64)
      STM_HIP(hipMemcpyAsync(energy_u64, eu, (size_t)nr * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    if (fell_back)
      STM_HIP(hipMemcpyAsync(fell_back, fell, (size_t)nr * sizeof(int32_t), hipMemcpyDeviceToHost, p->stream));
    STM_HIP(hipStreamSynchronize(p->stream));
  }
  return STM_OK;
}

}  // extern "C"

extern "C" {

int stm_plan_autotune(stm_plan* p, const char* cache_path, int32_t n_sample, int32_t* chosen) {
  err().clear();
  if (!p) return fail(STM_EINVAL, "null plan");
  const std::string key = plan_key(p);
  // chosen: the shape in effect (waves, workgroups per CU), whether it came
  // from the cache, the batch and the schedule variant
  auto report = [&](int cached) {
    if (!chosen) return;
    int32_t eff[4];
    (void)stm_plan_get_shape(p, eff);
    chosen[0] = eff[0];
    chosen[1] = eff[1];
    chosen[2] = cached;
    chosen[3] = eff[2];
    chosen[4] = eff[3];
  };
  // cache lookup: lines of the form
  //   "key": {"waves": W, "wgs_per_cu": G, "batch": B, "sched": S, "ms": T},
  std::vector<std::string> lines;
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char buf[512];
      while (std::fgets(buf, sizeof(buf), f)) {
        std::string line(buf);
        while (!line.empty() && (line.back() == '\n' || line.back() == '\r')) line.pop_back();
        char k[256];
        int w = 0, g = 0, bt = 0, sc = 0;
        double ms = 0;
        if (std::sscanf(line.c_str(),
                        " \"%255[^\"]\": {\"waves\": %d, \"wgs_per_cu\": %d, \"batch\": %d, \"sched\": %d, \"ms\": %lf}",
                        k, &w, &g, &bt, &sc, &ms) == 6) {
          if (key == k && !shape_error(w, g, bt, sc)) {
            std::fclose(f);
            STM_HIP(hipSetDevice(p->ctx->device));
            STM_HIP(hipStreamSynchronize(p->stream));
            int rc = plan_set_shape(p, w, g, bt, sc);
            if (rc) return rc;
            report(1);
            return STM_OK;
          }
          lines.push_back(line);
        }
      }
      std::fclose(f);
    }
  }
  STM_HIP(hipSetDevice(p->ctx->device));
  const hipStream_t st = p->stream;
  STM_HIP(hipStreamSynchronize(st));
  if (p->n_items == 0) {
    int rc = plan_set_shape(p, 8, 2, 0, -1);
    if (!rc) report(0);
    return rc;
  }
  const int w0 = p->waves, g0 = p->wgs_per_cu, b0 = p->batch_req, s0 = p->sched;
  int rc = STM_OK;
  // outputs for the timing runs
  float* e32 = p->o_e32;
  int32_t* asg = p->o_asg;
  if (p->device) {
    e32 = static_cast<float*>(plan_alloc(p, (size_t)p->row_off.back() * sizeof(float), &rc));
    asg = static_cast<int32_t*>(plan_alloc(p, (size_t)p->asg_off.back() * sizeof(int32_t), &rc));
    if (!e32 || !asg) return rc;
  }
  // evenly spaced sample of the cost-sorted list
  const int ns = n_sample > 0 ? std::min<int>(n_sample, p->n_items) : std::min<int>(p->n_items, p->n_cu * 24);
  std::vector<int2> all((size_t)p->n_items), sample((size_t)ns);
  STM_HIP(hipMemcpy(all.data(), p->items_dev, all.size() * sizeof(int2), hipMemcpyDeviceToHost));
  for (int k = 0; k < ns; ++k) sample[k] = all[(size_t)((long long)k * p->n_items / ns)];
  int2* sdev = static_cast<int2*>(plan_alloc(p, sample.size() * sizeof(int2), &rc));
  if (!sdev) return rc;
  STM_HIP(hipMemcpy(sdev, sample.data(), sample.size() * sizeof(int2), hipMemcpyHostToDevice));
  if ((rc = plan_enqueue_tables(p, st))) return rc;
  // the search space: (waves, workgroups per CU) x items per workgroup batch x
  // schedule variant (the packed one, 8 waves, wherever dummies are off)
  struct Cand { int w, g, b, s; };
  std::vector<Cand> cands;
  const int wg_pairs[][2] = {{4, 3}, {8, 2}, {8, 3}, {16, 1}, {16, 2}};
  const bool dum = dummy_on(&p->params);
  for (int sc = 0; sc <= (dum ? 0 : 1); ++sc)
    for (const auto& wg : wg_pairs) {
      if ((sc == 1 || dum) && wg[0] != 8) continue;  // those variants run 8 waves
      for (int bt = 1; bt <= std::min(stm::kMaxBatch, wg[0]); bt *= 2) cands.push_back({wg[0], wg[1], bt, sc});
    }
  hipEvent_t e0, e1;
  STM_HIP(hipEventCreate(&e0));
  STM_HIP(hipEventCreate(&e1));
  Cand best{8, 2, 0, -1};
  double best_ms = 1e300;
  for (const Cand& c : cands) {
    if (plan_set_shape(p, c.w, c.g, c.b, c.s)) {  // a batch whose scratch does not fit: skip it
      err().clear();
      continue;
    }
    const stm::BatchLaunch b = plan_launch(p, p->pairs_dev, sdev, ns, e32, asg);
    double ms_min = 1e300;
    for (int rep = 0; rep < 3 && !rc; ++rep) {
      if (stm::launch_fill_i32(p->counters, 3, 0, st) != hipSuccess) rc = fail(STM_EHIP, "fill failed");
      if (!rc && hipEventRecord(e0, st) != hipSuccess) rc = fail(STM_EHIP, "event failed");
      if (!rc && stm::launch_dp_persistent(b, p->n_cu * p->wgs_per_cu, st) != hipSuccess)
        rc = fail(STM_EHIP, "launch failed");
      if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = fail(STM_EHIP, "event failed");
      float ms = 0.f;
      if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = fail(STM_EHIP, "timing failed");
      if (rep > 0) ms_min = std::min<double>(ms_min, ms);  // the first run warms up
    }
    if (rc) break;
    if (ms_min < best_ms) { best_ms = ms_min; best = c; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    const std::string msg = err();
    (void)plan_set_shape(p, w0, g0, b0, s0);  // fits: its scratch is still owned
    err() = msg;
    return rc;
  }
  if ((rc = plan_set_shape(p, best.w, best.g, best.b, best.s))) {
    const std::string msg = err();
    (void)plan_set_shape(p, w0, g0, b0, s0);
    err() = msg;
    return rc;
  }
  report(0);
  if (cache_path) {
    char entry[512];
    std::snprintf(entry, sizeof(entry),
                  "  \"%s\": {\"waves\": %d, \"wgs_per_cu\": %d, \"batch\": %d, \"sched\": %d, \"ms\": %.4f}",
                  key.c_str(), best.w, best.g, best.b, best.s, best_ms);
    lines.push_back(entry);
    if (FILE* f = std::fopen(cache_path, "w")) {
      std::fputs("{\n", f);
      for (size_t k = 0; k < lines.size(); ++k) {
        std::string l = lines[k];
        while (!l.empty() && (l.back() == ',' || l.back() == ' ')) l.pop_back();
        std::fputs(l.c_str(), f);
        std::fputs(k + 1 < lines.size() ? ",\n" : "\n", f);
      }
      std::fputs("}\n", f);
      std::fclose(f);
    } else {
      return fail(STM_EINVAL, std::string("cannot write the tuning cache ") + cache_path);
    }
  }
  return STM_OK;
}

int stm_match_batch(stm_ctx* ctx, const stm_points* models, int32_t n_models, const stm_points* scenes,
                    int32_t n_scenes, const int32_t* pairs, int32_t n_pairs, const stm_params* params,
                    int64_t* row_offsets, float* energy32, double* energy64, int32_t* assign,
                    void* hip_stream) {
  stm_plan* p = nullptr;
  int rc = stm_plan_create(ctx, models, n_models, scenes, n_scenes, pairs, n_pairs, params, &p);
  if (rc) return rc;
  if (row_offsets) stm_plan_rows(p, row_offsets, nullptr, nullptr, nullptr);
  rc = stm_plan_run(p, energy32, energy64, nullptr, assign, hip_stream);
  if (!rc && p->device) {
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) rc = fail(STM_EHIP, hipGetErrorString(e));
  }
  std::string msg = err();
  plan_free(p);
  err() = msg;
  return rc;
}

}  // extern "C"

// ---- plan runs on caller-given candidate lists ---------------------------------

extern "C" {

int stm_plan_run_lists(stm_plan* p, const int32_t* const* cand, const int32_t* const* count, int32_t kc,
                       float* energy32, double* energy64, double* energy_u64, int32_t* assign, void* hip_stream) {
  err().clear();
  if (!p || !cand || !count) return fail(STM_EINVAL, "null plan or lists");
  if (p->params.flags & STM_CAUSAL_NODE)
    return fail(STM_EUNSUPPORTED, "node-order causality on given lists is not built");
  if (kc < 1 || kc > p->params.k_max) return fail(STM_EINVAL, "list stride kc must be in [1, k_max]");
  if (p->row_off.back() > 0 && (!energy32 || !assign)) return fail(STM_EINVAL, "energy32 and assign are required");
  STM_HIP(hipSetDevice(p->ctx->device));
  int rc = STM_OK;
  if (!p->ls_pairs_dev) {
    p->ls_pairs_dev = static_cast<stm::PairDev*>(
        plan_alloc(p, std::max<size_t>(1, p->pairs_host.size()) * sizeof(stm::PairDev), &rc));
    p->ls_bad = static_cast<int32_t*>(plan_alloc(p, sizeof(int32_t), &rc));
    if (rc) return rc;
  }
  const hipStream_t user = static_cast<hipStream_t>(hip_stream);
  STM_HIP(hipEventRecord(p->ev_in, user));
  STM_HIP(hipStreamWaitEvent(p->stream, p->ev_in, 0));
  const hipStream_t st = p->stream;
  // the lists: counts in [0, kc], ascending nodes of the pair's scene
  std::vector<stm::PairDev> ph = p->pairs_host;
  STM_HIP(stm::launch_fill_i32(p->ls_bad, 1, 0, st));
  for (size_t q = 0; q < ph.size(); ++q) {
    if (ph[q].n_tau > 0 && (!cand[q] || !count[q])) return fail(STM_EINVAL, "null list of a pair with offsets");
    STM_HIP(stm::launch_check_lists(cand[q], count[q], (long long)ph[q].n_tau * ph[q].m.M, kc, ph[q].s.S, p->ls_bad,
                                    st));
    ph[q].cand = cand[q];
    ph[q].ccount = count[q];
    ph[q].cstride = kc;
  }
  int32_t bad = 0;
  STM_HIP(hipMemcpyAsync(&bad, p->ls_bad, sizeof(bad), hipMemcpyDeviceToHost, st));
  if (!ph.empty())
    STM_HIP(hipMemcpyAsync(p->ls_pairs_dev, ph.data(), ph.size() * sizeof(stm::PairDev), hipMemcpyHostToDevice, st));
  STM_HIP(hipStreamSynchronize(st));
  if (bad) return fail(STM_EINVAL, "candidate lists: count outside [0, kc], node outside the scene or not ascending");

  float* e32 = p->device ? energy32 : p->o_e32;
  double* e64 = p->device ? energy64 : (energy64 ? p->o_e64 : nullptr);
  double* eu = p->device ? energy_u64 : (energy_u64 ? p->o_eu : nullptr);
  int32_t* asg = p->device ? assign : p->o_asg;
  if ((rc = plan_enqueue_tables(p, st))) return rc;
  STM_HIP(stm::launch_fill_i32(p->counters, 3, 0, st));
  stm::BatchLaunch b = plan_launch(p, p->ls_pairs_dev, p->items_dev, p->n_items, e32, asg);
  b.sp.K = kc;
  const bool timed = p->ctx->prof;
  if (timed) STM_HIP(hipEventRecord(p->ev_k0, st));
  STM_HIP(stm::launch_dp_persistent(b, p->n_cu * p->wgs_per_cu, st));
  if (timed) STM_HIP(hipEventRecord(p->ev_k1, st));
  STM_HIP(stm::launch_rescore_batch(p->pairs_dev, p->items_dev, p->n_items, stmh::search_params(&p->params, p->params.window), p->params.lambda1,
                                    p->params.lambda2, p->params.lambda3, w_dummy_of(&p->params), asg, e64, eu,
                                    st));
  STM_HIP(hipEventRecord(p->ev_out, st));
  STM_HIP(hipStreamWaitEvent(user, p->ev_out, 0));
  if (timed) {
    STM_HIP(hipEventSynchronize(p->ev_k1));
    float ms = 0.f;
    STM_HIP(hipEventElapsedTime(&ms, p->ev_k0, p->ev_k1));
    p->ctx->prof_plan_ms += ms;
    p->ctx->prof_plan_launches += 1;
    p->ctx->prof_matchings += p->row_off.back();
  }
  if (!p->device) {
    const int64_t nr = p->row_off.back(), na = p->asg_off.back();
    STM_HIP(hipMemcpyAsync(energy32, e32, (size_t)nr * sizeof(float), hipMemcpyDeviceToHost, st));
    STM_HIP(hipMemcpyAsync(assign, asg, (size_t)na * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (energy64) STM_HIP(hipMemcpyAsync(energy64, e64, (size_t)nr * sizeof(double), hipMemcpyDeviceToHost, st));
    if (energy_u64) STM_HIP(hipMemcpyAsync(energy_u64, eu, (size_t)nr * sizeof(double), hipMemcpyDeviceToHost, st));
    STM_HIP(hipStreamSynchronize(st));
  }
  return STM_OK;
}

}  // extern "C"
