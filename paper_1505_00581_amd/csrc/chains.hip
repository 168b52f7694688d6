// Multiple interest points per model frame, variant 2 of Section 4 (Table 4):
// the model is split into several single-point models (second-order chains),
// each solved independently by the exact recursion; the matching distance is
// the average of the chains' energies.
//
// The split (the paper leaves its details to another publication): chain c
// holds the c-th most salient point of every model frame with more than c
// points (salient = the detector's confidence, which the single-chain model
// uses to keep one point per frame, Section 2.1; equal confidences keep point
// order), for c < n_chains; chains of fewer than 3 points are dropped.  A
// model offset tau puts the model's first frame at scene frame tau; chain c is
// matched at tau + (its first frame - the model's first frame).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "host_common.h"
#include "stm_internal.h"

namespace stm {
namespace {

constexpr int32_t kUnchained = -3;  // a point that belongs to no kept chain

// Gathers points idx[j] of the model into row j of the chain arrays.
__global__ __launch_bounds__(64) void k_gather_points(const int32_t* __restrict__ idx, const float2* __restrict__ xy,
                                                      const int32_t* __restrict__ t, const float* __restrict__ desc,
                                                      int dim, float2* __restrict__ oxy, int32_t* __restrict__ ot,
                                                      float* __restrict__ odesc) {
  const int j = blockIdx.x;
  const int q = idx[j];
  if (threadIdx.x == 0) {
    oxy[j] = xy[q];
    ot[j] = t[q];
  }
  for (int d = threadIdx.x; d < dim; d += 64) odesc[(long long)j * dim + d] = desc[(long long)q * dim + d];
}

struct ChainRows {
  const float* e32;     // [n_chains][n_tau]
  const double* e64;    // [n_chains][n_tau]
  const double* eu;     // [n_chains][n_tau]
  const int32_t* as;    // chain c: [n_tau][len_c] from its point offset * n_tau
  const int32_t* idx;   // [n_used] model point of each chain point, chains in order
  const int32_t* off;   // [n_chains + 1] point offsets of the chains
};

// One workgroup per offset: the mean of the chains' energies (+inf if one is
// infeasible) and every point's node from its chain (kUnchained otherwise).
__global__ __launch_bounds__(256) void k_chain_combine(ChainRows c, int n_chains, int n_tau, int n_points,
                                                       float* __restrict__ e32, double* __restrict__ e64,
                                                       double* __restrict__ eu, int32_t* __restrict__ assign) {
  const int tau = blockIdx.x;
  if (threadIdx.x == 0) {
    float s32 = 0.f;
    double s64 = 0.0, su = 0.0;
    for (int q = 0; q < n_chains; ++q) {
      s32 += c.e32[(long long)q * n_tau + tau];
      s64 += c.e64[(long long)q * n_tau + tau];
      su += c.eu[(long long)q * n_tau + tau];
    }
    e32[tau] = s32 / static_cast<float>(n_chains);
    if (e64) e64[tau] = s64 / n_chains;
    if (eu) eu[tau] = su / n_chains;
  }
  int32_t* row = assign + (long long)tau * n_points;
  for (int p = threadIdx.x; p < n_points; p += 256) row[p] = kUnchained;
  __syncthreads();
  for (int q = 0; q < n_chains; ++q) {
    const int o = c.off[q], len = c.off[q + 1] - o;
    const int32_t* src = c.as + (long long)o * n_tau + (long long)tau * len;
    for (int j = threadIdx.x; j < len; j += 256) row[c.idx[o + j]] = src[j];
  }
}

}  // namespace
}  // namespace stm

using namespace stmh;

namespace {

template <class T>
int to_device(stm_ctx* ctx, DevBuf& b, const T* src, size_t count, bool src_device, hipStream_t st) {
  int rc = grow(ctx, b, std::max<size_t>(count, 1) * sizeof(T), st);
  if (rc) return rc;
  if (count)
    STM_HIP(hipMemcpyAsync(b.p, src, count * sizeof(T), src_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           st));
  return STM_OK;
}

}  // namespace

extern "C" int stm_match_chains(stm_ctx* ctx, const stm_points* model, const float* saliency, int32_t n_chains,
                                const stm_points* scene, const stm_params* params, int32_t tau_begin,
                                int32_t tau_end, float* energy32, double* energy64, double* energy_u64,
                                int32_t* assign, int32_t* chains_used, void* hip_stream) {
  err().clear();
  int rc = check_shapes(model, scene, params);
  if (rc) return rc;
  if (n_chains < 1 || n_chains > 64) return fail(STM_EINVAL, "n_chains must be in [1, 64]");
  if (!ctx) return fail(STM_EINVAL, "null context");
  STM_HIP(hipSetDevice(ctx->device));
  const hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const bool dev = (params->flags & STM_DEVICE_PTRS) != 0;
  const int n = model->n, dim = model->dim;

  // frames and confidences on the host, for the split
  std::vector<int32_t> t(n);
  std::vector<float> sal(saliency ? n : 0);
  if (dev) {
    STM_HIP(hipMemcpyAsync(t.data(), model->t, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (saliency) STM_HIP(hipMemcpyAsync(sal.data(), saliency, n * sizeof(float), hipMemcpyDeviceToHost, st));
    STM_HIP(hipStreamSynchronize(st));
  } else {
    std::copy(model->t, model->t + n, t.begin());
    if (saliency) std::copy(saliency, saliency + n, sal.begin());
  }
  for (int i = 1; i < n; ++i)
    if (t[i] < t[i - 1]) return fail(STM_EINVAL, "model frames must be non-decreasing");
  for (float v : sal)
    if (!std::isfinite(v)) return fail(STM_EINVAL, "non-finite saliency");

  std::vector<std::vector<int32_t>> chains(n_chains);
  for (int a = 0; a < n;) {
    int b = a;
    while (b < n && t[b] == t[a]) ++b;
    std::vector<int32_t> g(b - a);
    std::iota(g.begin(), g.end(), a);
    if (saliency)
      std::stable_sort(g.begin(), g.end(), [&](int32_t x, int32_t y) { return sal[x] > sal[y]; });
    for (int c = 0; c < n_chains && c < (int)g.size(); ++c) chains[c].push_back(g[c]);
    a = b;
  }
  std::vector<int32_t> idx, off{0};
  for (const auto& c : chains)
    if (c.size() >= 3) {
      idx.insert(idx.end(), c.begin(), c.end());
      off.push_back(static_cast<int32_t>(idx.size()));
    }
  const int nc = static_cast<int>(off.size()) - 1;
  if (nc == 0) return fail(STM_EINVAL, "no chain of 3 or more points");
  if (chains_used) *chains_used = nc;

  const long long n_off = std::max(0LL, (long long)scene->n_frames - ((long long)t[n - 1] - t[0]));
  if (tau_begin < 0 || tau_end < tau_begin || tau_end > n_off)
    return fail(STM_EINVAL, "offset range [" + std::to_string(tau_begin) + ", " + std::to_string(tau_end) +
                                ") outside [0, " + std::to_string(n_off) + ")");
  const int n_tau = tau_end - tau_begin;
  if (n_tau == 0) return STM_OK;
  if (!energy32 || !assign) return fail(STM_EINVAL, "energy32 and assign are required");

  // the model's points on the device, gathered chain by chain
  const int nu = static_cast<int>(idx.size());
  const float2* mxy = reinterpret_cast<const float2*>(model->xy);
  const int32_t* mt = model->t;
  const float* md = model->desc;
  if (!dev) {
    if ((rc = to_device(ctx, ctx->mxy, model->xy, (size_t)n * 2, false, st))) return rc;
    if ((rc = to_device(ctx, ctx->mt, model->t, (size_t)n, false, st))) return rc;
    if ((rc = to_device(ctx, ctx->mdesc, model->desc, (size_t)n * dim, false, st))) return rc;
    mxy = static_cast<const float2*>(ctx->mxy.p);
    mt = static_cast<const int32_t*>(ctx->mt.p);
    md = static_cast<const float*>(ctx->mdesc.p);
  }
  if ((rc = to_device(ctx, ctx->ch_idx, idx.data(), idx.size(), false, st))) return rc;
  if ((rc = grow(ctx, ctx->ch_xy, (size_t)nu * sizeof(float2), st))) return rc;
  if ((rc = grow(ctx, ctx->ch_t, (size_t)nu * sizeof(int32_t), st))) return rc;
  if ((rc = grow(ctx, ctx->ch_desc, (size_t)nu * dim * sizeof(float), st))) return rc;
  float2* cxy = static_cast<float2*>(ctx->ch_xy.p);
  int32_t* ct = static_cast<int32_t*>(ctx->ch_t.p);
  float* cd = static_cast<float*>(ctx->ch_desc.p);
  hipLaunchKernelGGL(stm::k_gather_points, dim3(nu), dim3(64), 0, st, static_cast<const int32_t*>(ctx->ch_idx.p),
                     mxy, mt, md, dim, cxy, ct, cd);
  STM_HIP(hipGetLastError());

  // the scene on the device
  stm_points sc = *scene;
  if (!dev) {
    const int S = scene->n;
    if ((rc = to_device(ctx, ctx->sxy, scene->xy, (size_t)S * 2, false, st))) return rc;
    if ((rc = to_device(ctx, ctx->st, scene->t, (size_t)S, false, st))) return rc;
    if ((rc = to_device(ctx, ctx->sdesc, scene->desc, (size_t)S * dim, false, st))) return rc;
    sc.xy = static_cast<const float*>(ctx->sxy.p);
    sc.t = static_cast<const int32_t*>(ctx->st.p);
    sc.desc = static_cast<const float*>(ctx->sdesc.p);
  }

  // every chain by the exact matching, at its own offsets
  if ((rc = grow(ctx, ctx->ch_e32, (size_t)nc * n_tau * sizeof(float), st))) return rc;
  if ((rc = grow(ctx, ctx->ch_e64, (size_t)nc * n_tau * sizeof(double), st))) return rc;
  if ((rc = grow(ctx, ctx->ch_eu, (size_t)nc * n_tau * sizeof(double), st))) return rc;
  if ((rc = grow(ctx, ctx->ch_as, (size_t)nu * n_tau * sizeof(int32_t), st))) return rc;
  float* e32c = static_cast<float*>(ctx->ch_e32.p);
  double* e64c = static_cast<double*>(ctx->ch_e64.p);
  double* euc = static_cast<double*>(ctx->ch_eu.p);
  int32_t* asc = static_cast<int32_t*>(ctx->ch_as.p);
  stm_params pc = *params;
  pc.flags |= STM_DEVICE_PTRS;
  for (int q = 0; q < nc; ++q) {
    const int o = off[q], len = off[q + 1] - o;
    stm_points cm;
    cm.n = len;
    cm.dim = dim;
    cm.n_frames = 0;
    cm.reserved = 0;
    cm.xy = reinterpret_cast<const float*>(cxy + o);
    cm.t = ct + o;
    cm.desc = cd + (size_t)o * dim;
    const int32_t delta = t[idx[o]] - t[0];
    if ((rc = stm_match(ctx, &cm, &sc, &pc, tau_begin + delta, tau_end + delta, e32c + (size_t)q * n_tau,
                        e64c + (size_t)q * n_tau, euc + (size_t)q * n_tau, asc + (size_t)o * n_tau, hip_stream)))
      return rc;
  }

  // the mean over chains, and the points' nodes in model order
  if ((rc = to_device(ctx, ctx->ch_off, off.data(), off.size(), false, st))) return rc;
  float* d_e32 = energy32;
  double* d_e64 = energy64;
  double* d_eu = energy_u64;
  int32_t* d_as = assign;
  if (!dev) {
    if ((rc = grow(ctx, ctx->o_e32, (size_t)n_tau * sizeof(float), st))) return rc;
    if ((rc = grow(ctx, ctx->o_e64, (size_t)n_tau * sizeof(double), st))) return rc;
    if ((rc = grow(ctx, ctx->o_eu, (size_t)n_tau * sizeof(double), st))) return rc;
    if ((rc = grow(ctx, ctx->o_assign, (size_t)n_tau * n * sizeof(int32_t), st))) return rc;
    d_e32 = static_cast<float*>(ctx->o_e32.p);
    d_e64 = static_cast<double*>(ctx->o_e64.p);
    d_eu = static_cast<double*>(ctx->o_eu.p);
    d_as = static_cast<int32_t*>(ctx->o_assign.p);
  }
  stm::ChainRows rows{e32c, e64c, euc, asc, static_cast<const int32_t*>(ctx->ch_idx.p),
                      static_cast<const int32_t*>(ctx->ch_off.p)};
  hipLaunchKernelGGL(stm::k_chain_combine, dim3(n_tau), dim3(256), 0, st, rows, nc, n_tau, n, d_e32, d_e64, d_eu,
                     d_as);
  STM_HIP(hipGetLastError());
  if (!dev) {
    STM_HIP(hipMemcpyAsync(energy32, d_e32, (size_t)n_tau * sizeof(float), hipMemcpyDeviceToHost, st));
    STM_HIP(hipMemcpyAsync(assign, d_as, (size_t)n_tau * n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (energy64)
      STM_HIP(hipMemcpyAsync(energy64, d_e64, (size_t)n_tau * sizeof(double), hipMemcpyDeviceToHost, st));
    if (energy_u64)
      STM_HIP(hipMemcpyAsync(energy_u64, d_eu, (size_t)n_tau * sizeof(double), hipMemcpyDeviceToHost, st));
    STM_HIP(hipStreamSynchronize(st));
  }
  return STM_OK;
}
