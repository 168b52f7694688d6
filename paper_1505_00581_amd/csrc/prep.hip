// Preparation kernels of the matching path: input validation, the scene
// frame index, candidate lists, the unary table and work counts.
#include <math.h>

#include "stm_internal.h"

namespace stm {
namespace {

constexpr int kBlock = 256;

inline int grid_for(long long n, int block, int cap = 65535 * 4) {
  long long g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<int>(g);
}

// ---- validation -------------------------------------------------------------
// bit 0: model frames not strictly increasing; bit 1: scene frames decreasing;
// bit 2: scene frame outside [0, F); bit 3: non-finite model data; bit 4:
// non-finite scene data.
__global__ void k_validate(ModelView m, SceneView s, int32_t* out) {
  const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  int32_t bits = 0;
  for (long long i = tid; i < m.M; i += stride) {
    if (i > 0 && m.t[i] <= m.t[i - 1]) bits |= 1;
    const float2 p = m.xy[i];
    if (!isfinite(p.x) || !isfinite(p.y)) bits |= 8;
  }
  for (long long i = tid; i < (long long)m.M * s.dim; i += stride)
    if (!isfinite(m.desc[i])) bits |= 8;
  for (long long i = tid; i < s.S; i += stride) {
    const int32_t ti = s.t[i];
    if (i > 0 && ti < s.t[i - 1]) bits |= 2;
    if (ti < 0 || ti >= s.F) bits |= 4;
    const float2 p = s.xy[i];
    if (!isfinite(p.x) || !isfinite(p.y)) bits |= 16;
  }
  for (long long i = tid; i < (long long)s.S * s.dim; i += stride)
    if (!isfinite(s.desc[i])) bits |= 16;
  if (bits) atomicOr(out, bits);
  if (tid == 0) out[1] = m.t[m.M - 1] - m.t[0];
}

// ---- frame index: fstart[f] = first node with frame >= f, f in [0, F] -------
__global__ void k_fstart(const int32_t* __restrict__ t, int32_t S, int32_t F,
                         int32_t* __restrict__ fstart) {
  const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f > F) return;
  int32_t lo = 0, hi = S;
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if (t[mid] < f) lo = mid + 1; else hi = mid;
  }
  fstart[f] = lo;
}

// ---- candidate lists (one 64-lane block per offset) ----------------------------
__global__ void k_candidates(ModelView m, SceneView s, SearchParams sp, int32_t tau0,
                             int32_t* __restrict__ cand, int32_t* __restrict__ count) {
  const int32_t tl = blockIdx.x, lane = threadIdx.x;
  const int32_t tau = tau0 + tl;
  for (int32_t i = 0; i < m.M; ++i) {
    const CandRange c = point_candidates(s.fstart, s.F, tau + m.t[i] - m.t[0], sp);
    const int32_t k = c.k1 + c.k2;
    int32_t* row = cand + ((long long)tl * m.M + i) * sp.K;
    for (int32_t a = lane; a < sp.K; a += 64) row[a] = a < k ? cand_node(c, a) : -1;
    if (lane == 0) count[(long long)tl * m.M + i] = k;
  }
}

// ---- unary table U[i][n] = ||f_i - g_n|| in FP32 (Eq. 2) -----------------------
// One thread per scene point, 16 model rows per block staged in LDS.  The
// scene rows of the block's 256 points are staged too, 32 dimensions at a
// time and read from global memory in 128-byte row segments (a thread
// streaming its own row would touch 64 lines per load across the wave).  Each
// distance is accumulated over the dimensions in ascending order.
constexpr int kUnaryRows = 16;
constexpr int kUnaryMaxDim = 256;
constexpr int kUnaryTile = 32;

__global__ __launch_bounds__(kBlock) void k_unary_f32(ModelView m, SceneView s, float* __restrict__ U) {
  __shared__ float fm[kUnaryRows][kUnaryMaxDim];
  __shared__ float gt[kBlock][kUnaryTile + 1];  // +1: lanes of one column hit distinct banks
  const int32_t dim = s.dim;
  const int32_t i0 = blockIdx.y * kUnaryRows;
  const int32_t rows = min(kUnaryRows, m.M - i0);
  for (int32_t e = threadIdx.x; e < kUnaryRows * dim; e += blockDim.x) {
    const int32_t r = e / dim, d = e - r * dim;
    fm[r][d] = r < rows ? m.desc[(long long)(i0 + r) * dim + d] : 0.0f;
  }
  const int32_t n0 = blockIdx.x * kBlock;
  const int32_t n = n0 + threadIdx.x;
  float acc[kUnaryRows];
#pragma unroll
  for (int r = 0; r < kUnaryRows; ++r) acc[r] = 0.0f;
  // the scene tile of dimensions [d0, d0 + 32) is read into registers one tile
  // ahead, so that its global reads overlap the arithmetic of the tile before.
  // Thread t reads dimension t % 32 of the tile for points t / 32 + 8 j.
  constexpr int kStride = kBlock / kUnaryTile;
  const int32_t tdd = threadIdx.x % kUnaryTile, tp = threadIdx.x / kUnaryTile;
  const float* src = s.desc + (long long)(n0 + tp) * dim + tdd;
  const long long jstep = (long long)kStride * dim;
  float pre[kUnaryTile];
  const auto fetch = [&](int32_t d0) {
    const bool dok = tdd < min(kUnaryTile, dim - d0);
#pragma unroll
    for (int32_t j = 0; j < kUnaryTile; ++j)
      pre[j] = dok && n0 + tp + kStride * j < s.S ? src[j * jstep + d0] : 0.0f;
  };
  fetch(0);
  for (int32_t d0 = 0; d0 < dim; d0 += kUnaryTile) {
    const int32_t w = min(kUnaryTile, dim - d0);
    __syncthreads();  // the previous tile is consumed (and fm is written, first time)
#pragma unroll
    for (int32_t j = 0; j < kUnaryTile; ++j) gt[tp + kStride * j][tdd] = pre[j];
    __syncthreads();
    if (d0 + kUnaryTile < dim) fetch(d0 + kUnaryTile);
    for (int32_t dd = 0; dd < w; ++dd) {
      const float v = gt[threadIdx.x][dd];
#pragma unroll
      for (int r = 0; r < kUnaryRows; ++r) {
        const float a0 = fm[r][d0 + dd] - v;
        acc[r] = fmaf(a0, a0, acc[r]);
      }
    }
  }
  if (n >= s.S) return;
#pragma unroll
  for (int r = 0; r < kUnaryRows; ++r)
    if (r < rows) U[(long long)(i0 + r) * s.S + n] = sqrtf(acc[r]);
}

// ---- model angles of the triangle ending at point i (FP64, then rounded) ------
// theta[i] = (angle at i-1 of (i, i-1, i-2), angle at i of (i-1, i, i-2)),
// oriented, 0 for a zero-length side (Eq. 6).
__global__ void k_model_angles(ModelView m, float2* __restrict__ theta) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.M) return;
  if (i < 2) { theta[i] = make_float2(0.f, 0.f); return; }
  const float2 pi = m.xy[i], pj = m.xy[i - 1], pk = m.xy[i - 2];
  const double mid = ang64(pi.x, pi.y, pj.x, pj.y, pk.x, pk.y);
  const double end = ang64(pj.x, pj.y, pi.x, pi.y, pk.x, pk.y);
  theta[i] = make_float2(static_cast<float>(mid), static_cast<float>(end));
}

// ---- work counts (one 64-lane block per offset) --------------------------------
__global__ void k_count(ModelView m, SceneView s, SearchParams sp, int32_t tau0,
                        unsigned long long* __restrict__ counts) {
  __shared__ int32_t tt[3][64];
  __shared__ int32_t nn[3][64];  // node ids (node-order causality)
  __shared__ int32_t kk[3];
  const int32_t tau = tau0 + blockIdx.x, lane = threadIdx.x;
  unsigned long long dc = 0, fc = 0, dr = 0, fr = 0;
  for (int32_t i = 0; i < m.M; ++i) {
    const CandRange c = point_candidates(s.fstart, s.F, tau + m.t[i] - m.t[0], sp);
    const int32_t k = c.k1 + c.k2;
    __syncthreads();
    if (lane < k) {
      tt[i % 3][lane] = s.t[cand_node(c, lane)];
      nn[i % 3][lane] = cand_node(c, lane);
    }
    if (lane == 0) kk[i % 3] = k;
    __syncthreads();
    if (i >= 1) {
      const int32_t kp = kk[(i - 1) % 3], kc = kk[i % 3];
      const int32_t T = pair_limit(sp), TS = span_limit(sp);
      // lane = candidate r of point i-1
      if (lane < kp) {
        const int32_t tr = tt[(i - 1) % 3][lane], nr = nn[(i - 1) % 3][lane];
        const int32_t* tcur = tt[i % 3];
        const int32_t* ncur = nn[i % 3];
        int32_t na = 0;
        for (int32_t a = 0; a < kc; ++a) na += consecutive_ok(sp, T, nr, tr, ncur[a], tcur[a]);
        dc += kc;
        fc += na;
        if (i >= 2) {
          const int32_t kq = kk[(i - 2) % 3];
          const int32_t* tprev = tt[(i - 2) % 3];
          const int32_t* nprev = nn[(i - 2) % 3];
          dr += (unsigned long long)kq * kc;
          if (TS <= 0) {
            int32_t nk = 0;
            for (int32_t q = 0; q < kq; ++q) nk += consecutive_ok(sp, T, nprev[q], tprev[q], nr, tr);
            fr += (unsigned long long)nk * na;
          } else {
            // span reading: for each admissible predecessor, the admissible
            // columns less than TS frames after it (frames ascend, so the
            // bound only moves forward)
            int32_t a = 0, n_below = 0;
            for (int32_t q = 0; q < kq; ++q) {
              if (!admissible(tprev[q], tr, T)) continue;
              for (; a < kc && tcur[a] - tprev[q] < TS; ++a) n_below += admissible(tr, tcur[a], T);
              fr += n_below;
            }
          }
        }
      }
    }
  }
  // wave reductions, then one atomic per counter
  for (int off = 32; off > 0; off >>= 1) {
    dc += __shfl_xor(dc, off);
    fc += __shfl_xor(fc, off);
    dr += __shfl_xor(dr, off);
    fr += __shfl_xor(fr, off);
  }
  if (lane == 0) {
    atomicAdd(counts + 0, dc);
    atomicAdd(counts + 1, fc);
    atomicAdd(counts + 2, dr);
    atomicAdd(counts + 3, fr);
  }
}

}  // namespace

hipError_t launch_validate(const ModelView& m, const SceneView& s, int32_t* out, hipStream_t st) {
  const long long n = (long long)(m.M > s.S ? m.M : s.S) * (s.dim > 1 ? s.dim : 1);
  hipLaunchKernelGGL(k_validate, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, st, m, s, out);
  return hipGetLastError();
}

hipError_t launch_fstart(const int32_t* t, int32_t S, int32_t F, int32_t* fstart, hipStream_t st) {
  hipLaunchKernelGGL(k_fstart, dim3(grid_for((long long)F + 1, kBlock)), dim3(kBlock), 0, st, t, S, F,
                     fstart);
  return hipGetLastError();
}

hipError_t launch_candidates(const ModelView& m, const SceneView& s, const SearchParams& sp,
                             int32_t tau0, int32_t n_tau, int32_t* cand, int32_t* count,
                             hipStream_t st) {
  if (n_tau <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_candidates, dim3(n_tau), dim3(64), 0, st, m, s, sp, tau0, cand, count);
  return hipGetLastError();
}

hipError_t launch_unary_f32(const ModelView& m, const SceneView& s, float* U, hipStream_t st) {
  if (s.dim > kUnaryMaxDim) return hipErrorInvalidValue;
  dim3 grid(grid_for(s.S, kBlock), (m.M + kUnaryRows - 1) / kUnaryRows);
  hipLaunchKernelGGL(k_unary_f32, grid, dim3(kBlock), 0, st, m, s, U);
  return hipGetLastError();
}

hipError_t launch_model_angles(const ModelView& m, float2* theta, hipStream_t st) {
  hipLaunchKernelGGL(k_model_angles, dim3((m.M + 63) / 64), dim3(64), 0, st, m, theta);
  return hipGetLastError();
}

hipError_t launch_count(const ModelView& m, const SceneView& s, const SearchParams& sp,
                        int32_t tau0, int32_t n_tau, unsigned long long* counts, hipStream_t st) {
  if (n_tau <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count, dim3(n_tau), dim3(64), 0, st, m, s, sp, tau0, counts);
  return hipGetLastError();
}

}  // namespace stm
