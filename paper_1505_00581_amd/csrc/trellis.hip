// The paper's own matching problem (Section 2.2): one trellis per (model,
// scene block) in which every model point may take any node of the block,
// pruned only by causality and closeness (Eq. 7, 8), whose consequences are
// the loop bounds of Section 3.4: with the block's nodes sorted by frame, the
// successors of a node (frames in (t, t + T)) and its predecessors (frames in
// (t - T, t)) are contiguous node ranges.
//
// Band layout.  A cell is a pair (r, c) of consecutive assignments with c a
// successor of r; the cells are numbered row after row (rowoff[r] + c -
// s_lo[r]), which is the layout of every step's value table V_i and of the
// cells' own directions A(r, c) = -phi(r -> c).  The (a_{i-2}, a_i) directions
// C(k, c) are needed for pairs two admissible steps apart (2 <= t_c - t_k <=
// 2T - 2), numbered row after row by k (qoff[k] + c - q_lo[k]); under the span
// reading of closeness a pair T or more frames apart holds +inf, which takes
// its terms out of every minimum.  The band and both direction tables depend
// on the scene block only and are built once.
//
// One launch per step i computes V_i from V_{i-1} for every model: a
// workgroup takes one tile, a rectangle of rows [r0, r1) by columns [c0, c1)
// holding at most 1024 cells (narrow bands: up to 64 consecutive rows whose
// successors span at most 128 nodes; wide bands: 32 rows by a 32-column
// window, so that a staged predecessor serves 32 rows and 32 columns), or at
// most 256 (8 rows by 32 columns) when 1024-cell tiles would give a launch few
// workgroups, thread t taking cells t, t + 256, ...  The predecessors of the
// tile's rows, a contiguous node range, are staged 20 or 24 at a time in LDS: the
// previous values with their directions va[k][r] (+inf where k is no
// predecessor of r) and the directions C[k][c] of the window's columns.  A
// wave runs over the union of its lanes' predecessor ranges; a lane outside
// its own range reads +inf, so the union changes no minimum.
//
// The last step's first row-major minimum is the optimum; backtracking
// recomputes each step's terms of the optimal cell over its predecessors with
// the same arithmetic (dp_math.h) and keeps the lowest node on ties.
#include <math.h>

#include "dp_math.h"
#include "stm_internal.h"

namespace stm {
namespace {

constexpr int kThreads = 256;                    // threads of a step workgroup
// Predecessors staged in LDS at a time and the occupancy target of a step
// launch: launches of many workgroups (several per CU) take 20 at a time at six
// waves per SIMD (80 registers), smaller ones 24 at five; on the whole video
// without a closeness limit 40.2 ms for 50 models against 42.6 (24) and 47.5
// (32 at four waves), and 7.8 ms for one model against 8.5 (20 at six).
constexpr int kChunkWide = 20, kWavesWide = 6;    // launches of >= kManyTiles workgroups
constexpr int kChunkSmall = 24, kWavesSmall = 5;
constexpr int kManyTiles = 1024;

// First index of the ascending a[0..n) whose value is >= x (n if none).
__device__ __forceinline__ int32_t lower_bound64(const int32_t* __restrict__ a, int32_t n, long long x) {
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if ((long long)a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// A cell's value at step 1, l1 U_0(r) + l1 U_1(c) + l2 |dt_model - dt_scene|, and
// at a later step, l1 U_i(c) + q_w |dt_model - dt_scene| + the minimum over the
// predecessors; the roundings are spelled out so that every kernel that forms a
// value gives the same bits.
__device__ __forceinline__ float first_value(const TrellisRun& a, float u0, float u1, int32_t dtm, int32_t dts) {
  return fmaf(a.lambda2, fabsf(static_cast<float>(dtm - dts)), fmaf(a.lambda1, u1, __fmul_rn(a.lambda1, u0)));
}
__device__ __forceinline__ float step_value(float cu, float qw, int32_t dtm, int32_t dts, float best) {
  return fmaf(qw, fabsf(static_cast<float>(dtm - dts)), cu) + best;
}

// ---- the band of a scene block -------------------------------------------------
__global__ __launch_bounds__(256) void k_trellis_band(const int32_t* __restrict__ t, int32_t n, SearchParams sp,
                                                      TrellisBand b) {
  const int32_t r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  const long long tr = t[r];
  const int32_t T = pair_limit(sp);
  const int32_t slo = lower_bound64(t, n, tr + 1);
  const int32_t shi = T > 0 ? lower_bound64(t, n, tr + T) : n;
  const int32_t qlo = lower_bound64(t, n, tr + 2);
  const int32_t qhi = T > 0 ? lower_bound64(t, n, tr + 2LL * T - 1) : n;
  b.s_lo[r] = slo;
  b.s_hi[r] = shi > slo ? shi : slo;
  b.p_hi[r] = lower_bound64(t, n, tr);
  b.p_lo[r] = T > 0 ? lower_bound64(t, n, tr - T + 1) : 0;
  b.q_lo[r] = qlo;
  b.q_hi[r] = qhi > qlo ? qhi : qlo;
  b.rowoff[r + 1] = shi > slo ? shi - slo : 0;  // widths; the scan makes offsets
  b.qoff[r + 1] = qhi > qlo ? qhi - qlo : 0;
  if (r == 0) {
    b.rowoff[0] = 0;
    b.qoff[0] = 0;
  }
}

// In-place inclusive scan of a[1..n] (a[0] = 0), one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan64(long long* __restrict__ a, int32_t n) {
  __shared__ long long wsum[16];
  __shared__ long long carry;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int32_t base = 1; base <= n; base += 1024) {
    const int32_t j = base + tid;
    long long v = j <= n ? a[j] : 0;
    for (int off = 1; off < 64; off <<= 1) {
      const long long u = __shfl_up(v, off);
      if (lane >= off) v += u;
    }
    if (lane == 63) wsum[wv] = v;
    __syncthreads();
    long long pre = carry;
    for (int q = 0; q < wv; ++q) pre += wsum[q];
    if (j <= n) a[j] = v + pre;
    __syncthreads();
    if (tid == 1023) carry = pre + v;
    __syncthreads();
  }
}

// Directions of the block: A (blockIdx.y = 0) over the cells of row r =
// blockIdx.x, C (blockIdx.y = 1) over the two-step pairs of row k = blockIdx.x.
// Coincident points give NaN and raise *flag; span-excluded C pairs are +inf.
__global__ __launch_bounds__(64) void k_trellis_dirs(TrellisBand b, const float2* __restrict__ xy,
                                                    const int32_t* __restrict__ t, int32_t span_lim,
                                                    int32_t* __restrict__ flag) {
  const int32_t r = blockIdx.x;
  const float2 pr = xy[r];
  int32_t same = 0;
  if (blockIdx.y == 0) {
    const int32_t lo = b.s_lo[r], hi = b.s_hi[r];
    float* out = b.A + b.rowoff[r] - lo;
    for (int32_t c = lo + threadIdx.x; c < hi; c += 64) {
      const float2 pc = xy[c];
      same |= pc.x == pr.x && pc.y == pr.y;
      out[c] = neg_dir<true>(pr, pc);
    }
  } else {
    const int32_t lo = b.q_lo[r], hi = b.q_hi[r];
    float* out = b.C + b.qoff[r] - lo;
    const int32_t tk = t[r];
    for (int32_t c = lo + threadIdx.x; c < hi; c += 64) {
      if (!span_ok(tk, t[c], span_lim)) {
        out[c] = __builtin_inff();
        continue;
      }
      const float2 pc = xy[c];
      same |= pc.x == pr.x && pc.y == pr.y;
      out[c] = neg_dir<true>(pr, pc);
    }
  }
  if (same) atomicOr(flag, 1);
}

// ---- the steps --------------------------------------------------------------------
// V_1(r, c) = l1 U_0(r) + l1 U_1(c) + l2 Delta(1, 0), row r = blockIdx.x of
// model blockIdx.y.
__global__ __launch_bounds__(64) void k_trellis_first(TrellisRun a) {
  const int32_t r = blockIdx.x;
  const TrellisModel md = a.models[blockIdx.y];
  const int32_t lo = a.band.s_lo[r], hi = a.band.s_hi[r];
  if (lo >= hi) return;
  const float* U0 = md.U;
  const float* U1 = md.U + a.n;
  const int32_t dtm = md.m.t[1] - md.m.t[0];
  const int32_t tr = a.t[r];
  float* out = md.V + a.band.rowoff[r] - lo;
  for (int32_t c = lo + threadIdx.x; c < hi; c += 64) out[c] = first_value(a, U0[r], U1[c], dtm, a.t[c] - tr);
}

template <int KC>
struct StepShared {
  float2 va[KC][kTrellisTileRows];  // (V_{i-1}(k, r), A(k, r)); +inf where k is no predecessor of r
  float ct[KC][kTrellisTileCols];   // C(k, c)
  int32_t plo[kTrellisTileRows], phi[kTrellisTileRows], slo[kTrellisTileRows], tr[kTrellisTileRows];
  int32_t cstart[kTrellisTileRows + 1];  // first tile cell of each row
  int16_t crow[kTrellisTileCells];       // row of each tile cell
  float cu[kTrellisTileCols];            // l1 U_i(c)
  int32_t tc[kTrellisTileCols];
};

// V_i for the tile blockIdx.x of model blockIdx.y (skipped when i >= M); tiles
// of at most SLOTS * 256 cells, SLOTS cells per thread.
template <bool DEGEN, int KC, int WAVES, int SLOTS>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(WAVES)))
void k_trellis_step(TrellisRun a, int32_t i) {
  constexpr int kChunk = KC;
  constexpr int kSlots = SLOTS;  // cells per thread
  __shared__ StepShared<KC> sh;
  const TrellisModel md = a.models[blockIdx.y];
  const int32_t M = md.m.M;
  if (i >= M) return;
  const TrellisTile tl = a.tiles[blockIdx.x];
  const int32_t R = tl.r1 - tl.r0, CW = tl.c1 - tl.c0;
  const int tid = threadIdx.x, lane = tid & 63;
  const float INF = __builtin_inff();
  const TrellisBand& b = a.band;
  const float* Ui = md.U + (long long)i * a.n;
  const float* Vp = md.V + (long long)(i - 2) * a.Q;  // V_{i-1}
  float* Vi = md.V + (long long)(i - 1) * a.Q;

  // rows: predecessor and successor ranges, cell counts inside the window
  int32_t cnt = 0;
  if (tid < R) {
    const int32_t r = tl.r0 + tid;
    sh.plo[tid] = b.p_lo[r];
    sh.phi[tid] = b.p_hi[r];
    const int32_t lo = max(b.s_lo[r], tl.c0), hi = min(b.s_hi[r], tl.c1);
    sh.slo[tid] = lo;
    sh.tr[tid] = a.t[r];
    cnt = hi > lo ? hi - lo : 0;
  }
  if (tid < CW) {
    const int32_t c = tl.c0 + tid;
    sh.cu[tid] = __fmul_rn(a.lambda1, Ui[c]);
    sh.tc[tid] = a.t[c];
  }
  if (tid < 64) {  // R <= 64: one wave scans the counts
    int32_t incl = cnt;
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t u = __shfl_up(incl, off);
      if (lane >= off) incl += u;
    }
    if (tid < R) sh.cstart[tid] = incl - cnt;
    if (tid == 63) sh.cstart[R] = incl;  // = tl.ncell
    if (tid < R)
      for (int32_t q = incl - cnt; q < incl; ++q) sh.crow[q] = static_cast<int16_t>(tid);
  }
  __syncthreads();

  const float2 th = md.theta[i];
  const int32_t dtm = md.m.t[i] - md.m.t[i - 1];
  const float qw = a.lambda2 * (i <= M - 2 ? 2.f : 1.f);
  const float w = a.w;
  const int32_t ncell = tl.ncell;
  int rr[kSlots], cc[kSlots];
  float bm[kSlots], be[kSlots], best[kSlots];
  bool same[kSlots];
  int32_t wlo[kSlots], whi[kSlots];  // wave-uniform predecessor union of each slot
#pragma unroll
  for (int j = 0; j < kSlots; ++j) {
    const int32_t cid = tid + kThreads * j;
    const bool valid = cid < ncell;
    const int32_t q = valid ? cid : 0;
    const int row = sh.crow[q];
    const int32_t c = sh.slo[row] + (q - sh.cstart[row]);
    rr[j] = row;
    cc[j] = c - tl.c0;
    best[j] = INF;
    const int32_t r = tl.r0 + row;
    const float arc = b.A[b.rowoff[r] + (c - b.s_lo[r])];
    cell_brackets(th, -arc, bm[j], be[j]);
    const float2 xr = a.xy[r], xc = a.xy[c];
    same[j] = xr.x == xc.x && xr.y == xc.y;
    int32_t lo = valid ? sh.plo[row] : 0x7fffffff, hi = valid ? sh.phi[row] : -1;
    for (int off = 32; off > 0; off >>= 1) {
      lo = min(lo, __shfl_xor(lo, off));
      hi = max(hi, __shfl_xor(hi, off));
    }
    if (hi <= lo) lo = hi = 0;  // no valid lane, or no predecessors: an empty range
    wlo[j] = __builtin_amdgcn_readfirstlane(lo);
    whi[j] = __builtin_amdgcn_readfirstlane(hi);
  }

  // staging: one wave per predecessor row of a table at a time, so that the
  // predecessor k and its band offsets are wave-uniform (scalar loads) and a
  // lane takes one row (va) or one of 64 columns (ct) of the tile
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int cgroups = (CW + 63) >> 6;  // 64-column groups of the window: 1 or 2
  for (int32_t k0 = tl.k0; k0 < tl.k1; k0 += kChunk) {
    const int32_t nk = min(kChunk, tl.k1 - k0);
    // rows kk = wv, wv + 4, ... of the chunk: every read of a table (of both
    // tables with one cell per thread, whose registers allow it) is issued
    // before the first store (fixed trip counts, unrolled; a lane without a
    // value reads index 0 and stores the default), so that a chunk waits for
    // one or two rounds of reads instead of one per row
    constexpr int kWaves = kThreads / 64;
    constexpr int kPerWave = kChunk / kWaves;
    static_assert(kChunk % kWaves == 0, "staged rows split evenly over the waves");
    float2 sv[kPerWave];
    bool okv[kPerWave];
#pragma unroll
    for (int s = 0; s < kPerWave; ++s) {
      const int kk = wv + kWaves * s;
      const int32_t k = kk < nk ? k0 + kk : tl.k1 - 1;  // wave-uniform, inside the band
      okv[s] = kk < nk && lane < R && k >= sh.plo[lane] && k < sh.phi[lane];
      const long long off = okv[s] ? b.rowoff[k] + (tl.r0 + lane - b.s_lo[k]) : 0;
      sv[s] = make_float2(Vp[off], b.A[off]);
    }
    const auto store_va = [&]() {
#pragma unroll
      for (int s = 0; s < kPerWave; ++s)
        if (lane < R) sh.va[wv + kWaves * s][lane] = okv[s] ? sv[s] : make_float2(INF, 0.f);
    };
    if constexpr (SLOTS > 1) store_va();
    float sc[kPerWave][2];
    bool okc[kPerWave][2];
#pragma unroll
    for (int s = 0; s < kPerWave; ++s) {
      const int kk = wv + kWaves * s;
      const int32_t k = kk < nk ? k0 + kk : tl.k1 - 1;
      const int32_t qlo = b.q_lo[k], qhi = b.q_hi[k];
      const long long qo = b.qoff[k];
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const int32_t c = tl.c0 + g * 64 + lane;
        okc[s][g] = kk < nk && g < cgroups && c < tl.c1 && c >= qlo && c < qhi;
        sc[s][g] = b.C[okc[s][g] ? qo + (c - qlo) : 0];
      }
    }
    if constexpr (SLOTS == 1) store_va();
#pragma unroll
    for (int s = 0; s < kPerWave; ++s)
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const int col = g * 64 + lane;
        if (g < cgroups && col < CW) sh.ct[wv + kWaves * s][col] = okc[s][g] ? sc[s][g] : 0.f;
      }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
      // bounds relative to the chunk, in [0, nk] (an empty range gives hi <= lo)
      const int32_t lo = max(wlo[j], k0) - k0, hi = min(whi[j], k0 + nk) - k0;
      const float2* vcol = &sh.va[0][rr[j]];
      const float* ccol = &sh.ct[0][cc[j]];
      float bj = best[j];
      int32_t kk = lo;
      for (; kk + 7 < hi; kk += 8) {
        const float2 v0 = vcol[kk * kTrellisTileRows], v1 = vcol[(kk + 1) * kTrellisTileRows];
        const float2 v2 = vcol[(kk + 2) * kTrellisTileRows], v3 = vcol[(kk + 3) * kTrellisTileRows];
        const float t0 = relax<DEGEN>(v0.x, v0.y, ccol[kk * kTrellisTileCols], bm[j], be[j], th, same[j], w);
        const float t1 = relax<DEGEN>(v1.x, v1.y, ccol[(kk + 1) * kTrellisTileCols], bm[j], be[j], th, same[j], w);
        const float t2 = relax<DEGEN>(v2.x, v2.y, ccol[(kk + 2) * kTrellisTileCols], bm[j], be[j], th, same[j], w);
        const float t3 = relax<DEGEN>(v3.x, v3.y, ccol[(kk + 3) * kTrellisTileCols], bm[j], be[j], th, same[j], w);
        bj = fminf(fminf(bj, fminf(fminf(t0, t1), t2)), t3);
        const float2 v4 = vcol[(kk + 4) * kTrellisTileRows], v5 = vcol[(kk + 5) * kTrellisTileRows];
        const float2 v6 = vcol[(kk + 6) * kTrellisTileRows], v7 = vcol[(kk + 7) * kTrellisTileRows];
        const float t4 = relax<DEGEN>(v4.x, v4.y, ccol[(kk + 4) * kTrellisTileCols], bm[j], be[j], th, same[j], w);
        const float t5 = relax<DEGEN>(v5.x, v5.y, ccol[(kk + 5) * kTrellisTileCols], bm[j], be[j], th, same[j], w);
        const float t6 = relax<DEGEN>(v6.x, v6.y, ccol[(kk + 6) * kTrellisTileCols], bm[j], be[j], th, same[j], w);
        const float t7 = relax<DEGEN>(v7.x, v7.y, ccol[(kk + 7) * kTrellisTileCols], bm[j], be[j], th, same[j], w);
        bj = fminf(fminf(bj, fminf(fminf(t4, t5), t6)), t7);
      }
      if (kk + 3 < hi) {
        const float2 v0 = vcol[kk * kTrellisTileRows], v1 = vcol[(kk + 1) * kTrellisTileRows];
        const float2 v2 = vcol[(kk + 2) * kTrellisTileRows], v3 = vcol[(kk + 3) * kTrellisTileRows];
        const float t0 = relax<DEGEN>(v0.x, v0.y, ccol[kk * kTrellisTileCols], bm[j], be[j], th, same[j], w);
        const float t1 = relax<DEGEN>(v1.x, v1.y, ccol[(kk + 1) * kTrellisTileCols], bm[j], be[j], th, same[j], w);
        const float t2 = relax<DEGEN>(v2.x, v2.y, ccol[(kk + 2) * kTrellisTileCols], bm[j], be[j], th, same[j], w);
        const float t3 = relax<DEGEN>(v3.x, v3.y, ccol[(kk + 3) * kTrellisTileCols], bm[j], be[j], th, same[j], w);
        bj = fminf(fminf(bj, fminf(fminf(t0, t1), t2)), t3);
        kk += 4;
      }
      for (; kk < hi; ++kk) {
        const float2 v0 = vcol[kk * kTrellisTileRows];
        bj = fminf(bj, relax<DEGEN>(v0.x, v0.y, ccol[kk * kTrellisTileCols], bm[j], be[j], th, same[j], w));
      }
      best[j] = bj;
    }
    __syncthreads();
  }

#pragma unroll
  for (int j = 0; j < kSlots; ++j) {
    const int32_t cid = tid + kThreads * j;
    if (cid < ncell) {
      const int32_t r = tl.r0 + rr[j], c = tl.c0 + cc[j];
      Vi[b.rowoff[r] + (c - b.s_lo[r])] = step_value(sh.cu[cc[j]], qw, dtm, sh.tc[cc[j]] - sh.tr[rr[j]], best[j]);
    }
  }
}

// ---- small bands: every step in one workgroup per model ---------------------------
// When the band's cells, the two-step pairs and the per-node offsets fit one
// workgroup's LDS (the whole video at T = 10: 7.5k cells, 14k pairs), one
// workgroup per model runs steps 1..M-1 with V_{i-1}, A, C and the offsets in
// LDS and a workgroup barrier between steps, instead of a launch per step whose
// dependent global reads make up most of its time.  Every term, and the order
// of the operations that form a cell's value, is that of k_trellis_first and
// k_trellis_step, so both give the same bits.
constexpr int kFusedThreads = 1024;
constexpr int kFusedSlots = 8;                                   // cells per thread
constexpr int kFusedLds = 160 * 1024 - 512;                      // bytes of the LDS pool

constexpr long long fused_bytes(long long Q, long long QC, long long n) {
  return 8 * n + 8 * n + 4 * Q + 4 * Q + 4 * QC + 2 * Q;
}

template <bool DEGEN>
__global__ __launch_bounds__(kFusedThreads) void k_trellis_fused(TrellisRun a) {
  __shared__ __align__(16) unsigned char pool[kFusedLds];
  const TrellisModel md = a.models[blockIdx.x];
  const int32_t M = md.m.M;
  const TrellisBand& b = a.band;
  const int32_t n = a.n, Q = static_cast<int32_t>(a.Q), QC = static_cast<int32_t>(a.QC);
  const int tid = threadIdx.x;
  const float INF = __builtin_inff();
  int2* kin = reinterpret_cast<int2*>(pool);           // (rowoff - s_lo, qoff - q_lo) of node k
  int2* prg = kin + n;                                 // predecessors [p_lo, p_hi) of node r
  float2* VA = reinterpret_cast<float2*>(prg + n);     // (V_{i-1}, A(r, c)) of every cell: one read per term
  float* C = reinterpret_cast<float*>(VA + Q);         // C(k, c) of every two-step pair
  int16_t* crow = reinterpret_cast<int16_t*>(C + QC);  // row of every cell
  for (int32_t k = tid; k < n; k += kFusedThreads) {
    const int32_t r0 = static_cast<int32_t>(b.rowoff[k]), r1 = static_cast<int32_t>(b.rowoff[k + 1]);
    kin[k] = make_int2(r0 - b.s_lo[k], static_cast<int32_t>(b.qoff[k]) - b.q_lo[k]);
    prg[k] = make_int2(b.p_lo[k], b.p_hi[k]);
    for (int32_t q = r0; q < r1; ++q) crow[q] = static_cast<int16_t>(k);
  }
  for (int32_t q = tid; q < Q; q += kFusedThreads) VA[q].y = b.A[q];
  for (int32_t q = tid; q < QC; q += kFusedThreads) C[q] = b.C[q];
  __syncthreads();

  // the thread's cells and step 1: V_1(r, c) = l1 (U_0(r) + U_1(c)) + l2 |dt|
  int32_t cr[kFusedSlots], cc[kFusedSlots], lo[kFusedSlots], hi[kFusedSlots], dt[kFusedSlots];
  float arc[kFusedSlots];
  bool same[kFusedSlots];
  const int32_t dtm1 = md.m.t[1] - md.m.t[0];
#pragma unroll
  for (int j = 0; j < kFusedSlots; ++j) {
    const int32_t q = tid + kFusedThreads * j;
    const bool valid = q < Q;
    const int32_t r = valid ? crow[q] : 0;
    const int32_t c = valid ? q - kin[r].x : 0;  // s_lo[r] + (q - rowoff[r])
    const int2 p = prg[r];
    cr[j] = r;
    cc[j] = c;
    lo[j] = valid ? p.x : 0;
    hi[j] = valid ? p.y : 0;
    dt[j] = a.t[c] - a.t[r];
    arc[j] = valid ? VA[q].y : 0.f;
    if (DEGEN) {
      const float2 xr = a.xy[r], xc = a.xy[c];
      same[j] = xr.x == xc.x && xr.y == xc.y;
    } else {
      same[j] = false;
    }
    if (valid) {
      const float v = first_value(a, md.U[r], md.U[n + c], dtm1, dt[j]);
      VA[q].x = v;
      md.V[q] = v;
    }
  }
  __syncthreads();

  for (int32_t i = 2; i < M; ++i) {
    const float2 th = md.theta[i];
    const int32_t dtm = md.m.t[i] - md.m.t[i - 1];
    const float qw = a.lambda2 * (i <= M - 2 ? 2.f : 1.f);
    const float* Ui = md.U + (long long)i * n;
    float* Vi = md.V + (long long)(i - 1) * a.Q;
    float nv[kFusedSlots];
#pragma unroll
    for (int j = 0; j < kFusedSlots; ++j) {
      nv[j] = INF;
      if (tid + kFusedThreads * j < Q) {
        float bm, be;
        cell_brackets(th, -arc[j], bm, be);
        const int32_t r = cr[j], c = cc[j];
        float best = INF;
        // unrolled by two (the whole video at T = 10, one model: 0.49 ms per run,
        // against 0.53 not unrolled and 0.52 by four)
#pragma unroll 2
        for (int32_t k = lo[j]; k < hi[j]; ++k) {
          const int2 kk = kin[k];
          const int32_t off = kk.x + r;  // cell (k, r)
          const float2 va = VA[off];
          best = fminf(best, relax<DEGEN>(va.x, va.y, C[kk.y + c], bm, be, th, same[j], a.w));
        }
        nv[j] = step_value(__fmul_rn(a.lambda1, Ui[c]), qw, dtm, dt[j], best);
      }
    }
    __syncthreads();  // every read of V_{i-1} done
#pragma unroll
    for (int j = 0; j < kFusedSlots; ++j) {
      const int32_t q = tid + kFusedThreads * j;
      if (q < Q) {
        VA[q].x = nv[j];
        Vi[q] = nv[j];
      }
    }
    __syncthreads();
  }
}

// ---- optimum and backtracking, one workgroup per model ---------------------------
template <bool DEGEN>
__global__ __launch_bounds__(256) void k_trellis_final(TrellisRun a) {
  __shared__ float red_v[4];
  __shared__ long long red_i[4];
  __shared__ float res_v;
  __shared__ long long res_i;
  const int32_t q = blockIdx.x;
  const TrellisModel md = a.models[q];
  const int32_t M = md.m.M;
  const TrellisBand& b = a.band;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const float INF = __builtin_inff();
  const float* VM = md.V + (long long)(M - 2) * a.Q;  // V_{M-1}
  float bv = INF;
  long long bi = 0x7fffffffffffffffLL;
  for (long long x = tid; x < a.Q; x += 256) {
    const float v = VM[x];
    if (v < bv) { bv = v; bi = x; }  // x ascends: the first minimum of this thread
  }
  for (int off = 32; off > 0; off >>= 1) {
    const float ov = __shfl_xor(bv, off);
    const long long oi = __shfl_xor(bi, off);
    if (ov < bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  if (lane == 0) { red_v[wv] = bv; red_i[wv] = bi; }
  __syncthreads();
  if (tid == 0) {
    for (int w2 = 1; w2 < 4; ++w2)
      if (red_v[w2] < bv || (red_v[w2] == bv && red_i[w2] < bi)) { bv = red_v[w2]; bi = red_i[w2]; }
    res_v = bv;
    res_i = bi;
    a.e32[q] = bv;
  }
  __syncthreads();
  if (wv != 0) return;
  int32_t* out = a.assign + md.assign0;
  if (!(res_v < INF)) {
    for (int i = lane; i < M; i += 64) out[i] = -1;
    return;
  }
  // the optimal final cell: row = last r with rowoff[r] <= index
  const long long idx = res_i;
  int32_t lo = 0, hi = a.n;  // rowoff[lo] <= idx < rowoff[hi]
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (b.rowoff[mid] <= idx) lo = mid; else hi = mid;
  }
  int32_t r = lo, c = b.s_lo[lo] + static_cast<int32_t>(idx - b.rowoff[lo]);
  if (lane == 0) {
    out[M - 1] = a.node0 + c;
    out[M - 2] = a.node0 + r;
  }
  const int32_t TS = a.span_lim;
  for (int32_t i = M - 1; i >= 2; --i) {
    const float* Vp = md.V + (long long)(i - 2) * a.Q;  // V_{i-1}
    const float2 th = md.theta[i];
    const float arc = b.A[b.rowoff[r] + (c - b.s_lo[r])];
    float bm, be;
    cell_brackets(th, -arc, bm, be);
    const float2 xr = a.xy[r], xc = a.xy[c];
    const bool same = xr.x == xc.x && xr.y == xc.y;
    const int32_t tcv = a.t[c];
    float tot = INF;
    int32_t bk = 0x7fffffff;
    for (int32_t k0 = b.p_lo[r]; k0 < b.p_hi[r]; k0 += 64) {
      const int32_t k = k0 + lane;
      if (k < b.p_hi[r] && span_ok(a.t[k], tcv, TS)) {
        const long long off = b.rowoff[k] + (r - b.s_lo[k]);
        const float v = relax<DEGEN>(Vp[off], b.A[off], b.C[b.qoff[k] + (c - b.q_lo[k])], bm, be, th, same, a.w);
        if (v < tot) { tot = v; bk = k; }  // k ascends: the lowest k of this lane's minimum
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const float ot = __shfl_xor(tot, off);
      const int32_t ok = __shfl_xor(bk, off);
      if (ot < tot || (ot == tot && ok < bk)) { tot = ot; bk = ok; }
    }
    if (bk == 0x7fffffff) {  // no predecessor: cannot happen on a finite optimum
      for (int j = lane; j < M; j += 64) out[j] = -1;
      return;
    }
    if (lane == 0) out[i - 2] = a.node0 + bk;
    c = r;
    r = bk;
  }
}

}  // namespace

hipError_t launch_trellis_band(const int32_t* t, int32_t n, const SearchParams& sp, const TrellisBand& b,
                               hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trellis_band, dim3((n + 255) / 256), dim3(256), 0, st, t, n, sp, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan64, dim3(1), dim3(1024), 0, st, b.rowoff, n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan64, dim3(1), dim3(1024), 0, st, b.qoff, n);
  return hipGetLastError();
}

hipError_t launch_trellis_dirs(const TrellisBand& b, int32_t n, const float2* xy, const int32_t* t, int32_t span_lim,
                               int32_t* flag, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trellis_dirs, dim3(n, 2), dim3(64), 0, st, b, xy, t, span_lim, flag);
  return hipGetLastError();
}

bool trellis_fits_fused(long long Q, long long QC, int32_t n) {
  return Q > 0 && Q <= (long long)kFusedThreads * kFusedSlots && n <= 32767 && fused_bytes(Q, QC, n) <= kFusedLds;
}

hipError_t launch_trellis_run(const TrellisRun& a, int32_t n_tiles, int32_t tile_cells, int32_t m_max, bool degen,
                              bool fused, hipStream_t st) {
  if (a.n_models <= 0) return hipSuccess;
  if (fused) {
    if (!trellis_fits_fused(a.Q, a.QC, a.n)) return hipErrorInvalidValue;
    if (degen)
      hipLaunchKernelGGL(k_trellis_fused<true>, dim3(a.n_models), dim3(kFusedThreads), 0, st, a);
    else
      hipLaunchKernelGGL(k_trellis_fused<false>, dim3(a.n_models), dim3(kFusedThreads), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  } else if (a.Q > 0) {
    hipLaunchKernelGGL(k_trellis_first, dim3(a.n, a.n_models), dim3(64), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (tile_cells != kTrellisTileCells && tile_cells != kTrellisSmallTileCells) return hipErrorInvalidValue;
    const bool small_tiles = tile_cells == kTrellisSmallTileCells;
    for (int32_t i = 2; i < m_max && n_tiles > 0; ++i) {
      const dim3 grid(n_tiles, a.n_models);
      // (1024-cell tiles are cut only for launches of many workgroups)
      const bool many = (long long)n_tiles * a.n_models >= kManyTiles;
      constexpr int kS = kTrellisSmallTileCells / kThreads, kL = kTrellisTileCells / kThreads;
      if (degen && !small_tiles)
        hipLaunchKernelGGL((k_trellis_step<true, kChunkWide, kWavesWide, kL>), grid, dim3(kThreads), 0, st, a, i);
      else if (degen && many)
        hipLaunchKernelGGL((k_trellis_step<true, kChunkWide, kWavesWide, kS>), grid, dim3(kThreads), 0, st, a, i);
      else if (degen)
        hipLaunchKernelGGL((k_trellis_step<true, kChunkSmall, kWavesSmall, kS>), grid, dim3(kThreads), 0, st, a, i);
      else if (!small_tiles)
        hipLaunchKernelGGL((k_trellis_step<false, kChunkWide, kWavesWide, kL>), grid, dim3(kThreads), 0, st, a, i);
      else if (many)
        hipLaunchKernelGGL((k_trellis_step<false, kChunkWide, kWavesWide, kS>), grid, dim3(kThreads), 0, st, a, i);
      else
        hipLaunchKernelGGL((k_trellis_step<false, kChunkSmall, kWavesSmall, kS>), grid, dim3(kThreads), 0, st, a, i);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  if (degen)
    hipLaunchKernelGGL(k_trellis_final<true>, dim3(a.n_models), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_trellis_final<false>, dim3(a.n_models), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace stm
