// Internal declarations shared by the HIP sources of libstm.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace stm {

// Device view of one model and one scene.  Scene nodes are sorted by frame;
// fstart[f] is the first node of frame f (the paper's minnode(f), Section
// 3.4), fstart[F] = S.
struct SceneView {
  const float2* xy;
  const int32_t* t;
  const float* desc;
  const int32_t* fstart;
  int32_t S, F, dim;
};

struct ModelView {
  const float2* xy;
  const int32_t* t;
  const float* desc;
  int32_t M;
};

struct SearchParams {
  int32_t T, W, K, kdensity;
  int32_t span;  // closeness as the span of each triangle (Section 3.4, Eq. 14)
  int32_t uns;   // unsigned triangle angles (the magnitudes of Eq. 6's angles)
  int32_t node;  // causality by scene node order, z_{i-1} < z_i (equal frames allowed)
};

// Closeness limit of consecutive points: T of Eq. 8, or under the span reading
// T - 1, since a pair inside a triangle whose first and last frames are less
// than T apart is at most T - 2 frames apart (T = 1, 2: no pair); <= 0: none.
__host__ __device__ __forceinline__ int32_t pair_limit(const SearchParams& sp) {
  return sp.span && sp.T > 0 ? (sp.T > 2 ? sp.T - 1 : 1) : sp.T;
}

// Limit on the first and last frames of a triangle under the span reading
// (t'(z_i) - t'(z_{i-2}) < limit); 0 when it does not apply.
__host__ __device__ __forceinline__ int32_t span_limit(const SearchParams& sp) {
  return sp.span && sp.T > 0 ? sp.T : 0;
}

// Candidate list of one model point at one offset, as two ascending node
// ranges: [s1, s1 + k1) then [s2, s2 + k2), with s1 + k1 <= s2.
struct CandRange {
  int32_t s1, k1, s2, k2;
};

// Reads an input that no kernel writes while the reader runs (points, frame
// starts, unary tables, model angles, given lists) through the constant address
// space: a wave-uniform address becomes a scalar load and a divergent one a
// global load, where a pointer fetched from memory would otherwise be read with
// flat loads, which also hold up the wave's LDS waits.
template <class T>
__device__ __forceinline__ T ro(const T* p) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte elements");
  using Word = typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type;
  return __builtin_bit_cast(T, *(const __attribute__((address_space(4))) Word*)p);
}

__device__ __forceinline__ int32_t fs_at(const int32_t* __restrict__ fstart, int32_t F, int32_t f) {
  f = f < 0 ? 0 : (f > F ? F : f);
  return ro(fstart + f);
}

// Per-point cap from the local density: rho = nodes in frames f0-1..f0+1,
// K = clamp(floor((56 rho - 1170) / 60), 8, 64) (8 + 56 (rho - 30) / 60 rounded
// half up), never above k_max.  bnd(d) is the first node of frame f0 + d,
// clamped (fstart[0] below frame 0, fstart[F] above frame F).
template <class Bnd>
__device__ __forceinline__ int32_t density_cap_by(const Bnd& bnd, int32_t kmax) {
  int32_t rho = bnd(2) - bnd(-1);
  int32_t num = 56 * rho - 1170;
  int32_t k = num >= 0 ? num / 60 : -((-num + 59) / 60);
  k = k < 8 ? 8 : (k > 64 ? 64 : k);
  return k < kmax ? k : kmax;
}

// The first K nodes within W frames of frame f0, ordered by (|frame - f0|,
// node id), returned in ascending node order.  Frames are visited in the
// order f0, f0-1, f0+1, f0-2, f0+2, ...: whole frames are taken while they fit,
// the first frame that does not fit contributes its lowest node ids.  The
// whole frames form one contiguous frame interval, so the kept set is at most
// two contiguous node ranges.  A frame outside the scene has bnd(d + 1) =
// bnd(d), no nodes.  kW > 0 unrolls the visiting loop for windows W <= kW,
// so that bnd sees compile-time offsets only.
template <int kW, class Bnd>
__device__ __forceinline__ CandRange cand_range_by(const Bnd& bnd, int32_t W, int32_t K) {
  int32_t taken = 0;
  int32_t a = bnd(0), b = a;  // nodes [a, b) of the whole frames taken so far
  CandRange r;
  // one visited frame; true once the range is complete
  const auto visit = [&](int32_t step) {
    const int32_t d = step == 0 ? 0 : ((step & 1) ? -((step + 1) >> 1) : (step >> 1));
    const int32_t s = bnd(d), e = bnd(d + 1);
    if (taken + (e - s) <= K) {
      taken += e - s;
      if (d <= 0) a = s;
      if (d >= 0) b = e;
      return false;
    }
    const int32_t kp = K - taken;
    if (d < 0) {
      r.s1 = s; r.k1 = kp; r.s2 = a; r.k2 = b - a;
    } else {
      r.s1 = a; r.k1 = b - a; r.s2 = s; r.k2 = kp;
    }
    return true;
  };
  if constexpr (kW > 0) {
#pragma unroll
    for (int32_t step = 0; step <= 2 * kW; ++step)
      if (step > 2 * W || visit(step)) return step > 2 * W ? CandRange{a, b - a, b, 0} : r;
  } else {
    for (int32_t step = 0; step <= 2 * W; ++step)
      if (visit(step)) return r;
  }
  return CandRange{a, b - a, b, 0};
}

// Windows up to this half-width read all their frame boundaries in one round
// of independent loads before the rule runs, instead of one load per visited
// frame.
constexpr int32_t kWindowPreload = 3;

__device__ __forceinline__ CandRange point_candidates(const int32_t* __restrict__ fstart, int32_t F,
                                                      int32_t f0, const SearchParams& sp) {
  if (sp.W <= kWindowPreload) {
    constexpr int kW = kWindowPreload;
    int32_t bd[2 * kW + 4];  // first nodes of frames f0 - kW - 1 .. f0 + kW + 2
#pragma unroll
    for (int l = 0; l < 2 * kW + 4; ++l) bd[l] = fs_at(fstart, F, f0 - kW - 1 + l);
    const auto bnd = [&](int32_t d) { return bd[d + kW + 1]; };
    const int32_t K = sp.kdensity ? density_cap_by(bnd, sp.K) : sp.K;
    return cand_range_by<kW>(bnd, sp.W, K);
  }
  const auto bnd = [&](int32_t d) { return fs_at(fstart, F, f0 + d); };
  const int32_t K = sp.kdensity ? density_cap_by(bnd, sp.K) : sp.K;
  return cand_range_by<0>(bnd, sp.W, K);
}

__device__ __forceinline__ int32_t cand_node(const CandRange& c, int32_t a) {
  return a < c.k1 ? c.s1 + a : c.s2 + (a - c.k1);
}

// Causality (strictly increasing scene frames, Eq. 7) and temporal closeness
// (consecutive scene frames less than T apart, Eq. 8; T <= 0: no limit).
__device__ __forceinline__ bool admissible(int32_t tp_prev, int32_t tp_cur, int32_t T) {
  return tp_prev < tp_cur && (T <= 0 || tp_cur - tp_prev < T);
}

// The same for consecutive points (z_prev, z_cur) under the search's reading
// of causality: frames as above, or with node order increasing node ids and
// Eq. 8's closeness.
__device__ __forceinline__ bool consecutive_ok(const SearchParams& sp, int32_t T, int32_t n_prev, int32_t t_prev,
                                               int32_t n_cur, int32_t t_cur) {
  return sp.node ? n_prev < n_cur && (T <= 0 || t_cur - t_prev < T) : admissible(t_prev, t_cur, T);
}

// Entries <= x (below: < x) of the ascending windowed list c of scene nodes.
__device__ __forceinline__ int32_t range_count_le(const CandRange& c, int32_t x) {
  return min(max(x - c.s1 + 1, 0), c.k1) + min(max(x - c.s2 + 1, 0), c.k2);
}
__device__ __forceinline__ int32_t range_count_lt(const CandRange& c, int32_t x) { return range_count_le(c, x - 1); }

// The span reading's condition on a triangle's first and last scene frames
// (limit from span_limit; 0: always true).
__device__ __forceinline__ bool span_ok(int32_t tp_first, int32_t tp_last, int32_t limit) {
  return limit <= 0 || tp_last - tp_first < limit;
}

// Oriented angle at vertex b of the triangle (a, b, c), from ray b->a to ray
// b->c, in FP64; 0 when a side has zero length (Eq. 6).
__device__ __forceinline__ double ang64(double ax, double ay, double bx, double by, double cx,
                                        double cy) {
  const double ux = ax - bx, uy = ay - by, vx = cx - bx, vy = cy - by;
  if ((ux == 0.0 && uy == 0.0) || (vx == 0.0 && vy == 0.0)) return 0.0;
  return atan2(ux * vy - uy * vx, ux * vx + uy * vy);
}

// ---- launchers (return hipError_t of the launch) ---------------------------

// Validation of inputs: flags bits (see api.cpp) are OR-ed into out[0]; the
// model span t[M-1] - t[0] is written to out[1] by one thread.
hipError_t launch_validate(const ModelView& m, const SceneView& s, int32_t* out, hipStream_t st);
hipError_t launch_fstart(const int32_t* t, int32_t S, int32_t F, int32_t* fstart, hipStream_t st);
hipError_t launch_candidates(const ModelView& m, const SceneView& s, const SearchParams& sp,
                             int32_t tau0, int32_t n_tau, int32_t* cand, int32_t* count,
                             hipStream_t st);
hipError_t launch_unary_f32(const ModelView& m, const SceneView& s, float* U, hipStream_t st);
hipError_t launch_count(const ModelView& m, const SceneView& s, const SearchParams& sp,
                        int32_t tau0, int32_t n_tau, unsigned long long* counts, hipStream_t st);
hipError_t launch_model_angles(const ModelView& m, float2* theta, hipStream_t st);

// BF16 split-precision unary table.  launch_to_bf16 writes x [n_valid][dim]
// rounded to BF16 into out [np][bf16_padded_dim(dim)] (zero padding) and the
// squared norms of the rounded rows into norm2 [np].  launch_unary_bf16 reads
// fb/fn padded to a multiple of 16 rows and gb/gn padded to a multiple of 256.
int32_t bf16_padded_dim(int32_t dim);
hipError_t launch_to_bf16(const float* x, int32_t n_valid, int32_t dim, int32_t np, uint16_t* out,
                          float* norm2, hipStream_t st);
hipError_t launch_unary_bf16(const uint16_t* fb, const float* fn, int32_t M, const uint16_t* gb,
                             const float* gn, int32_t S, int32_t dim, float* U, hipStream_t st);

struct DPLaunch {
  ModelView m;
  SceneView s;
  SearchParams sp;
  const float* U;       // [M][S] raw distances
  const float2* theta;  // [M] model angles (mid, end) of the triangle ending at i
  float lambda1, lambda2, w;  // w = lambda2 * lambda3
  int32_t tau0, n_tau;
  float* vt;            // [n_tau][M-2][V][V] cell values V_i, i = 1..M-2; V = K (+1 with dummies)
  float* e32;           // [n_tau]
  int2* last2;          // [n_tau]
  int32_t* degen;       // [n_tau], written by the fast variant
  int32_t waves;        // waves per workgroup of the recursion: 4, 8 or 16
  // explicit candidate lists (null: the windowed rule): offset tl, point j has
  // the nodes cand[(tl * M + j) * cstride + a], a < ccount[tl * M + j], ascending
  const int32_t* cand = nullptr;
  const int32_t* ccount = nullptr;
  int32_t cstride = 0;
  // explicit offsets (null: tau0 + tl): matching tl of the launch is offset taus[tl]
  const int32_t* taus = nullptr;
  // dummy assignments (Eq. 2): enabled flag and lambda1 * W^d in FP32
  int32_t dummy = 0;
  float cw = 0.f;
  // packed schedules (sparse scenes, long lists; no dummies): every cell of a
  // step on its own lane, chunk after chunk
  int32_t packed = 0;
};
// The fast variant over every matching of the launch, then the variant for
// degenerate triangles, which only recomputes the matchings flagged by the first.
hipError_t launch_dp_fast(const DPLaunch& a, hipStream_t st);
hipError_t launch_dp_degenerate(const DPLaunch& a, hipStream_t st);

hipError_t launch_backtrack(const DPLaunch& a, int32_t* assign, hipStream_t st);

// FP64 energy of each assignment row; w_dummy is W^d, the unary cost of a
// dummy (node id -2 in assign; never present when dummies are off).
hipError_t launch_rescore(const ModelView& m, const SceneView& s, const SearchParams& sp, double lambda1,
                          double lambda2, double lambda3, double w_dummy, const int32_t* assign,
                          int32_t n_tau, double* e64, double* eu64, hipStream_t st);

// ---- batched persistent launch ---------------------------------------------------

// One (model, scene) pair of a batch.
struct PairDev {
  ModelView m;
  SceneView s;
  const float* U;       // this model's rows of the scene's unary table
  long long us;         // row stride of U (the scene's point count)
  const float2* theta;  // this model's angles
  long long row0;       // first output row (offset 0) of the pair
  long long assign0;    // first assignment element of the pair
  int32_t n_tau;
  // explicit candidate lists (null: the windowed rule): offset tau, point j has
  // cand[(tau * M + j) * cstride + a], a < ccount[tau * M + j], ascending
  const int32_t* cand = nullptr;
  const int32_t* ccount = nullptr;
  int32_t cstride = 0;
};

struct BatchLaunch {
  const PairDev* pairs;
  const int2* items;    // (pair, offset), in the order workgroups take them
  int32_t n_items;
  int32_t* counter;     // two work counters (fast, degenerate), 0 at launch
  int32_t* degen_count; // items whose matching has coincident points, 0 at launch
  int32_t* degen_items; // [n_items] their indices into items
  // the fast variant's items: all of items (list null), or items[list[q]] for
  // q < *list_count (read on the device)
  const int32_t* list = nullptr;
  const int32_t* list_count = nullptr;
  SearchParams sp;
  float lambda1, lambda2, w;
  float* vt;            // value-table scratch: batch slots of vt_stride floats per workgroup
  long long vt_stride;
  int32_t batch = 1;    // items a workgroup takes at a time (1..kMaxBatch)
  int32_t dummy = 0;    // dummy assignments (Eq. 2) enabled
  float cw = 0.f;       // lambda1 * W^d in FP32
  int32_t packed = 0;   // packed schedules (sparse scenes; no dummies)
  float* e32;           // [rows]
  int32_t* assign;      // [sum over pairs of n_tau * M]
  int32_t waves;        // 4, 8 or 16 waves per workgroup
};

// Most items a persistent workgroup takes at a time.
constexpr int kMaxBatch = 8;

// The fast variant over all items, then the degenerate variant over the items
// the first one flagged; n_wg workgroups each.
hipError_t launch_dp_persistent(const BatchLaunch& b, int n_wg, hipStream_t st);
hipError_t launch_item_cost(const PairDev* pairs, const int2* items, int n_items, const SearchParams& sp,
                            long long* cost, hipStream_t st);
hipError_t launch_fill_i32(int* p, int n, int v, hipStream_t st);
// Items whose matching is infeasible (e32 of its row is +inf): their indices
// appended to list (order unspecified) and counted in *count; fell[row] = 1
// for them when fell is given (rows of the other items are left as they are).
hipError_t launch_collect_infeasible(const PairDev* pairs, const int2* items, int n_items, const float* e32,
                                     int32_t* list, int32_t* count, int32_t* fell, hipStream_t st);
hipError_t launch_rescore_batch(const PairDev* pairs, const int2* items, int n_items, const SearchParams& sp,
                                double lambda1, double lambda2, double lambda3, double w_dummy,
                                const int32_t* assign, double* e64, double* eu64, hipStream_t st);

// ---- the trellis over a scene block ---------------------------------------------------

// Tiles of a step: rows [r0, r1) by columns [c0, c1) of the band, ncell >= 1
// cells (c a successor of r inside the window), predecessors [k0, k1).
constexpr int kTrellisTileRows = 64;
constexpr int kTrellisTileCols = 128;
constexpr int kTrellisTileCells = 1024;
constexpr int kTrellisSmallTileCells = 256;  // tiles of launches with few workgroups
struct TrellisTile {
  int32_t r0, r1, c0, c1, k0, k1, ncell, pad;
};

// The band of a scene block of n nodes (local ids, sorted by frame): successors
// [s_lo, s_hi) (frames in (t, t + T)), predecessors [p_lo, p_hi) (frames in
// (t - T, t)), two-step pairs [q_lo, q_hi) (frames in [t + 2, t + 2T - 2]), with
// T the limit of consecutive points (pair_limit); rowoff [n + 1] and qoff
// [n + 1] number the cells and the pairs row after row; A [rowoff[n]] holds
// -phi(r -> c) of every cell, C [qoff[n]] -phi(k -> c) of every pair (+inf
// for pairs the span reading excludes; NaN for coincident points).
struct TrellisBand {
  int32_t *s_lo, *s_hi, *p_lo, *p_hi, *q_lo, *q_hi;
  long long *rowoff, *qoff;
  float *A, *C;
};

// One model of a trellis run: U [M][n] raw distances to the block's nodes,
// V [(M - 1)][Q] the value tables of steps 1..M-1, assignments from
// assign + assign0.
struct TrellisModel {
  ModelView m;
  const float2* theta;
  const float* U;
  float* V;
  long long assign0;
};

struct TrellisRun {
  const TrellisModel* models;
  int32_t n_models;
  TrellisBand band;
  const TrellisTile* tiles;
  const int32_t* t;     // [n] the block's frames
  const float2* xy;     // [n] the block's coordinates
  int32_t n;            // block nodes
  int32_t node0;        // scene id of the block's first node
  long long Q;          // cells per step
  long long QC;         // two-step direction pairs
  int32_t span_lim;     // span_limit of the search parameters
  float lambda1, lambda2, w;
  float* e32;           // [n_models]
  int32_t* assign;      // scene node ids, -1 rows when infeasible
};

// The band of the block (t [n] sorted): ranges, then offsets by two scans.
hipError_t launch_trellis_band(const int32_t* t, int32_t n, const SearchParams& sp, const TrellisBand& b,
                               hipStream_t st);
// The direction tables A and C; *flag |= 1 when coincident points take part.
hipError_t launch_trellis_dirs(const TrellisBand& b, int32_t n, const float2* xy, const int32_t* t, int32_t span_lim,
                               int32_t* flag, hipStream_t st);
// Steps 1..M-1 of every model, then the optimum and backtracking (degen: the
// variant that handles coincident points; fused: every step in one workgroup
// per model, for bands that trellis_fits_fused accepts; tile_cells: the cell
// cap the tiles were cut with, kTrellisTileCells or kTrellisSmallTileCells).
hipError_t launch_trellis_run(const TrellisRun& a, int32_t n_tiles, int32_t tile_cells, int32_t m_max, bool degen,
                              bool fused, hipStream_t st);
// Whether a band of n nodes, Q cells and QC two-step pairs fits one
// workgroup's LDS for the fused run.
bool trellis_fits_fused(long long Q, long long QC, int32_t n);

// ---- learned candidate pruner -------------------------------------------------------

constexpr int kPrunerHidden = 128;

// Candidate nodes, features and the neighbours' chosen candidates of groups
// (tau, i) = groups[g], or (tau0 + g / M, g % M) without a list: node [G * 64]
// (-1 past the list), phi [G * 64][8], q [G][2] (nullable).
hipError_t launch_group_rows(const ModelView& m, const SceneView& s, const float* U, long long us,
                             const SearchParams& sp, const int2* groups, int tau0, long long G, int32_t* node,
                             float* phi, int32_t* q, hipStream_t st);

// One FP32 training pass over G groups (rows = 64 G): forward, scores and
// per-group losses; with labels also the gradient of the mean loss into grad
// (packed like theta).  Buffers: h1, h2, dz1, dz2 [rows][128], ds [rows],
// part [pruner_part_floats(G, D)].
struct PrunerTrain {
  const float* mdesc;
  const float* sdesc;
  const int2* groups;
  const int32_t* node;
  const float* phi;
  const int32_t* labels;  // null: forward only
  int D, G;
  const float* theta;
  float* grad;
  float *h1, *h2, *dz1, *dz2, *ds, *loss, *scores, *part;
};
hipError_t launch_pruner_train(const PrunerTrain& t, hipStream_t st);
long long pruner_part_floats(int G, int D);
hipError_t launch_adam(float* theta, const float* g, float* m, float* v, long long n, float lr, float beta1,
                       float beta2, float eps, float c1, float c2, hipStream_t st);

// BF16 inference.
hipError_t launch_cast_rows_bf16(const float* W, int rows, int ld, int off, int D, int dp, uint16_t* out,
                                 hipStream_t st);
hipError_t launch_project_bf16(const uint16_t* Xb, int n, int dp, const uint16_t* Wb, float scale,
                               const float* bias, float* P, hipStream_t st);
struct PrunerInfer {
  ModelView m;
  SceneView s;
  const float* U;
  long long us;
  SearchParams sp;
  const int2* groups;  // null: groups (tau0 + g / M, g % M)
  long long n_groups;
  int tau0;
  int32_t* node;        // scratch [n_groups][64]: candidate of each slot (written here)
  float* phi;           // scratch [n_groups][64][8]: its features (written here)
  const float* theta;  // FP32 parameters (W1 phi columns, W2, b2, w3, b3)
  int D;
  const float* A;       // [M][128] model projection W1[:, 0:D] (D f) + b1
  const float* B;       // [S][128] scene projection W1[:, D:2D] (D g)
  int topk;
  int rule;             // 0: top-k by score; 1: nearest frames first, score inside; 2: nearest frames, then slot
  int32_t* cand;        // [n_groups][topk]
  int32_t* count;       // [n_groups]
  float* scores;        // [n_groups][64], nullable
};
hipError_t launch_pruner_infer(const PrunerInfer& q, hipStream_t st);
// Checks caller-given lists [rows][kc] with counts [rows]; ORs error bits into *bad.
hipError_t launch_check_lists(const int32_t* cand, const int32_t* count, long long rows, int kc, int S, int32_t* bad,
                              hipStream_t st);
// Exact re-solves of n offsets taus[] (rows r) back into outputs indexed by tau - tau0.
hipError_t launch_scatter_fallback(const int32_t* taus, int n, int tau0, int M, const float* e32, const double* e64,
                                  const double* eu, const int32_t* as, float* o32, double* o64, double* ou,
                                  int32_t* oas, int32_t* fell, hipStream_t st);

}  // namespace stm
