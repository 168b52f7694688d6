/*
 * stm.h — C ABI of libstm.so: exact space-time hypergraph matching on AMD
 * MI355X (gfx950).
 *
 * The library solves the matching problem of Lombardi, Wolf, Celiktutan and
 * Sankur, "Activity recognition from videos with parallel hypergraph matching
 * on GPUs" (arXiv 1505.00581), Section 2: assign each of the M time-ordered
 * points of a model action to a scene point so that the energy
 *
 *   E(z) = lambda1 * sum_i U(z_i) + lambda2 * sum_{i>=3} D(z_i, z_{i-1}, z_{i-2})   (Eq. 1, 9)
 *
 * is minimal, where U is the Euclidean descriptor distance (Eq. 2) and
 * D = D^t + lambda3 * D^g is the temporal plus angular distortion of the
 * triangle of three consecutive points (Eq. 3-6), under causality (Eq. 7:
 * consecutive points map to strictly increasing scene frames) and temporal
 * closeness (Eq. 8: consecutive scene frames less than T apart).  The exact
 * minimum is found by the second-order min-sum dynamic programme with
 * backtracking of Section 2.2 (Eq. 10-13), solved here in forward form.
 *
 * One "matching" is one model against one scene at one time offset tau: model
 * point i is searched among the scene points whose frame is within `window`
 * frames of tau + (t_i - t_1), keeping at most k_max of them (the first by
 * |frame difference|, then node id).  This bounded per-point search replaces
 * the paper's pruning of the trellis by causality and closeness (Sections 3.2
 * and 3.4).  Every offset is an independent matching.
 *
 * Conventions
 *  - Every function returns an int status: STM_OK (0) or a negative code; it
 *    never throws and never aborts.  stm_last_error() describes the last
 *    failure of the calling thread.
 *  - The caller owns every input and output buffer.  The context owns its
 *    device scratch (frame index, unary table, the recursion's value tables),
 *    grows it on demand and frees it in stm_destroy.  On STM_ENOMEM nothing
 *    was written.
 *  - Pointers are host pointers unless params->flags has STM_DEVICE_PTRS;
 *    then every input and output pointer of the call is a device pointer on
 *    the context's device, the work is queued on `hip_stream` (NULL: the HIP
 *    default stream) and the call returns once the inputs have been
 *    validated (one small device-to-host read) and the kernels are queued.
 *    With host pointers the call is synchronous.
 *  - One context per host thread; calls on one context must not overlap.
 *  - An offset with no admissible assignment is not an error: its energies
 *    are +inf and its assignment row is all -1.
 *  - Indices are 0-based: model points 0..M-1, scene nodes 0..S-1 in the
 *    order given (sorted by frame), offsets tau in [0, n_frames - span) with
 *    span = t_{M-1} - t_0.
 */
#ifndef STM_H
#define STM_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define STM_API __attribute__((visibility("default")))
#else
#define STM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define STM_OK            0
#define STM_EINVAL       -1  /* invalid argument or input data (see stm_last_error) */
#define STM_ENOMEM       -2  /* device or host allocation failed; nothing written   */
#define STM_EHIP         -3  /* a HIP runtime call failed (message has its string)  */
#define STM_EUNSUPPORTED -4  /* flag combination or size this library does not support  */

/* ---- limits ------------------------------------------------------------- */
/* Candidate cap: one 64-lane wavefront covers the candidates of one model
 * point.  A larger k_max gives STM_EUNSUPPORTED; the trellis over a scene
 * block (stm_trellis_*) searches every node of the block instead. */
#define STM_K_LIMIT 64

/* ---- flags (stm_params.flags) ------------------------------------------- */
#define STM_DEVICE_PTRS 0x1u  /* all pointers of the call are device pointers           */
#define STM_UNARY_BF16  0x2u  /* unary table as sqrt(|f|^2 + |g|^2 - 2 f.g) with the
                                 descriptors rounded to BF16, dot products on MFMA with
                                 FP32 accumulation, squared norms of the rounded vectors
                                 in FP32, the descriptor zero-padded to a multiple of 32;
                                 the recursion stays FP32 and the re-score FP64 from the
                                 FP32 descriptors                                          */
#define STM_K_DENSITY   0x4u  /* per-point cap from the local density of scene points:
                                 rho = points in frames f-1..f+1 around the shifted
                                 model frame f, K = clamp(floor((56 rho - 1170) / 60),
                                 8, 64), never above k_max                                */
#define STM_DUMMY       0x8u  /* dummy assignments (Eq. 2): a model point may stay
                                 unmatched (node id STM_DUMMY_NODE) at unary cost
                                 w_dummy.  The paper defines only that cost; here a
                                 Delta term of D^t (Eq. 4-5) counts only when both of
                                 its points are matched, D^g (Eq. 6) only when all
                                 three are, and causality and closeness (Eq. 7-8)
                                 bind matched consecutive points only.  Every offset
                                 is then feasible.  stm_match, stm_match_lists and
                                 plans (stm_plan_run) take it; the pruned entry
                                 points return STM_EUNSUPPORTED.                       */

#define STM_CLOSENESS_SPAN 0x10u  /* temporal closeness read from the loop bounds of
                                 Section 3.4 (Eq. 14): the first and last scene
                                 frames of every triangle (z_{i-2}, z_{i-1}, z_i)
                                 lie less than T apart, and consecutive points keep
                                 causality (Eq. 7) only, instead of Eq. 8's limit on
                                 consecutive points.  Consecutive points are then at
                                 most T - 2 frames apart.  No effect with T <= 0;
                                 not with STM_DUMMY (STM_EUNSUPPORTED).             */
#define STM_TRELLIS_STEPWISE 0x20u  /* trellis (stm_trellis_*) only: one launch per
                                 step even where the band fits one workgroup's LDS
                                 and all steps would run in one launch; the two give
                                 the same bits                                      */
#define STM_ANGLE_UNSIGNED 0x40u  /* the angles of Eq. 6 read as magnitudes in [0, pi]
                                 (unoriented), so that a triangle and its mirror
                                 image match; the default reads them oriented
                                 (atan2 of cross and dot products).  Exact path,
                                 lists and plans (stm_match, stm_match_lists,
                                 stm_match_batch, stm_plan_*, stm_match_noalloc,
                                 stm_match_chains);
                                 not with STM_DUMMY, the pruner or the trellis
                                 (STM_EUNSUPPORTED)                                 */
#define STM_CAUSAL_NODE 0x80u  /* causality (Eq. 7) read as increasing scene node ids,
                                 z_{i-1} < z_i, which in a scene sorted by frame lets
                                 consecutive points share a frame; closeness as Eq.
                                 8.  The default reads strictly increasing frames.
                                 Exact path and plans on the windowed lists
                                 (stm_match, stm_match_batch, stm_plan_run,
                                 stm_match_noalloc, stm_match_chains); not with
                                 STM_DUMMY, STM_CLOSENESS_SPAN, given lists, the
                                 pruner or the trellis (STM_EUNSUPPORTED)             */

/* Node id of a dummy assignment in assignment rows (STM_DUMMY); -1 marks the
 * rows of infeasible offsets. */
#define STM_DUMMY_NODE (-2)

/* ---- types -------------------------------------------------------------- */
typedef struct stm_ctx stm_ctx;

/* A point set (Section 2): `n` points with image coordinates, frame numbers and
 * appearance descriptors.  Models: t strictly increasing (one point per model
 * frame, Section 2.1), n >= 3.  Scenes: t non-decreasing with 0 <= t <
 * n_frames (points sorted by frame), n >= 1.  All arrays row-major,
 * caller-owned, read-only. */
typedef struct {
  int32_t n;            /* number of points                                      */
  int32_t dim;          /* descriptor length (the paper's HoG/HoF: 162)          */
  int32_t n_frames;     /* scenes: frame count; models: ignored                  */
  int32_t reserved;     /* must be 0                                             */
  const float* xy;      /* [n][2] pixel coordinates (x, y)                        */
  const int32_t* t;     /* [n] frame numbers                                     */
  const float* desc;    /* [n][dim] descriptors                                  */
} stm_points;

/* Energy weights and search limits.  The paper's values (Section 4):
 * lambda1 = 0.6, lambda2 = 0.2, lambda3 = 5, T = 10. */
typedef struct {
  double lambda1;       /* weight of the appearance term U (Eq. 1), >= 0           */
  double lambda2;       /* weight of the geometric term D (Eq. 1), >= 0            */
  double lambda3;       /* weight of D^g inside D (Eq. 3), >= 0                    */
  int32_t T;            /* temporal closeness in frames (Eq. 8); <= 0: no limit    */
  int32_t window;       /* candidate window half-width in frames, >= 0             */
  int32_t k_max;        /* candidate cap K, 1..STM_K_LIMIT                         */
  uint32_t flags;       /* STM_DEVICE_PTRS | STM_UNARY_BF16 | STM_K_DENSITY |
                           STM_DUMMY | STM_CLOSENESS_SPAN                          */
  double w_dummy;       /* W^d, the unary cost of a dummy (Eq. 2), finite, >= 0;
                           read only with STM_DUMMY                                 */
} stm_params;

/* ---- context ------------------------------------------------------------ */

/* Creates a context on HIP device `hip_device`.  *out receives the context.
 * Work is queued on the stream each call names (NULL: the HIP default
 * stream). */
STM_API int stm_create(stm_ctx** out, int hip_device);

/* Waits for the device, then frees the context and all its device scratch.
 * NULL is a no-op. */
STM_API void stm_destroy(stm_ctx* ctx);

/* Message of the last failed call on this thread ("" if none).  The string
 * stays valid until the next call on this thread. */
STM_API const char* stm_last_error(void);

/* ---- offsets ------------------------------------------------------------ */

/* The offsets at which the whole model fits in the scene: [*begin, *end) =
 * [0, max(0, scene->n_frames - (t_{M-1} - t_0))).  `flags` may hold
 * STM_DEVICE_PTRS (then model->t is read from the device of `ctx`). */
STM_API int stm_offsets(stm_ctx* ctx, const stm_points* model, const stm_points* scene, uint32_t flags,
                int32_t* begin, int32_t* end);

/* ---- the exact matching ------------------------------------------------- */

/* Exact optimum of E(z) (Eq. 1 and 9 under Eq. 7 and 8) at every offset in
 * [tau_begin, tau_end), found by the min-sum recursion with backtracking of
 * Section 2.2 (Eq. 10-13).  The recursion runs in FP32; the returned
 * assignment is re-scored from the definition in FP64.
 * Outputs, each [n_tau] with n_tau = tau_end - tau_begin (assign [n_tau][M]):
 *   energy32   FP32 optimum of the recursion, +inf if infeasible     (required)
 *   energy64   FP64 energy of the returned assignment (Eq. 1)         (nullable)
 *   energy_u64 FP64 appearance part lambda1 * sum_i U(z_i) (Eq. 2)    (nullable)
 *   assign     scene node id of every model point, -1 if infeasible,  (required)
 *              STM_DUMMY_NODE for a dummy (STM_DUMMY)
 * Ties are broken towards the lowest candidate index inside each minimum and
 * the first (row-major) final state pair; the dummy state counts after every
 * candidate.
 * Errors: STM_EINVAL for n < 3 (model) or < 1 (scene), dim mismatch, model
 * frames not strictly increasing, scene frames decreasing or outside
 * [0, n_frames), non-finite coordinates or descriptors, window < 0, k_max
 * < 1, a negative or non-finite lambda or w_dummy (with STM_DUMMY), or an
 * offset range outside [0, n_frames - span); STM_EUNSUPPORTED for k_max above
 * STM_K_LIMIT. */
STM_API int stm_match(stm_ctx* ctx, const stm_points* model, const stm_points* scene,
              const stm_params* params, int32_t tau_begin, int32_t tau_end,
              float* energy32, double* energy64, double* energy_u64, int32_t* assign,
              void* hip_stream);

/* ---- the exact matching without allocation -------------------------------
 *
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels, results and tie rules as stm_match, with all device scratch taken
 * from one fixed array of STM_NOALLOC_SCRATCH_BYTES per device, which the
 * library holds from the first stm_create on that device until the process
 * ends.  It never calls hipMalloc or hipFree.
 *
 * params->flags must hold STM_DEVICE_PTRS: every input and output is a
 * caller-owned device pointer, the work is queued on `hip_stream` (NULL: the
 * HIP default stream) and the call returns after the input validation (one
 * small device-to-host read, so the call itself cannot be captured into a
 * graph).  The offsets run in chunks of as many as the array holds beside the
 * frame index, model angles and unary table (and the BF16 copies with
 * STM_UNARY_BF16).
 *
 * Every call on a device shares that device's array and leaves its contents
 * behind; calls that overlap on one device (from several host threads, or on
 * streams not ordered with each other) race on it and must be serialised by
 * the caller.
 * Errors: as stm_match; STM_EINVAL without STM_DEVICE_PTRS, or when the
 * frame index, angles and unary table plus the buffers of one offset exceed
 * the array (M * S * 4 bytes of unary table, (M - 2) * K^2 * 4 bytes per
 * offset, (K + 1)^2 with STM_DUMMY); STM_EHIP if the array's device address
 * could not be looked up at context creation. */
#define STM_NOALLOC_SCRATCH_BYTES (256u << 20)
STM_API int stm_match_noalloc(stm_ctx* ctx, const stm_points* model, const stm_points* scene,
                              const stm_params* params, int32_t tau_begin, int32_t tau_end,
                              float* energy32, double* energy64, double* energy_u64, int32_t* assign,
                              void* hip_stream);

/* ---- several points per model frame ------------------------------------------
 *
 * The multiple-points model, variant 2 of Section 4 (Table 4): the model is
 * split into single-point models (second-order chains), each matched
 * independently by stm_match, and the matching distance is the mean of the
 * chains' energies.  The paper leaves the split to another publication; here
 * chain c (c < n_chains) holds the c-th most salient point of every model
 * frame with more than c points (saliency: the detector's confidence, higher
 * first, equal values in point order; NULL: point order), and chains of fewer
 * than 3 points are dropped.
 *
 * model: frames non-decreasing (several points may share a frame), n >= 3;
 * saliency [n] in the same memory as the other pointers (nullable).  Offsets
 * are those of the whole model (stm_offsets): tau puts its first frame at
 * scene frame tau, and chain c is matched at tau + (first frame of c - first
 * frame of the model).  Outputs as stm_match, per offset:
 *   energy32, energy64, energy_u64  the mean over the kept chains (+inf if one
 *                                   of them is infeasible);
 *   assign [n_tau][n]               each point's node in its chain's optimum,
 *                                   STM_UNCHAINED_NODE for points of no kept
 *                                   chain (-1 for the points of an infeasible
 *                                   chain);
 *   chains_used                     the number of kept chains (nullable).
 * Errors as stm_match, plus STM_EINVAL for decreasing model frames, a
 * non-finite saliency, n_chains outside 1..64, or no chain of 3 points. */
#define STM_UNCHAINED_NODE (-3)
STM_API int stm_match_chains(stm_ctx* ctx, const stm_points* model, const float* saliency, int32_t n_chains,
                             const stm_points* scene, const stm_params* params, int32_t tau_begin,
                             int32_t tau_end, float* energy32, double* energy64, double* energy_u64,
                             int32_t* assign, int32_t* chains_used, void* hip_stream);

/* ---- many matchings in one launch ------------------------------------------
 *
 * A plan matches every offset of every (model, scene) pair of a batch.  At
 * creation it validates all point sets once, builds the scenes' frame indices,
 * a pair table and a work list of (pair, offset) items sorted by decreasing
 * cost (the dense relaxation count sum_i K_{i-2} K_{i-1} K_i of the item), and
 * allocates its scratch.  A run queues, as one HIP graph captured at the first
 * run and replayed afterwards: the frame indices, the model angles, the unary
 * tables (every model against every scene of the plan), one persistent
 * recursion kernel whose workgroups pull items from the cost-sorted list with
 * an atomic counter (a second launch redoes the items with coincident points),
 * and the FP64 re-score.  This is the paper's suggestion of matching several
 * models and spreading several trellises over the GPU at once (Section 5),
 * for the under-used GPU it measures on small scene blocks (Section 3.9).
 * The largest scratch is the recursion's value tables: each resident
 * workgroup keeps those of up to 8 items ((M_max - 2) x K^2 floats each, K + 1
 * per side with dummies) and backtracks them together, as many items as fit
 * an eighth of the free device memory and at most 16 GiB in all (at least
 * one; STM_ENOMEM if one does not fit).
 *
 * Output rows: pair p owns the energy rows [row_offsets[p], row_offsets[p+1])
 * (one per offset, in offset order) and the assignment elements
 * [assign_offsets[p], assign_offsets[p+1]) (n_tau x M of its model).
 * With STM_DEVICE_PTRS the point sets are referenced, not copied: they must stay
 * allocated and unchanged while the plan lives; outputs of a run are device
 * pointers and the run is queued on `hip_stream` (NULL: the HIP default
 * stream).  Without it the plan keeps device copies and runs synchronously. */
typedef struct stm_plan stm_plan;

/* pairs: [n_pairs][2] (model index, scene index), host memory.  All models
 * and scenes share one descriptor dim.  Errors as for stm_match, plus
 * STM_EINVAL for a pair index out of range. */
STM_API int stm_plan_create(stm_ctx* ctx, const stm_points* models, int32_t n_models,
                    const stm_points* scenes, int32_t n_scenes, const int32_t* pairs,
                    int32_t n_pairs, const stm_params* params, stm_plan** out);

/* Frees the plan, its graph and its scratch (waits for the device).  NULL is a no-op. */
STM_API void stm_plan_destroy(stm_plan* plan);

/* Prefix offsets of the outputs, host memory, [n_pairs + 1] each (nullable),
 * and the totals (nullable). */
STM_API int stm_plan_rows(const stm_plan* plan, int64_t* row_offsets, int64_t* assign_offsets,
                  int64_t* n_rows, int64_t* n_assign);

/* One run over the whole batch.  energy32 [n_rows] and assign [n_assign] are
 * required; energy64 and energy_u64 [n_rows] are nullable.  Same meaning and
 * tie rules as stm_match. */
STM_API int stm_plan_run(stm_plan* plan, float* energy32, double* energy64, double* energy_u64,
                 int32_t* assign, void* hip_stream);

/* One run over the whole batch on caller-given candidate lists: the recursion
 * of stm_match_lists for every pair in one persistent launch (for instance
 * many models against the paper's streaming scene blocks, Table 2).  cand[q]
 * [n_tau_q][M_q][kc] and count[q] [n_tau_q][M_q] are device pointers for pair
 * q, n_tau_q its row count (stm_plan_rows); point j of offset tau has the
 * nodes cand[q][(tau * M_q + j) * kc + a], a < count, ascending.  kc <= the
 * plan's k_max.  The offsets matter only through the lists.  Outputs as
 * stm_plan_run.  Errors: STM_EINVAL for null arguments, kc outside
 * [1, k_max], or lists that fail the device check (count outside [0, kc], a
 * node outside the pair's scene, not ascending; one read-back). */
STM_API int stm_plan_run_lists(stm_plan* plan, const int32_t* const* cand, const int32_t* const* count,
                               int32_t kc, float* energy32, double* energy64, double* energy_u64,
                               int32_t* assign, void* hip_stream);

/* Launch shape of the persistent recursion kernel: waves per workgroup (4, 8
 * or 16) and workgroups per compute unit (1..3; 16-wave workgroups at most 2).
 * The plan keeps its batch and schedule requests (stm_plan_set_shape).
 * Results do not depend on the shape.  The shape is taken only once the
 * value-table scratch it needs is allocated: on STM_ENOMEM the plan keeps its
 * previous shape and scratch.  Graphs captured with the previous shape (plain
 * and pruned runs) are dropped and captured again at the next run. */
STM_API int stm_plan_set_tuning(stm_plan* plan, int32_t waves, int32_t wgs_per_cu);

/* The full launch shape, shape [4] host memory: waves, workgroups per CU (as
 * stm_plan_set_tuning), items per workgroup batch (1..8, whose backtracking
 * walks run together, one wave each; 0: the largest that fits an eighth of
 * the free device memory and 16 GiB) and the schedule variant of a step's
 * cells (0: dense chunks of one frame group, 1: packed chunks with a
 * predecessor range per lane, -1: packed when every scene has at most 3
 * points per frame).  Plans with STM_DUMMY always run the dense schedule,
 * and the dummy and packed variants run 8 waves per workgroup.  Same
 * allocation and graph rules as stm_plan_set_tuning; a given batch must fit
 * as it is (STM_ENOMEM otherwise, the plan unchanged). */
STM_API int stm_plan_set_shape(stm_plan* plan, const int32_t* shape);

/* The shape in effect, shape [4] host memory: waves the kernel runs,
 * workgroups per CU, batch, schedule variant (0 dense, 1 packed). */
STM_API int stm_plan_get_shape(const stm_plan* plan, int32_t* shape);

/* Picks the launch shape: looks up the key (GPU architecture, K bucket = k_max
 * rounded up to a power of two, M bucket = the largest model rounded up to a
 * multiple of 32, density flag, unary precision, dummies, whether the scenes
 * are sparse) in the cache file `cache_path` (nullable; one JSON object, one
 * entry per line); if absent, times every candidate shape (waves and
 * workgroups per CU in {(4,3), (8,2), (8,3), (16,1), (16,2)}, batch in 1, 2,
 * 4, 8 up to the waves, dense and packed schedules) on an evenly spaced
 * sample of at most `n_sample` items (<= 0: 24 per compute unit) of the work
 * list, keeps the fastest and writes it to the cache.  chosen [5] (nullable)
 * receives the shape in effect: waves, workgroups per CU, 1 if it came from
 * the cache, batch, schedule variant.  On an error the plan keeps its
 * previous shape. */
STM_API int stm_plan_autotune(stm_plan* plan, const char* cache_path, int32_t n_sample, int32_t* chosen);

/* One-shot batch: plan, run once, destroy.  row_offsets [n_pairs + 1]
 * (nullable, host) receives the energy row prefix. */
STM_API int stm_match_batch(stm_ctx* ctx, const stm_points* models, int32_t n_models,
                    const stm_points* scenes, int32_t n_scenes, const int32_t* pairs,
                    int32_t n_pairs, const stm_params* params, int64_t* row_offsets,
                    float* energy32, double* energy64, int32_t* assign, void* hip_stream);

/* ---- the trellis over a scene block (the paper's own problem) -------------
 *
 * Section 2.2 matches a model against a scene block without offsets or
 * windows: every model point may take any node of the block, the trellis is
 * pruned only by causality and closeness (Eq. 7, 8), and the loop bounds of
 * Section 3.4 follow from them: with nodes sorted by frame, the successors of
 * a node (frames in (t, t + T)) and its predecessors (frames in (t - T, t))
 * are contiguous node ranges.  Here the cells of every step are stored as that
 * band (cells (r, c) with c a successor of r, row after row), so the work is
 * the number of admissible (a_{i-2}, a_{i-1}, a_i) triples, not K^3 per step;
 * T <= 0 (no closeness limit) is the full upper-triangular trellis.  This is
 * the whole-video workload of the paper's Table 2 (M = 30 against 754 nodes)
 * and its T sweep (Fig. 7).
 *
 * A trellis object holds n_models models against the nodes [node_begin,
 * node_end) of one scene: the band, its tiles, the direction tables and the
 * value tables (sum over models of (M - 1) x cells floats).  A run solves
 * every model: the unary tables, the min-sum recursion (forward form of Eq.
 * 10-11) over all models (one launch for all steps, one workgroup per model,
 * when the band fits a workgroup's LDS; else one launch per step), the
 * optimum and backtracking
 * (Eq. 12-13) on the device, and the FP64 re-score (Eq. 1).
 * Outputs: energy32, energy64, energy_u64 [n_models] (nullable: the FP64 ones)
 * and assign [sum of model sizes] (model q's points from the sum of the sizes
 * before it), scene node ids (-1 rows when a model has no admissible
 * assignment in the block).  Ties: the first row-major minimum of the last
 * step, the lowest node inside each minimum.
 * params: lambda1..3 and T as for stm_match; window and k_max are not used;
 * flags: STM_DEVICE_PTRS (device inputs, referenced by the object and the
 * scene not copied; device outputs; runs queued on `hip_stream`),
 * STM_CLOSENESS_SPAN and STM_TRELLIS_STEPWISE; STM_UNARY_BF16, STM_K_DENSITY
 * and STM_DUMMY give
 * STM_EUNSUPPORTED.  Errors as stm_match, plus STM_EINVAL for an empty or
 * out-of-range node range, STM_ENOMEM when the value tables do not fit. */
typedef struct stm_trellis stm_trellis;
STM_API int stm_trellis_create(stm_ctx* ctx, const stm_points* models, int32_t n_models, const stm_points* scene,
                               int32_t node_begin, int32_t node_end, const stm_params* params, stm_trellis** out);
STM_API void stm_trellis_destroy(stm_trellis* trellis);
STM_API int stm_trellis_run(stm_trellis* trellis, float* energy32, double* energy64, double* energy_u64,
                            int32_t* assign, void* hip_stream);
/* info [10], host memory: cells per step, two-step direction pairs, tiles per
 * step launch, 1 if the degenerate variant runs (coincident points), then the
 * work of one run over all models: dense cells (M - 1) n^2, feasible cells
 * (M - 1) x band cells, dense relaxations (M - 2) n^3, feasible relaxations
 * (admissible triples), the sum of the model sizes, and 1 if every step runs
 * in one launch (one workgroup per model, the band in LDS), 0 if each step is
 * a launch of its own. */
STM_API int stm_trellis_info(const stm_trellis* trellis, int64_t* info);
/* One-shot: create, run once, destroy (waits for the run). */
STM_API int stm_match_trellis(stm_ctx* ctx, const stm_points* models, int32_t n_models, const stm_points* scene,
                              int32_t node_begin, int32_t node_end, const stm_params* params, float* energy32,
                              double* energy64, double* energy_u64, int32_t* assign, void* hip_stream);

/* ---- the steps of the path, exposed for checking ------------------------- */

/* Candidate lists of every model point at every offset in [tau_begin,
 * tau_end): cand [n_tau][M][k_max] scene node ids in ascending order (unused
 * slots -1) and count [n_tau][M].  Same rule and validation as stm_match. */
STM_API int stm_candidates(stm_ctx* ctx, const stm_points* model, const stm_points* scene,
                   const stm_params* params, int32_t tau_begin, int32_t tau_end,
                   int32_t* cand, int32_t* count, void* hip_stream);

/* Unary table U [M][S]: U[i][n] = ||f_i - g_n||_2 (Eq. 2, without lambda1),
 * the look-up table of Section 3.3; FP32, or split-precision BF16 with
 * STM_UNARY_BF16. */
STM_API int stm_unary(stm_ctx* ctx, const stm_points* model, const stm_points* scene,
              const stm_params* params, float* U, void* hip_stream);

/* Work of the recursion over [tau_begin, tau_end), written to counts[4]
 * (host memory, always): dense cells sum_i K_{i-1} K_i, feasible cells (the
 * pair is admissible), dense relaxations sum_i K_{i-2} K_{i-1} K_i and
 * feasible relaxations (both consecutive pairs admissible).  Synchronous. */
STM_API int stm_count_work(stm_ctx* ctx, const stm_points* model, const stm_points* scene,
                   const stm_params* params, int32_t tau_begin, int32_t tau_end,
                   int64_t* counts, void* hip_stream);

/* ---- learned candidate pruner ------------------------------------------------
 *
 * Not part of the paper.  A small network scores each candidate scene node n
 * of model point i at offset tau and keeps the best `topk`, so that the exact
 * recursion (Section 2.2) runs on candidate lists of at most topk nodes (a
 * subset of the windowed lists, kept in ascending node order).  Since every
 * pruned list is a subset of the exact one, a pruned optimum is an admissible
 * assignment of the exact problem and its energy is never below the exact
 * optimum.  Offsets left with no admissible assignment are solved again
 * exactly (the fallback).
 *
 * A group is the candidate list of one (tau, i); it has 64 slots (slot a holds
 * the a-th node of the windowed list, slots past the list are empty).  Row
 * input x = [dim f_i, dim g_n, phi (8)] (descriptors scaled by their
 * dimension):
 *   phi0  (t'_n - (tau + t_i - t_0)) / 4                frame offset
 *   phi1,2 ((p'_n - p'_{q_a}) - (p_i - p_a)) / 64        x, y against neighbour a
 *   phi3,4 the same against neighbour b
 *   phi5  log((|p'_n - p'_{q_a}| + 1) / (|p_i - p_a| + 1)) scale ratio
 *   phi6  U(i, n) - min over the group's candidates n' of U(i, n') (Eq. 2)
 *   phi7  i / (M - 1)
 * with a = i - 1, b = i + 1 (the one neighbour twice at the chain ends) and q_j
 * the candidate of neighbour j with the smallest U (lowest slot on ties; no
 * candidate: its terms are 0).  Network: h1 = relu(W1 x + b1), h2 =
 * relu(W2 h1 + b2), score = w3 . h2 + b3, 128 hidden units.  Parameters are
 * packed FP32 as [W1 (128 x (2 dim + 8), row-major), b1 (128), W2 (128 x 128),
 * b2 (128), w3 (128), b3 (1)].
 *
 * Training: FP32 forward and backward on the device; the loss of a group is
 * the softmax cross-entropy of its scores against the slot of the label node
 * (the exact optimum's a*_i), the batch loss the mean over groups; Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8).  Inference: BF16 inputs and weights on
 * MFMA with FP32 accumulation (the first layer split into a model part, a
 * scene part and the feature part, which stays FP32).
 *
 * Group lists `groups` are host arrays of G (tau, i) int32 pairs and `labels`
 * host arrays of G node ids, whatever params->flags says; model and scene
 * follow params->flags as in stm_match.  All pruner calls are synchronous.
 */
typedef struct stm_pruner stm_pruner;

/* Number of packed parameters for descriptor dimension dim (no GPU needed). */
STM_API int64_t stm_pruner_num_params(int32_t dim);

/* A pruner for descriptors of dimension dim on ctx's device, parameters zero;
 * set them with stm_pruner_set_params.  The pruner keeps ctx; destroy it
 * before ctx. */
STM_API int stm_pruner_create(stm_ctx* ctx, int32_t dim, stm_pruner** out);
STM_API void stm_pruner_destroy(stm_pruner* pruner);

/* Selection rule of the kept candidates (the ranking of stm_pruner_infer,
 * stm_match_pruned and stm_plan_run_pruned):
 *   STM_PRUNE_SCORE         the topk highest scores (lower slot first on ties);
 *   STM_PRUNE_FRAMES_FIRST  candidates in frames nearer the shifted model frame
 *                           first (|t'_n - (tau + t_i - t_0)|), the score rule
 *                           among candidates of one frame distance;
 *   STM_PRUNE_TIME_NEAREST  (default) the first topk candidates of the windowed
 *                           rule, i.e. nearer frames first, lower slot inside a
 *                           frame; the network is not evaluated by
 *                           stm_match_pruned / stm_plan_run_pruned, which then
 *                           equal stm_match at k_max = topk plus the exact
 *                           fallback.  On the synthetic workloads the learned
 *                           score reaches the 1% mean-gap target at the same
 *                           list size as this rule and costs the inference, so
 *                           this rule is the default; the two score rules stay
 *                           selectable for descriptors that carry signal. */
#define STM_PRUNE_SCORE 0
#define STM_PRUNE_FRAMES_FIRST 1
#define STM_PRUNE_TIME_NEAREST 2
STM_API int stm_pruner_set_rule(stm_pruner* pruner, int32_t rule);

/* Copies n = stm_pruner_num_params(dim) FP32 parameters from / to host
 * memory.  Setting them also resets the Adam moments and step count. */
STM_API int stm_pruner_set_params(stm_pruner* pruner, const float* theta, int64_t n);
STM_API int stm_pruner_get_params(stm_pruner* pruner, float* theta, int64_t n);

/* Parameters to / from a file: 8-byte tag "STMPRUN1", int32 dim, int32 0,
 * int64 n, then n little-endian FP32 values. */
STM_API int stm_pruner_save(stm_pruner* pruner, const char* path);
STM_API int stm_pruner_load(stm_pruner* pruner, const char* path);

/* The rows of G groups (host outputs): node [G][64] (-1 for empty slots), phi
 * [G][64][8] (zeros for empty slots), q [G][2] (q_a, q_b node ids or -1).
 * Every (tau, i) must be a valid offset and model point. */
STM_API int stm_pruner_features(stm_pruner* pruner, const stm_points* model, const stm_points* scene,
                                const stm_params* params, const int32_t* groups, int32_t G,
                                int32_t* node, float* phi, int32_t* q, void* hip_stream);

/* FP32 forward and backward over G groups: loss (mean over groups) into
 * *loss, and optionally the gradient [n_params] and the scores [G][64]
 * (-inf for empty slots), host memory.  STM_EINVAL if a label is not among
 * its group's candidates.  No parameter changes. */
STM_API int stm_pruner_gradient(stm_pruner* pruner, const stm_points* model, const stm_points* scene,
                                const stm_params* params, const int32_t* groups, const int32_t* labels,
                                int32_t G, float* loss, float* grad, float* scores, void* hip_stream);

/* stm_pruner_gradient followed by one Adam step with learning rate lr. */
STM_API int stm_pruner_train_step(stm_pruner* pruner, const stm_points* model, const stm_points* scene,
                                  const stm_params* params, const int32_t* groups, const int32_t* labels,
                                  int32_t G, float lr, float* loss, void* hip_stream);

/* BF16 inference over G groups: scores [G][64] (-inf for empty slots), and the
 * kept nodes cand [G][topk] (ascending; entries past count are unspecified)
 * with count [G] (min(topk, list length)).  Kept: the first topk in the order
 * of the pruner's selection rule.  1 <= topk <= 64.  Host outputs; any may be
 * NULL. */
STM_API int stm_pruner_infer(stm_pruner* pruner, const stm_points* model, const stm_points* scene,
                             const stm_params* params, const int32_t* groups, int32_t G, int32_t topk,
                             float* scores, int32_t* cand, int32_t* count, void* hip_stream);

/* stm_match on the pruned candidate lists: outputs as in stm_match (host or
 * device per params->flags), plus fell_back [tau_end - tau_begin] (same
 * memory kind, may be NULL): 1 where the pruned lists admitted no assignment
 * and the offset was solved exactly instead.  Synchronous (the fallback reads
 * the pruned energies back). */
STM_API int stm_match_pruned(stm_ctx* ctx, stm_pruner* pruner, const stm_points* model,
                             const stm_points* scene, const stm_params* params, int32_t topk,
                             int32_t tau_begin, int32_t tau_end, float* energy32, double* energy64,
                             double* energy_u64, int32_t* assign, int32_t* fell_back, void* hip_stream);

/* stm_match on caller-given candidate lists: cand [n_tau][M][kc] and count
 * [n_tau][M] (offset-major, then model point), each list ascending scene node
 * ids, count <= kc <= 64; the same memory kind as the other pointers (checked
 * on the device with STM_DEVICE_PTRS).  The recursion, tie rules and re-score
 * are those of stm_match; an offset whose lists admit no assignment gets +inf
 * and a -1 row (no fallback).  With the windowed lists this reproduces
 * stm_match. */
STM_API int stm_match_lists(stm_ctx* ctx, const stm_points* model, const stm_points* scene,
                            const stm_params* params, int32_t tau_begin, int32_t tau_end,
                            const int32_t* cand, const int32_t* count, int32_t kc, float* energy32,
                            double* energy64, double* energy_u64, int32_t* assign, void* hip_stream);

/* A plan run on pruned candidate lists (the batched form of stm_match_pruned):
 * the pruner's lists of every (pair, offset, point), one persistent launch of
 * the recursion on them, the items they left infeasible solved again exactly
 * in a second persistent launch, the FP64 re-score; all on the device, as one
 * captured graph (replayed while the outputs, pruner, topk and rule are the
 * same; the pruner's current parameters are read at each run).  Outputs as
 * stm_plan_run plus fell_back [rows] (nullable): 1 where the exact fallback
 * answered.  The pruner must belong to the plan's context and match its
 * descriptor dimension; plans with STM_UNARY_BF16 are not supported
 * (STM_EUNSUPPORTED).  Rows equal stm_match_pruned's for each pair. */
STM_API int stm_plan_run_pruned(stm_plan* plan, stm_pruner* pruner, int32_t topk, float* energy32,
                                double* energy64, double* energy_u64, int32_t* assign, int32_t* fell_back,
                                void* hip_stream);

/* ---- tuning ----------------------------------------------------------------- */

/* Waves per workgroup of the recursion kernel (one workgroup per matching):
 * 4, 8 or 16; 0 restores the default (8).  Results do not depend on it. */
STM_API int stm_set_dp_waves(stm_ctx* ctx, int waves);

/* ---- kernel timing for benchmarks -------------------------------------------- */

/* Enables (1) or disables (0) timing and resets the totals.  While enabled,
 * every launch of the recursion kernel (the fast variant) is bracketed by two
 * HIP events recorded on the stream it is launched on.  A plan run launches
 * its kernels directly on the plan's stream instead of replaying its graph,
 * with two events around its persistent recursion launches (the fast kernel
 * and the re-run of flagged degenerate matchings), and waits for the second
 * event to read the time. */
STM_API int stm_profile_enable(stm_ctx* ctx, int enable);

/* Waits for the recorded events and writes the summed kernel time in
 * milliseconds, the number of launches and the number of matchings they
 * processed.  Any output pointer may be NULL. */
STM_API int stm_profile_read(stm_ctx* ctx, double* dp_ms, int64_t* dp_launches, int64_t* dp_matchings);

#ifdef __cplusplus
}
#endif

#endif /* STM_H */
