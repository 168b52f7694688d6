// The exact min-sum recursion of the matching (Section 2.2), one workgroup per
// (model, scene, offset) matching, with the triplet cost fused into the
// minimisation; backtracking and the FP64 re-score of the result.
//
// The forward pass keeps only running minima: each step's cell values are
// written to device memory, and backtracking (Eq. 12) recomputes, along the
// optimal path only, the minimising predecessor of each step with the same
// arithmetic as the forward pass, so ties resolve to the lowest index.
//
// Forward form of Eq. 10-13.  With a_i the candidate index of model point i:
//   V_1(a_0, a_1) = l1 U_0 + l1 U_1 + Q_1(a_0, a_1)
//   V_i(a_{i-1}, a_i) = l1 U_i(a_i) + Q_i(a_{i-1}, a_i)
//       + min_{a_{i-2}} [ V_{i-1}(a_{i-2}, a_{i-1}) + l2 l3 D^g_i(a_{i-2}, a_{i-1}, a_i) ]
// where Q_i = l2 c_i Delta(i, i-1), +inf unless the pair is admissible (Eq. 7,
// 8), and c_i counts the triangles holding the pair (i, i-1) (2 inside the
// chain, 1 at its ends), so every D^t term of Eq. 4 is charged exactly once.
// The optimum is min V_{M-1}; the argmin a_{i-2} of each step on the optimal
// path is found again during backtracking.
//
// D^g from pairwise directions.  With phi(p -> q) the direction of q - p, the
// oriented angle at b of (a, b, c) is phi(b -> c) - phi(b -> a) mod 2 pi, and
// reversing a direction adds pi.  Hence, for the triangle (i, i-1, i-2) with
// model angles th_mid (at i-1) and th_end (at i):
//   delta_mid = wrap( -phi(z_{i-2} -> z_{i-1}) + [th_mid - pi + phi(z_{i-1} -> z_i)] )
//   delta_end = wrap( -phi(z_{i-2} -> z_i)     + [th_end + phi(z_{i-1} -> z_i)] )
// The first addend depends on (a_{i-2}, a_{i-1}) resp. (a_{i-2}, a_i) and is a
// table of K x K directions; the bracket depends only on the cell (a_{i-1},
// a_i).  So atan2 runs K^2 times per step and the K^3 relaxations need only
// adds, |wrap| via pi - |pi - |x|| (valid for |x| <= 2 pi), a square root,
// fused multiply-adds and a compare.
//
// Layout.  Candidates are sorted by frame, so the rows a_{i-1} of one frame
// share one contiguous range of admissible columns a_i and one contiguous
// range of admissible predecessors a_{i-2} (the paper's loop bounds of
// Section 3.4).  Each step builds a schedule of 64-cell chunks over the
// admissible cells only, frame group by frame group; a lane takes one cell of
// a chunk, the waves take chunks round-robin, and every lane of a chunk shares
// the predecessor loop bounds.  For explicit lists on sparse scenes (about
// one point per frame, lists spanning many frames) a group has only a few
// cells, so the packed variant numbers all cells of a step across the chunks
// and gives lane l of packed chunk p cell 64 p + l, each lane with its own
// predecessor range; the minima, and so every result, are the same.  Per step the LDS holds the previous V cells
// with their directions and the (a_{i-2}, a_i) direction table; the new cells
// stay in registers until every wave has finished reading, then replace the
// old ones.  Only admissible cells are ever read back.
//
// Degenerate triangles.  A zero-length side gives a scene angle of 0 in the
// definition, which the direction form does not reproduce.  The fast variant
// detects coincident points on pairs that can be admissible and flags the
// matching; the flagged matchings are recomputed by the variant that marks
// coincident directions as NaN and substitutes the model angle.
//
// Dummy assignments (Eq. 2).  With dummies every point also has the state
// epsilon at unary cost W^d; a Delta term needs both of its points matched,
// D^g all three, and the constraints bind matched consecutive points only.
// So a triangle holding epsilon adds no D^g, and the cells with epsilon follow
// from the step before without the K^3 loop:
//   V_i(r, c)     = l1 U_i(c) + Q_i(r, c) + min(V_{i-1}(eps, r), min_k [...])
//   V_i(r, eps)   = l1 W^d + min(V_{i-1}(eps, r), min_{k admissible} V_{i-1}(k, r))
//   V_i(eps, c)   = l1 U_i(c) + m_{i-1},   V_i(eps, eps) = l1 W^d + m_{i-1}
// with m_{i-1} = min(V_{i-1}(eps, eps), min_k V_{i-1}(k, eps)).  Each step keeps
// these as two K-vectors and a scalar beside the K x K cells; epsilon is index
// 64 in the final argmin and in backtracking (after every candidate, so ties
// go to candidates) and index K in the value tables, whose rows then have
// K + 1 entries.
//
// Alternative readings.  Unsigned angles (a template variant): the terms
// compare magnitudes, the scene's angles at z_{i-1} and z_i being wrap(pi +
// anew - A) and wrap(anew - C) of the same stored directions (dp_math.h).
// Node-order causality (a run-time switch of the schedule): consecutive points
// take increasing node ids, so within a frame every row has its own columns
// (the nodes above it) and its own predecessors (the nodes below it); every row
// is then a group of its own, its ranges counted from the windowed lists' node
// ranges, and the chunk loop is unchanged.
#include <math.h>

#include "dp_math.h"
#include "stm_internal.h"

namespace stm {
namespace {

constexpr int kMaxList = 64;  // longest candidate list = wavefront lanes
constexpr int kEps = kMaxList;  // index of the dummy state epsilon
constexpr int32_t kDummyNode = -2;  // epsilon in assignments

// A chunk of the cells of one step: the admissible cells (a_{i-1}, a_i) of the
// rows r0.. r0+nr-1 of one frame group, flattened row-major over their common
// column range [clo, clo + nc); the chunk covers flat cells [e0, e0 + 64).  All
// rows of the group share the predecessor range [lo, hi).
struct Chunk {
  int r0, clo, nc, e0, lo, hi, ncell;
};

__device__ __forceinline__ uint2 pack_chunk(int r0, int clo, int nc, int e0, int lo, int hi, int ncell) {
  return make_uint2(static_cast<uint32_t>(r0) | (static_cast<uint32_t>(clo) << 6) |
                        (static_cast<uint32_t>(nc) << 12) | (static_cast<uint32_t>(e0) << 19),
                    static_cast<uint32_t>(lo) | (static_cast<uint32_t>(hi) << 7) |
                        (static_cast<uint32_t>(ncell) << 14));
}

// Decodes a descriptor read from LDS; the fields are wave-uniform, so they are
// moved to scalar registers and the loops over them stay scalar.
__device__ __forceinline__ Chunk unpack_chunk(uint2 d) {
  const uint32_t x = __builtin_amdgcn_readfirstlane(d.x), y = __builtin_amdgcn_readfirstlane(d.y);
  Chunk c;
  c.r0 = x & 63;
  c.clo = (x >> 6) & 63;
  c.nc = (x >> 12) & 127;
  c.e0 = x >> 19;
  c.lo = y & 127;
  c.hi = (y >> 7) & 127;
  c.ncell = y >> 14;
  return c;
}

// Number of entries < x in the ascending list a[0..n).
// Lists hold at most 64 entries, so seven probes at fixed strides suffice; the
// probes do not branch on the data, and independent searches interleave their
// reads.
__device__ __forceinline__ int count_lt(const int32_t* a, int n, int x) {
  if (n <= 0) return 0;
  int pos = 0;
#pragma unroll
  for (int step = 64; step > 0; step >>= 1) {
    const int probe = pos + step;
    const int32_t v = a[(probe <= n ? probe : n) - 1];
    if (probe <= n && v < x) pos = probe;
  }
  return pos;
}

// Cell of lane `lane` in chunk c: row r and column a; false past the last cell.
__device__ __forceinline__ bool chunk_cell(const Chunk& c, int lane, int& r, int& a) {
  const int e = c.e0 + lane;
  // e < 4096 and nc <= 64: (e + 1/2) / nc stays >= 1/128 away from an integer,
  // far above the float rounding, so the truncation is the exact quotient.
  const int q = static_cast<int>((static_cast<float>(e) + 0.5f) * __builtin_amdgcn_rcpf(static_cast<float>(c.nc)));
  r = c.r0 + q;
  a = c.clo + (e - q * c.nc);
  return e < c.ncell;
}

// Builds the chunk schedule of one step, run by one wave (lane = row).  Rows
// are the candidates of point i-1 (frames trow, ascending), columns those of
// point i (tcol), predecessors those of point i-2 (tprev, or none for the
// first pair).  The rows of one frame f share the admissible columns (frames in
// (f, f + T)) and predecessors (frames in (f - T, f)).  Each group gives
// ceil(rows * columns / 64) <= rows chunks, so a step has at most K chunks.
// With pstart (packed variant): pstart[j] = number of the first cell of chunk
// j when the step's cells are numbered chunk after chunk, pstart[n] = the
// step's cell count, also stored in *ptot.
__device__ void build_schedule(const int32_t* trow, int nrow, const int32_t* tcol, int ncol,
                               const int32_t* tprev, int nprev, int T, uint2* out, int32_t* nout,
                               int lane, int16_t* pstart, int32_t* ptot, const CandRange* ring, int sr, int sc,
                               int sp) {
  const int f = lane < nrow ? trow[lane] : 0;
  // node-order causality (ring: the windowed node ranges of the candidate
  // ring in LDS, sr, sc, sp: the rows', columns' and predecessors' slots;
  // null for frame order): every row is a group of its own, its columns the
  // nodes above its own within T frames, its predecessors the nodes below it
  // within T frames
  const bool node = ring != nullptr;
  const bool start = lane < nrow && (node || lane == 0 || trow[lane - 1] != f);
  const unsigned long long starts = __ballot(start);
  int nchunk = 0, nr = 0, nc = 0, clo = 0, chi = 0, lo = 0, hi = 0;
  if (node) {
    if (start) {
      const int nd = cand_node(ring[sr], lane);
      clo = range_count_le(ring[sc], nd);
      chi = T > 0 ? count_lt(tcol, ncol, f > 0x7fffffff - T ? 0x7fffffff : f + T) : ncol;
      if (tprev) {
        hi = range_count_lt(ring[sp], nd);
        lo = T > 0 ? count_lt(tprev, nprev, f - T + 1) : 0;
      }
    }
  } else if (__popcll(starts) <= 16) {
    // few frame groups: each lane holds one column and one predecessor frame,
    // and every count is a ballot, one group after the other
    const int32_t tc = lane < ncol ? tcol[lane] : 0x7fffffff;  // frames are < 0x7fffffff
    const int32_t tp = tprev && lane < nprev ? tprev[lane] : 0x7fffffff;
    unsigned long long rem = starts;
    while (rem) {
      const int g = __ffsll(static_cast<long long>(rem)) - 1;
      rem &= rem - 1;
      const int fg = __builtin_amdgcn_readlane(f, g);
      const int c0 = __popcll(__ballot(tc < fg + 1));
      const int c1 = T > 0 ? __popcll(__ballot(tc < (fg > 0x7fffffff - T ? 0x7fffffff : fg + T))) : ncol;
      const int p1 = __popcll(__ballot(tp < fg));
      const int p0 = T > 0 ? __popcll(__ballot(tp < fg - T + 1)) : 0;
      if (lane == g) {
        clo = c0;
        chi = c1;
        hi = p1;
        lo = p0;
      }
    }
  } else if (start) {
    // many groups (sparse scenes): binary searches, one group per lane
    clo = count_lt(tcol, ncol, f + 1);
    chi = T > 0 ? count_lt(tcol, ncol, f > 0x7fffffff - T ? 0x7fffffff : f + T) : ncol;
    if (tprev) {
      hi = count_lt(tprev, nprev, f);
      lo = T > 0 ? count_lt(tprev, nprev, f - T + 1) : 0;
    }
  }
  if (start) {
    const unsigned long long later = starts & ~((2ull << lane) - 1ull);
    const int next = later ? __ffsll(static_cast<long long>(later)) - 1 : nrow;
    nr = next - lane;
    nc = chi > clo ? chi - clo : 0;
    nchunk = (nr * nc + 63) >> 6;
  }
  int incl = nchunk;
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off);
    if (lane >= off) incl += v;
  }
  if (start)
    for (int c = 0; c < nchunk; ++c) out[incl - nchunk + c] = pack_chunk(lane, clo, nc, c * 64, lo, hi, nr * nc);
  const int total = __shfl(incl, 63);
  if (lane == 0) *nout = total;
  if (pstart) {
    int cells = nr * nc;  // inclusive scan of the groups' cell counts
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(cells, off);
      if (lane >= off) cells += v;
    }
    if (start)
      for (int c = 0; c < nchunk; ++c) pstart[incl - nchunk + c] = static_cast<int16_t>(cells - nr * nc + c * 64);
    const int ncells = __shfl(cells, 63);
    if (lane == 0) {
      pstart[total] = static_cast<int16_t>(ncells);
      *ptot = ncells;
    }
  }
}

// Cell 64 p + lane of a packed schedule: its chunk j (the last with pstart[j]
// <= the number), row r, column a and predecessor range [lo, hi).  A number
// past the step's cells decodes cell 0 (in-range reads) and returns false.
__device__ __forceinline__ bool packed_cell(const uint2* sched, const int16_t* pstart, int n_chunks, int n_cells,
                                            int num, int& r, int& a, int& lo, int& hi) {
  const bool valid = num < n_cells;
  const int e_all = valid ? num : 0;
  int j = 0, j1 = n_chunks;  // pstart[j] <= e_all < pstart[j1]
  while (j1 - j > 1) {
    const int mid = (j + j1) >> 1;
    if (pstart[mid] <= e_all) j = mid; else j1 = mid;
  }
  const uint2 d = sched[j];
  const int r0 = d.x & 63, clo = (d.x >> 6) & 63, nc = (d.x >> 12) & 127, e0 = d.x >> 19;
  lo = d.y & 127;
  hi = (d.y >> 7) & 127;
  const int e = e0 + (e_all - pstart[j]);
  const int q = static_cast<int>((static_cast<float>(e) + 0.5f) * __builtin_amdgcn_rcpf(static_cast<float>(nc)));
  r = r0 + q;
  a = clo + (e - q * nc);
  return valid;
}

// Per-step vectors of the dummy state, double-buffered by step parity:
// de[b][c] = V(eps, c), df[b][r] = V(r, eps), dg[b] = V(eps, eps).
template <int KL, bool DUMMY>
struct DummyShared {};
template <int KL>
struct DummyShared<KL, true> {
  float de[2][KL];
  float df[2][KL];
  float dg[2];
};

// Packed schedules: first cell number of every chunk, and the step's cell count.
template <int KL, bool PACKED>
struct PackedShared {};
template <int KL>
struct PackedShared<KL, true> {
  int16_t pstart[2][KL + 1];
  int32_t ptot[2];
};

template <int NW, int KL, bool DUMMY = false, bool PACKED = false>
struct DPShared : DummyShared<KL, DUMMY>, PackedShared<KL, PACKED> {
  float2 va[KL * KL];   // [a_{i-2}][a_{i-1}]: (V_{i-1}, -phi(z_{i-2} -> z_{i-1}))
  float ct[KL * KL];    // [a_{i-2}][a_i]: -phi(z_{i-2} -> z_i)
  float2 cxy[4][KL];    // candidate ring: coordinates,
  int32_t ctt[4][KL];   //   frames,
  float cu[4][KL];      //   l1 * U
  uint2 sched[2][KL];   // chunk schedules of the current and the previous step
  int32_t nch[2];
  int32_t ck[4];        //   list lengths
  CandRange crange[4];  //   the windowed lists' node ranges (node-order causality)
  int32_t flag;         // coincident points seen (fast variant)
  float red_v[NW];
  int32_t red_i[NW];
  float res_v;
  int32_t res_i;
};

// One matching: a model against a scene at offset tau.
struct MatchView {
  ModelView m;
  SceneView s;
  SearchParams sp;
  const float* U;       // unary table: row j = model point j, row stride us
  long long us;
  const float2* theta;  // model angles of the triangle ending at each point
  float lambda1, lambda2, w;
  float cw;             // l1 * W^d, the unary cost of the dummy
  int vs;               // value-table row length: K, or K + 1 with dummies
  int tau;
  // explicit candidate lists of this matching (null: the windowed rule):
  // point j's nodes are cand[j * cstride + a], a < ccount[j], ascending
  const int32_t* cand;
  const int32_t* ccount;
  int cstride;
};

// Candidate list of point j of a matching: explicit, or the windowed rule.
struct Cands {
  CandRange r;
  const int32_t* list;
  int n;
  __device__ __forceinline__ int count() const { return list ? n : r.k1 + r.k2; }
  __device__ __forceinline__ int node(int a) const { return list ? ro(list + a) : cand_node(r, a); }
};

__device__ __forceinline__ Cands cands_of(const MatchView& a, int j) {
  Cands c;
  if (a.cand) {
    c.list = a.cand + (long long)j * a.cstride;
    c.n = ro(a.ccount + j);
    c.r = CandRange{0, 0, 0, 0};
  } else {
    c.list = nullptr;
    c.n = 0;
    c.r = point_candidates(a.s.fstart, a.s.F, a.tau + ro(a.m.t + j) - ro(a.m.t), a.sp);
  }
  return c;
}

// Value table of step i (cells V_i(a_{i-1}, a_i), i = 1..M-2) inside the
// matching's scratch vt [M-2][vs][vs], stored by column: V_i(r, c) at c * vs +
// r, so that backtracking reads the values of one column (every predecessor of
// the chosen cell) contiguously (with dummies, index K holds the epsilon state
// on either side).
__device__ __forceinline__ float* vtable(float* vt, const MatchView& a, int i) {
  return vt + (long long)(i - 1) * a.vs * a.vs;
}
__device__ __forceinline__ const float* vtable(const float* vt, const MatchView& a, int i) {
  return vt + (long long)(i - 1) * a.vs * a.vs;
}

struct DPResult {
  float v;   // optimum (+inf if infeasible)
  int idx;   // r * KL + c of the first minimising final pair (a_{M-2}, a_{M-1});
             // with dummies r * (KL + 1) + c, epsilon = KL
  int flag;  // coincident points seen (fast variant)
};

// Forward pass of one matching by the whole workgroup (NW waves): writes the
// value tables of steps 1..M-2 to vtm and returns the optimum to every thread.
template <int NW, bool DEGEN, int KL, bool DUMMY = false, bool PACKED = false, bool UNS = false>
__device__ DPResult dp_forward(DPShared<NW, KL, DUMMY, PACKED>& sh, const MatchView& a, float* vtm) {
  static_assert(KL == 16 || KL == 32 || KL == 64, "list capacity");
  static_assert(!DUMMY || KL == kMaxList, "dummies use the 64-slot layout");
  static_assert(!PACKED || (KL == kMaxList && !DUMMY), "packed schedules: 64-slot layout, no dummies");
  constexpr int RPW = KL / NW;  // chunk slots per wave (a step has <= KL chunks)
  const int tau = a.tau;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int M = a.m.M;
  const int T = pair_limit(a.sp);   // consecutive points
  const int TS = span_limit(a.sp);  // first and last points of a triangle (span reading)
  const int Kc = a.sp.K;
  const int VS = a.vs;
  const int tm0 = ro(a.m.t);
  const float INF = __builtin_inff();
  constexpr int kBuilder = NW - 1;  // wave that builds the schedules

  // chunk slots of schedule b, and the cell of this lane in slot ch (packed
  // schedules: cell number 64 ch + lane; lo/hi only set there)
  auto n_slots = [&](int b) {
    if constexpr (PACKED) return (sh.ptot[b] + 63) >> 6;
    else return sh.nch[b];
  };
  auto slot_cell = [&](int b, int ch, int& r, int& col) {
    if constexpr (PACKED) {
      int lo, hi;
      return packed_cell(sh.sched[b], sh.pstart[b], sh.nch[b], sh.ptot[b], ch * 64 + lane, r, col, lo, hi);
    } else {
      return chunk_cell(unpack_chunk(sh.sched[b][ch]), lane, r, col);
    }
  };
  // the same, with an in-range cell for lanes past the last one (their reads)
  auto slot_cell_safe = [&](int b, int ch, int& r, int& col) {
    if constexpr (PACKED) {
      return slot_cell(b, ch, r, col);
    } else {
      const Chunk c = unpack_chunk(sh.sched[b][ch]);
      const bool valid = chunk_cell(c, lane, r, col);
      if (!valid) { r = c.r0; col = c.clo; }  // in-range reads; results unused
      return valid;
    }
  };
  // sr, sc, sp: ring slots of the rows', columns' and predecessors' lists
  auto schedule = [&](int sr, int sc, int spv, int b) {
    const int32_t* trow = sh.ctt[sr];
    const int32_t* tcol = sh.ctt[sc];
    const int32_t* tprev = spv >= 0 ? sh.ctt[spv] : nullptr;
    const int nrow = sh.ck[sr], ncol = sh.ck[sc], nprev = spv >= 0 ? sh.ck[spv] : 0;
    const CandRange* ring = a.sp.node ? sh.crange : nullptr;
    if constexpr (PACKED)
      build_schedule(trow, nrow, tcol, ncol, tprev, nprev, T, sh.sched[b], &sh.nch[b], lane, sh.pstart[b],
                     &sh.ptot[b], ring, sr, sc, spv);
    else
      build_schedule(trow, nrow, tcol, ncol, tprev, nprev, T, sh.sched[b], &sh.nch[b], lane, nullptr, nullptr,
                     ring, sr, sc, spv);
  };

  // The candidates of list j, read by wave 0 in two halves: fetch_slot issues
  // the reads into registers (its frame boundaries, then its nodes' position,
  // frame and unary cost) a step before commit_slot stores them into ring slot
  // j & 3, so that their latency overlaps the recursion of the step between.
  struct SlotRegs {
    Cands c;
    float2 xy;
    int32_t t;
    float u;
  };
  auto fetch_slot = [&](int j) {
    SlotRegs f;
    if (wv == 0) {
      f.c = cands_of(a, j);
      if (lane < f.c.count()) {
        const int n = f.c.node(lane);
        f.xy = ro(a.s.xy + n);
        f.t = ro(a.s.t + n);
        f.u = ro(a.U + (long long)j * a.us + n);
      }
    }
    return f;
  };
  auto commit_slot = [&](int j, const SlotRegs& f) {
    if (wv == 0) {
      const int k = f.c.count();
      const int sl = j & 3;
      if (lane < k) {
        sh.cxy[sl][lane] = f.xy;
        sh.ctt[sl][lane] = f.t;
        sh.cu[sl][lane] = a.lambda1 * f.u;
      }
      if (lane == 0) {
        sh.ck[sl] = k;
        sh.crange[sl] = f.c.r;
      }
    }
  };
  auto load_slot = [&](int j) { commit_slot(j, fetch_slot(j)); };

  if (threadIdx.x == 0) sh.flag = 0;
  load_slot(0);
  load_slot(1);
  load_slot(2);
  __syncthreads();
  if (wv == kBuilder) schedule(0, 1, -1, 1);
  __syncthreads();
  SlotRegs next;  // list i + 1 in flight during step i - 1's recursion and step i's phase 1
  if (3 < M) next = fetch_slot(3);

  float vr[RPW], ar[RPW];
  int pi[RPW];  // LDS index (row * KL + column) of each slot's cell, -1: none
#pragma unroll
  for (int s = 0; s < RPW; ++s) { vr[s] = INF; ar[s] = 0.f; pi[s] = -1; }

  // ---- the first pair (points 0, 1) ------------------------------------------
  {
    const int dtm = ro(a.m.t + 1) - ro(a.m.t);
    const int nch = n_slots(1);
    float* vt = vtable(vtm, a, 1);
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int ch = wv + NW * s;
      if (ch < nch) {
        int r, col;
        const bool valid = slot_cell_safe(1, ch, r, col);
        const int tr = sh.ctt[0][r], tp = sh.ctt[1][col];
        const float2 xr = sh.cxy[0][r], xa = sh.cxy[1][col];
        const bool same = xa.x == xr.x && xa.y == xr.y;
        if (!DEGEN && same && valid) sh.flag = 1;
        const float q = a.lambda2 * fabsf(static_cast<float>(dtm - (tp - tr)));
        vr[s] = (sh.cu[0][r] + sh.cu[1][col]) + q;
        ar[s] = neg_dir<DEGEN>(xr, xa);
        if (valid) vt[col * VS + r] = vr[s];
        pi[s] = valid ? r * KL + col : -1;
      }
    }
    if constexpr (DUMMY) {
      if (wv == 0) {
        const float cw = a.cw;
        if (lane < sh.ck[1]) {
          const float e = cw + sh.cu[1][lane];
          sh.de[1][lane] = e;
          vt[lane * VS + Kc] = e;
        }
        if (lane < sh.ck[0]) {
          const float f = sh.cu[0][lane] + cw;
          sh.df[1][lane] = f;
          vt[Kc * VS + lane] = f;
        }
        if (lane == 0) {
          sh.dg[1] = cw + cw;
          vt[Kc * VS + Kc] = cw + cw;
        }
      }
    }
  }

  // ---- points 2 .. M-1 -----------------------------------------------------------
  for (int i = 2; i < M; ++i) {
    const int s2 = (i - 2) & 3, s1 = (i - 1) & 3, s0 = i & 3;
    const int Kq = sh.ck[s2], Kp = sh.ck[s1], Kn = sh.ck[s0];
    const int cur = i & 1, prv = cur ^ 1;

    // Phase 1: publish the previous step's cells, build this step's schedule and
    // (a_{i-2}, a_i) direction table, prefetch the next candidate list.
    {
      const int nprev = n_slots(prv);
#pragma unroll
      for (int s = 0; s < RPW; ++s) {
        const int ch = wv + NW * s;
        if (ch < nprev && pi[s] >= 0) sh.va[pi[s]] = make_float2(vr[s], ar[s]);
      }
    }
    if (wv == kBuilder) schedule(s1, s0, s2, cur);
    {
      // the (a_{i-2}, a_i) direction of row k, column c; a pair is used only
      // if some z_{i-1} fits strictly between its frames and within T of
      // both: 2 <= t_i - t_{i-2} <= 2T - 2 (node order: between its nodes,
      // so the frames may be equal).  Under the span reading a pair whose
      // frames are TS or more apart gets +inf, which takes its terms out of
      // every minimum.
      const int gap_min = a.sp.node ? 0 : 2;
      const auto direction = [&](int k, int c, int tc, float2 pc) {
        const int gap = tc - sh.ctt[s2][k];
        if (gap >= gap_min && (T <= 0 || gap <= 2 * T - 2)) {
          if (TS > 0 && gap >= TS) {
            sh.ct[k * KL + c] = INF;
            return;
          }
          const float2 pk = sh.cxy[s2][k];
          if (!DEGEN && pk.x == pc.x && pk.y == pc.y) sh.flag = 1;
          sh.ct[k * KL + c] = neg_dir<DEGEN>(pk, pc);
        }
      };
      if (KL == kMaxList && !PACKED && Kn <= 48) {
        // short lists (density caps): the Kq x Kn pairs spread over the
        // threads (with 8 or more waves, all but the builder's, which has the
        // schedule to build: 2% faster than sharing the table with it);
        // p < 4096 and Kn <= 64 keep (p + 1/2) / Kn at least 1/128 from an
        // integer, so the truncated float quotient is exact
        const float rn = __builtin_amdgcn_rcpf(static_cast<float>(Kn));
        const int stride = NW >= 8 ? (NW - 1) * 64 : NW * 64;
        for (int p = (NW >= 8 && wv == kBuilder) ? Kq * Kn : threadIdx.x; p < Kq * Kn; p += stride) {
          const int k = static_cast<int>((static_cast<float>(p) + 0.5f) * rn);
          const int c = p - k * Kn;
          direction(k, c, sh.ctt[s0][c], sh.cxy[s0][c]);
        }
      } else if (KL == kMaxList && NW >= 8) {
        // each wave but the schedule's builder keeps one column c per lane and
        // walks the rows k
        if (wv != kBuilder && lane < Kn) {
          const int tc = sh.ctt[s0][lane];
          const float2 pc = sh.cxy[s0][lane];
          for (int k = wv; k < Kq; k += NW - 1) direction(k, lane, tc, pc);
        }
      } else {
        // each thread keeps one column c and walks the rows k
        constexpr int kRowsPerPass = NW * 64 / KL;
        const int c = threadIdx.x & (KL - 1);
        if (c < Kn) {
          const int tc = sh.ctt[s0][c];
          const float2 pc = sh.cxy[s0][c];
          for (int k = threadIdx.x / KL; k < Kq; k += kRowsPerPass) direction(k, c, tc, pc);
        }
      }
    }
    if (i + 1 < M) commit_slot(i + 1, next);
    __syncthreads();
    if (i + 2 < M) next = fetch_slot(i + 2);

    // Phase 2: the minima over a_{i-2} of every admissible cell, chunk by chunk.
    const float2 th = ro(a.theta + i);
    const int dtm = ro(a.m.t + i) - ro(a.m.t + (i - 1));
    const float qw = a.lambda2 * (i <= M - 2 ? 2.f : 1.f);
    float* vt = i <= M - 2 ? vtable(vtm, a, i) : nullptr;
    const float w = a.w;
    const int nch = n_slots(cur);
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int ch = wv + NW * s;
      float vnew = INF, anew = 0.f;
      if constexpr (PACKED) {
        if (ch < nch) {
          // lane-own cell and predecessor range; the wave runs to the longest
          // range, a lane past its own repeats its last predecessor, masked
          int r, col, lo, hi;
          const bool valid = packed_cell(sh.sched[cur], sh.pstart[cur], sh.nch[cur], sh.ptot[cur], ch * 64 + lane, r,
                                         col, lo, hi);
          const int tr = sh.ctt[s1][r], tp = sh.ctt[s0][col];
          const float2 xr = sh.cxy[s1][r], xa = sh.cxy[s0][col];
          const bool same = xa.x == xr.x && xa.y == xr.y;
          if (!DEGEN && same && valid) sh.flag = 1;
          anew = neg_dir<DEGEN>(xr, xa);
          float bm, be;
          cell_consts<UNS>(th, anew, bm, be);
          const float2* vcol = sh.va + r;
          const float* ccol = sh.ct + col;
          const int len = hi - lo;
          int longest = len;
          for (int off = 32; off > 0; off >>= 1) longest = max(longest, __shfl_xor(longest, off));
          longest = __builtin_amdgcn_readfirstlane(longest);
          const int last = max(len - 1, 0);
          float best = INF;
          for (int j = 0; j < longest; ++j) {
            const int kk = min(lo + min(j, last), KL - 1);
            const float2 v0 = vcol[kk * KL];
            const float t0 = relax<DEGEN, UNS>(v0.x, v0.y, ccol[kk * KL], bm, be, th, same, w);
            best = fminf(best, j < len ? t0 : INF);
          }
          const float q = qw * fabsf(static_cast<float>(dtm - (tp - tr)));
          vnew = (sh.cu[s0][col] + q) + best;
          if (valid && vt) vt[col * VS + r] = vnew;
          pi[s] = valid ? r * KL + col : -1;
          vr[s] = vnew;
          ar[s] = anew;
        }
      } else {
        if (ch < nch) {
          const Chunk c = unpack_chunk(sh.sched[cur][ch]);
          int r, col;
          const bool valid = chunk_cell(c, lane, r, col);
          if (!valid) { r = c.r0; col = c.clo; }  // in-range reads; results unused
          const int tr = sh.ctt[s1][r], tp = sh.ctt[s0][col];
          const float2 xr = sh.cxy[s1][r], xa = sh.cxy[s0][col];
          const bool same = xa.x == xr.x && xa.y == xr.y;
          if (!DEGEN && same && valid) sh.flag = 1;
          anew = neg_dir<DEGEN>(xr, xa);
          float bm, be;
          cell_consts<UNS>(th, anew, bm, be);
          const float2* vcol = sh.va + r;
          const float* ccol = sh.ct + col;
          float best = INF;
          if constexpr (DUMMY) best = sh.de[prv][r];  // predecessor epsilon: no D^g
          // eight predecessors per trip (one address step per table; the wide
          // layouts only, where few chunk slots leave registers for it), then
          // four, then one at a time
          int k = c.lo;
          constexpr bool kEight = NW >= 8 && KL == kMaxList;
          for (; kEight && k + 7 < c.hi; k += 8) {
            const float2 v0 = vcol[k * KL], v1 = vcol[(k + 1) * KL];
            const float2 v2 = vcol[(k + 2) * KL], v3 = vcol[(k + 3) * KL];
            const float t0 = relax<DEGEN, UNS>(v0.x, v0.y, ccol[k * KL], bm, be, th, same, w);
            const float t1 = relax<DEGEN, UNS>(v1.x, v1.y, ccol[(k + 1) * KL], bm, be, th, same, w);
            const float t2 = relax<DEGEN, UNS>(v2.x, v2.y, ccol[(k + 2) * KL], bm, be, th, same, w);
            const float t3 = relax<DEGEN, UNS>(v3.x, v3.y, ccol[(k + 3) * KL], bm, be, th, same, w);
            best = fminf(fminf(best, fminf(fminf(t0, t1), t2)), t3);
            const float2 v4 = vcol[(k + 4) * KL], v5 = vcol[(k + 5) * KL];
            const float2 v6 = vcol[(k + 6) * KL], v7 = vcol[(k + 7) * KL];
            const float t4 = relax<DEGEN, UNS>(v4.x, v4.y, ccol[(k + 4) * KL], bm, be, th, same, w);
            const float t5 = relax<DEGEN, UNS>(v5.x, v5.y, ccol[(k + 5) * KL], bm, be, th, same, w);
            const float t6 = relax<DEGEN, UNS>(v6.x, v6.y, ccol[(k + 6) * KL], bm, be, th, same, w);
            const float t7 = relax<DEGEN, UNS>(v7.x, v7.y, ccol[(k + 7) * KL], bm, be, th, same, w);
            best = fminf(fminf(best, fminf(fminf(t4, t5), t6)), t7);
          }
          if (k + 3 < c.hi) {
            const float2 v0 = vcol[k * KL], v1 = vcol[(k + 1) * KL];
            const float2 v2 = vcol[(k + 2) * KL], v3 = vcol[(k + 3) * KL];
            const float t0 = relax<DEGEN, UNS>(v0.x, v0.y, ccol[k * KL], bm, be, th, same, w);
            const float t1 = relax<DEGEN, UNS>(v1.x, v1.y, ccol[(k + 1) * KL], bm, be, th, same, w);
            const float t2 = relax<DEGEN, UNS>(v2.x, v2.y, ccol[(k + 2) * KL], bm, be, th, same, w);
            const float t3 = relax<DEGEN, UNS>(v3.x, v3.y, ccol[(k + 3) * KL], bm, be, th, same, w);
            best = fminf(fminf(best, fminf(fminf(t0, t1), t2)), t3);
            k += 4;
          }
          for (; k < c.hi; ++k) {
            const float2 v0 = vcol[k * KL];
            best = fminf(best, relax<DEGEN, UNS>(v0.x, v0.y, ccol[k * KL], bm, be, th, same, w));
          }
          const float q = qw * fabsf(static_cast<float>(dtm - (tp - tr)));
          vnew = (sh.cu[s0][col] + q) + best;
          if (valid && vt) vt[col * VS + r] = vnew;
          pi[s] = valid ? r * KL + col : -1;
          vr[s] = vnew;
          ar[s] = anew;
        }
      }
      // a slot past the step's chunk count keeps stale registers: every reader
      // (publication, the final minimum) checks the slot against that count
    }
    if constexpr (DUMMY) {
      // the epsilon cells of step i, from step i-1's cells and epsilon cells
      const float cw = a.cw;
      // V_i(r, eps): over the admissible predecessors of row r, no D^g; eight
      // lanes per row split its predecessors, the rows spread over the waves
      for (int r0 = wv * 8; r0 < Kp; r0 += NW * 8) {
        const int r = r0 + (lane >> 3), sub = lane & 7;
        float m = INF;
        if (r < Kp) {
          const int f = sh.ctt[s1][r];
          const int hi = count_lt(sh.ctt[s2], Kq, f);
          const int lo = T > 0 ? count_lt(sh.ctt[s2], Kq, f - T + 1) : 0;
          for (int k = lo + sub; k < hi; k += 8) m = fminf(m, sh.va[k * KL + r].x);
        }
        m = fminf(m, __shfl_xor(m, 1));
        m = fminf(m, __shfl_xor(m, 2));
        m = fminf(m, __shfl_xor(m, 4));
        if (r < Kp && sub == 0) {
          const float v = cw + fminf(sh.de[prv][r], m);
          sh.df[cur][r] = v;
          if (vt) vt[Kc * VS + r] = v;
        }
      }
      if (wv == kBuilder) {
        float m = lane < Kq ? sh.df[prv][lane] : INF;
        for (int off = 32; off > 0; off >>= 1) m = fminf(m, __shfl_xor(m, off));
        m = fminf(m, sh.dg[prv]);
        if (lane < Kn) {
          const float v = sh.cu[s0][lane] + m;
          sh.de[cur][lane] = v;
          if (vt) vt[lane * VS + Kc] = v;
        }
        if (lane == 0) {
          sh.dg[cur] = cw + m;
          if (vt) vt[Kc * VS + Kc] = cw + m;
        }
      }
    }
    __syncthreads();
  }

  // ---- optimum: first row-major minimum of V_{M-1}(a_{M-2}, a_{M-1}) ------------
  {
    constexpr int RS = KL + (DUMMY ? 1 : 0);  // row stride of the result index
    const int last = (M - 1) & 1;
    const int nch = n_slots(last);
    float bv = INF;
    int bi = 0x7fffffff;
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int ch = wv + NW * s;
      if (ch < nch) {
        int r, col;
        if (slot_cell(last, ch, r, col)) {
          const int idx = r * RS + col;
          if (vr[s] < bv || (vr[s] == bv && idx < bi)) { bv = vr[s]; bi = idx; }
        }
      }
    }
    if constexpr (DUMMY) {
      if (wv == 0) {
        auto take = [&](float v, int idx) {
          if (v < bv || (v == bv && idx < bi)) { bv = v; bi = idx; }
        };
        if (lane < sh.ck[(M - 2) & 3]) take(sh.df[last][lane], lane * RS + kEps);
        if (lane < sh.ck[(M - 1) & 3]) take(sh.de[last][lane], kEps * RS + lane);
        if (lane == 0) take(sh.dg[last], kEps * RS + kEps);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const float ov = __shfl_xor(bv, off);
      const int oi = __shfl_xor(bi, off);
      if (ov < bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { sh.red_v[wv] = bv; sh.red_i[wv] = bi; }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 1; q < NW; ++q) {
        const float ov = sh.red_v[q];
        const int oi = sh.red_i[q];
        if (ov < bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      }
      sh.res_v = bv;
      sh.res_i = bi == 0x7fffffff ? 0 : bi;
    }
    __syncthreads();
  }
  DPResult res;
  res.v = sh.res_v;
  res.idx = sh.res_i;
  res.flag = DEGEN ? 0 : sh.flag;
  return res;
}

// ---- backtracking (Eq. 12), one wave per matching ---------------------------------
// From the optimal final pair (r, c) = (a_{M-2}, a_{M-1}), each step recomputes
// the terms of the optimal cell over its admissible predecessors (lanes) with
// the forward pass's arithmetic and keeps the lowest index of the minimum.
// With dummies r and c may be kEps; the epsilon predecessor comes last, so it
// is taken only when its term is strictly smaller.
//
// The candidates of a list do not depend on the path, so each lane holds one
// candidate (node, frame, coordinates) of the three lists of the current
// step, and the next list is fetched while the current step runs; the chosen
// nodes' data come from their lanes by shuffles.  The one read that waits for
// the previous step's choice is the value-table column of the chosen cell.
struct LaneCand {
  int node;   // scene node of this lane's candidate, -1 past the list
  int t;      // its frame
  float2 xy;  // its coordinates
  int n;      // list length
};

__device__ __forceinline__ LaneCand lane_cand(const MatchView& a, int j, int lane) {
  const Cands q = cands_of(a, j);
  LaneCand L;
  L.n = q.count();
  L.node = lane < L.n ? q.node(lane) : -1;
  L.t = L.node >= 0 ? ro(a.s.t + L.node) : 0;
  L.xy = L.node >= 0 ? ro(a.s.xy + L.node) : make_float2(0.f, 0.f);
  return L;
}

template <bool DEGEN, bool DUMMY = false, bool UNS = false>
__device__ void backtrack_wave(const MatchView& a, const float* vtm, int r, int c, int lane,
                               int32_t* out) {
  const int M = a.m.M, Kc = a.sp.K, VS = a.vs;
  const int T = pair_limit(a.sp), TS = span_limit(a.sp);
  const float INF = __builtin_inff();
  // candidate index idx of a list held in lanes -> its node (dummy: kDummyNode)
  auto node_at = [&](const LaneCand& L, int idx) {
    return DUMMY && idx == kEps ? kDummyNode : __shfl(L.node, idx);
  };
  LaneCand Lc = lane_cand(a, M - 1, lane);
  LaneCand Lr = lane_cand(a, M - 2, lane);
  LaneCand Lk = lane_cand(a, M - 3, lane);
  {
    const int nc0 = node_at(Lc, c), nr0 = node_at(Lr, r);
    if (lane == 0) {
      out[M - 1] = nc0;
      out[M - 2] = nr0;
    }
  }
  for (int i = M - 1; i >= 2; --i) {
    const int nk = Lk.n;
    const float* vp = vtable(vtm, a, i - 1);
    // the column of the chosen cell: V_{i-1}(k, r) for every candidate k
    float vcol = INF;
    if (lane < nk && !(DUMMY && r == kEps)) vcol = vp[r * VS + lane];
    // the next list, fetched while this step runs
    LaneCand Ln;
    if (i >= 3) Ln = lane_cand(a, i - 3, lane);
    float tot = INF, teps = INF;
    if (DUMMY && r == kEps) {
      // V_i(eps, .) = ... + min(V_{i-1}(eps, eps), min_k V_{i-1}(k, eps))
      if (lane < nk) tot = vp[Kc * VS + lane];
      teps = vp[Kc * VS + Kc];
    } else {
      const float2 xr = make_float2(__shfl(Lr.xy.x, r), __shfl(Lr.xy.y, r));
      const int tr = __shfl(Lr.t, r);
      const int nr = __shfl(Lr.node, r);
      if (DUMMY) teps = vp[r * VS + Kc];
      if (DUMMY && c == kEps) {
        // V_i(r, eps) = l1 W^d + min(V_{i-1}(eps, r), min_k V_{i-1}(k, r))
        if (lane < nk && admissible(Lk.t, tr, T)) tot = vcol;
      } else {
        const float2 xa = make_float2(__shfl(Lc.xy.x, c), __shfl(Lc.xy.y, c));
        const int tc = __shfl(Lc.t, c);
        const float2 th = ro(a.theta + i);
        const bool same = xa.x == xr.x && xa.y == xr.y;
        float bm, be;
        cell_consts<UNS>(th, neg_dir<DEGEN>(xr, xa), bm, be);
        if (lane < nk && consecutive_ok(a.sp, T, Lk.node, Lk.t, nr, tr) && span_ok(Lk.t, tc, TS))
          tot = relax<DEGEN, UNS>(vcol, neg_dir<DEGEN>(Lk.xy, xr), neg_dir<DEGEN>(Lk.xy, xa), bm, be, th, same, a.w);
      }
    }
    int bk = lane;
    for (int off = 32; off > 0; off >>= 1) {
      const float ot = __shfl_xor(tot, off);
      const int ok = __shfl_xor(bk, off);
      if (ot < tot || (ot == tot && ok < bk)) { tot = ot; bk = ok; }
    }
    if (DUMMY && teps < tot) bk = kEps;
    const int nbk = node_at(Lk, bk);
    if (lane == 0) out[i - 2] = nbk;
    c = r;
    r = bk;
    Lc = Lr;
    Lr = Lk;
    if (i >= 3) Lk = Ln;
  }
}

// ---- per-offset kernels: one workgroup per offset of one (model, scene) pair ------
__device__ __forceinline__ MatchView view_of(const DPLaunch& a, int tl) {
  MatchView v;
  v.m = a.m;
  v.s = a.s;
  v.sp = a.sp;
  v.U = a.U;
  v.us = a.s.S;
  v.theta = a.theta;
  v.lambda1 = a.lambda1;
  v.lambda2 = a.lambda2;
  v.w = a.w;
  v.cw = a.cw;
  v.vs = a.sp.K + (a.dummy ? 1 : 0);
  v.tau = a.taus ? a.taus[tl] : a.tau0 + tl;
  v.cand = a.cand ? a.cand + (long long)tl * a.m.M * a.cstride : nullptr;
  v.ccount = a.cand ? a.ccount + (long long)tl * a.m.M : nullptr;
  v.cstride = a.cstride;
  return v;
}

__device__ __forceinline__ float* scratch_of(const DPLaunch& a, int tl) {
  const long long vs = a.sp.K + (a.dummy ? 1 : 0);
  return a.vt + (long long)tl * (a.m.M - 2) * vs * vs;
}

template <int NW, bool DEGEN, int KL, bool DUMMY = false, bool PACKED = false, bool UNS = false>
__global__ __launch_bounds__(NW * 64)
__attribute__((amdgpu_waves_per_eu(KL == kMaxList && NW == 8 ? 4 : 1)))
void k_dp(DPLaunch a) {
  __shared__ DPShared<NW, KL, DUMMY, PACKED> sh;
  const int tl = blockIdx.x;
  if (DEGEN && a.degen[tl] == 0) return;
  const DPResult r = dp_forward<NW, DEGEN, KL, DUMMY, PACKED, UNS>(sh, view_of(a, tl), scratch_of(a, tl));
  if (threadIdx.x == 0) {
    constexpr int RS = KL + (DUMMY ? 1 : 0);
    a.e32[tl] = r.v;
    a.last2[tl] = make_int2(r.idx / RS, r.idx % RS);
    if (!DEGEN) a.degen[tl] = r.flag;
  }
}

__global__ __launch_bounds__(64) void k_backtrack(DPLaunch a, int32_t* __restrict__ assign) {
  const int tl = blockIdx.x, lane = threadIdx.x;
  const int M = a.m.M;
  int32_t* out = assign + (long long)tl * M;
  if (!(a.e32[tl] < __builtin_inff())) {
    for (int i = lane; i < M; i += 64) out[i] = -1;
    return;
  }
  const MatchView v = view_of(a, tl);
  const int2 l2 = a.last2[tl];
  float* vt = scratch_of(a, tl);
  if (a.dummy) {
    if (a.degen[tl]) backtrack_wave<true, true>(v, vt, l2.x, l2.y, lane, out);
    else backtrack_wave<false, true>(v, vt, l2.x, l2.y, lane, out);
  } else if (a.sp.uns) {
    if (a.degen[tl]) backtrack_wave<true, false, true>(v, vt, l2.x, l2.y, lane, out);
    else backtrack_wave<false, false, true>(v, vt, l2.x, l2.y, lane, out);
  } else {
    if (a.degen[tl]) backtrack_wave<true>(v, vt, l2.x, l2.y, lane, out);
    else backtrack_wave<false>(v, vt, l2.x, l2.y, lane, out);
  }
}

// ---- batched persistent launch ------------------------------------------------------
// Workgroups pull (pair, offset) items from a cost-sorted list with an atomic
// counter until it runs out; each solves its item with the forward pass, re-runs
// the degenerate variant when coincident points were flagged, and backtracks in
// wave 0 from its own value-table scratch before taking the next item.
__device__ __forceinline__ MatchView view_of(const BatchLaunch& b, const PairDev& pd, int tau) {
  MatchView v;
  v.m = pd.m;
  v.s = pd.s;
  v.sp = b.sp;
  v.U = pd.U;
  v.us = pd.us;
  v.theta = pd.theta;
  v.lambda1 = b.lambda1;
  v.lambda2 = b.lambda2;
  v.w = b.w;
  v.cw = b.cw;
  v.vs = b.sp.K + (b.dummy ? 1 : 0);
  v.tau = tau;
  v.cand = pd.cand ? pd.cand + (long long)tau * pd.m.M * pd.cstride : nullptr;
  v.ccount = pd.cand ? pd.ccount + (long long)tau * pd.m.M : nullptr;
  v.cstride = pd.cstride;
  return v;
}

// A workgroup runs the forward passes of up to b.batch items (at most one per
// wave) one after the other, each into its own value tables, then wave q
// backtracks the q-th of them.  A backtracking walk is a
// chain of dependent memory reads, so the batch's walks overlap instead of
// each leaving the other waves idle.  The fast variant takes every item; an
// item whose matching has coincident points is appended to the degenerate
// list instead of being backtracked, and the degenerate variant (a second
// launch) takes the items of that list.  Occupancy target: two 8-wave
// workgroups per CU (four waves per SIMD), which leaves 128 registers per lane;
// the LDS of one matching would allow three, but at 80 registers the kernel
// spills and runs slower (1.3% on the realistic workload, 3.9% on the batched
// one).
template <int NW, bool DEGEN, int KL = kMaxList, bool DUMMY = false, bool PACKED = false, bool UNS = false>
__global__ __launch_bounds__(NW * 64)
__attribute__((amdgpu_waves_per_eu(DUMMY || PACKED ? 4 : (NW >= 8 ? 4 : 3))))
void k_dp_persistent(BatchLaunch b) {
  __shared__ DPShared<NW, KL, DUMMY, PACKED> sh;
  __shared__ int item_sh;
  __shared__ int bt_item[NW];  // item of each batch slot, -1: not backtracked here
  __shared__ int bt_idx[NW];   // its first minimising final pair, -1: infeasible
  constexpr int RS = KL + (DUMMY ? 1 : 0);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nb_max = b.batch < 1 ? 1 : (b.batch < NW ? b.batch : NW);
  float* vwg = b.vt + (long long)blockIdx.x * b.batch * b.vt_stride;
  const int n_items = DEGEN ? *b.degen_count : (b.list ? *b.list_count : b.n_items);
  int32_t* counter = DEGEN ? b.counter + 1 : b.counter;
  int slot = 0;  // forward passes waiting for their backtracking
  for (;;) {
    if (threadIdx.x == 0) item_sh = atomicAdd(counter, 1);
    __syncthreads();
    const bool done = item_sh >= n_items;
    if (!done) {
      const int item = DEGEN ? b.degen_items[item_sh] : b.list ? b.list[item_sh] : item_sh;
      const int2 it = b.items[item];
      const PairDev pd = b.pairs[it.x];
      const MatchView mv = view_of(b, pd, it.y);
      const DPResult r = dp_forward<NW, DEGEN, KL, DUMMY, PACKED, UNS>(sh, mv, vwg + slot * b.vt_stride);
      if (threadIdx.x == 0) {
        if (!DEGEN && r.flag) {
          b.degen_items[atomicAdd(b.degen_count, 1)] = item;
          bt_item[slot] = -1;
        } else {
          b.e32[pd.row0 + it.y] = r.v;
          bt_item[slot] = item;
          bt_idx[slot] = r.v < __builtin_inff() ? r.idx : -1;
        }
      }
      ++slot;
    }
    if (slot == nb_max || (done && slot > 0)) {
      __syncthreads();
      if (wv < slot && bt_item[wv] >= 0) {
        const int2 it = b.items[bt_item[wv]];
        const PairDev pd = b.pairs[it.x];
        int32_t* out = b.assign + pd.assign0 + (long long)it.y * pd.m.M;
        const int idx = bt_idx[wv];
        if (idx >= 0) {
          backtrack_wave<DEGEN, DUMMY, UNS>(view_of(b, pd, it.y), vwg + wv * b.vt_stride, idx / RS, idx % RS, lane,
                                       out);
        } else {
          for (int i = lane; i < pd.m.M; i += 64) out[i] = -1;
        }
      }
      slot = 0;
    }
    if (done) break;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_collect_infeasible(const PairDev* __restrict__ pairs,
                                                           const int2* __restrict__ items, int n_items,
                                                           const float* __restrict__ e32, int32_t* __restrict__ list,
                                                           int32_t* __restrict__ count, int32_t* __restrict__ fell) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n_items) return;
  const int2 it = items[q];
  const long long row = pairs[it.x].row0 + it.y;
  if (!(e32[row] < __builtin_inff())) {
    list[atomicAdd(count, 1)] = q;
    if (fell) fell[row] = 1;
  }
}

// Dense relaxations sum_i K_{i-2} K_{i-1} K_i of each item (one wave per item),
// the cost the work list is sorted by.
__global__ __launch_bounds__(64) void k_item_cost(const PairDev* __restrict__ pairs,
                                                 const int2* __restrict__ items, int n_items,
                                                 SearchParams sp, long long* __restrict__ cost) {
  const int item = blockIdx.x, lane = threadIdx.x;
  if (item >= n_items) return;
  const int2 it = items[item];
  const PairDev pd = pairs[it.x];
  const int M = pd.m.M, t0 = pd.m.t[0];
  long long acc = 0;
  for (int i = 2 + lane; i < M; i += 64) {
    long long prod = 1;
    for (int q = i - 2; q <= i; ++q) {
      const CandRange c = point_candidates(pd.s.fstart, pd.s.F, it.y + pd.m.t[q] - t0, sp);
      prod *= c.k1 + c.k2;
    }
    acc += prod;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) cost[item] = acc;
}

__global__ void k_fill_i32(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---- FP64 re-score of an assignment from the definition (Eq. 1-8) ---------------
__device__ __forceinline__ double wrap64(double x) {
  const double two_pi = 6.283185307179586476925286766559;
  return x - two_pi * rint(x / two_pi);
}

// One wave re-scores the assignment z of one matching into e64[row], eu64[row].
// A dummy (kDummyNode) costs wd; a Delta term needs both of its points
// matched, D^g all three, and only matched consecutive points are checked.
// The descriptor distances are taken four points at a time, 16 lanes per
// point striding its descriptor (coalesced reads; partial sums joined by a
// 16-lane tree); the triangle terms one point per lane.
__device__ void rescore_wave(const ModelView& m, const SceneView& s, const SearchParams& sp, double l1, double l2,
                             double l3, double wd, const int32_t* __restrict__ z, long long tl,
                             double* __restrict__ e64, double* __restrict__ eu64) {
  const int lane = threadIdx.x & 63;
  const int32_t T = pair_limit(sp), TS = span_limit(sp);
  const int M = m.M, dim = s.dim;
  const double inf = __builtin_inf();
  if (ro(z) == -1) {
    if (lane == 0) {
      if (e64) e64[tl] = inf;
      if (eu64) eu64[tl] = inf;
    }
    return;
  }
  double su = 0.0, sd = 0.0;
  int bad = 0;
  const int grp = lane >> 4, gl = lane & 15;
  for (int i0 = 0; i0 < M; i0 += 4) {
    const int i = i0 + grp;
    const int n = i < M ? ro(z + i) : kDummyNode;
    double acc = 0.0;
    if (n != kDummyNode) {
      const float* f = m.desc + (long long)i * dim;
      const float* g = s.desc + (long long)n * dim;
      for (int d = gl; d < dim; d += 16) {
        const double v = (double)ro(f + d) - (double)ro(g + d);
        acc = fma(v, v, acc);
      }
    }
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (gl == 0 && i < M) su += n == kDummyNode ? wd : sqrt(acc);
  }
  for (int i = lane; i < M; i += 64) {
    const int n = ro(z + i);
    const int nj = i >= 1 ? ro(z + (i - 1)) : kDummyNode;
    const int nk = i >= 2 ? ro(z + (i - 2)) : kDummyNode;
    if (n != kDummyNode && nj != kDummyNode && !consecutive_ok(sp, T, nj, ro(s.t + nj), n, ro(s.t + n))) bad = 1;
    // the span reading (no dummies): the triangle's first and last frames
    if (TS > 0 && i >= 2 && !span_ok(ro(s.t + ro(z + (i - 2))), ro(s.t + n), TS)) bad = 1;
    if (i >= 2 && (n == kDummyNode || nj == kDummyNode || nk == kDummyNode)) {
      // the Delta terms whose points are both matched; no D^g
      if (n != kDummyNode && nj != kDummyNode) {
        const long d1 = (long)(ro(m.t + i) - ro(m.t + (i - 1))) - (long)(ro(s.t + n) - ro(s.t + nj));
        sd += (double)(d1 < 0 ? -d1 : d1);
      }
      if (nj != kDummyNode && nk != kDummyNode) {
        const long d2 = (long)(ro(m.t + (i - 1)) - ro(m.t + (i - 2))) - (long)(ro(s.t + nj) - ro(s.t + nk));
        sd += (double)(d2 < 0 ? -d2 : d2);
      }
    } else if (i >= 2) {
      const long dt1 = (long)(ro(m.t + i) - ro(m.t + (i - 1))) - (long)(ro(s.t + n) - ro(s.t + nj));
      const long dt2 = (long)(ro(m.t + (i - 1)) - ro(m.t + (i - 2))) - (long)(ro(s.t + nj) - ro(s.t + nk));
      const float2 pi = ro(m.xy + i), pj = ro(m.xy + (i - 1)), pk = ro(m.xy + (i - 2));
      const float2 qi = ro(s.xy + n), qj = ro(s.xy + nj), qk = ro(s.xy + nk);
      double mid_m = ang64(pi.x, pi.y, pj.x, pj.y, pk.x, pk.y);
      double mid_s = ang64(qi.x, qi.y, qj.x, qj.y, qk.x, qk.y);
      double end_m = ang64(pj.x, pj.y, pi.x, pi.y, pk.x, pk.y);
      double end_s = ang64(qj.x, qj.y, qi.x, qi.y, qk.x, qk.y);
      if (sp.uns) {  // the unsigned reading: magnitudes of the angles
        mid_m = fabs(mid_m);
        mid_s = fabs(mid_s);
        end_m = fabs(end_m);
        end_s = fabs(end_s);
      }
      const double d1 = wrap64(mid_m - mid_s), d2 = wrap64(end_m - end_s);
      sd += (double)(dt1 < 0 ? -dt1 : dt1) + (double)(dt2 < 0 ? -dt2 : dt2) +
            l3 * sqrt(d1 * d1 + d2 * d2);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    su += __shfl_xor(su, off);
    sd += __shfl_xor(sd, off);
    bad |= __shfl_xor(bad, off);
  }
  if (lane == 0) {
    if (e64) e64[tl] = bad ? inf : l1 * su + l2 * sd;
    if (eu64) eu64[tl] = bad ? inf : l1 * su;
  }
}

__global__ __launch_bounds__(64) void k_rescore(ModelView m, SceneView s, SearchParams sp, double l1, double l2,
                                               double l3, double wd, const int32_t* __restrict__ assign,
                                               double* __restrict__ e64, double* __restrict__ eu64) {
  const int tl = blockIdx.x;
  rescore_wave(m, s, sp, l1, l2, l3, wd, assign + (long long)tl * m.M, tl, e64, eu64);
}

__global__ __launch_bounds__(64) void k_rescore_batch(const PairDev* __restrict__ pairs,
                                                     const int2* __restrict__ items, int n_items,
                                                     SearchParams sp, double l1, double l2, double l3, double wd,
                                                     const int32_t* __restrict__ assign,
                                                     double* __restrict__ e64, double* __restrict__ eu64) {
  const int item = blockIdx.x;
  if (item >= n_items) return;
  const int2 it = items[item];
  const PairDev pd = pairs[it.x];
  rescore_wave(pd.m, pd.s, sp, l1, l2, l3, wd, assign + pd.assign0 + (long long)it.y * pd.m.M,
               pd.row0 + it.y, e64, eu64);
}

// Lists of at most 16 or 32 candidates take a smaller LDS layout and fewer
// waves per matching (more matchings resident per CU); longer lists take the
// 64-slot layout with the requested number of waves.  The arithmetic of every
// cell is the same, so the results do not depend on the variant.
template <bool DEGEN>
hipError_t launch_dp_waves(const DPLaunch& a, hipStream_t st) {
  if (a.n_tau <= 0) return hipSuccess;
  if (a.dummy) {  // dummies: one variant, 8 waves and the 64-slot layout
    hipLaunchKernelGGL((k_dp<8, DEGEN, 64, true>), dim3(a.n_tau), dim3(8 * 64), 0, st, a);
    return hipGetLastError();
  }
  if (a.sp.uns) {  // unsigned angles: one variant, 8 waves, the 64-slot layout and dense schedules
    hipLaunchKernelGGL((k_dp<8, DEGEN, 64, false, false, true>), dim3(a.n_tau), dim3(8 * 64), 0, st, a);
    return hipGetLastError();
  }
  if (a.packed && a.sp.K > 32) {  // sparse scenes, long lists: packed schedules
    hipLaunchKernelGGL((k_dp<8, DEGEN, 64, false, true>), dim3(a.n_tau), dim3(8 * 64), 0, st, a);
    return hipGetLastError();
  }
  if (a.sp.K <= 16) {
    hipLaunchKernelGGL((k_dp<1, DEGEN, 16>), dim3(a.n_tau), dim3(64), 0, st, a);
    return hipGetLastError();
  }
  if (a.sp.K <= 32) {
    hipLaunchKernelGGL((k_dp<2, DEGEN, 32>), dim3(a.n_tau), dim3(2 * 64), 0, st, a);
    return hipGetLastError();
  }
  switch (a.waves) {
    case 4:
      hipLaunchKernelGGL((k_dp<4, DEGEN, 64>), dim3(a.n_tau), dim3(4 * 64), 0, st, a);
      break;
    case 16:
      hipLaunchKernelGGL((k_dp<16, DEGEN, 64>), dim3(a.n_tau), dim3(16 * 64), 0, st, a);
      break;
    default:
      hipLaunchKernelGGL((k_dp<8, DEGEN, 64>), dim3(a.n_tau), dim3(8 * 64), 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_dp_fast(const DPLaunch& a, hipStream_t st) { return launch_dp_waves<false>(a, st); }

hipError_t launch_dp_degenerate(const DPLaunch& a, hipStream_t st) { return launch_dp_waves<true>(a, st); }

template <bool DEGEN>
hipError_t launch_persistent_variant(const BatchLaunch& b, int n_wg, hipStream_t st) {
  if (b.dummy) {  // dummies: 8 waves whatever the tuning says
    hipLaunchKernelGGL((k_dp_persistent<8, DEGEN, kMaxList, true>), dim3(n_wg), dim3(8 * 64), 0, st, b);
    return hipGetLastError();
  }
  if (b.sp.uns) {  // unsigned angles: one variant, 8 waves, dense schedules
    hipLaunchKernelGGL((k_dp_persistent<8, DEGEN, kMaxList, false, false, true>), dim3(n_wg), dim3(8 * 64), 0, st,
                       b);
    return hipGetLastError();
  }
  if (b.packed) {  // sparse scenes: packed schedules, 8 waves
    hipLaunchKernelGGL((k_dp_persistent<8, DEGEN, kMaxList, false, true>), dim3(n_wg), dim3(8 * 64), 0, st, b);
    return hipGetLastError();
  }
  switch (b.waves) {
    case 4:
      hipLaunchKernelGGL((k_dp_persistent<4, DEGEN>), dim3(n_wg), dim3(4 * 64), 0, st, b);
      break;
    case 16:
      hipLaunchKernelGGL((k_dp_persistent<16, DEGEN>), dim3(n_wg), dim3(16 * 64), 0, st, b);
      break;
    default:
      hipLaunchKernelGGL((k_dp_persistent<8, DEGEN>), dim3(n_wg), dim3(8 * 64), 0, st, b);
  }
  return hipGetLastError();
}

hipError_t launch_dp_persistent(const BatchLaunch& b, int n_wg, hipStream_t st) {
  hipError_t e = launch_persistent_variant<false>(b, n_wg, st);
  if (e != hipSuccess) return e;
  return launch_persistent_variant<true>(b, n_wg, st);
}

hipError_t launch_item_cost(const PairDev* pairs, const int2* items, int n_items, const SearchParams& sp,
                            long long* cost, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_item_cost, dim3(n_items), dim3(64), 0, st, pairs, items, n_items, sp, cost);
  return hipGetLastError();
}

hipError_t launch_collect_infeasible(const PairDev* pairs, const int2* items, int n_items, const float* e32,
                                     int32_t* list, int32_t* count, int32_t* fell, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_collect_infeasible, dim3((n_items + 255) / 256), dim3(256), 0, st, pairs, items, n_items, e32,
                     list, count, fell);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int n, int v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_rescore_batch(const PairDev* pairs, const int2* items, int n_items, const SearchParams& sp,
                                double lambda1, double lambda2, double lambda3, double w_dummy,
                                const int32_t* assign, double* e64, double* eu64, hipStream_t st) {
  if (n_items <= 0 || (!e64 && !eu64)) return hipSuccess;
  hipLaunchKernelGGL(k_rescore_batch, dim3(n_items), dim3(64), 0, st, pairs, items, n_items, sp,
                     lambda1, lambda2, lambda3, w_dummy, assign, e64, eu64);
  return hipGetLastError();
}

hipError_t launch_backtrack(const DPLaunch& a, int32_t* assign, hipStream_t st) {
  if (a.n_tau <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_backtrack, dim3(a.n_tau), dim3(64), 0, st, a, assign);
  return hipGetLastError();
}

hipError_t launch_rescore(const ModelView& m, const SceneView& s, const SearchParams& sp, double lambda1,
                          double lambda2, double lambda3, double w_dummy, const int32_t* assign,
                          int32_t n_tau, double* e64, double* eu64, hipStream_t st) {
  if (n_tau <= 0 || (!e64 && !eu64)) return hipSuccess;
  hipLaunchKernelGGL(k_rescore, dim3(n_tau), dim3(64), 0, st, m, s, sp, lambda1, lambda2, lambda3,
                     w_dummy, assign, e64, eu64);
  return hipGetLastError();
}

}  // namespace stm
