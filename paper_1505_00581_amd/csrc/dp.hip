// The exact min-sum recursion of the matching (Section 2.2), one workgroup per
// (model, scene, offset) matching, with the triplet cost fused into the
// minimisation; backtracking and the FP64 re-score of the result.
//
// Forward form of Eq. 10-13.  With a_i the candidate index of model point i:
//   V_1(a_0, a_1) = l1 U_0 + l1 U_1 + Q_1(a_0, a_1)
//   V_i(a_{i-1}, a_i) = l1 U_i(a_i) + Q_i(a_{i-1}, a_i)
//       + min_{a_{i-2}} [ V_{i-1}(a_{i-2}, a_{i-1}) + l2 l3 D^g_i(a_{i-2}, a_{i-1}, a_i) ]
// where Q_i = l2 c_i Delta(i, i-1), +inf unless the pair is admissible (Eq. 7,
// 8), and c_i counts the triangles holding the pair (i, i-1) (2 inside the
// chain, 1 at its ends), so every D^t term of Eq. 4 is charged exactly once.
// The optimum is min V_{M-1}; B_i = argmin a_{i-2} is kept for backtracking.
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
// Layout.  Lanes of a 64-wide wavefront are the candidates a_i of the current
// point; the waves of the workgroup take the rows a_{i-1} round-robin.  The
// admissible predecessors a_{i-2} of a row form one contiguous index range
// (candidates are sorted by frame), found with two ballots, so the inner loop
// has wave-uniform bounds (the paper's loop bounds of Section 3.4).  Per step
// the LDS holds the previous V column pairs with their directions and the
// (a_{i-2}, a_i) direction table; the new cells stay in registers until every
// wave has finished reading, then replace the old ones.
//
// Degenerate triangles.  A zero-length side gives a scene angle of 0 in the
// definition, which the direction form does not reproduce.  The fast variant
// detects coincident points on pairs that can be admissible and flags the
// matching; the flagged matchings are recomputed by the variant that marks
// coincident directions as NaN and substitutes the model angle.
#include <math.h>

#include "stm_internal.h"

namespace stm {
namespace {

constexpr int KL = 64;  // candidate slots = wavefront lanes
constexpr float kPi = 3.14159265358979323846f;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr float kInvTwoPi = 0.15915494309189533577f;

__device__ __forceinline__ float wrap_pi(float x) { return fmaf(-kTwoPi, rintf(x * kInvTwoPi), x); }

// |wrap(x)| for |x| <= 2 pi.
__device__ __forceinline__ float abs_wrap(float x) { return kPi - fabsf(kPi - fabsf(x)); }

template <int NW>
struct DPShared {
  float2 va[KL * KL];   // [a_{i-2}][a_{i-1}]: (V_{i-1}, -phi(z_{i-2} -> z_{i-1}))
  float ct[KL * KL];    // [a_{i-2}][a_i]: -phi(z_{i-2} -> z_i)
  float2 cxy[4][KL];    // candidate ring: coordinates,
  int32_t ctt[4][KL];   //   frames,
  float cu[4][KL];      //   l1 * U
  int32_t ck[4];        //   list lengths
  int32_t flag;         // coincident points seen (fast variant)
  float red_v[NW];
  int32_t red_i[NW];
};

template <int NW, bool DEGEN>
__global__ __launch_bounds__(NW * 64) void k_dp(DPLaunch a) {
  __shared__ DPShared<NW> sh;
  constexpr int RPW = KL / NW;  // rows per wave
  const int tl = blockIdx.x;
  if (DEGEN && a.degen[tl] == 0) return;
  const int tau = a.tau0 + tl;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int M = a.m.M;
  const int S = a.s.S;
  const int T = a.sp.T;
  const int Kc = a.sp.K;
  const int tm0 = a.m.t[0];
  const float INF = __builtin_inff();
  const float QNAN = __builtin_nanf("");

  auto load_slot = [&](int j) {
    if (wv == 0) {
      const CandRange c = point_candidates(a.s.fstart, a.s.F, tau + a.m.t[j] - tm0, a.sp);
      const int k = c.k1 + c.k2;
      const int sl = j & 3;
      if (lane < k) {
        const int n = cand_node(c, lane);
        sh.cxy[sl][lane] = a.s.xy[n];
        sh.ctt[sl][lane] = a.s.t[n];
        sh.cu[sl][lane] = a.lambda1 * a.U[(long long)j * S + n];
      }
      if (lane == 0) sh.ck[sl] = k;
    }
  };

  if (threadIdx.x == 0) sh.flag = 0;
  load_slot(0);
  load_slot(1);
  load_slot(2);
  __syncthreads();

  float vr[RPW], ar[RPW];
#pragma unroll
  for (int s = 0; s < RPW; ++s) { vr[s] = INF; ar[s] = 0.f; }

  // ---- the first pair (points 0, 1) ------------------------------------------
  {
    const int K0 = sh.ck[0], K1 = sh.ck[1];
    const bool valid_a = lane < K1;
    const int tp = valid_a ? sh.ctt[1][lane] : 0;
    const float2 xa = valid_a ? sh.cxy[1][lane] : make_float2(0.f, 0.f);
    const float ua = valid_a ? sh.cu[1][lane] : 0.f;
    const int dtm = a.m.t[1] - a.m.t[0];
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int r = wv + NW * s;
      if (r < K0) {
        const int tr = sh.ctt[0][r];
        const float2 xr = sh.cxy[0][r];
        const bool adm = valid_a && admissible(tr, tp, T);
        const bool same = xa.x == xr.x && xa.y == xr.y;
        const float phi = same ? 0.f : atan2f(xa.y - xr.y, xa.x - xr.x);
        if (!DEGEN && same && adm) sh.flag = 1;
        const float q = a.lambda2 * fabsf(static_cast<float>(dtm - (tp - tr)));
        vr[s] = adm ? (sh.cu[0][r] + ua) + q : INF;
        ar[s] = (DEGEN && same) ? QNAN : -phi;
      }
    }
  }

  // ---- points 2 .. M-1 -----------------------------------------------------------
  for (int i = 2; i < M; ++i) {
    const int s2 = (i - 2) & 3, s1 = (i - 1) & 3, s0 = i & 3;
    const int Kq = sh.ck[s2], Kp = sh.ck[s1], Kn = sh.ck[s0];

    // Phase 1: publish the previous cells, build the (a_{i-2}, a_i) direction
    // table, prefetch the next candidate list.
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int k = wv + NW * s;
      if (k < Kq && lane < Kp) sh.va[k * KL + lane] = make_float2(vr[s], ar[s]);
    }
    for (int e = threadIdx.x; e < Kq * KL; e += NW * 64) {
      const int k = e >> 6, c = e & 63;
      if (c < Kn) {
        const float2 pk = sh.cxy[s2][k], pc = sh.cxy[s0][c];
        const bool same = pk.x == pc.x && pk.y == pc.y;
        float v = same ? 0.f : -atan2f(pc.y - pk.y, pc.x - pk.x);
        if (DEGEN && same) v = QNAN;
        if (!DEGEN && same && sh.ctt[s2][k] < sh.ctt[s0][c]) sh.flag = 1;
        sh.ct[e] = v;
      }
    }
    if (i + 1 < M) load_slot(i + 1);
    __syncthreads();

    // Phase 2: the relaxations of every cell (a_{i-1} = row, a_i = lane).
    const float2 th = a.theta[i];
    const int dtm = a.m.t[i] - a.m.t[i - 1];
    const float qw = a.lambda2 * (i <= M - 2 ? 2.f : 1.f);
    const bool valid_a = lane < Kn;
    const int tp = valid_a ? sh.ctt[s0][lane] : 0;
    const float2 xa = valid_a ? sh.cxy[s0][lane] : make_float2(0.f, 0.f);
    const float ua = valid_a ? sh.cu[s0][lane] : 0.f;
    const int tk_lane = lane < Kq ? sh.ctt[s2][lane] : 0x7fffffff;
    uint8_t* bprow = a.bp + ((long long)tl * (M - 2) + (i - 2)) * Kc * Kc;
    const float w = a.w;
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int r = wv + NW * s;
      float vnew = INF, anew = 0.f;
      if (r < Kp) {
        const int tr = sh.ctt[s1][r];
        const float2 xr = sh.cxy[s1][r];
        const bool adm = valid_a && admissible(tr, tp, T);
        const bool same = xa.x == xr.x && xa.y == xr.y;
        const float phi = same ? 0.f : atan2f(xa.y - xr.y, xa.x - xr.x);
        if (!DEGEN && same && adm) sh.flag = 1;
        const int hi = __popcll(__ballot(tk_lane < tr));
        const int lo = T > 0 ? __popcll(__ballot(tk_lane <= tr - T)) : 0;
        float best = INF;
        int arg = 0;
        if (adm) {
          const float bm = wrap_pi(th.x - kPi + phi), be = wrap_pi(th.y + phi);
          const float2* vcol = sh.va + r;
          const float* ccol = sh.ct + lane;
#pragma unroll 4
          for (int k = lo; k < hi; ++k) {
            const float2 v = vcol[k * KL];
            const float c = ccol[k * KL];
            float x1, x2;
            if (DEGEN) {
              x1 = (same || isnan(v.y)) ? th.x : v.y + bm;
              x2 = (same || isnan(c)) ? th.y : c + be;
            } else {
              x1 = v.y + bm;
              x2 = c + be;
            }
            const float z1 = abs_wrap(x1), z2 = abs_wrap(x2);
            const float d = __builtin_amdgcn_sqrtf(fmaf(z2, z2, z1 * z1));
            const float tot = fmaf(w, d, v.x);
            if (tot < best) { best = tot; arg = k; }
          }
          const float q = qw * fabsf(static_cast<float>(dtm - (tp - tr)));
          vnew = (ua + q) + best;
        }
        anew = (DEGEN && same) ? QNAN : -phi;
        if (valid_a) bprow[r * Kc + lane] = static_cast<uint8_t>(arg);
      }
      vr[s] = vnew;
      ar[s] = anew;
    }
    __syncthreads();
  }

  // ---- optimum: first row-major minimum of V_{M-1}(a_{M-2}, a_{M-1}) ------------
  {
    const int Kq = sh.ck[(M - 2) & 3], Kn = sh.ck[(M - 1) & 3];
    float bv = INF;
    int bi = 0x7fffffff;
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const int r = wv + NW * s;
      if (r < Kq && lane < Kn) {
        const int idx = r * KL + lane;
        if (vr[s] < bv || (vr[s] == bv && idx < bi)) { bv = vr[s]; bi = idx; }
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
      a.e32[tl] = bv;
      a.last2[tl] = bi == 0x7fffffff ? make_int2(0, 0) : make_int2(bi / KL, bi % KL);
      if (!DEGEN) a.degen[tl] = sh.flag;
    }
  }
}

// ---- backtracking (Eq. 12), one thread per matching -----------------------------
__global__ void k_backtrack(DPLaunch a, int32_t* __restrict__ assign) {
  const int tl = blockIdx.x * blockDim.x + threadIdx.x;
  if (tl >= a.n_tau) return;
  const int M = a.m.M, K = a.sp.K;
  int32_t* out = assign + (long long)tl * M;
  if (!(a.e32[tl] < __builtin_inff())) {
    for (int i = 0; i < M; ++i) out[i] = -1;
    return;
  }
  const int tau = a.tau0 + tl, tm0 = a.m.t[0];
  int r = a.last2[tl].x, c = a.last2[tl].y;  // a_{M-2}, a_{M-1}
  out[M - 1] = cand_node(point_candidates(a.s.fstart, a.s.F, tau + a.m.t[M - 1] - tm0, a.sp), c);
  out[M - 2] = cand_node(point_candidates(a.s.fstart, a.s.F, tau + a.m.t[M - 2] - tm0, a.sp), r);
  for (int i = M - 1; i >= 2; --i) {
    const uint8_t* bprow = a.bp + ((long long)tl * (M - 2) + (i - 2)) * K * K;
    const int k = bprow[r * K + c];
    out[i - 2] = cand_node(point_candidates(a.s.fstart, a.s.F, tau + a.m.t[i - 2] - tm0, a.sp), k);
    c = r;
    r = k;
  }
}

// ---- FP64 re-score of an assignment from the definition (Eq. 1-8) ---------------
__device__ __forceinline__ double wrap64(double x) {
  const double two_pi = 6.283185307179586476925286766559;
  return x - two_pi * rint(x / two_pi);
}

__global__ void k_rescore(ModelView m, SceneView s, int32_t T, double l1, double l2, double l3,
                          const int32_t* __restrict__ assign, double* __restrict__ e64,
                          double* __restrict__ eu64) {
  const int tl = blockIdx.x, lane = threadIdx.x;
  const int M = m.M, dim = s.dim;
  const int32_t* z = assign + (long long)tl * M;
  const double inf = __builtin_inf();
  if (z[0] < 0) {
    if (lane == 0) {
      if (e64) e64[tl] = inf;
      if (eu64) eu64[tl] = inf;
    }
    return;
  }
  double su = 0.0, sd = 0.0;
  int bad = 0;
  for (int i = lane; i < M; i += 64) {
    const int n = z[i];
    const float* f = m.desc + (long long)i * dim;
    const float* g = s.desc + (long long)n * dim;
    double acc = 0.0;
    for (int d = 0; d < dim; ++d) {
      const double v = (double)f[d] - (double)g[d];
      acc += v * v;
    }
    su += sqrt(acc);
    if (i >= 1 && !admissible(s.t[z[i - 1]], s.t[n], T)) bad = 1;
    if (i >= 2) {
      const int nj = z[i - 1], nk = z[i - 2];
      const long dt1 = (long)(m.t[i] - m.t[i - 1]) - (long)(s.t[n] - s.t[nj]);
      const long dt2 = (long)(m.t[i - 1] - m.t[i - 2]) - (long)(s.t[nj] - s.t[nk]);
      const float2 pi = m.xy[i], pj = m.xy[i - 1], pk = m.xy[i - 2];
      const float2 qi = s.xy[n], qj = s.xy[nj], qk = s.xy[nk];
      const double mid_m = ang64(pi.x, pi.y, pj.x, pj.y, pk.x, pk.y);
      const double mid_s = ang64(qi.x, qi.y, qj.x, qj.y, qk.x, qk.y);
      const double end_m = ang64(pj.x, pj.y, pi.x, pi.y, pk.x, pk.y);
      const double end_s = ang64(qj.x, qj.y, qi.x, qi.y, qk.x, qk.y);
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

constexpr int kDPWaves = 4;

}  // namespace

hipError_t launch_dp_fast(const DPLaunch& a, hipStream_t st) {
  if (a.n_tau <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_dp<kDPWaves, false>), dim3(a.n_tau), dim3(kDPWaves * 64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_dp_degenerate(const DPLaunch& a, hipStream_t st) {
  if (a.n_tau <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_dp<kDPWaves, true>), dim3(a.n_tau), dim3(kDPWaves * 64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_backtrack(const DPLaunch& a, int32_t* assign, hipStream_t st) {
  if (a.n_tau <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_backtrack, dim3((a.n_tau + 63) / 64), dim3(64), 0, st, a, assign);
  return hipGetLastError();
}

hipError_t launch_rescore(const ModelView& m, const SceneView& s, int32_t T, double lambda1,
                          double lambda2, double lambda3, const int32_t* assign, int32_t n_tau,
                          double* e64, double* eu64, hipStream_t st) {
  if (n_tau <= 0 || (!e64 && !eu64)) return hipSuccess;
  hipLaunchKernelGGL(k_rescore, dim3(n_tau), dim3(64), 0, st, m, s, T, lambda1, lambda2, lambda3,
                     assign, e64, eu64);
  return hipGetLastError();
}

}  // namespace stm
