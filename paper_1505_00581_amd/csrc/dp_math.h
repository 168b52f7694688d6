// Device arithmetic of the recursion's terms shared by the per-offset kernels
// and the trellis kernels: the scene directions (a project-written atan2),
// the wrap of angle differences and one relaxation term V + l2 l3 D^g.  Both
// evaluate every term through these functions, so a term has the same bits
// wherever it is computed.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace stm {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr float kInvTwoPi = 0.15915494309189533577f;

__device__ __forceinline__ float wrap_pi(float x) { return fmaf(-kTwoPi, rintf(x * kInvTwoPi), x); }

// |wrap(x)| for |x| <= 2 pi.
__device__ __forceinline__ float abs_wrap(float x) { return kPi - fabsf(kPi - fabsf(x)); }

// Coefficients of atan(t) ~ t * P(t^2) on [0, 1]: degree-7 minimax fit by the
// Remez exchange algorithm (gen_atan_poly.py prints them).
constexpr float kAtanC0 = 0.9999993443489075f;
constexpr float kAtanC1 = -0.33329859375953674f;
constexpr float kAtanC2 = 0.19946566224098206f;
constexpr float kAtanC3 = -0.1390862911939621f;
constexpr float kAtanC4 = 0.0964219719171524f;
constexpr float kAtanC5 = -0.0559123270213604f;
constexpr float kAtanC6 = 0.021862957626581192f;
constexpr float kAtanC7 = -0.004054567310959101f;
constexpr float kHalfPi = 1.57079632679489661923f;

// -atan2(y, x) for (x, y) != (0, 0): reduction to t = min(|x|,|y|) / max(|x|,|y|)
// in [0, 1], the polynomial, then the octant and quadrant corrections.  The
// largest error over the plane is below 3.5e-7 rad (mostly the final rounding
// of values near pi).
__device__ __forceinline__ float neg_atan2(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float t = fminf(ax, ay) * __builtin_amdgcn_rcpf(fmaxf(ax, ay));
  const float s = t * t;
  float p = kAtanC7;
  p = fmaf(p, s, kAtanC6);
  p = fmaf(p, s, kAtanC5);
  p = fmaf(p, s, kAtanC4);
  p = fmaf(p, s, kAtanC3);
  p = fmaf(p, s, kAtanC2);
  p = fmaf(p, s, kAtanC1);
  p = fmaf(p, s, kAtanC0);
  float a = t * p;
  a = ay > ax ? kHalfPi - a : a;
  a = x < 0.f ? kPi - a : a;
  return y < 0.f ? a : -a;
}

// -phi(p -> q), the stored (negated) direction of q - p; -0 for coincident
// points in the fast variant, NaN in the degenerate variant.
template <bool DEGEN>
__device__ __forceinline__ float neg_dir(float2 p, float2 q) {
  const bool same = p.x == q.x && p.y == q.y;
  if (DEGEN && same) return __builtin_nanf("");
  return same ? -0.f : neg_atan2(q.y - p.y, q.x - p.x);
}

// The per-cell brackets of delta_mid and delta_end, pre-wrapped; phi is the
// direction z_{i-1} -> z_i of the cell.
__device__ __forceinline__ void cell_brackets(float2 th, float phi, float& bm, float& be) {
  bm = wrap_pi(th.x - kPi + phi);
  be = wrap_pi(th.y + phi);
}

// The per-cell constants of relax from the cell's stored direction anew =
// -phi(z_{i-1} -> z_i): the brackets above (oriented angles), or with unsigned
// angles pi + anew and anew, from which the scene triangle's angles at z_{i-1}
// and z_i are wrap(pi + anew - A) and wrap(anew - C).
template <bool UNS>
__device__ __forceinline__ void cell_consts(float2 th, float anew, float& bm, float& be) {
  if constexpr (UNS) {
    bm = kPi + anew;
    be = anew;
  } else {
    cell_brackets(th, -anew, bm, be);
  }
}

// One relaxation term V_{i-1}(a_{i-2}, a_{i-1}) + l2 l3 D^g_i.  A = -phi(z_{i-2}
// -> z_{i-1}), C = -phi(z_{i-2} -> z_i); same_rc: z_{i-1} and z_i coincide; bm,
// be from cell_consts<UNS>.  UNS: the unsigned reading of the angles, each
// difference taken between the magnitudes of the model's and the scene's
// angle.  The forward pass and backtracking both evaluate terms through this
// function, so they agree bit for bit.
template <bool DEGEN, bool UNS = false>
__device__ __forceinline__ float relax(float v, float A, float C, float bm, float be, float2 th,
                                       bool same_rc, float w) {
  if constexpr (UNS) {
    const float am = fabsf(th.x), ae = fabsf(th.y);
    float z1 = am - fabsf(wrap_pi(bm - A)), z2 = ae - fabsf(wrap_pi(be - C));
    if (DEGEN) {  // a zero-length side makes the scene's angle 0
      z1 = (same_rc || isnan(A)) ? am : z1;
      z2 = (same_rc || isnan(C)) ? ae : z2;
    }
    const float t = fmaf(w, __builtin_amdgcn_sqrtf(fmaf(z2, z2, z1 * z1)), v);
    // +inf marks a triangle the span reading of closeness excludes
    return C == __builtin_inff() ? __builtin_inff() : t;
  }
  float x1, x2;
  if (DEGEN) {
    // +inf marks a triangle the span reading of closeness excludes (the fast
    // variant reaches +inf or NaN through the arithmetic, both ignored by the
    // minimum)
    if (C == __builtin_inff()) return __builtin_inff();
    x1 = (same_rc || isnan(A)) ? th.x : A + bm;
    x2 = (same_rc || isnan(C)) ? th.y : C + be;
  } else {
    x1 = A + bm;
    x2 = C + be;
  }
  const float z1 = abs_wrap(x1), z2 = abs_wrap(x2);
  return fmaf(w, __builtin_amdgcn_sqrtf(fmaf(z2, z2, z1 * z1)), v);
}

}  // namespace stm
