// Learned candidate pruner: features, FP32 training kernels (forward,
// listwise loss, backward, Adam) and the BF16 inference kernel with top-k
// selection.  Not part of the paper: it shortens the candidate lists the
// exact recursion (Section 2.2) runs on; the exact recursion stays the
// fallback and the reference for the energy gap.
//
// One group = the candidates of one model point i at one offset tau; a group
// occupies 64 rows (one per candidate slot; slots past the list are invalid).
// Row input x = [D f_i (D), D g_n (D), phi (8)] (descriptors are L1-normalised;
// the factor D brings their entries to order 1) with phi:
//   0  (t'_n - (tau + t_i - t_0)) / 4
//   1,2 ((p'_n - p'_{q_a}) - (p_i - p_a)) / 64,  3,4 the same for neighbour b
//   5  log((|p'_n - p'_{q_a}| + 1) / (|p_i - p_a| + 1))
//   6  U(i, n) - min over the group's candidates of U(i, .)
//   7  i / (M - 1)
// with a = i - 1, b = i + 1 (the one neighbour twice at the chain ends) and q_j
// the candidate of neighbour j with the smallest U (lowest index on ties).
// Network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), s = w3 . h2 + b3, 128
// hidden units; parameters packed as [W1 (128 x NI), b1, W2 (128 x 128), b2,
// w3, b3], NI = 2 D + 8.
#include <math.h>

#include "stm_internal.h"

namespace stm {
namespace {

constexpr int H = kPrunerHidden;

// ---- features --------------------------------------------------------------------

__device__ __forceinline__ int wave_argmin_node(const CandRange& c, const float* __restrict__ Urow, int lane) {
  const int k = c.k1 + c.k2;
  float v = __builtin_inff();
  int idx = 0x7fffffff;
  if (lane < k) {
    v = Urow[cand_node(c, lane)];
    idx = lane;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const float ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(idx, off);
    if (ov < v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  }
  return k > 0 ? cand_node(c, idx) : -1;
}

// Candidate node and features of lane `lane` of group (tau, i); node -1 past
// the list.  Returns the neighbours' chosen candidates in qa, qb.
__device__ void group_features(const ModelView& m, const SceneView& s, const float* __restrict__ U,
                               long long us, const SearchParams& sp, int tau, int i, int lane, int& node,
                               float phi[8], int& qa, int& qb) {
  const int M = m.M, t0 = m.t[0];
  const int a = i >= 1 ? i - 1 : i + 1;
  const int b = i <= M - 2 ? i + 1 : i - 1;
  const CandRange ci = point_candidates(s.fstart, s.F, tau + m.t[i] - t0, sp);
  const CandRange ca = point_candidates(s.fstart, s.F, tau + m.t[a] - t0, sp);
  const CandRange cb = point_candidates(s.fstart, s.F, tau + m.t[b] - t0, sp);
  qa = wave_argmin_node(ca, U + (long long)a * us, lane);
  qb = wave_argmin_node(cb, U + (long long)b * us, lane);
  const int k = ci.k1 + ci.k2;
  node = lane < k ? cand_node(ci, lane) : -1;
  const int best = wave_argmin_node(ci, U + (long long)i * us, lane);
#pragma unroll
  for (int f = 0; f < 8; ++f) phi[f] = 0.f;
  if (node < 0) return;
  const float2 pn = s.xy[node], pi = m.xy[i], pa = m.xy[a], pb = m.xy[b];
  phi[0] = static_cast<float>(s.t[node] - (tau + m.t[i] - t0)) * 0.25f;
  if (qa >= 0) {
    const float2 q = s.xy[qa];
    phi[1] = ((pn.x - q.x) - (pi.x - pa.x)) * (1.f / 64.f);
    phi[2] = ((pn.y - q.y) - (pi.y - pa.y)) * (1.f / 64.f);
    phi[5] = logf((sqrtf((pn.x - q.x) * (pn.x - q.x) + (pn.y - q.y) * (pn.y - q.y)) + 1.f) /
                  (sqrtf((pi.x - pa.x) * (pi.x - pa.x) + (pi.y - pa.y) * (pi.y - pa.y)) + 1.f));
  }
  if (qb >= 0) {
    const float2 q = s.xy[qb];
    phi[3] = ((pn.x - q.x) - (pi.x - pb.x)) * (1.f / 64.f);
    phi[4] = ((pn.y - q.y) - (pi.y - pb.y)) * (1.f / 64.f);
  }
  phi[6] = U[(long long)i * us + node] - U[(long long)i * us + best];
  phi[7] = static_cast<float>(i) / static_cast<float>(M - 1);
}

// One 64-lane block per group: rows node [G*64], phi [G*64][8], q [G][2].
// Groups are groups[g] = (tau, i), or (tau0 + g / M, g % M) when groups is
// null; q may be null.
__global__ __launch_bounds__(64) void k_group_rows(ModelView m, SceneView s, const float* __restrict__ U,
                                                  long long us, SearchParams sp, const int2* __restrict__ groups,
                                                  int tau0, int32_t* __restrict__ node, float* __restrict__ phi,
                                                  int32_t* __restrict__ q) {
  const long long g = blockIdx.x;
  const int lane = threadIdx.x;
  const int2 gi = groups ? groups[g] : make_int2(tau0 + static_cast<int>(g / m.M), static_cast<int>(g % m.M));
  int n, qa, qb;
  float f[8];
  group_features(m, s, U, us, sp, gi.x, gi.y, lane, n, f, qa, qb);
  const long long r = g * 64 + lane;
  node[r] = n;
  float4* ph = reinterpret_cast<float4*>(phi + r * 8);
  ph[0] = make_float4(f[0], f[1], f[2], f[3]);
  ph[1] = make_float4(f[4], f[5], f[6], f[7]);
  if (q && lane == 0) {
    q[2 * g] = qa;
    q[2 * g + 1] = qb;
  }
}

// ---- FP32 layer kernels ------------------------------------------------------------

// Row loader of the first layer: x = [f_i, g_n, phi, 0...] gathered on the fly.
struct GatherX {
  const float* mdesc;   // [M][D]
  const int2* groups;   // (tau, i) per group
  const float* sdesc;   // [S][D]
  const int32_t* node;  // [rows]
  const float* phi;     // [rows][8]
  int D;
  float scale;          // D, the descriptor input factor
  __device__ __forceinline__ float operator()(long long r, int c) const {
    const int n = node[r];
    if (n < 0) return 0.f;
    if (c < D) return scale * mdesc[(long long)groups[r >> 6].y * D + c];
    if (c < 2 * D) return scale * sdesc[(long long)n * D + (c - D)];
    if (c < 2 * D + 8) return phi[r * 8 + (c - 2 * D)];
    return 0.f;
  }
};

struct PlainX {
  const float* x;
  int ld;
  __device__ __forceinline__ float operator()(long long r, int c) const { return x[r * ld + c]; }
};

// C[r][o] = act(sum_k A(r, k) B(o, k) + bias[o]) for o < 128, with B(o, k) =
// W[o * ldw + k] (TRANS = false) or W[k * ldw + o] (TRANS = true); act = relu
// when `relu`, times [mask[r][o] > 0] when mask is given.  64 rows per block,
// 256 threads, each 4 rows x 8 columns; K in tiles of 16 through LDS.
template <class Loader, bool TRANS>
__global__ __launch_bounds__(256) void k_layer(Loader ld, long long R, int I, const float* __restrict__ W, int ldw,
                                              const float* __restrict__ bias, const float* __restrict__ mask,
                                              int relu, float* __restrict__ C) {
  __shared__ float As[16][64 + 1];
  __shared__ float Bs[16][H + 1];
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  const long long r0 = (long long)blockIdx.x * 64;
  float acc[4][8];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[j][c] = 0.f;
  for (int k0 = 0; k0 < I; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q, row = e >> 4, kk = e & 15;
      As[kk][row] = (r0 + row < R && k0 + kk < I) ? ld(r0 + row, k0 + kk) : 0.f;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + 256 * q, col = e >> 4, kk = e & 15;
      float v = 0.f;
      if (k0 + kk < I) v = TRANS ? W[(long long)(k0 + kk) * ldw + col] : W[(long long)col * ldw + k0 + kk];
      Bs[kk][col] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[8];
#pragma unroll
      for (int j = 0; j < 4; ++j) a[j] = As[kk][tr + 16 * j];
#pragma unroll
      for (int c = 0; c < 8; ++c) b[c] = Bs[kk][tc + 16 * c];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[j][c] = fmaf(a[j], b[c], acc[j][c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const long long r = r0 + tr + 16 * j;
    if (r >= R) continue;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int o = tc + 16 * c;
      float v = acc[j][c] + (bias ? bias[o] : 0.f);
      if (relu) v = fmaxf(v, 0.f);
      if (mask && !(mask[r * H + o] > 0.f)) v = 0.f;
      C[r * H + o] = v;
    }
  }
}

// Weight gradient, partial over a chunk of kWgradRows rows:
// part[chunk][o][c] = sum_{r in chunk} dZ[r][o] X(r, c), o < 128, c < I.
constexpr int kWgradRows = 512;

template <class Loader>
__global__ __launch_bounds__(256) void k_wgrad(const float* __restrict__ dZ, Loader ld, long long R, int I,
                                              float* __restrict__ part) {
  __shared__ float Zs[16][H + 1];
  __shared__ float Xs[16][32 + 1];
  const int tid = threadIdx.x, to = tid >> 3, tcc = tid & 7;  // o = to + 32 j, c = tcc + 8 q
  const int c0 = blockIdx.x * 32;
  const long long rbeg = (long long)blockIdx.y * kWgradRows;
  const long long rend = rbeg + kWgradRows < R ? rbeg + kWgradRows : R;
  float acc[4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[j][q] = 0.f;
  for (long long r0 = rbeg; r0 < rend; r0 += 16) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + 256 * q, rr = e >> 7, o = e & 127;
      Zs[rr][o] = r0 + rr < rend ? dZ[(r0 + rr) * H + o] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = tid + 256 * q, rr = e >> 5, c = e & 31;
      Xs[rr][c] = (r0 + rr < rend && c0 + c < I) ? ld(r0 + rr, c0 + c) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      float z[4], x[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) z[j] = Zs[rr][to + 32 * j];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = Xs[rr][tcc + 8 * q];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[j][q] = fmaf(z[j], x[q], acc[j][q]);
    }
    __syncthreads();
  }
  float* out = part + (long long)blockIdx.y * H * I;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = c0 + tcc + 8 * q;
      if (c < I) out[(long long)(to + 32 * j) * I + c] = acc[j][q];
    }
}

// Column sums, partial over chunks of rows: part[chunk][c] = sum_r s(r) Y[r][c]
// (s = 1 when scale is null).
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ Y, int ncol, long long R,
                                               const float* __restrict__ scale, float* __restrict__ part) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= ncol) return;
  const long long rbeg = (long long)blockIdx.y * kWgradRows;
  const long long rend = rbeg + kWgradRows < R ? rbeg + kWgradRows : R;
  float acc = 0.f;
  for (long long r = rbeg; r < rend; ++r) acc = fmaf(scale ? scale[r] : 1.f, Y[r * ncol + c], acc);
  part[(long long)blockIdx.y * ncol + c] = acc;
}

// out[j] = sum over chunks of part[chunk][j], in chunk order.
__global__ __launch_bounds__(256) void k_reduce_chunks(const float* __restrict__ part, int nchunk, long long n,
                                                      float* __restrict__ out) {
  const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  float acc = 0.f;
  for (int c = 0; c < nchunk; ++c) acc += part[(long long)c * n + j];
  out[j] = acc;
}

// Listwise loss of each group (one 64-lane block): scores s = w3 . h2 + b3,
// softmax over the valid candidates, loss = -log p[label] with label the slot
// of node labels[g]; ds = (p - onehot) / G; dZ2 = ds w3 [h2 > 0].
__global__ __launch_bounds__(64) void k_loss(const float* __restrict__ H2, const float* __restrict__ w3,
                                            const float* __restrict__ b3, const int32_t* __restrict__ node,
                                            const int32_t* __restrict__ labels, int G, float* __restrict__ scores,
                                            float* __restrict__ loss, float* __restrict__ ds,
                                            float* __restrict__ dZ2) {
  const int g = blockIdx.x, lane = threadIdx.x;
  const long long r = (long long)g * 64 + lane;
  const bool valid = node[r] >= 0;
  float s = b3[0];
  for (int k = 0; k < H; ++k) s = fmaf(H2[r * H + k], w3[k], s);
  if (scores) scores[r] = valid ? s : -__builtin_inff();
  if (!labels) return;
  float mx = valid ? s : -__builtin_inff();
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
  const float e = valid ? expf(s - mx) : 0.f;
  float z = e;
  for (int off = 32; off > 0; off >>= 1) z += __shfl_xor(z, off);
  // the label is a node id; its slot is the lane holding it (none: NaN loss, no gradient)
  const unsigned long long hit = __ballot(valid && node[r] == labels[g]);
  const int lab = hit ? __ffsll(static_cast<long long>(hit)) - 1 : -1;
  const float sl = __shfl(s, lab < 0 ? 0 : lab);
  if (lane == 0) loss[g] = lab < 0 ? __builtin_nanf("") : -(sl - mx - logf(z));
  const float d = lab < 0 ? 0.f : ((valid ? e / z : 0.f) - (lane == lab ? 1.f : 0.f)) / static_cast<float>(G);
  ds[r] = d;
  for (int k = 0; k < H; ++k) dZ2[r * H + k] = H2[r * H + k] > 0.f ? d * w3[k] : 0.f;
}

// Adam (Kingma and Ba) on the packed parameters; c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ theta, const float* __restrict__ g,
                                             float* __restrict__ m, float* __restrict__ v, long long n, float lr,
                                             float beta1, float beta2, float eps, float c1, float c2) {
  const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const float gj = g[j];
  const float mj = beta1 * m[j] + (1.f - beta1) * gj;
  const float vj = beta2 * v[j] + (1.f - beta2) * gj * gj;
  m[j] = mj;
  v[j] = vj;
  theta[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}


// ---- BF16 inference ------------------------------------------------------------------

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float x) {
  const uint32_t b = __float_as_uint(x);
  return static_cast<uint16_t>((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}

// out [rows][dp] BF16 of W[o * ld + off + d] (d < D), zero for D <= d < dp.
__global__ void k_cast_rows_bf16(const float* __restrict__ W, int rows, int ld, int off, int D, int dp,
                                 uint16_t* __restrict__ out) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long long)rows * dp) return;
  const int o = static_cast<int>(e / dp), d = static_cast<int>(e % dp);
  out[e] = d < D ? to_bf16(W[(long long)o * ld + off + d]) : 0;
}

// P[n][o] = scale * sum_d X[n][d] Wp[o][d] + bias[o] for o < 128 (bias
// nullable): BF16 inputs on MFMA, FP32 accumulation and output.
// Xb [np][dp] zero-padded to a multiple of 16 rows; one 4-wave block per 16
// rows, each wave 32 output columns (two 16x16 tiles).
__global__ __launch_bounds__(256) void k_project_bf16(const uint16_t* __restrict__ Xb, int n, int dp,
                                                     const uint16_t* __restrict__ Wb, float scale,
                                                     const float* __restrict__ bias, float* __restrict__ P) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int row0 = blockIdx.x * 16, lr = lane & 15, kq = (lane >> 4) * 8;
  f32x4_t acc[2] = {f32x4_t{0.f, 0.f, 0.f, 0.f}, f32x4_t{0.f, 0.f, 0.f, 0.f}};
  for (int k0 = 0; k0 < dp; k0 += 32) {
    const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(Xb + (long long)(row0 + lr) * dp + k0 + kq);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int col = wv * 32 + t * 16 + lr;
      const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(Wb + (long long)col * dp + k0 + kq);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = row0 + (lane >> 4) * 4 + j;
      if (row < n) {
        const int o = wv * 32 + t * 16 + lr;
        P[(long long)row * H + o] = scale * acc[t][j] + (bias ? bias[o] : 0.f);
      }
    }
}

// Inference: one wave per group, no block barriers after the set-up.
//
// Layer 1 runs transposed, Z1^T [hidden k][candidate c], per 16 x 16 tile
// (kt, ct): the accumulator starts at A'_i[k] + B_n[k] (A' = W1a (D f) + b1,
// B = W1b (D g), both from the BF16 projections) and takes W1c phi on
// v_mfma_f32_16x16x4_f32 (K = 8 as two steps, FP32).  Its accumulator layout
// (lane l: k = 16 kt + 4 (l / 16) + j, c = 16 ct + l % 16) is used directly as
// the B operand of layer 2 on v_mfma_f32_16x16x32_bf16: the 32-wide K block p
// takes tiles kt = 2p and 2p + 1, so lane l supplies hidden units
// 32p + 16h + 4 (l / 16) + j (h, j in {0,1} x {0..3}); W2 sits in LDS permuted
// to the same order, so no data moves between the layers.
constexpr int kInferWaves = 8;
constexpr int kW2Row = H + 8;  // bf16 per permuted W2 row (padding against bank conflicts)

struct alignas(16) InferShared {
  uint16_t w2p[H * kW2Row];   // W2 rows o, K order of the MFMA operand
  float b2[H], w3[H];
  float phi[kInferWaves][64][9];  // per wave: features of the 64 slots (+ pad)
  int32_t node[kInferWaves][64];
  unsigned long long key[kInferWaves][64];  // per wave: selection keys of the 64 slots
};

// Selection key of a slot: smaller is kept first.  Frame distance (0 under the
// score rule), then the score descending, then the slot; unique per slot.
__device__ __forceinline__ unsigned long long select_key(int df, float sc, int slot) {
  unsigned int u = __float_as_uint(sc + 0.f);  // -0 counts as +0
  u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);  // order-preserving map of floats to unsigned
  return (static_cast<unsigned long long>(df) << 38) | (static_cast<unsigned long long>(~u) << 6) |
         static_cast<unsigned long long>(slot);
}

// Position of hidden unit u inside a permuted W2 row.
__device__ __forceinline__ int w2_pos(int u) {
  const int p = u >> 5, r = u & 31, h = r >> 4, g = (r & 15) >> 2, j = r & 3;
  return ((p * 4 + g) * 8) + h * 4 + j;
}

__global__ __launch_bounds__(kInferWaves * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_pruner_infer(
    ModelView m, SceneView s, const int32_t* __restrict__ gnode, const float* __restrict__ gphi,
    const int2* __restrict__ groups, long long n_groups, int tau0, const float* __restrict__ theta, int D,
    const float* __restrict__ A, const float* __restrict__ B, int topk, int rule, int32_t* __restrict__ cand,
    int32_t* __restrict__ count, float* __restrict__ scores) {
  __shared__ InferShared sh;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int NI = 2 * D + 8;
  const float* W1 = theta;
  const float* b1 = W1 + (long long)H * NI;
  const float* W2 = b1 + H;
  const float* b2 = W2 + H * H;
  const float* w3 = b2 + H;
  const float b3 = w3[H];
  for (int e = tid; e < H * H; e += kInferWaves * 64) {
    const int o = e >> 7, u = e & 127;
    sh.w2p[o * kW2Row + w2_pos(u)] = __builtin_bit_cast(uint16_t, static_cast<__bf16>(W2[e]));
  }
  for (int e = tid; e < H; e += kInferWaves * 64) {
    sh.b2[e] = b2[e];
    sh.w3[e] = w3[e];
  }
  // layer-1 A operands (W1 phi columns): lane l holds W1c[16 kt + l % 16][l / 16 + 4 h]
  float w1c[8][2];
  const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
  for (int kt = 0; kt < 8; ++kt)
#pragma unroll
    for (int h = 0; h < 2; ++h) w1c[kt][h] = W1[(long long)(16 * kt + lr) * NI + 2 * D + lq + 4 * h];
  __syncthreads();

  float(*phi)[9] = sh.phi[wv];
  int32_t* node = sh.node[wv];
  const long long stride = (long long)gridDim.x * kInferWaves;
  for (long long g = (long long)blockIdx.x * kInferWaves + wv; g < n_groups; g += stride) {
    const int2 gi = groups ? groups[g] : make_int2(tau0 + static_cast<int>(g / m.M), static_cast<int>(g % m.M));
    const int n = gnode[g * 64 + lane];
    {
      const float4* gp = reinterpret_cast<const float4*>(gphi + (g * 64 + lane) * 8);
      const float4 f0 = gp[0], f1 = gp[1];
      node[lane] = n;
      phi[lane][0] = f0.x; phi[lane][1] = f0.y; phi[lane][2] = f0.z; phi[lane][3] = f0.w;
      phi[lane][4] = f1.x; phi[lane][5] = f1.y; phi[lane][6] = f1.z; phi[lane][7] = f1.w;
    }
    // the wave's LDS writes above are read by other lanes of the same wave below
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // A'_i rows for this lane's hidden units: k = 16 kt + 4 lq + j
    float4 arow[8];
#pragma unroll
    for (int kt = 0; kt < 8; ++kt) arow[kt] = *reinterpret_cast<const float4*>(A + (long long)gi.y * H + 16 * kt + 4 * lq);
    float sc = -__builtin_inff();
#pragma unroll 1
    for (int ct = 0; ct < 4; ++ct) {
      const int c = 16 * ct + lr;  // this lane's candidate in the tile
      const int nc = node[c];
      const float p0 = phi[c][lq], p1 = phi[c][lq + 4];
      const float* brow = B + (long long)(nc < 0 ? 0 : nc) * H + 4 * lq;
      bf16x8_t hb[4];
#pragma unroll
      for (int kt = 0; kt < 8; ++kt) {
        const float4 bv = *reinterpret_cast<const float4*>(brow + 16 * kt);
        f32x4_t z = {arow[kt].x + bv.x, arow[kt].y + bv.y, arow[kt].z + bv.z, arow[kt].w + bv.w};
        z = __builtin_amdgcn_mfma_f32_16x16x4f32(w1c[kt][0], p0, z, 0, 0, 0);
        z = __builtin_amdgcn_mfma_f32_16x16x4f32(w1c[kt][1], p1, z, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float hv = nc < 0 ? 0.f : fmaxf(z[j], 0.f);
          hb[kt >> 1][(kt & 1) * 4 + j] = static_cast<__bf16>(hv);  // v_cvt_pk_bf16_f32, nearest even
        }
      }
      float part = 0.f;
#pragma unroll 2
      for (int ot = 0; ot < 8; ++ot) {
        f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
        const uint16_t* wrow = sh.w2p + (16 * ot + lr) * kW2Row + lq * 8;
#pragma unroll
        for (int pb = 0; pb < 4; ++pb) {
          const bf16x8_t wa = *reinterpret_cast<const bf16x8_t*>(wrow + pb * 32);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, hb[pb], acc, 0, 0, 0);
        }
        // rows of acc: output units o = 16 ot + 4 lq + j, column: candidate c
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int o = 16 * ot + 4 * lq + j;
          part = fmaf(fmaxf(acc[j] + sh.b2[o], 0.f), sh.w3[o], part);
        }
      }
      part += __shfl_xor(part, 16);
      part += __shfl_xor(part, 32);
      if (ct == lq) sc = part + b3;  // lane l = 16 ct + l % 16 owns candidate l
    }
    if (n < 0) sc = -__builtin_inff();
    if (scores) scores[g * 64 + lane] = sc;
    // rank: candidates ahead in the selection order.  Score rule: a higher
    // score, or an equal score and a lower slot.  Frames-first rule: a frame
    // nearer the shifted model frame, then the score rule inside a frame.
    // Time-nearest rule: a nearer frame, then the lower slot (the score is
    // not consulted).  Empty slots carry -inf and the largest frame distance:
    // ranked last.
    const int df = n < 0 ? (1 << 25) : abs(s.t[n] - (gi.x + m.t[gi.y] - m.t[0]));
    const unsigned long long key = select_key(rule ? df : (n < 0 ? 1 : 0), rule == 2 ? 0.f : sc, lane);
    sh.key[wv][lane] = key;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int rank = 0;
    const ulonglong2* kk = reinterpret_cast<const ulonglong2*>(sh.key[wv]);
#pragma unroll 8
    for (int j = 0; j < 32; ++j) {
      const ulonglong2 o = kk[j];  // the same address in every lane: a broadcast read
      rank += (o.x < key) + (o.y < key);
    }
    const bool keep = n >= 0 && rank < topk;
    const unsigned long long mask = __ballot(keep);
    const int pos = __popcll(mask & ((1ull << lane) - 1ull));
    if (keep) cand[g * topk + pos] = n;
    if (lane == 0) count[g] = __popcll(mask);
    // every lane has read this group's LDS rows before the next group rewrites them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Rows of the exact re-solve of offsets taus[r] back into the outputs of the
// offset range starting at tau0; fell_back[tau - tau0] = 1.
__global__ __launch_bounds__(64) void k_scatter_fallback(const int32_t* __restrict__ taus, int tau0, int M,
                                                        const float* __restrict__ e32, const double* __restrict__ e64,
                                                        const double* __restrict__ eu, const int32_t* __restrict__ as,
                                                        float* __restrict__ o32, double* __restrict__ o64,
                                                        double* __restrict__ ou, int32_t* __restrict__ oas,
                                                        int32_t* __restrict__ fell) {
  const int r = blockIdx.x, lane = threadIdx.x;
  const long long d = taus[r] - tau0;
  for (int i = lane; i < M; i += 64) oas[d * M + i] = as[(long long)r * M + i];
  if (lane == 0) {
    o32[d] = e32[r];
    if (o64) o64[d] = e64[r];
    if (ou) ou[d] = eu[r];
    if (fell) fell[d] = 1;
  }
}

// Caller-given candidate lists: bad |= 1 for a count outside [0, kc], 2 for a
// node outside [0, S), 4 for a list not strictly ascending.
__global__ __launch_bounds__(256) void k_check_lists(const int32_t* __restrict__ cand,
                                                    const int32_t* __restrict__ count, long long rows, int kc, int S,
                                                    int32_t* __restrict__ bad) {
  const long long r = (long long)blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  const int n = count[r];
  int b = 0;
  if (n < 0 || n > kc) {
    b = 1;
  } else {
    int prev = -1;
    for (int a = 0; a < n; ++a) {
      const int v = cand[r * kc + a];
      if (v < 0 || v >= S) b |= 2;
      else if (v <= prev) b |= 4;
      prev = v;
    }
  }
  if (b) atomicOr(bad, b);
}

inline int blocks(long long n, int per) { return static_cast<int>((n + per - 1) / per); }

}  // namespace

hipError_t launch_group_rows(const ModelView& m, const SceneView& s, const float* U, long long us,
                             const SearchParams& sp, const int2* groups, int tau0, long long G, int32_t* node,
                             float* phi, int32_t* q, hipStream_t st) {
  if (G <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_group_rows, dim3(static_cast<unsigned>(G)), dim3(64), 0, st, m, s, U, us, sp, groups, tau0,
                     node, phi, q);
  return hipGetLastError();
}

hipError_t launch_pruner_train(const PrunerTrain& t, hipStream_t st) {
  const long long R = (long long)t.G * 64;
  const int NI = 2 * t.D + 8;
  const float* W1 = t.theta;
  const float* b1 = W1 + (long long)H * NI;
  const float* W2 = b1 + H;
  const float* b2 = W2 + H * H;
  const float* w3 = b2 + H;
  const float* b3 = w3 + H;
  float* gW1 = t.grad;
  float* gb1 = gW1 + (long long)H * NI;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + H * H;
  float* gw3 = gb2 + H;
  float* gb3 = gw3 + H;
  const GatherX gx{t.mdesc, t.groups, t.sdesc, t.node, t.phi, t.D, static_cast<float>(t.D)};
  const int nb = blocks(R, 64);
  hipLaunchKernelGGL((k_layer<GatherX, false>), dim3(nb), dim3(256), 0, st, gx, R, NI, W1, NI, b1,
                     (const float*)nullptr, 1, t.h1);
  hipLaunchKernelGGL((k_layer<PlainX, false>), dim3(nb), dim3(256), 0, st, PlainX{t.h1, H}, R, H, W2, H, b2,
                     (const float*)nullptr, 1, t.h2);
  hipLaunchKernelGGL(k_loss, dim3(t.G), dim3(64), 0, st, t.h2, w3, b3, t.node, t.labels, t.G, t.scores, t.loss,
                     t.ds, t.dz2);
  if (!t.labels) return hipGetLastError();
  const int nch = blocks(R, kWgradRows);
  // layer 3: dw3 = sum_r ds_r h2_r, db3 = sum_r ds_r
  hipLaunchKernelGGL(k_colsum, dim3(1, nch), dim3(256), 0, st, t.h2, H, R, t.ds, t.part);
  hipLaunchKernelGGL(k_reduce_chunks, dim3(1), dim3(256), 0, st, t.part, nch, (long long)H, gw3);
  hipLaunchKernelGGL(k_colsum, dim3(1, nch), dim3(256), 0, st, t.ds, 1, R, (const float*)nullptr, t.part);
  hipLaunchKernelGGL(k_reduce_chunks, dim3(1), dim3(256), 0, st, t.part, nch, 1LL, gb3);
  // layer 2: dW2 = dZ2^T h1, db2 = colsum dZ2, dZ1 = (dZ2 W2) [h1 > 0]
  hipLaunchKernelGGL(k_wgrad<PlainX>, dim3(H / 32, nch), dim3(256), 0, st, t.dz2, PlainX{t.h1, H}, R, H, t.part);
  hipLaunchKernelGGL(k_reduce_chunks, dim3(blocks((long long)H * H, 256)), dim3(256), 0, st, t.part, nch,
                     (long long)H * H, gW2);
  hipLaunchKernelGGL(k_colsum, dim3(1, nch), dim3(256), 0, st, t.dz2, H, R, (const float*)nullptr, t.part);
  hipLaunchKernelGGL(k_reduce_chunks, dim3(1), dim3(256), 0, st, t.part, nch, (long long)H, gb2);
  hipLaunchKernelGGL((k_layer<PlainX, true>), dim3(nb), dim3(256), 0, st, PlainX{t.dz2, H}, R, H, W2, H,
                     (const float*)nullptr, t.h1, 0, t.dz1);
  // layer 1: dW1 = dZ1^T X, db1 = colsum dZ1
  hipLaunchKernelGGL(k_wgrad<GatherX>, dim3(blocks(NI, 32), nch), dim3(256), 0, st, t.dz1, gx, R, NI, t.part);
  hipLaunchKernelGGL(k_reduce_chunks, dim3(blocks((long long)H * NI, 256)), dim3(256), 0, st, t.part, nch,
                     (long long)H * NI, gW1);
  hipLaunchKernelGGL(k_colsum, dim3(1, nch), dim3(256), 0, st, t.dz1, H, R, (const float*)nullptr, t.part);
  hipLaunchKernelGGL(k_reduce_chunks, dim3(1), dim3(256), 0, st, t.part, nch, (long long)H, gb1);
  return hipGetLastError();
}

long long pruner_part_floats(int G, int D) {
  const long long R = (long long)G * 64;
  const long long nch = (R + kWgradRows - 1) / kWgradRows;
  return nch * (long long)H * (2 * D + 8 > H ? 2 * D + 8 : H);
}

hipError_t launch_adam(float* theta, const float* g, float* m, float* v, long long n, float lr, float beta1,
                       float beta2, float eps, float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(blocks(n, 256)), dim3(256), 0, st, theta, g, m, v, n, lr, beta1, beta2, eps, c1,
                     c2);
  return hipGetLastError();
}

hipError_t launch_cast_rows_bf16(const float* W, int rows, int ld, int off, int D, int dp, uint16_t* out,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_cast_rows_bf16, dim3(blocks((long long)rows * dp, 256)), dim3(256), 0, st, W, rows, ld, off,
                     D, dp, out);
  return hipGetLastError();
}

hipError_t launch_project_bf16(const uint16_t* Xb, int n, int dp, const uint16_t* Wb, float scale,
                               const float* bias, float* P, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_project_bf16, dim3(blocks(n, 16)), dim3(256), 0, st, Xb, n, dp, Wb, scale, bias, P);
  return hipGetLastError();
}

hipError_t launch_pruner_infer(const PrunerInfer& q, hipStream_t st) {
  if (q.n_groups <= 0) return hipSuccess;
  int n_cu = 256, dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  const long long want = (q.n_groups + kInferWaves - 1) / kInferWaves;
  const long long grid = want < (long long)n_cu * 2 ? want : (long long)n_cu * 2;
  hipError_t e = launch_group_rows(q.m, q.s, q.U, q.us, q.sp, q.groups, q.tau0, q.n_groups, q.node, q.phi, nullptr,
                                  st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pruner_infer, dim3(static_cast<unsigned>(grid)), dim3(kInferWaves * 64), 0, st, q.m, q.s,
                     q.node, q.phi, q.groups, q.n_groups, q.tau0, q.theta, q.D, q.A, q.B, q.topk, q.rule, q.cand,
                     q.count, q.scores);
  return hipGetLastError();
}

hipError_t launch_scatter_fallback(const int32_t* taus, int n, int tau0, int M, const float* e32, const double* e64,
                                  const double* eu, const int32_t* as, float* o32, double* o64, double* ou,
                                  int32_t* oas, int32_t* fell, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_fallback, dim3(n), dim3(64), 0, st, taus, tau0, M, e32, e64, eu, as, o32, o64, ou,
                     oas, fell);
  return hipGetLastError();
}

hipError_t launch_check_lists(const int32_t* cand, const int32_t* count, long long rows, int kc, int S, int32_t* bad,
                              hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_lists, dim3(blocks(rows, 256)), dim3(256), 0, st, cand, count, rows, kc, S, bad);
  return hipGetLastError();
}

}  // namespace stm
