// Split-precision unary table: U[i][n] = sqrt(max(|f_i|^2 + |g_n|^2 - 2 f_i . g_n, 0))
// with descriptors rounded to BF16 (Eq. 2 expanded; Section 3.3's look-up
// table).  The dot products run on MFMA (BF16 inputs, FP32 accumulation), the
// squared norms are taken in FP32 from the same BF16-rounded vectors, and the
// descriptor length is zero-padded to a multiple of 32 (162 -> 192).
#include "stm_internal.h"

namespace stm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bf16 bits, round to nearest even (inputs are finite).
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  const uint32_t b = __float_as_uint(x);
  return static_cast<uint16_t>((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

// out [np][dp] BF16 (zero rows n >= n_valid, zero columns d >= dim), norm2[n] =
// sum of squares of the rounded row in FP32, index order.  One thread per row.
__global__ void k_to_bf16(const float* __restrict__ x, int32_t n_valid, int32_t dim, int32_t np,
                          int32_t dp, uint16_t* __restrict__ out, float* __restrict__ norm2) {
  const int32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= np) return;
  uint16_t* row = out + (long long)n * dp;
  float acc = 0.f;
  for (int32_t d = 0; d < dp; ++d) {
    uint16_t h = 0;
    if (n < n_valid && d < dim) h = bf16_bits(x[(long long)n * dim + d]);
    row[d] = h;
    const float v = bf16_value(h);
    acc = fmaf(v, v, acc);
  }
  norm2[n] = acc;
}

// One wave computes a 16 (model rows) x 64 (scene points) block with four
// 16x16 MFMA tiles; K runs over dp in steps of 32.  Operand layout of
// v_mfma_f32_16x16x32_bf16: lane l holds row (l % 16) of A and column (l % 16)
// of B at k = 8 (l / 16) .. 8 (l / 16) + 7 of the step; the accumulator holds
// rows 4 (l / 16) + j, j = 0..3, of column l % 16.
constexpr int kWavesPerBlock = 4;

__global__ __launch_bounds__(kWavesPerBlock * 64) void k_unary_bf16(
    const uint16_t* __restrict__ fb, const float* __restrict__ fn, int32_t M,
    const uint16_t* __restrict__ gb, const float* __restrict__ gn, int32_t S, int32_t dp,
    float* __restrict__ U) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int row0 = blockIdx.y * 16;
  const int col0 = (blockIdx.x * kWavesPerBlock + wv) * 64;
  const int lr = lane & 15, kq = (lane >> 4) * 8;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* arow = fb + (long long)(row0 + lr) * dp + kq;
  for (int k0 = 0; k0 < dp; k0 += 32) {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(arow + k0);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(gb + (long long)(col0 + t * 16 + lr) * dp + kq + k0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int col = col0 + t * 16 + lr;
    const float g2 = gn[col];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = row0 + (lane >> 4) * 4 + j;
      const float d2 = fn[row] + g2 - 2.f * acc[t][j];
      if (row < M && col < S) U[(long long)row * S + col] = __builtin_sqrtf(fmaxf(d2, 0.f));
    }
  }
}

}  // namespace

int32_t bf16_padded_dim(int32_t dim) { return (dim + 31) / 32 * 32; }

hipError_t launch_to_bf16(const float* x, int32_t n_valid, int32_t dim, int32_t np, uint16_t* out,
                          float* norm2, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3((np + 127) / 128), dim3(128), 0, st, x, n_valid, dim, np,
                     bf16_padded_dim(dim), out, norm2);
  return hipGetLastError();
}

hipError_t launch_unary_bf16(const uint16_t* fb, const float* fn, int32_t M, const uint16_t* gb,
                             const float* gn, int32_t S, int32_t dim, float* U, hipStream_t st) {
  const int32_t cols_per_block = kWavesPerBlock * 64;
  dim3 grid((S + cols_per_block - 1) / cols_per_block, (M + 15) / 16);
  hipLaunchKernelGGL(k_unary_bf16, grid, dim3(kWavesPerBlock * 64), 0, st, fb, fn, M, gb, gn, S,
                     bf16_padded_dim(dim), U);
  return hipGetLastError();
}

}  // namespace stm
