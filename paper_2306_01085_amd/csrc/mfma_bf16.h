// bfloat16 conversion and the 32x32x8 bf16 MFMA tile used by the network kernels and
// the BF16 J(u)v element pass (v_mfma_f32_32x32x8 bf16 with FP32 accumulators).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

namespace dg {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

// float -> bfloat16, round to nearest even (inf and nan kept)
__host__ __device__ inline uint16_t f2bf(float f) {
  uint32_t b;
  memcpy(&b, &f, 4);
  if ((b & 0x7f800000u) == 0x7f800000u) return (uint16_t)(b >> 16);
  const uint32_t lsb = (b >> 16) & 1u;
  b += 0x7fffu + lsb;
  return (uint16_t)(b >> 16);
}
__host__ __device__ inline float bf2f(uint16_t h) {
  uint32_t b = ((uint32_t)h) << 16;
  float f;
  memcpy(&f, &b, 4);
  return f;
}

// one 32x32 tile: acc += A(32 x K, rows of a_ld) * B^T (B: 32 x K, rows of b_ld), all bf16.
// Lane layout: A row = lane % 32, k = 4 (lane / 32) + v (v = 0..3); B likewise with its
// row = output column; acc[a] holds output row (a / 4) * 8 + (lane / 32) * 4 + a % 4,
// column lane % 32. K, a_ld and b_ld are multiples of 8 and A, B are 16-byte aligned,
// so each lane's four k-consecutive operands are one 8-byte load.
__device__ inline void mfma_tile_lds_global(v16f& acc, const uint16_t* A, int a_ld, const uint16_t* B, int b_ld, int K) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 31, kq = (lane >> 5) * 4;
  for (int k0 = 0; k0 < K; k0 += 8) {
    const v4s a = *reinterpret_cast<const v4s*>(A + r * a_ld + k0 + kq);
    const v4s b = *reinterpret_cast<const v4s*>(B + r * b_ld + k0 + kq);
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
  }
}

__device__ inline int mfma_out_row(int a) { return (a / 4) * 8 + ((threadIdx.x & 63) >> 5) * 4 + (a % 4); }

}  // namespace dg
