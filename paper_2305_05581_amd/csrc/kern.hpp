// Device helpers shared by the kernels of the library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

namespace tns {

// Element-wise kernels walk their array with a grid stride: operator arrays
// exceed the 2^32 work items that one dispatch can address.
#define GRID_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// --- BF16 split: round to nearest even, NaN kept quiet --------------------
__host__ __device__ inline uint16_t f32_to_bf16_rne(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float x;
  memcpy(&x, &u, 4);
  return x;
}

// BF16X3 operand arrays keep each element as a high and a low BF16 half,
// interleaved in groups of 8 elements: the 8 high halves of a group, then its
// 8 low halves.  Element e's high half sits at u16 index bfx_hi(e), its low
// half 8 further; an aligned run of 32 elements (a row step of the ring) is
// 128 contiguous bytes.
__host__ __device__ inline int64_t bfx_hi(int64_t e) { return 2 * e - (e & 7); }

// --- MFMA wrappers ------------------------------------------------------------
// 16 x 16 output tile; lane l supplies A[l % 16][k-slot l / 16] and
// B[k-slot l / 16][l % 16].  Element v (0..3) of lane l's accumulator is
// D[mrow(l / 16, v)][l % 16]: rows 4 (l / 16) + v for the FP32 and BF16
// instructions, rows l / 16 + 4 v for the FP64 one.
__device__ inline d4 mfma(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline f4 mfma(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
// BF16: lane l supplies 8 consecutive k of row (column) l % 16, k-group l / 16.
__device__ inline f4 mfma_bf(u16x8 a, u16x8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0,
                                                 0);
}

__device__ inline int mrow(d4, int lg, int v) { return lg + 4 * v; }
__device__ inline int mrow(f4, int lg, int v) { return 4 * lg + v; }

template <class T> __device__ inline T vzero();
template <> __device__ inline d4 vzero<d4>() { return d4{0.0, 0.0, 0.0, 0.0}; }
template <> __device__ inline f4 vzero<f4>() { return f4{0.f, 0.f, 0.f, 0.f}; }

}  // namespace tns
