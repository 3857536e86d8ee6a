// Device-side helpers shared by the FCTN kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fctn {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kWave = 64;

// 16x16 output tile owned by one wave: lane l, register i holds element
// (row(l, i), col l%16) of the tile, with row(l, i) = 4*(l/16) + i for the
// float forms and 4*i + l/16 for the double form.  A-operand lane l carries
// (row l%16, k l/16); B-operand lane l carries (k l/16, col l%16).
template <typename Acc> struct Mfma;

template <> struct Mfma<float> {
  typedef f32x4 acc_t;
  static constexpr int kStep = 4;  // k consumed per instruction
  __device__ static inline acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

template <> struct Mfma<double> {
  typedef f64x4 acc_t;
  static constexpr int kStep = 4;
  __device__ static inline acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int i) { return 4 * i + (lane >> 4); }
};

// bf16 x bf16 -> f32, k = 32 per instruction: lane l carries 8 consecutive
// k values 8*(l/16) .. 8*(l/16)+7 of row (A) or column (B) l%16.
struct MfmaBf16 {
  typedef f32x4 acc_t;
  static constexpr int kStep = 32;
  __device__ static inline acc_t mma(bf16x8 a, bf16x8 b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

// Round-to-nearest-even float -> bf16 bits (finite inputs).
__device__ __host__ inline uint16_t bf16_bits_rne(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
__device__ __host__ inline float bf16_bits_to_float(uint16_t h) {
  return __builtin_bit_cast(float, ((uint32_t)h) << 16);
}

// Wave-wide sum of a double (all 64 lanes take part).
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Value of a double held by lane `src` (wave-uniform src), via two readlanes.
__device__ inline double bcast_lane(double v, int src) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Value held by lane G of each group of four lanes, for every lane of the
// group (DPP quad permutation; G is a compile-time constant).
template <int G>
__device__ inline double quad_bcast(double v) {
  constexpr int ctrl = G * 0x55;  // quad_perm [G, G, G, G]
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, ctrl, 0xF, 0xF, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), ctrl, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ inline double quad_bcast(double v, int g) {
  switch (g) {
    case 0: return quad_bcast<0>(v);
    case 1: return quad_bcast<1>(v);
    case 2: return quad_bcast<2>(v);
    default: return quad_bcast<3>(v);
  }
}

// 1/sqrt(d) for d > 0: hardware estimate refined by two Newton steps
// (quadratic convergence to full double precision).
__device__ inline double rsqrt_f64(double d) {
  double y = __builtin_amdgcn_rsq(d);
  y = y * (1.5 - 0.5 * d * y * y);
  y = y * (1.5 - 0.5 * d * y * y);
  return y;
}

// 1/d for d > 0: hardware estimate refined by two Newton steps.
__device__ inline double rcp_f64(double d) {
  double y = __builtin_amdgcn_rcp(d);
  y = fma(y, fma(-d, y, 1.0), y);
  y = fma(y, fma(-d, y, 1.0), y);
  return y;
}

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace fctn
