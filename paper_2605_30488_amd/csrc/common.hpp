// Device-side building blocks shared by the HIP kernels of the dense Sim(3) back-end (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/ds3.h"

namespace ds3 {

constexpr int kWave = 64;

// --------------------------------------------------------------------------------------------------
// xyzc arena access: float4 (16 B) or 4 x bfloat16 (8 B) per pixel
// --------------------------------------------------------------------------------------------------
template <int DT>
struct Px;

template <>
struct Px<DS3_F32> {
  static constexpr int bytes = 16;
  using raw_t = float4;
  __device__ static inline float4 load(const void* base, int64_t px) {
    return reinterpret_cast<const float4*>(base)[px];
  }
  __device__ static inline raw_t load_raw(const void* base, int64_t px) {
    return reinterpret_cast<const float4*>(base)[px];
  }
  __device__ static inline float4 unpack(raw_t r) { return r; }
  __device__ static inline float conf(const void* base, int64_t px) {
    return reinterpret_cast<const float*>(base)[4 * px + 3];
  }
};

__device__ inline float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

template <>
struct Px<DS3_BF16> {
  static constexpr int bytes = 8;
  using raw_t = uint2;
  __device__ static inline float4 load(const void* base, int64_t px) {
    uint2 w = reinterpret_cast<const uint2*>(base)[px];
    return make_float4(bf16_lo(w.x), bf16_hi(w.x), bf16_lo(w.y), bf16_hi(w.y));
  }
  __device__ static inline raw_t load_raw(const void* base, int64_t px) {
    return reinterpret_cast<const uint2*>(base)[px];
  }
  __device__ static inline float4 unpack(raw_t w) {
    return make_float4(bf16_lo(w.x), bf16_hi(w.x), bf16_lo(w.y), bf16_hi(w.y));
  }
  __device__ static inline float conf(const void* base, int64_t px) {
    return bf16_hi(reinterpret_cast<const uint32_t*>(base)[2 * px + 1]);
  }
};

// Round-to-nearest-even float32 -> bfloat16 bits; NaN stays a quiet NaN.
__device__ inline uint32_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// --------------------------------------------------------------------------------------------------
// Wave reductions (64 lanes)
// --------------------------------------------------------------------------------------------------
__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sum over the 64 lanes with DPP moves (cross-lane operands of ordinary VALU adds, no LDS round trip):
// pairs and quads (quad_perm), rows of 16 (row_shr 4 and 8), then row 15 broadcast into rows 1 and 3 and
// lane 31 into rows 2 and 3; the total ends in lane 63 (the other lanes hold partial sums). Sources outside
// a row or in a masked row contribute 0 (bound_ctrl, old = 0).
__device__ inline float wave_sum_to_lane63(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xb1, 0xf, 0xf, true));   // quad_perm [1,0,3,2]
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4e, 0xf, 0xf, true));   // quad_perm [2,3,0,1]
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, true));  // row_shr:4
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, true));  // row_shr:8
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xa, 0xf, true));  // row_bcast:15
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xc, 0xf, true));  // row_bcast:31
  return v;
}

__device__ inline int wave_sum(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline bool finite3(float a, float b, float c) {
  return isfinite(a) && isfinite(b) && isfinite(c);
}

}  // namespace ds3
