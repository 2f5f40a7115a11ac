// 16-bit storage of a wavefield level with a per-level scale s = max |u|: stored value
// RNE(u / s) as bfloat16 or IEEE half (subnormals kept); decoded as value * s.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace awe {

__device__ __forceinline__ unsigned short enc16(float y, int bf16) {
  return bf16 ? __bfloat16_as_ushort(__float2bfloat16(y)) : __half_as_ushort(__float2half_rn(y));
}

__device__ __forceinline__ float dec16(unsigned short b, int bf16) {
  return bf16 ? __uint_as_float(((unsigned)b) << 16) : __half2float(__ushort_as_half(b));
}

// 1 / s for encoding; 0 when the level is identically zero (its codes are then 0).
__device__ __forceinline__ float inv_scale(float s) { return s > 0.f ? 1.f / s : 0.f; }

// Max over the 64 lanes of a wave (all lanes must call).
__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

}  // namespace awe
