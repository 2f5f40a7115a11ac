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

// The scale of a FULL-stored level is kept as kScaleSlots partial maxima (one per XCD,
// chosen by the workgroup id), so the per-workgroup atomic maxima of one level do not all
// serialise on one address; readers take the max of the slots.
constexpr int kScaleSlots = 8;

__device__ __forceinline__ float level_scale(const float* scl, int level) {
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < kScaleSlots; ++i) s = fmaxf(s, scl[level * kScaleSlots + i]);
  return s;
}

// Max over the workgroup (all threads must call; uses one small LDS array), then one atomic
// max on the float bits (exact and order independent for non-negative values) into the
// workgroup's slot of this level.
__device__ __forceinline__ void block_max_to_slot(float v, float* scl, int level) {
  __shared__ float red[16];
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, red[w]);
    atomicMax(reinterpret_cast<unsigned*>(scl) + level * kScaleSlots + (blockIdx.x & (kScaleSlots - 1)),
              __float_as_uint(m));
  }
}

}  // namespace awe
