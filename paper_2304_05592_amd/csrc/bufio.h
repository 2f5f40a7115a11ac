// Buffer-resource loads and stores for the step kernels (gfx950 raw buffer instructions).
//
// A field is read through a 128-bit buffer resource (base address and size in bytes, held in
// scalar registers) with a 32-bit per-lane byte offset plus a wave-uniform byte offset.  The
// hardware checks every access against the size: an access past it loads 0 and stores
// nothing, and sends no memory request.  The kernels use this in two ways:
//   * a lane whose point lies outside the grid passes the offset kOOB (past every field, which
//     is smaller than 2 GiB), so its loads read 0 and its stores are dropped;
//   * a plane (3D) or row (2D) outside the grid, or a whole level that is zero by definition,
//     is read through a resource of size 0.
// Offsets are 32-bit and mostly loop-invariant per lane, so no 64-bit address arithmetic,
// clamping or masking is spent per access.
#pragma once

#include <hip/hip_runtime.h>

namespace awe {

typedef __amdgpu_buffer_rsrc_t brsrc;

// Word 3 of a raw (unswizzled, 32-bit data format) buffer resource on gfx9-class GPUs.
constexpr int kBufWord3 = 0x00020000;
// Per-lane offset of a point outside the grid: 2^31, past every field (at most 2^30 bytes, see
// Planes) also after a wave-uniform offset of at most 2^30 is added (no 32-bit wrap).
constexpr int kOOB = (int)0x80000000u;
// Cache policy bit of the instructions: nontemporal (streamed once).
constexpr int kNT = 2;

// Index of the calling thread's wave in its workgroup, as a wave-uniform (scalar) value: row
// offsets derived from it then stay in scalar registers, as the buffer instructions need.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

__device__ __forceinline__ brsrc make_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, bytes, kBufWord3);
}

// The same for a base and size that are wave-uniform although the compiler cannot prove it: a
// resource it takes for divergent makes every access loop over the lanes' distinct resources.
__device__ __forceinline__ brsrc make_rsrc_uniform(const void* base, int bytes) {
  const unsigned long long b = reinterpret_cast<unsigned long long>(base);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b), hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return make_rsrc(reinterpret_cast<const void*>(((unsigned long long)hi << 32) | lo), __builtin_amdgcn_readfirstlane(bytes));
}

__device__ __forceinline__ float ldb(brsrc r, int voff, int soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ float ldb_nt(brsrc r, int voff, int soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, kNT));
}
__device__ __forceinline__ unsigned short ldb16_nt(brsrc r, int voff, int soff) {
  return __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, kNT);
}
__device__ __forceinline__ double ldb64(brsrc r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

__device__ __forceinline__ void stb(brsrc r, float v, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
}
__device__ __forceinline__ void stb_nt(brsrc r, float v, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, kNT);
}
__device__ __forceinline__ void stb16_nt(brsrc r, unsigned short v, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b16(v, r, voff, soff, kNT);
}
__device__ __forceinline__ double ldb64_nt(brsrc r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, kNT));
}
__device__ __forceinline__ void stb64_nt(brsrc r, double v, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v),
                                        r, voff, soff, kNT);
}
__device__ __forceinline__ void stb64(brsrc r, double v, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v),
                                        r, voff, soff, 0);
}

// A field read slice by slice along its slowest axis (x-y planes in 3D, rows in 2D): slice z
// lies at byte offset z * plane of the resource r (the whole field, at most kMaxField bytes);
// slices outside [0, nzv) read as zero, nzv = 0 for a level that is zero by definition.  Such a
// slice gets the wave-uniform offset kZOOB, which puts every lane past the field (a lane offset
// below 2^30 plus 2^30, or kOOB plus 2^30, stays below 2^32), so the resource and the lane
// offsets stay the same for every slice.
constexpr int kZOOB = 1 << 30;
constexpr long long kMaxField = 1LL << 30;

struct Planes {
  brsrc r;
  int plane, nzv;
};

__device__ __forceinline__ Planes planes(const void* base, int nz, int nzv, long long plane_bytes) {
  return Planes{make_rsrc(base, (int)(nz * plane_bytes)), (int)plane_bytes, nzv};
}

__device__ __forceinline__ int slice_off(const Planes& f, int z) {
  return (unsigned)z < (unsigned)f.nzv ? z * f.plane : kZOOB;
}
__device__ __forceinline__ float ldp(const Planes& f, int voff, int z) { return ldb(f.r, voff, slice_off(f, z)); }
__device__ __forceinline__ float ldp_nt(const Planes& f, int voff, int z) {
  return ldb_nt(f.r, voff, slice_off(f, z));
}
__device__ __forceinline__ unsigned short ldp16_nt(const Planes& f, int voff, int z) {
  return ldb16_nt(f.r, voff, slice_off(f, z));
}
__device__ __forceinline__ double ldp64(const Planes& f, int voff, int z) { return ldb64(f.r, voff, slice_off(f, z)); }
__device__ __forceinline__ double ldp64_nt(const Planes& f, int voff, int z) {
  return ldb64_nt(f.r, voff, slice_off(f, z));
}
// Any point of the field by its own full offset (kOOB when it lies outside the grid); the whole
// field reads as zero when nzv = 0.
__device__ __forceinline__ float ldp_at(const Planes& f, int off) {
  return ldb(f.r, off, f.nzv > 0 ? 0 : kZOOB);
}

// Byte offset of column (x, y) within a plane of row pitch px for elements of esz bytes, or
// kOOB when (x, y) lies outside the nx x ny grid (in 2D: y = 0, ny = 1).
__device__ __forceinline__ int col_off(int x, int y, int nx, int ny, int px, int esz) {
  return ((unsigned)x < (unsigned)nx && (unsigned)y < (unsigned)ny) ? (y * px + x) * esz : kOOB;
}

}  // namespace awe
