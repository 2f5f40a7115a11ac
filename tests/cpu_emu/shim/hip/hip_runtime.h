// CPU build of the library's HIP sources (a test tool, not a product path).
//
// Supplies, for an ordinary host compiler, the parts of the HIP device language and of the
// HIP runtime that the library uses.  A kernel launch runs synchronously on the calling
// thread: the blocks of the grid one after another, the threads of a block as cooperative
// fibers that switch at barriers (__syncthreads) and at cross-lane exchanges (__shfl_xor).
// Device memory is host memory.  Built with AddressSanitizer, every out-of-bounds access of
// a kernel or of the host code becomes a report that names the access.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <functional>
#include <type_traits>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline __attribute__((always_inline))
#define __launch_bounds__(...)
// register-budget hints of kernels mean nothing on the host (the attribute list is left empty)
#define amdgpu_waves_per_eu(...)
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) (&(x))

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned x_ = 1, unsigned y_ = 1, unsigned z_ = 1) : x(x_), y(y_), z(z_) {}
};
struct uint3_emu { unsigned x, y, z; };

namespace emu {
extern uint3_emu thread_idx, block_idx, block_dim, grid_dim;
void syncthreads();
void launch(dim3 grid, dim3 block, const std::function<void()>& body);
// exchange slot of the calling thread (8 bytes per thread of the block)
unsigned long long* xchg_slots();
}  // namespace emu

#define threadIdx (::emu::thread_idx)
#define blockIdx (::emu::block_idx)
#define blockDim (::emu::block_dim)
#define gridDim (::emu::grid_dim)

inline void __syncthreads() { ::emu::syncthreads(); }
// lane 0's value of a wave-uniform operand (every lane holds the same value where it is used)
inline int __builtin_amdgcn_readfirstlane(int v) { return v; }
inline unsigned __builtin_amdgcn_readfirstlane(unsigned v) { return v; }
#define __builtin_amdgcn_s_waitcnt(x) ((void)(x))

template <class T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  static_assert(sizeof(T) <= 8, "exchange of at most 8 bytes");
  unsigned long long* slot = ::emu::xchg_slots();
  const unsigned tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  unsigned long long bits = 0;
  std::memcpy(&bits, &v, sizeof(T));
  slot[tid] = bits;
  __syncthreads();
  const unsigned src = (tid & ~(unsigned)(width - 1)) | ((tid & (unsigned)(width - 1)) ^ (unsigned)mask);
  bits = slot[src];
  __syncthreads();
  T r;
  std::memcpy(&r, &bits, sizeof(T));
  return r;
}

template <class A, class B>
inline auto min(A a, B b) -> std::common_type_t<A, B> {
  using C = std::common_type_t<A, B>;
  return (C)a < (C)b ? (C)a : (C)b;
}
template <class A, class B>
inline auto max(A a, B b) -> std::common_type_t<A, B> {
  using C = std::common_type_t<A, B>;
  return (C)a < (C)b ? (C)b : (C)a;
}

inline unsigned __float_as_uint(float f) { unsigned u; std::memcpy(&u, &f, 4); return u; }
inline float __uint_as_float(unsigned u) { float f; std::memcpy(&f, &u, 4); return f; }
inline unsigned atomicMax(unsigned* p, unsigned v) { const unsigned o = *p; if (v > o) *p = v; return o; }
inline int atomicMax(int* p, int v) { const int o = *p; if (v > o) *p = v; return o; }
inline unsigned atomicAdd(unsigned* p, unsigned v) { const unsigned o = *p; *p = o + v; return o; }
inline double atomicAdd(double* p, double v) { const double o = *p; *p = o + v; return o; }
inline float atomicAdd(float* p, float v) { const float o = *p; *p = o + v; return o; }
inline unsigned long long atomicAdd(unsigned long long* p, unsigned long long v) { const unsigned long long o = *p; *p = o + v; return o; }

struct uint4 { unsigned x, y, z, w; };
inline uint4 make_uint4(unsigned x, unsigned y, unsigned z, unsigned w) { return {x, y, z, w}; }

// ---------------------------------------------------------------- buffer resources
// A raw buffer resource: base and size in bytes.  An access whose byte offset (per-lane plus
// uniform part, summed without wrapping) reaches past the size loads 0 and stores nothing; a
// sum that would wrap 32 bits is reported, since the hardware's 32-bit sum would then differ.
struct __amdgpu_buffer_rsrc_t {
  char* base;
  unsigned bytes;
};
namespace emu {
char* buffer_at(const __amdgpu_buffer_rsrc_t& r, int voff, int soff, unsigned size);
}
inline __amdgpu_buffer_rsrc_t __builtin_amdgcn_make_buffer_rsrc(void* p, short stride, int bytes, int flags) {
  (void)stride;
  (void)flags;
  return {static_cast<char*>(p), (unsigned)bytes};
}
inline unsigned __builtin_amdgcn_raw_buffer_load_b32(__amdgpu_buffer_rsrc_t r, int voff, int soff, int aux) {
  (void)aux;
  unsigned v = 0;
  if (char* p = ::emu::buffer_at(r, voff, soff, 4)) std::memcpy(&v, p, 4);
  return v;
}
inline unsigned short __builtin_amdgcn_raw_buffer_load_b16(__amdgpu_buffer_rsrc_t r, int voff, int soff, int aux) {
  (void)aux;
  unsigned short v = 0;
  if (char* p = ::emu::buffer_at(r, voff, soff, 2)) std::memcpy(&v, p, 2);
  return v;
}
typedef unsigned emu_u32x2 __attribute__((ext_vector_type(2)));
inline emu_u32x2 __builtin_amdgcn_raw_buffer_load_b64(__amdgpu_buffer_rsrc_t r, int voff, int soff, int aux) {
  (void)aux;
  emu_u32x2 v = {0u, 0u};
  if (char* p = ::emu::buffer_at(r, voff, soff, 8)) std::memcpy(&v, p, 8);
  return v;
}
inline void __builtin_amdgcn_raw_buffer_store_b32(unsigned v, __amdgpu_buffer_rsrc_t r, int voff, int soff, int aux) {
  (void)aux;
  if (char* p = ::emu::buffer_at(r, voff, soff, 4)) std::memcpy(p, &v, 4);
}
inline void __builtin_amdgcn_raw_buffer_store_b16(unsigned short v, __amdgpu_buffer_rsrc_t r, int voff, int soff, int aux) {
  (void)aux;
  if (char* p = ::emu::buffer_at(r, voff, soff, 2)) std::memcpy(p, &v, 2);
}
inline void __builtin_amdgcn_raw_buffer_store_b64(emu_u32x2 v, __amdgpu_buffer_rsrc_t r, int voff, int soff, int aux) {
  (void)aux;
  if (char* p = ::emu::buffer_at(r, voff, soff, 8)) std::memcpy(p, &v, 8);
}

// ---------------------------------------------------------------- runtime
typedef int hipError_t;
enum : int { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorMemoryAllocation = 2,
             hipErrorInvalidSymbol = 13, hipErrorNotSupported = 801 };
typedef struct emu_stream* hipStream_t;
typedef struct emu_event* hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
                     hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 };
struct hipDeviceProp_t { char name[256]; char gcnArchName[256]; size_t totalGlobalMem; int multiProcessorCount; };

hipError_t hipMalloc(void** p, size_t n);
template <class T> inline hipError_t hipMalloc(T** p, size_t n) { return hipMalloc((void**)p, n); }
hipError_t hipFree(void* p);
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st);
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st);
hipError_t hipMemGetInfo(size_t* free_b, size_t* total_b);
hipError_t hipGetDevice(int* dev);
hipError_t hipSetDevice(int dev);
hipError_t hipGetDeviceCount(int* n);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int dev);
hipError_t hipGetSymbolAddress(void** p, const void* sym);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipDeviceSynchronize();
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
