// CPU build of the library's HIP sources (a test tool): kernel launches, fibers, memory.
//
// A launch runs the blocks of the grid in order (or in reverse order when EMU_REVERSE_BLOCKS
// is set, to expose a dependence between blocks of one launch).  The threads of a block are
// fibers run one after another until each reaches a barrier or returns; when every live
// fiber waits at the barrier, all are released (threads that returned no longer take part,
// as waves that ended do not on the GPU).  Fibers switch with a small x86-64 routine that
// saves the callee-saved registers and the floating-point control words (no system call).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#include <sanitizer/asan_interface.h>
#include <sanitizer/common_interface_defs.h>
#define EMU_ASAN 1
#endif
#endif

namespace emu {

uint3_emu thread_idx{0, 0, 0}, block_idx{0, 0, 0}, block_dim{1, 1, 1}, grid_dim{1, 1, 1};

// switch stacks: save callee-saved state on the current stack, store its pointer in *save,
// continue on the stack `load` (x86-64 System V)
extern "C" void emu_ctx_switch(void** save, void* load);
asm(R"(
  .text
  .globl emu_ctx_switch
  .type emu_ctx_switch,@function
emu_ctx_switch:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  subq $8, %rsp
  stmxcsr (%rsp)
  fnstcw 4(%rsp)
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  ldmxcsr (%rsp)
  fldcw 4(%rsp)
  addq $8, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
  .size emu_ctx_switch, .-emu_ctx_switch
)");

namespace {

constexpr size_t kStack = 256 * 1024;

struct Fiber {
  void* sp = nullptr;
  char* stack = nullptr;
  bool done = false;
  uint3_emu tid{0, 0, 0};
};

std::vector<Fiber> fibers;
void* sched_sp = nullptr;
int cur = -1;
const std::function<void()>* body = nullptr;
std::vector<unsigned long long> slots;
bool reverse_blocks = false;
long long launches = 0;
#ifdef EMU_ASAN
const void* sched_bottom = nullptr;
size_t sched_size = 0;
#endif

void to_scheduler(bool finished) {
#ifdef EMU_ASAN
  void* fake = nullptr;
  __sanitizer_start_switch_fiber(finished ? nullptr : &fake, sched_bottom, sched_size);
  emu_ctx_switch(&fibers[cur].sp, sched_sp);
  __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#else
  (void)finished;
  emu_ctx_switch(&fibers[cur].sp, sched_sp);
#endif
}

extern "C" void emu_fiber_start() {
#ifdef EMU_ASAN
  __sanitizer_finish_switch_fiber(nullptr, &sched_bottom, &sched_size);
#endif
  (*body)();
  fibers[cur].done = true;
  to_scheduler(true);
  std::abort();   // a finished fiber is never resumed
}

// Initial stack of a fiber: the frame emu_ctx_switch pops (control words, six registers) and
// emu_fiber_start as its return address.
void init_fiber(Fiber& F) {
#ifdef EMU_ASAN
  // a fiber that returned leaves its frames' redzones poisoned on the reused stack
  __asan_unpoison_memory_region(F.stack, kStack);
#endif
  uintptr_t top = reinterpret_cast<uintptr_t>(F.stack + kStack) & ~(uintptr_t)15;
  uint64_t* sp = reinterpret_cast<uint64_t*>(top - 72);   // sp % 16 == 8 after the 8 pops + ret
  uint32_t mx;
  uint16_t cw;
  asm volatile("stmxcsr %0" : "=m"(mx));
  asm volatile("fnstcw %0" : "=m"(cw));
  sp[0] = (uint64_t)mx | ((uint64_t)cw << 32);
  for (int i = 1; i <= 6; ++i) sp[i] = 0;
  sp[7] = reinterpret_cast<uint64_t>(&emu_fiber_start);
  sp[8] = 0;
  F.sp = sp;
}

void resume(int t) {
  cur = t;
  thread_idx = fibers[t].tid;
#ifdef EMU_ASAN
  void* fake = nullptr;
  __sanitizer_start_switch_fiber(&fake, fibers[t].stack, kStack);
  emu_ctx_switch(&sched_sp, fibers[t].sp);
  __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#else
  emu_ctx_switch(&sched_sp, fibers[t].sp);
#endif
  cur = -1;
}

}  // namespace

unsigned long long* xchg_slots() { return slots.data(); }

char* buffer_at(const __amdgpu_buffer_rsrc_t& r, int voff, int soff, unsigned size) {
  const unsigned long long off = (unsigned long long)(unsigned)voff + (unsigned)soff;
  if (off >> 32) {
    std::fprintf(stderr, "emu: buffer offset %u + %u wraps 32 bits\n", (unsigned)voff, (unsigned)soff);
    std::abort();
  }
  if ((off & (size - 1)) != 0) {
    std::fprintf(stderr, "emu: misaligned buffer access at offset %llu (size %u)\n", off, size);
    std::abort();
  }
  if (off + size > r.bytes) return nullptr;
  return r.base + off;
}

void syncthreads() {
  if (cur < 0) {
    std::fprintf(stderr, "emu: __syncthreads outside a kernel\n");
    std::abort();
  }
  to_scheduler(false);
}

void launch(dim3 grid, dim3 block, const std::function<void()>& f) {
  static bool init = false;
  if (!init) {
    reverse_blocks = std::getenv("EMU_REVERSE_BLOCKS") != nullptr;
    init = true;
  }
  const unsigned nth = block.x * block.y * block.z;
  if (nth == 0 || nth > 1024 || grid.x == 0 || grid.y == 0 || grid.z == 0) {
    std::fprintf(stderr, "emu: invalid launch grid (%u,%u,%u) block (%u,%u,%u)\n", grid.x, grid.y,
                 grid.z, block.x, block.y, block.z);
    std::abort();
  }
  ++launches;
  if (fibers.size() < nth) fibers.resize(nth);
  for (unsigned i = 0; i < nth; ++i)
    if (!fibers[i].stack) fibers[i].stack = static_cast<char*>(std::malloc(kStack));
  slots.assign(nth, 0ull);
  body = &f;
  block_dim = {block.x, block.y, block.z};
  grid_dim = {grid.x, grid.y, grid.z};
  const long long nblocks = (long long)grid.x * grid.y * grid.z;
  for (long long bi = 0; bi < nblocks; ++bi) {
    const long long b = reverse_blocks ? nblocks - 1 - bi : bi;
    block_idx = {(unsigned)(b % grid.x), (unsigned)((b / grid.x) % grid.y),
                 (unsigned)(b / ((long long)grid.x * grid.y))};
    for (unsigned t = 0; t < nth; ++t) {
      Fiber& F = fibers[t];
      F.done = false;
      F.tid = {t % block.x, (t / block.x) % block.y, t / (block.x * block.y)};
      init_fiber(F);
    }
    for (;;) {
      int live = 0;
      for (unsigned t = 0; t < nth; ++t)
        if (!fibers[t].done) {
          resume((int)t);
          live += !fibers[t].done;
        }
      if (live == 0) break;
    }
  }
  body = nullptr;
  thread_idx = {0, 0, 0};
}

}  // namespace emu

extern "C" long long emu_launch_count() { return emu::launches; }

// ---------------------------------------------------------------- runtime calls
namespace {
std::map<void*, size_t> allocs;
hipError_t last_error = hipSuccess;
struct emu_event_t { int recorded = 0; };
}  // namespace

hipError_t hipMalloc(void** p, size_t n) {
  if (!p) return hipErrorInvalidValue;
  const size_t cap = (n + 255) / 256 * 256 + 256;
  void* q = std::aligned_alloc(256, cap);
  if (!q) return hipErrorMemoryAllocation;
  // Device memory is not cleared by hipMalloc; EMU_FILL=<byte> gives it a known non-zero content
  // so a read before the first write shows up (the driver fills workspaces the same way).
  if (const char* f = std::getenv("EMU_FILL")) {
    if (std::strcmp(f, "random") == 0) {
      unsigned long long x = 0x9E3779B97F4A7C15ull ^ (unsigned long long)allocs.size();
      for (size_t i = 0; i < cap; ++i) {
        x ^= x << 13; x ^= x >> 7; x ^= x << 17;
        static_cast<unsigned char*>(q)[i] = (unsigned char)x;
      }
    } else {
      std::memset(q, (int)std::strtol(f, nullptr, 0), cap);
    }
  }
  allocs[q] = n;
  *p = q;
  return hipSuccess;
}

hipError_t hipFree(void* p) {
  if (!p) return hipSuccess;
  auto it = allocs.find(p);
  if (it == allocs.end()) {
    std::fprintf(stderr, "emu: hipFree of an address hipMalloc did not return\n");
    std::abort();
  }
  allocs.erase(it);
  std::free(p);
  return hipSuccess;
}

hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  if (n) std::memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t) {
  return hipMemcpy(d, s, n, k);
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
  if (n) std::memset(d, v, n);
  return hipSuccess;
}
hipError_t hipMemGetInfo(size_t* free_b, size_t* total_b) {
  const char* e = std::getenv("EMU_FREE_BYTES");
  const size_t f = e ? (size_t)std::strtoull(e, nullptr, 10) : (size_t)64 << 30;
  if (free_b) *free_b = f;
  if (total_b) *total_b = (size_t)288 << 30;
  return hipSuccess;
}
hipError_t hipGetDevice(int* dev) { if (dev) *dev = 0; return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDeviceCount(int* n) { if (n) *n = 1; return hipSuccess; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  if (!p) return hipErrorInvalidValue;
  *p = hipDeviceProp_t{};
  std::snprintf(p->name, sizeof p->name, "CPU emulation");
  std::snprintf(p->gcnArchName, sizeof p->gcnArchName, "emu");
  p->totalGlobalMem = (size_t)288 << 30;
  p->multiProcessorCount = 1;
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  if (!p || !sym) return hipErrorInvalidSymbol;
  *p = const_cast<void*>(sym);
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = reinterpret_cast<hipEvent_t>(new emu_event_t());
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete reinterpret_cast<emu_event_t*>(e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  if (!e) return hipErrorInvalidValue;
  reinterpret_cast<emu_event_t*>(e)->recorded = 1;
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) { return e ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  if (!ms || !a || !b) return hipErrorInvalidValue;
  *ms = 0.f;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError() {
  const hipError_t e = last_error;
  last_error = hipSuccess;
  return e;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated HIP error"; }
