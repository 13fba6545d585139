// Host emulation runtime for the bounds test of libsgspm's kernels: a fiber per
// work-item, __syncthreads and wave shuffles as scheduling points, device memory
// as exact-size host allocations (test infrastructure only).
#include <hip/hip_runtime.h>
#include <sanitizer/asan_interface.h>
#include <sys/mman.h>

#include <cstdio>
#include <string>
#include <vector>

// tell AddressSanitizer about every stack switch (no-ops in a build without it)
#ifdef __SANITIZE_ADDRESS__
#define SWITCH_START(save, bottom, size) __sanitizer_start_switch_fiber(save, bottom, size)
#define SWITCH_FINISH(save, bottom, size) __sanitizer_finish_switch_fiber(save, bottom, size)
#else
#define SWITCH_START(save, bottom, size) ((void)0)
#define SWITCH_FINISH(save, bottom, size) ((void)0)
#endif

dim3 threadIdx, blockIdx, blockDim, gridDim;

namespace sgspm {
// the dynamic LDS of every kernel (declared extern in each kernel body)
alignas(256) unsigned char smem_raw[160 * 1024];
}

namespace {
constexpr size_t LDS_CAP = sizeof(sgspm::smem_raw);
constexpr size_t STACK = 512 * 1024;
constexpr int MAXT = 1024;
enum { RUN, BAR, WSYNC, DONE };

// Stack switch: saves the callee-saved registers on the current stack, stores
// the stack pointer in *save, loads `next` and restores the registers saved
// there.  A new fiber's stack is laid out so that the first switch to it
// "returns" into fiber_start.
extern "C" void emu_switch(void** save, void* next);
asm(R"(
  .text
  .globl emu_switch
  .type emu_switch, @function
emu_switch:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
  .size emu_switch, .-emu_switch
)");

struct Fiber {
  void* sp = nullptr;  // saved stack pointer while switched out
  char* stack = nullptr;
  int state = DONE;
  void* fake = nullptr;
  int tid = 0;
  unsigned wphase = 0;
};

Fiber fibers[MAXT];
void* sched_sp = nullptr;
void* sched_fake = nullptr;
const void* sched_bottom = nullptr;
size_t sched_size = 0;
Fiber* cur = nullptr;
const emu::Launch* cur_launch = nullptr;
uint64_t slot[2][MAXT];
hipError_t last_error = hipSuccess;
long launches = 0, groups_run = 0;

long max_groups() {
  const char* e = getenv("EMU_MAX_GROUPS");
  return e ? atol(e) : 0;
}

void fail(const char* what, const char* name) {
  fprintf(stderr, "EMU ERROR: %s in launch %ld (%s)\n", what, launches, name);
  fflush(stderr);
  abort();
}

void set_thread_index(int t) {
  threadIdx.x = t % blockDim.x;
  threadIdx.y = (t / blockDim.x) % blockDim.y;
  threadIdx.z = t / (blockDim.x * blockDim.y);
}

// fiber -> scheduler; returns when the scheduler resumes this fiber
void yield(int st) {
  Fiber* me = cur;
  me->state = st;
  SWITCH_START(&me->fake, sched_bottom, sched_size);
  emu_switch(&me->sp, sched_sp);
  SWITCH_FINISH(me->fake, &sched_bottom, &sched_size);
}

// every fiber runs work-items for the life of the process: one per workgroup
extern "C" void fiber_start() {
  Fiber* me = cur;
  SWITCH_FINISH(nullptr, &sched_bottom, &sched_size);
  for (;;) {
    cur_launch->body(cur_launch->ctx);
    yield(DONE);
  }
  (void)me;
}

void init_fiber(Fiber& f, const char* name) {
  void* p = mmap(nullptr, STACK, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
  if (p == MAP_FAILED) fail("fiber stack allocation", name);
  f.stack = static_cast<char*>(p);
  // top of stack, 16-byte aligned: [6 saved registers][return address = fiber_start][pad]
  uintptr_t top = (reinterpret_cast<uintptr_t>(f.stack) + STACK - 64) & ~uintptr_t(15);
  void** sp = reinterpret_cast<void**>(top);
  *--sp = nullptr;  // alignment: at fiber_start entry rsp + 8 is 16-byte aligned
  *--sp = reinterpret_cast<void*>(&fiber_start);
  for (int i = 0; i < 6; ++i) *--sp = nullptr;
  f.sp = sp;
}

void resume(Fiber& f) {
  cur = &f;
  set_thread_index(f.tid);
  SWITCH_START(&sched_fake, f.stack, STACK);
  emu_switch(&sched_sp, f.sp);
  SWITCH_FINISH(sched_fake, nullptr, nullptr);
}

void run_group(int n, const char* name) {
  for (int t = 0; t < n; ++t) {
    Fiber& f = fibers[t];
    if (!f.stack) init_fiber(f, name);
    f.state = RUN;
    f.tid = t;
    f.wphase = 0;
  }
  for (;;) {
    for (int t = 0; t < n; ++t)
      if (fibers[t].state == RUN) resume(fibers[t]);
    bool all_done = true, released = false;
    for (int t = 0; t < n; ++t) all_done &= fibers[t].state == DONE;
    if (all_done) break;
    // a wave whose live work-items all wait in a shuffle goes on
    for (int w0 = 0; w0 < n; w0 += 64) {
      bool any = false, all = true;
      for (int t = w0; t < std::min(n, w0 + 64); ++t) {
        if (fibers[t].state == DONE) continue;
        any = true;
        all &= fibers[t].state == WSYNC;
      }
      if (any && all) {
        for (int t = w0; t < std::min(n, w0 + 64); ++t)
          if (fibers[t].state == WSYNC) fibers[t].state = RUN;
        released = true;
      }
    }
    if (released) continue;
    // the workgroup goes on when every live work-item waits at the barrier
    bool all_bar = true;
    for (int t = 0; t < n; ++t)
      if (fibers[t].state != DONE) all_bar &= fibers[t].state == BAR;
    if (!all_bar) fail("work-items wait at different synchronisation points", name);
    for (int t = 0; t < n; ++t)
      if (fibers[t].state == BAR) fibers[t].state = RUN;
  }
}

template <typename V> V shfl(V v, unsigned d, int width) {
  if (!cur) fail("shuffle outside a kernel", "");
  if (width != 64) fail("shuffle width other than 64", "");
  const int t = cur->tid;
  const unsigned ph = cur->wphase++ & 1;
  uint64_t bits = 0;
  memcpy(&bits, &v, sizeof(V));
  slot[ph][t] = bits;
  yield(WSYNC);
  const int n = blockDim.x * blockDim.y * blockDim.z;
  const int lane = t & 63;
  const int src = (lane + (int)d < 64 && t + (int)d < n) ? t + (int)d : t;
  V r;
  memcpy(&r, &slot[ph][src], sizeof(V));
  return r;
}
}  // namespace

void __syncthreads() {
  if (!cur) fail("barrier outside a kernel", "");
  yield(BAR);
}
float __shfl_down(float v, unsigned d, int w) { return shfl(v, d, w); }
double __shfl_down(double v, unsigned d, int w) { return shfl(v, d, w); }
int __shfl_down(int v, unsigned d, int w) { return shfl(v, d, w); }

namespace emu {
void run_launch(const char* name, dim3 grid, dim3 block, size_t lds, const Launch& l) {
  ++launches;
  if (getenv("EMU_TRACE")) fprintf(stderr, "launch %ld %s grid %u %u %u block %u lds %zu\n", launches, name, grid.x, grid.y, grid.z, block.x, lds);
  const long nthreads = (long)block.x * block.y * block.z;
  const long ngroups = (long)grid.x * grid.y * grid.z;
  if (nthreads <= 0 || nthreads > MAXT) fail("workgroup size outside 1..1024", name);
  if (ngroups <= 0) fail("empty grid", name);
  if (grid.y > 65535 || grid.z > 65535) fail("grid y or z above 65535", name);
  if (lds > LDS_CAP) fail("dynamic LDS above 160 KiB", name);
  ASAN_UNPOISON_MEMORY_REGION(sgspm::smem_raw, LDS_CAP);
  memset(sgspm::smem_raw, 0xff, LDS_CAP);
  if (lds < LDS_CAP) ASAN_POISON_MEMORY_REGION(sgspm::smem_raw + lds, LDS_CAP - lds);
  gridDim = grid;
  blockDim = block;
  cur_launch = &l;
  const long mg = max_groups();
  std::vector<long> ids;
  if (mg <= 0 || ngroups <= mg) {
    for (long g = 0; g < ngroups; ++g) ids.push_back(g);
  } else {
    // the first and last workgroups along every grid axis, and a spread between
    for (long k = 0; k < mg; ++k) ids.push_back(k * (ngroups - 1) / (mg - 1));
    const long gx = grid.x, gy = grid.y, gz = grid.z;
    for (long z : {0L, gz - 1})
      for (long y : {0L, gy - 1})
        for (long x : {0L, gx - 1}) ids.push_back(x + gx * (y + gy * z));
    std::sort(ids.begin(), ids.end());
    ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
  }
  for (long g : ids) {
    blockIdx.x = g % grid.x;
    blockIdx.y = (g / grid.x) % grid.y;
    blockIdx.z = g / ((long)grid.x * grid.y);
    run_group((int)nthreads, name);
    ++groups_run;
  }
  cur = nullptr;
  cur_launch = nullptr;
}
}  // namespace emu

extern "C" long emu_launch_count() { return launches; }
extern "C" long emu_group_count() { return groups_run; }

// ---- runtime API
hipError_t hipMalloc(void** p, size_t n) {
  if (posix_memalign(p, 256, n ? n : 1)) return hipErrorOutOfMemory;
  memset(*p, 0xff, n);  // uninitialised device memory reads as NaN
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  free(p);
  return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t) { return hipMemcpy(d, s, n, k); }
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
  memset(d, v, n);
  return hipSuccess;
}
hipError_t hipMemset(void* d, int v, size_t n) { return hipMemsetAsync(d, v, n, nullptr); }
static int stream_token;
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = reinterpret_cast<hipStream_t>(&stream_token);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError() {
  hipError_t e = last_error;
  last_error = hipSuccess;
  return e;
}
hipError_t hipPeekAtLastError() { return last_error; }
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated HIP error"; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
static int event_token;
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = reinterpret_cast<hipEvent_t>(&event_token);
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.0f;
  return hipSuccess;
}
// graph capture is not emulated: the graph entry point reports an error
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t*) { return hipErrorNotSupported; }
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, hipGraphNode_t*, char*, size_t) { return hipErrorNotSupported; }
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  *p = const_cast<void*>(sym);
  return hipSuccess;
}
