// Host emulation of the HIP runtime for the engine's sources (test
// infrastructure only; see hip/hip_runtime.h for what is emulated).
#include <hip/hip_runtime.h>
#include <sanitizer/asan_interface.h>
#include <sanitizer/common_interface_defs.h>
#include <sys/mman.h>
#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "emu.hpp"
#include "kernels.hpp"

emu_uint3 threadIdx, blockIdx, blockDim, gridDim;

namespace emu {

[[noreturn]] void die(const std::string& msg) {
  std::fprintf(stderr, "EMU ERROR: %s\n", msg.c_str());
  std::fflush(stderr);
  std::abort();
}

}  // namespace emu

using emu::die;

[[noreturn]] void emu_buffer_fault(int op, unsigned long offset, unsigned bytes) {
  die(std::string(op == 0 ? "buffer load" : "buffer store") + " at byte " + std::to_string(offset) +
      " of a " + std::to_string(bytes) + "-byte buffer");
}

// ---------------------------------------------------------------------------
// handles: never freed, only marked dead, so that any later use is reported
// ---------------------------------------------------------------------------
struct emu_graph {
  bool alive = true;
  std::vector<std::function<void()>> ops;
  hipStream_t origin = nullptr;
};
struct emu_graph_exec {
  bool alive = true;
  std::vector<std::function<void()>> ops;
  int pending = 0;   // launches enqueued and not yet run
};
struct emu_stream {
  bool alive = true;
  int id = 0;
  std::deque<std::pair<unsigned long long, std::function<void()>>> q;
  unsigned long long enq = 0, done = 0;
  emu_graph* cap = nullptr;    // capture in progress (origin or joined)
  bool origin = false;
};
struct emu_event {
  bool alive = true;
  emu_stream* s = nullptr;     // stream and position of the last record
  unsigned long long seq = 0;
  emu_graph* cap = nullptr;    // recorded during a capture into this graph
  size_t cap_pos = 0;
};

namespace {

emu_stream g_null;
std::vector<emu_stream*> g_streams{&g_null};
hipError_t g_last = hipSuccess;
int g_captures = 0;

emu_stream* S(hipStream_t s, const char* where) {
  emu_stream* p = s ? s : &g_null;
  if (!p->alive) die(std::string(where) + ": stream used after hipStreamDestroy");
  return p;
}

void check_event(hipEvent_t e, const char* where) {
  if (e == nullptr) die(std::string(where) + ": NULL event");
  if (!e->alive) die(std::string(where) + ": event used after hipEventDestroy");
}

void enqueue(emu_stream* s, std::function<void()> fn) {
  if (s->cap) {
    s->cap->ops.push_back(std::move(fn));
    return;
  }
  s->q.emplace_back(++s->enq, std::move(fn));
}

void drain(emu_stream* s, unsigned long long upto) {
  while (s->done < upto) {
    if (s->q.empty()) die("stream queue underflow");
    auto op = std::move(s->q.front());
    s->q.pop_front();
    op.second();
    s->done = op.first;
  }
}

void drain_all() {
  for (bool again = true; again;) {
    again = false;
    for (emu_stream* s : g_streams)
      if (s->alive && s->done < s->enq) {
        drain(s, s->enq);
        again = true;
      }
  }
}

// ---------------------------------------------------------------------------
// fibers: the threads of one block, switched by a small x86-64 routine that
// saves the callee-saved registers, MXCSR and the x87 control word
// ---------------------------------------------------------------------------
extern "C" void emu_swap(void** save_sp, void* new_sp);
extern "C" void emu_trampoline();
extern "C" void emu_fiber_main();
asm(R"(
.text
.globl emu_swap
.type emu_swap,@function
emu_swap:
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
.size emu_swap, .-emu_swap
.globl emu_trampoline
.type emu_trampoline,@function
emu_trampoline:
  call emu_fiber_main
  ud2
.size emu_trampoline, .-emu_trampoline
)");

constexpr size_t kStack = 512 * 1024;

struct Fiber {
  void* sp = nullptr;
  void* fake = nullptr;    // ASan's fake stack of the fiber while it is switched out
  char* stack = nullptr;
  bool done = false;
  bool waiting = false;
  emu_uint3 tid{};
};

void* g_sched_sp = nullptr;
Fiber* g_cur = nullptr;
void* g_sched_fake_stack = nullptr;
const void* g_sched_bottom = nullptr;
size_t g_sched_size = 0;
std::function<void()>* g_body = nullptr;
std::vector<Fiber> g_fibers;

// A fresh fiber's stack: the frame emu_swap pops, returning into the
// trampoline with a 16-byte aligned stack.
void* initial_sp(char* stack) {
  uintptr_t top = (reinterpret_cast<uintptr_t>(stack) + kStack) & ~uintptr_t(15);
  uint64_t* a = reinterpret_cast<uint64_t*>(top - 24);   // return address slot, = 8 mod 16
  a[0] = reinterpret_cast<uint64_t>(&emu_trampoline);
  for (int k = 1; k <= 6; ++k) a[-k] = 0;                 // rbp, rbx, r12 .. r15
  uint32_t* ctl = reinterpret_cast<uint32_t*>(a - 7);
  ctl[0] = 0x1F80u;                                        // MXCSR default
  ctl[1] = 0x037Fu;                                        // x87 control word default
  return a - 7;
}

void resume(Fiber& f) {
  g_cur = &f;
  threadIdx = f.tid;
  __sanitizer_start_switch_fiber(&g_sched_fake_stack, f.stack, kStack);
  emu_swap(&g_sched_sp, f.sp);
  __sanitizer_finish_switch_fiber(g_sched_fake_stack, nullptr, nullptr);
}

void run_block(std::function<void()>& body, dim3 block, const char* name) {
  const unsigned n = block.x * block.y * block.z;
  if (g_fibers.size() < n) g_fibers.resize(n);
  g_body = &body;
  for (unsigned t = 0; t < n; ++t) {
    Fiber& f = g_fibers[t];
    if (!f.stack) f.stack = static_cast<char*>(std::malloc(kStack));
    f.done = false;
    f.waiting = false;
    f.tid = emu_uint3{t % block.x, (t / block.x) % block.y, t / (block.x * block.y)};
    f.sp = initial_sp(f.stack);
  }
  for (;;) {
    for (unsigned t = 0; t < n; ++t)
      if (!g_fibers[t].done) resume(g_fibers[t]);
    unsigned done = 0, waiting = 0;
    for (unsigned t = 0; t < n; ++t) {
      done += g_fibers[t].done;
      waiting += g_fibers[t].waiting;
    }
    if (done == n) break;
    if (done != 0) die(std::string(name) + ": threads of a block left while others wait at a barrier");
    if (waiting != n) die(std::string(name) + ": barrier not reached by every thread");
    for (unsigned t = 0; t < n; ++t) g_fibers[t].waiting = false;
  }
  g_cur = nullptr;
}

}  // namespace

extern "C" void emu_fiber_main() {
  __sanitizer_finish_switch_fiber(nullptr, &g_sched_bottom, &g_sched_size);
  (*g_body)();
  Fiber* f = g_cur;
  f->done = true;
  __sanitizer_start_switch_fiber(nullptr, g_sched_bottom, g_sched_size);
  emu_swap(&f->sp, g_sched_sp);
  die("a finished fiber was resumed");
}

void __syncthreads() {
  if (g_cur == nullptr) die("__syncthreads outside a kernel");
  Fiber* f = g_cur;
  f->waiting = true;
  __sanitizer_start_switch_fiber(&f->fake, g_sched_bottom, g_sched_size);
  emu_swap(&f->sp, g_sched_sp);
  __sanitizer_finish_switch_fiber(f->fake, &g_sched_bottom, &g_sched_size);
  threadIdx = f->tid;
}

namespace emu {

long long g_launches = 0;

void launch(hipStream_t st, dim3 grid, dim3 block, int site, std::function<void()> body,
            std::function<void(dim3)> check) {
  const std::string name = "kernel launched at line " + std::to_string(site);
  emu_stream* s = S(st, "hipLaunchKernelGGL");
  if (grid.x == 0 || grid.y == 0 || grid.z == 0 || block.x * block.y * block.z == 0 ||
      block.x * block.y * block.z > 1024 || grid.y > 65536 || grid.z > 65536) {
    std::fprintf(stderr, "EMU: invalid launch geometry of %s (%u %u %u)\n", name.c_str(), grid.x, grid.y,
                 grid.z);
    g_last = hipErrorInvalidValue;
    return;
  }
  const std::string nm(name);
  enqueue(s, [grid, block, nm, body, check]() mutable {
    ++g_launches;
    check(grid);
    gridDim = emu_uint3{grid.x, grid.y, grid.z};
    blockDim = emu_uint3{block.x, block.y, block.z};
    for (unsigned z = 0; z < grid.z; ++z)
      for (unsigned y = 0; y < grid.y; ++y)
        for (unsigned x = 0; x < grid.x; ++x) {
          blockIdx = emu_uint3{x, y, z};
          run_block(body, block, nm.c_str());
        }
  });
}

// ---------------------------------------------------------------------------
// memory regions registered by the test, with the problem that owns them
// ---------------------------------------------------------------------------
struct Region {
  const char* lo;
  size_t bytes;
  int owner;
  std::string what;
};
std::vector<Region> g_regions;

void register_region(const void* p, size_t bytes, int owner, const char* what) {
  g_regions.push_back(Region{static_cast<const char*>(p), bytes, owner, what});
}
void clear_regions() { g_regions.clear(); }

// The owner of [p, p + bytes), which must lie inside one registered region.
int owner_of(const void* p, size_t bytes, const std::string& what) {
  const char* c = static_cast<const char*>(p);
  for (const Region& r : g_regions)
    if (c >= r.lo && c + bytes <= r.lo + r.bytes) return r.owner;
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s: range %p + %zu bytes lies in no registered region", what.c_str(), p, bytes);
  die(buf);
}

void same_owner(int& owner, int o, const std::string& what) {
  if (o < 0) return;   // shared region (descriptors)
  if (owner < 0) owner = o;
  if (owner != o) die(what + ": argument ranges of one problem span two problems' memory");
}

// The ranges one pass reads and writes (see PassArgs and axis_pass_body).
void check_pass(const brahms::PassArgs& a, int nf, const std::string& what) {
  const long plane = long(a.nx) * a.ny;
  const size_t field_bytes = sizeof(float2) * size_t(plane) * size_t(a.nt);
  int n = 0;
  if (a.axis_off == 0) n = a.nx;
  else if (a.axis_off == a.nx) n = a.ny;
  else if (a.axis_off == a.nx + a.ny) n = a.nt;
  else die(what + ": axis_off names no axis");
  if (a.field_stride != a.nx + a.ny + a.nt) die(what + ": field_stride is not nx + ny + nt");
  int owner = -1;
  for (int j = 0; j < nf; ++j) {
    same_owner(owner, owner_of(a.f[j], field_bytes, what + " field in"), what);
    same_owner(owner, owner_of(a.fo[j], field_bytes, what + " field out"), what);
    if (a.pre[0] != nullptr) owner_of(a.pre[j], field_bytes, what + " pre");
  }
  auto table = [&](const float2* t, size_t entries, const char* nm) {
    same_owner(owner, owner_of(t, sizeof(float2) * entries, what + " " + nm), what);
  };
  table(a.tw, size_t(n), "twiddles");
  for (int j = 0; j < nf; ++j)
    table(a.prop + size_t(j) * a.field_stride + a.axis_off, size_t(n), "propagator");
  same_owner(owner, owner_of(a.consts, sizeof(brahms::DftConsts), what + " consts"), what);
  table(a.nl, size_t(nf) * brahms::kNlCoef, "rk4 coefficients");
  table(a.nl2, size_t(nf) * brahms::kNlCoef, "rk4 coefficients 2");
  if (a.tw2 != nullptr) {
    table(a.tw2, size_t(n), "next twiddles");
    for (int j = 0; j < nf; ++j)
      table(a.prop2 + size_t(j) * a.field_stride + a.axis_off, size_t(n), "next propagator");
    same_owner(owner, owner_of(a.consts2, sizeof(brahms::DftConsts), what + " next consts"), what);
  }
  if (a.map != nullptr) table(a.map, size_t(3) * size_t(plane), "map factors");
  if (a.tiles == 0 || a.tile_mul == 0) die(what + ": tile map with zero tiles");
}

void check_tables(const brahms::TableArgs& t, const std::string& what) {
  int owner = -1;
  if (t.count < 0) die(what + ": negative row count");
  const long long n0 = t.n0_dev != nullptr ? t.n0_dev[0] : t.n0;
  if (t.row_stride != brahms::table_row_stride(t.nf, t.nx, t.ny, t.nt)) die(what + ": row stride");
  if (t.count == 0) return;
  same_owner(owner, owner_of(t.rows, sizeof(float2) * size_t(t.count) * t.row_stride, what + " rows"), what);
  same_owner(owner, owner_of(t.nl, sizeof(float2) * size_t(t.count) * 2 * t.nf * brahms::kNlCoef,
                             what + " rk4 rows"), what);
  if (t.dk != nullptr) {
    same_owner(owner, owner_of(t.dk + n0, sizeof(double) * size_t(t.count), what + " dk"), what);
    same_owner(owner, owner_of(t.phi0 + n0, sizeof(double) * size_t(t.count), what + " phi0"), what);
  }
}

long long g_checked_passes = 0, g_checked_tables = 0;

void check_args(dim3 grid, const brahms::PassArgs& a) {
  int nf = 0;
  while (nf < 3 && a.f[nf] != nullptr) ++nf;
  // a linear pass of one field per block takes its field from blockIdx.z
  if (grid.z > 1 && int(grid.z) != nf) die("plain pass: gridDim.z is not the field count");
  check_pass(a, nf, "plain pass");
  ++g_checked_passes;
}

void check_args(dim3 grid, const brahms::PassArgs* const& descs, const long long& step, const int& nf) {
  const bool per_field = grid.z > 1;
  if (per_field && grid.z % unsigned(nf) != 0) die("batched pass: gridDim.z is not a multiple of nf");
  const unsigned m = per_field ? grid.z / unsigned(nf) : grid.y;
  owner_of(descs, sizeof(brahms::PassArgs) * m, "batched pass descriptors");
  for (unsigned i = 0; i < m; ++i) {
    const brahms::PassArgs& a = descs[i];
    if (step >= a.nz) continue;
    check_pass(a, nf, "batched pass, instance " + std::to_string(i));
    ++g_checked_passes;
  }
}

void check_args(dim3, const brahms::TableArgs& a) {
  check_tables(a, "tables");
  ++g_checked_tables;
}

void check_args(dim3 grid, const brahms::TableArgs* const& targs) {
  owner_of(targs, sizeof(brahms::TableArgs) * grid.y, "batched table arguments");
  for (unsigned i = 0; i < grid.y; ++i) {
    check_tables(targs[i], "batched tables, instance " + std::to_string(i));
    ++g_checked_tables;
  }
}

// ---------------------------------------------------------------------------
// "device" memory: page-aligned mappings with an inaccessible page after the
// end (the buffer ends exactly at it) and before the start
// ---------------------------------------------------------------------------
struct Mapping {
  char* base;
  size_t total;
};
std::map<const void*, Mapping> g_maps;

void* device_alloc(size_t bytes) {
  const size_t pg = size_t(sysconf(_SC_PAGESIZE));
  const size_t body = (bytes + pg - 1) / pg * pg;
  const size_t total = body + 2 * pg;
  char* base = static_cast<char*>(mmap(nullptr, total, PROT_NONE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0));
  if (base == MAP_FAILED) die("mmap failed");
  if (mprotect(base + pg, body, PROT_READ | PROT_WRITE) != 0) die("mprotect failed");
  // 256-byte aligned start as close to the guard page after the end as allowed
  char* p = base + pg + (body - bytes) / 256 * 256;
  std::memset(base + pg, 0x7f, body);
  g_maps[p] = Mapping{base, total};
  return p;
}

void device_free(void* p) {
  auto it = g_maps.find(p);
  if (it == g_maps.end()) die("device_free of an unknown pointer");
  munmap(it->second.base, it->second.total);
  g_maps.erase(it);
}

}  // namespace emu

// ---------------------------------------------------------------------------
// runtime API
// ---------------------------------------------------------------------------
hipError_t hipGetDevice(int* dev) {
  *dev = 0;
  return hipSuccess;
}

hipError_t hipGetLastError() {
  const hipError_t e = g_last;
  g_last = hipSuccess;
  return e;
}

const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated error"; }

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  auto* p = new emu_stream();
  p->id = int(g_streams.size());
  g_streams.push_back(p);
  *s = p;
  return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s) {
  if (s == nullptr) die("hipStreamDestroy(NULL)");
  emu_stream* p = S(s, "hipStreamDestroy");
  if (p->cap) die("hipStreamDestroy of a capturing stream");
  drain(p, p->enq);
  p->alive = false;
  return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s) {
  emu_stream* p = S(s, "hipStreamSynchronize");
  if (p->cap) return hipErrorStreamCaptureUnsupported;
  if (g_captures > 0 && p == &g_null) die("hipStreamSynchronize(NULL) during a capture");
  drain(p, p->enq);
  return hipSuccess;
}

hipError_t hipDeviceSynchronize() {
  if (g_captures > 0) die("hipDeviceSynchronize during a capture");
  drain_all();
  return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new emu_event();
  return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }

hipError_t hipEventDestroy(hipEvent_t e) {
  check_event(e, "hipEventDestroy");
  e->alive = false;
  return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t st) {
  check_event(e, "hipEventRecord");
  emu_stream* s = S(st, "hipEventRecord");
  if (s->cap) {
    e->cap = s->cap;
    e->cap_pos = s->cap->ops.size();
    e->s = s;
    return hipSuccess;
  }
  e->cap = nullptr;
  e->s = s;
  e->seq = s->enq;
  return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t st, hipEvent_t e, unsigned) {
  check_event(e, "hipStreamWaitEvent");
  emu_stream* s = S(st, "hipStreamWaitEvent");
  if (e->cap != nullptr) {
    // an event recorded in a capture: the waiting stream joins that capture
    if (s->cap != nullptr && s->cap != e->cap) die("hipStreamWaitEvent across two captures");
    if (s->cap == nullptr) {
      if (!s->q.empty() && s->done < s->enq) die("stream joins a capture with work still queued");
      s->cap = e->cap;
      ++g_captures;
    }
    return hipSuccess;
  }
  if (s->cap != nullptr && e->s != nullptr && e->s->cap == nullptr && e->seq > e->s->done)
    die("captured wait on an event of uncaptured, unfinished work");
  if (e->s == nullptr) return hipSuccess;   // never recorded: no dependency
  emu_stream* src = e->s;
  const unsigned long long seq = e->seq;
  enqueue(s, [src, seq]() { drain(src, seq); });
  return hipSuccess;
}

hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  check_event(a, "hipEventElapsedTime");
  check_event(b, "hipEventElapsedTime");
  if (a->s) drain(a->s, a->seq);
  if (b->s) drain(b->s, b->seq);
  *ms = 0.01f;
  return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t st) {
  emu_stream* s = S(st, "hipMemcpyAsync");
  if (s->cap) die("hipMemcpyAsync captured into a graph");
  // the copy reads its source when the stream reaches it, as the runtime does
  enqueue(s, [dst, src, bytes]() { std::memcpy(dst, src, bytes); });
  return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t st, hipStreamCaptureMode) {
  emu_stream* s = S(st, "hipStreamBeginCapture");
  if (s == &g_null) return hipErrorStreamCaptureUnsupported;
  if (s->cap) return hipErrorIllegalState;
  drain(s, s->enq);
  s->cap = new emu_graph();
  s->cap->origin = s;
  s->origin = true;
  ++g_captures;
  return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t st, hipGraph_t* g) {
  emu_stream* s = S(st, "hipStreamEndCapture");
  if (!s->origin || s->cap == nullptr) return hipErrorIllegalState;
  emu_graph* graph = s->cap;
  for (emu_stream* o : g_streams)
    if (o->cap == graph) {
      o->cap = nullptr;
      o->origin = false;
      --g_captures;
    }
  *g = graph;
  return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t g, void*, char*, size_t) {
  if (g == nullptr || !g->alive) die("hipGraphInstantiate of a destroyed graph");
  auto* x = new emu_graph_exec();
  x->ops = g->ops;
  *exec = x;
  return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t st) {
  if (exec == nullptr || !exec->alive) die("hipGraphLaunch of a destroyed graph exec");
  emu_stream* s = S(st, "hipGraphLaunch");
  if (s->cap) die("hipGraphLaunch into a capture");
  ++exec->pending;
  enqueue(s, [exec]() {
    if (!exec->alive) die("a graph exec was destroyed before its launch ran");
    for (auto& op : exec->ops) op();
    --exec->pending;
  });
  return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t exec) {
  if (exec == nullptr || !exec->alive) die("hipGraphExecDestroy of a destroyed graph exec");
  if (exec->pending > 0) die("hipGraphExecDestroy while a launch of it has not run (no wait before it)");
  exec->alive = false;
  exec->ops.clear();
  return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g) {
  if (g == nullptr || !g->alive) die("hipGraphDestroy of a destroyed graph");
  g->alive = false;
  g->ops.clear();
  return hipSuccess;
}

hipError_t hipGetSymbolAddress(void** ptr, const void* symbol) {
  *ptr = const_cast<void*>(symbol);
  return hipSuccess;
}
