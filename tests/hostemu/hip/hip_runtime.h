// Host emulation of the parts of the HIP runtime and device language that the
// engine uses (test infrastructure only).
//
// The engine's own sources (csrc/*.hip, *.hpp) are compiled unchanged as host
// C++ against this header, so their host logic and their kernels run on the
// CPU under AddressSanitizer / UndefinedBehaviorSanitizer:
//   * kernels run block after block; the threads of a block are fibers that
//     switch at __syncthreads(), __shared__ arrays are block-shared statics;
//   * streams are FIFO queues executed lazily (at synchronisation points), so
//     a host buffer released before its asynchronous copy ran is read after
//     its release, which ASan reports;
//   * events, stream capture and graphs follow the HIP rules the engine relies
//     on, and every handle is checked for use after destruction;
//   * each batched or plain pass launch is checked before it runs: every
//     range its arguments let a block read or write must lie in memory the
//     test registered for the same problem (emu::register_region).
#pragma once

#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <cmath>
#include <functional>
#include <tuple>
#include <utility>

// ---------------------------------------------------------------------------
// device-language qualifiers and vector types
// ---------------------------------------------------------------------------
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))

struct alignas(8) float2 {
  float x, y;
};
struct alignas(16) double2 {
  double x, y;
};
struct alignas(16) float4 {
  float x, y, z, w;
};
inline float2 make_float2(float x, float y) { return float2{x, y}; }
inline double2 make_double2(double x, double y) { return double2{x, y}; }
inline float4 make_float4(float x, float y, float z, float w) { return float4{x, y, z, w}; }

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct emu_uint3 {
  unsigned x, y, z;
};
extern emu_uint3 threadIdx, blockIdx, blockDim, gridDim;

void __syncthreads();

inline float __int_as_float(int v) {
  float f;
  memcpy(&f, &v, 4);
  return f;
}
inline int __float_as_int(float f) {
  int v;
  memcpy(&v, &f, 4);
  return v;
}
#define __builtin_amdgcn_readfirstlane(x) (x)
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
// a wavefront-scope exchange point: every thread of the block reaches it
// together here, so the block barrier (which switches fibers) stands in
#define __builtin_amdgcn_fence(order, scope) ((void)0)
#define __builtin_amdgcn_wave_barrier() __syncthreads()

// Buffer resources (raw, untyped): a base and a size in bytes.  The engine
// never relies on the hardware's out-of-range handling, so an access that
// does not lie wholly inside [base, base + size) stops the run.
struct emu_buffer_rsrc {
  char* base;
  unsigned bytes;
};
typedef float emu_f32x2 __attribute__((ext_vector_type(2)));
// (op 0: load, 1: store; an int rather than a string literal, whose copies in
// every translation unit ASan would report as an ODR violation)
[[noreturn]] void emu_buffer_fault(int op, unsigned long offset, unsigned bytes);
inline emu_buffer_rsrc emu_make_buffer_rsrc(const void* base, short, int num_records, int) {
  return emu_buffer_rsrc{static_cast<char*>(const_cast<void*>(base)), unsigned(num_records)};
}
inline emu_f32x2 emu_raw_buffer_load_b64(emu_buffer_rsrc r, unsigned voffset, unsigned soffset, int) {
  const unsigned long off = (unsigned long)voffset + soffset;
  if (off + 8 > r.bytes) emu_buffer_fault(0, off, r.bytes);
  emu_f32x2 v;
  memcpy(&v, r.base + off, 8);
  return v;
}
inline void emu_raw_buffer_store_b64(emu_f32x2 v, emu_buffer_rsrc r, unsigned voffset, unsigned soffset, int) {
  const unsigned long off = (unsigned long)voffset + soffset;
  if (off + 8 > r.bytes) emu_buffer_fault(1, off, r.bytes);
  memcpy(r.base + off, &v, 8);
}
#define __amdgpu_buffer_rsrc_t emu_buffer_rsrc
#define __builtin_amdgcn_make_buffer_rsrc emu_make_buffer_rsrc
#define __builtin_amdgcn_raw_buffer_load_b64 emu_raw_buffer_load_b64
#define __builtin_amdgcn_raw_buffer_store_b64 emu_raw_buffer_store_b64

inline int atomicOr(int* p, int v) {
  const int old = *p;
  *p = old | v;
  return old;
}
inline void sincospi(double x, double* s, double* c) {
  *s = sin(M_PI * x);
  *c = cos(M_PI * x);
}
inline unsigned min(unsigned a, unsigned b) { return a < b ? a : b; }
inline unsigned max(unsigned a, unsigned b) { return a > b ? a : b; }
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline long min(long a, long b) { return a < b ? a : b; }
inline long max(long a, long b) { return a > b ? a : b; }
inline long long min(long long a, long long b) { return a < b ? a : b; }
inline long long max(long long a, long long b) { return a > b ? a : b; }

// ---------------------------------------------------------------------------
// runtime API
// ---------------------------------------------------------------------------
typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorInvalidResourceHandle = 400,
  hipErrorStreamCaptureUnsupported = 900,
  hipErrorStreamCaptureInvalidated = 901,
  hipErrorIllegalState = 401,
  hipErrorUnknown = 999,
} hipError_t;

typedef struct emu_stream* hipStream_t;
typedef struct emu_event* hipEvent_t;
typedef struct emu_graph* hipGraph_t;
typedef struct emu_graph_exec* hipGraphExec_t;

enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
};
enum hipStreamCaptureMode {
  hipStreamCaptureModeGlobal = 0,
  hipStreamCaptureModeThreadLocal = 1,
  hipStreamCaptureModeRelaxed = 2
};
#define hipStreamNonBlocking 1u
#define hipEventDisableTiming 2u
#define hipEventDefault 0u
#define HIP_SYMBOL(s) (reinterpret_cast<const void*>(&(s)))

hipError_t hipGetDevice(int* dev);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
hipError_t hipDeviceSynchronize();
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t g, void* err_node, char* log, size_t n);
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t exec);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGetSymbolAddress(void** ptr, const void* symbol);

namespace brahms {
struct PassArgs;
struct TableArgs;
}  // namespace brahms

namespace emu {

// Enqueue one kernel launch (run later, in stream order).  `check` runs with
// the launch geometry when the launch executes, before the kernel body.
// `site` is the source line of the launch (a kernel name string would be one
// literal repeated in many template instantiations, which ASan's global
// registration mistakes for an ODR violation).
void launch(hipStream_t s, dim3 grid, dim3 block, int site, std::function<void()> body,
            std::function<void(dim3)> check);

// Range checks of the engine's pass and table launches (tests/hostemu/emu.cpp);
// other argument lists are not checked.
template <typename... A>
inline void check_args(dim3, const A&...) {}
void check_args(dim3 grid, const brahms::PassArgs& a);
void check_args(dim3 grid, const brahms::PassArgs* const& descs, const long long& step, const int& nf);
void check_args(dim3 grid, const brahms::TableArgs& a);
void check_args(dim3 grid, const brahms::TableArgs* const& targs);

}  // namespace emu

#define hipLaunchKernelGGL(K, G, B, SHMEM, ST, ...)                                     \
  ::emu::launch((ST), dim3(G), dim3(B), __LINE__, [=]() { K(__VA_ARGS__); },            \
                [=](dim3 grid_) { ::emu::check_args(grid_, __VA_ARGS__); })
