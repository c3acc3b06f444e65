// Diagnostics behind the C ABI (brahms_diagnose, brahms_set_monitor,
// brahms_set_snapshots; see include/brahms.h): the output quantities of
// Sec. 6 taken on the device while the z-loop runs.
//
// A record describes the fields at one step index n (z = n dz):
//   [0]                      n
//   [1, 1 + nf nt)           P_j(tau) = sum_{x,y} |A_j|^2 dx dy, field-major
//   [1 + nf nt, + nf)        E_j = sum_tau P_j(tau) dtau
//   [1 + nf (nt + 1), + 3)   Manley-Rowe combinations: nf = 3:
//                            E_p/k_p + E_s/k_s, E_p/k_p + E_i/k_i,
//                            E_s/k_s - E_i/k_i;  nf = 2: E_F/k_F + E_S/k_S,
//                            then NaN, NaN (NaN wherever a kappa is 0)
// Every sum runs in FP64 in a fixed order, so records are reproducible bit
// for bit.  Reading the fields costs 8 nf bytes per grid point per record.
// The slice sums are split into fixed chunks (partials in the plan
// workspace) so that the reduction fills the chip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/brahms.h"
#include "plan.hpp"

using brahms::detail::check_plan;
using brahms::detail::fail;

namespace {

constexpr int kDiagBlock = 256;

struct FieldPtrs {
  const float2* f[3];
};

// Partial sums of |A|^2: block (c, tau, j) sums chunk c of the (tau, j)
// slice with a fixed thread -> element assignment (two values per 16-byte
// load, four independent accumulators) and a fixed tree; part[(j nt + tau)
// nchunk + c] receives the block's sum.
__global__ __launch_bounds__(kDiagBlock) void power_partials(FieldPtrs fp, long plane, int nt,
                                                             long chunk, int nchunk, int pairs,
                                                             double* part) {
  const int c = blockIdx.x;
  const int tau = blockIdx.y;
  const int j = blockIdx.z;
  const float2* s = fp.f[j] + long(tau) * plane;
  const long lo = long(c) * chunk;
  const long hi = lo + chunk < plane ? lo + chunk : plane;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  long i = lo + 2 * long(threadIdx.x);
  if (pairs) {
    // pairs of values per 16-byte load (plane and chunk even, fields 16-byte
    // aligned); 2 * kDiagBlock values per sweep
    const float4* s4 = reinterpret_cast<const float4*>(s);
    for (; i + 6 * kDiagBlock + 1 < hi; i += 8 * kDiagBlock) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float4 v = s4[(i + 2 * u * kDiagBlock) / 2];
        acc[u] = fma(double(v.x), double(v.x), fma(double(v.y), double(v.y), acc[u]));
        acc[u] = fma(double(v.z), double(v.z), fma(double(v.w), double(v.w), acc[u]));
      }
    }
    for (; i + 1 < hi; i += 2 * kDiagBlock) {
      const float4 v = s4[i / 2];
      acc[0] = fma(double(v.x), double(v.x), fma(double(v.y), double(v.y), acc[0]));
      acc[0] = fma(double(v.z), double(v.z), fma(double(v.w), double(v.w), acc[0]));
    }
  } else {
    for (i = lo + threadIdx.x; i < hi; i += kDiagBlock) {
      const float2 v = s[i];
      acc[0] = fma(double(v.x), double(v.x), fma(double(v.y), double(v.y), acc[0]));
    }
  }
  __shared__ double red[kDiagBlock];
  red[threadIdx.x] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  for (int w = kDiagBlock / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long(j) * nt + tau) * nchunk + c] = red[0];
}

// P_j(tau) from the partial sums, in chunk order.
__global__ void power_traces(const double* part, int nf, int nt, int nchunk, double cell_xy,
                             double* rec) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nf * nt) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[long(k) * nchunk + c];
  rec[1 + k] = s * cell_xy;
}

struct Kappas {
  double k[3];
};

// Step index, energies and Manley-Rowe combinations of one record (one
// block of 64 threads: strided partial sums over tau, then a fixed tree).
constexpr int kFinishThreads = 64;

__global__ __launch_bounds__(kFinishThreads) void finish_record(double* rec, long long step, int nf,
                                                                int nt, double dt, Kappas ka) {
  __shared__ double part[3][kFinishThreads];
  const int t = threadIdx.x;
  for (int j = 0; j < 3; ++j) {
    double s = 0.0;
    if (j < nf)
      for (int k = t; k < nt; k += kFinishThreads) s += rec[1 + long(j) * nt + k];
    part[j][t] = s;
  }
  __syncthreads();
  for (int w = kFinishThreads / 2; w > 0; w >>= 1) {
    if (t < w)
      for (int j = 0; j < 3; ++j) part[j][t] += part[j][t + w];
    __syncthreads();
  }
  if (t != 0) return;
  rec[0] = double(step);
  double e[3] = {0.0, 0.0, 0.0};
  for (int j = 0; j < nf; ++j) {
    e[j] = part[j][0] * dt;
    rec[1 + long(nf) * nt + j] = e[j];
  }
  const double qnan = __builtin_nan("");
  double q[3];
  for (int j = 0; j < nf; ++j) q[j] = ka.k[j] != 0.0 ? e[j] / ka.k[j] : qnan;
  double* mr = rec + 1 + long(nf) * (nt + 1);
  if (nf == 3) {
    mr[0] = q[0] + q[1];
    mr[1] = q[0] + q[2];
    mr[2] = q[1] - q[2];
  } else {
    mr[0] = q[0] + q[1];
    mr[1] = qnan;
    mr[2] = qnan;
  }
}

__global__ void copy_state(float2* dst, const float2* src, long n) {
  for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

// Chunks per slice: about 4096 blocks in all, at most kDiagChunks (the
// partial sums live in the plan workspace).
int chunks_for(const brahms_plan_s& p) {
  const long plane = long(p.nx) * p.ny;
  const long slices = long(p.nt) * p.nf;
  long want = (4096 + slices - 1) / slices;              // about 4096 blocks in all
  want = std::min<long>(want, std::max<long>(1, plane / (8 * kDiagBlock)));
  return int(std::max<long>(1, std::min<long>(want, brahms::detail::kDiagChunks)));
}

brahms_status write_record(brahms_plan_s& p, long long step, double* rec) {
  FieldPtrs fp{};
  for (int j = 0; j < 3; ++j) fp.f[j] = p.fields[j];
  const long plane = long(p.nx) * p.ny;
  const int nchunk = chunks_for(p);
  long chunk = (plane + nchunk - 1) / nchunk;
  chunk += chunk & 1;                                    // keep chunks on 16-byte boundaries
  double* part = reinterpret_cast<double*>(p.ws + p.off_diag);
  int pairs = (plane % 2 == 0) ? 1 : 0;
  for (int j = 0; j < p.nf; ++j)
    if (reinterpret_cast<uintptr_t>(p.fields[j]) % 16 != 0) pairs = 0;
  hipLaunchKernelGGL(power_partials, dim3(unsigned(nchunk), unsigned(p.nt), unsigned(p.nf)),
                     dim3(kDiagBlock), 0, p.stream, fp, plane, p.nt, chunk, nchunk, pairs, part);
  HIP_TRY(hipGetLastError());
  const int nk = p.nf * p.nt;
  hipLaunchKernelGGL(power_traces, dim3(unsigned((nk + 255) / 256)), dim3(256), 0, p.stream, part,
                     p.nf, p.nt, nchunk, p.dx * p.dy, rec);
  HIP_TRY(hipGetLastError());
  Kappas ka{};
  for (int j = 0; j < p.nf; ++j) ka.k[j] = p.fp[j].kappa;
  hipLaunchKernelGGL(finish_record, dim3(1), dim3(kFinishThreads), 0, p.stream, rec, step, p.nf, p.nt,
                     p.dt, ka);
  HIP_TRY(hipGetLastError());
  return BRAHMS_OK;
}

long record_doubles(const brahms_plan_s& p) { return 1 + long(p.nf) * (p.nt + 1) + 3; }

}  // namespace

namespace brahms {
namespace detail {

brahms_status after_step(brahms_plan_s& p, long long step_done) {
  if (p.mon_every > 0 && p.mon_count < p.mon_capacity && step_done % p.mon_every == 0) {
    if (brahms_status st = write_record(p, step_done, p.mon_records + long(p.mon_count) * record_doubles(p)))
      return st;
    ++p.mon_count;
  }
  for (size_t i = 0; i < p.snap_steps.size(); ++i) {
    if (p.snap_steps[i] != step_done) continue;
    const long n = long(p.nx) * p.ny * p.nt;
    const unsigned blocks = unsigned(std::min<long>((n + 255) / 256, 4096));
    for (int j = 0; j < p.nf; ++j) {
      hipLaunchKernelGGL(copy_state, dim3(blocks), dim3(256), 0, p.stream,
                         p.snap_buffers[i * size_t(p.nf) + j], p.fields[j], n);
      HIP_TRY(hipGetLastError());
    }
  }
  return BRAHMS_OK;
}

}  // namespace detail
}  // namespace brahms

extern "C" {

brahms_status brahms_record_size(brahms_plan plan, int* ndoubles) {
  if (brahms_status st = check_plan(plan)) return st;
  if (ndoubles == nullptr) return fail(BRAHMS_E_INVALID_ARG, "ndoubles is NULL");
  *ndoubles = int(record_doubles(*plan));
  return BRAHMS_OK;
}

brahms_status brahms_diagnose(brahms_plan plan, double* record) {
  if (brahms_status st = check_plan(plan)) return st;
  if (!plan->bound) return fail(BRAHMS_E_STATE, "brahms_diagnose before brahms_plan_bind");
  if (record == nullptr) return fail(BRAHMS_E_INVALID_ARG, "record is NULL");
  return write_record(*plan, plan->step, record);
}

brahms_status brahms_set_monitor(brahms_plan plan, int every, double* records, int capacity) {
  if (brahms_status st = check_plan(plan)) return st;
  if (every < 0 || capacity < 0) return fail(BRAHMS_E_INVALID_ARG, "every and capacity must be >= 0");
  if (every > 0 && (records == nullptr || capacity == 0))
    return fail(BRAHMS_E_INVALID_ARG, "a monitor needs a records buffer and capacity >= 1");
  plan->mon_every = every;
  plan->mon_records = every > 0 ? records : nullptr;
  plan->mon_capacity = every > 0 ? capacity : 0;
  plan->mon_count = 0;
  return BRAHMS_OK;
}

brahms_status brahms_get_monitor_count(brahms_plan plan, int* count) {
  if (brahms_status st = check_plan(plan)) return st;
  if (count == nullptr) return fail(BRAHMS_E_INVALID_ARG, "count is NULL");
  *count = plan->mon_count;
  return BRAHMS_OK;
}

brahms_status brahms_set_snapshots(brahms_plan plan, int n, const long long* steps,
                                   void* const* buffers) {
  if (brahms_status st = check_plan(plan)) return st;
  if (n < 0 || (n > 0 && (steps == nullptr || buffers == nullptr)))
    return fail(BRAHMS_E_INVALID_ARG, "need n >= 0 and, for n > 0, steps and buffers");
  std::vector<long long> st(steps, steps + n);
  std::vector<float2*> bufs(size_t(n) * plan->nf);
  for (int i = 0; i < n; ++i) {
    if (st[i] < 1) return fail(BRAHMS_E_INVALID_ARG, "snapshot steps must be >= 1");
    for (int j = 0; j < plan->nf; ++j) {
      void* b = buffers[size_t(i) * plan->nf + j];
      if (b == nullptr) return fail(BRAHMS_E_INVALID_ARG, "snapshot buffer is NULL");
      bufs[size_t(i) * plan->nf + j] = static_cast<float2*>(b);
    }
  }
  plan->snap_steps = std::move(st);
  plan->snap_buffers = std::move(bufs);
  return BRAHMS_OK;
}

}  // extern "C"
