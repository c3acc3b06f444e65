// Adjoint of the z-loop behind the C ABI (brahms_adjoint_*; see
// include/brahms.h and adjoint.hpp).
//
// Forward: the plain z-loop, with the state copied to a checkpoint every K
// steps.  Backward, one K-step segment at a time from the last: recompute the
// segment out of place from its checkpoint, keeping every step's input and
// the input of its second RK4 half-step (for K <= 32 on a second stream,
// into a second set of buffers, while the previous segment is swept back);
// then for each step in reverse apply
// the adjoint passes (reverse second half-step + conj-propagator transforms
// along the last axis, conj-propagator transforms along y, conj-propagator
// transforms along the first axis + reverse first half-step).  dJ/dPhi at the
// six stage positions of every step is reduced on the device in a fixed
// order and turned into dJ/ddk_n on the host: with Phi(z) = Phi_n +
// dk_n (z - z_n) and Phi_n = dz sum_{m<n} dk_m,
//   dJ/ddk_n = sum_stages (z_s - z_n) dJ/dPhi(z_s) [stages of step n]
//            + dz sum_{m>n} sum_stages dJ/dPhi(z_s) [stages of later steps].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/brahms.h"
#include "adjoint.hpp"
#include "launch.hpp"
#include "plan.hpp"

using namespace brahms;
using brahms::detail::align_up;
using brahms::detail::check_plan;
using brahms::detail::fail;
using brahms::detail::kChunk;

namespace {

// Segment buffers come in two sets when a segment fits half of the table
// ring (every <= 32): the reverse sweep of one segment then runs while the
// next one is recomputed into the other set, on its own table rows.
struct AdjLayout {
  size_t ckpt = 0, dphi = 0, total = 0;
  size_t seg[2] = {0, 0}, pre[2] = {0, 0}, parts[2] = {0, 0};
  int nsets = 1;
  int nckpt = 0, every = 0, nsteps = 0;
  size_t field_bytes = 0;
  int max_blocks = 0;
};

constexpr int kSetRows = kChunk / 2;   // table rows of the second set start here

int pass_blocks(int axis, const brahms_plan_s& p) {
  const int n = axis == AX_X ? p.nx : p.nt;
  const long lines = axis == AX_X ? long(p.ny) * p.nt : long(p.nx) * p.ny;
  const int lpb = lines_per_block(n);
  return int((lines + lpb - 1) / lpb);
}

AdjLayout adj_layout(const brahms_plan_s& p, int nsteps, int every) {
  AdjLayout L;
  L.every = every;
  L.nsteps = nsteps;
  L.nckpt = (nsteps + every - 1) / every;
  L.field_bytes = sizeof(float2) * size_t(p.nx) * p.ny * p.nt;
  const size_t state = align_up(L.field_bytes) * p.nf;
  L.max_blocks = std::max(pass_blocks(AX_X, p), pass_blocks(AX_T, p));
  L.nsets = (every <= kSetRows && L.nckpt > 1) ? 2 : 1;
  size_t off = 0;
  L.ckpt = off;
  off += state * L.nckpt;
  for (int s = 0; s < L.nsets; ++s) {
    L.seg[s] = off;
    off += state * (every + 1);
    L.pre[s] = off;
    off += state * every;
    L.parts[s] = off;
    off = align_up(off + sizeof(double) * 3 * L.max_blocks * 2 * every);
  }
  L.dphi = off;
  off = align_up(off + sizeof(double) * 6 * nsteps);
  L.total = off;
  return L;
}

float2* state_field(char* base, const AdjLayout& L, const brahms_plan_s& p, int slot, int j) {
  return reinterpret_cast<float2*>(base + (size_t(slot) * p.nf + j) * align_up(L.field_bytes));
}

hipError_t dispatch_adj(int axis, int at, const brahms_plan_s& p, const AdjArgs& a) {
  const int n = axis == AX_X ? p.nx : p.nt;
  switch (n) {
#define BRAHMS_CASE_(N, N1, N2) \
  case N: brahms::detail::launch_adj_axis<N1, N2>(axis, at, p, a); break;
    BRAHMS_LENGTHS(BRAHMS_CASE_)
#undef BRAHMS_CASE_
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

brahms_status copy_state(const brahms_plan_s& p, float2* const* dst, float2* const* src) {
  const long n = long(p.nx) * p.ny * p.nt;
  for (int j = 0; j < p.nf; ++j)
    hipLaunchKernelGGL(copy_field, dim3(unsigned(std::min<long>((n + 255) / 256, 4096))), dim3(256), 0,
                       p.stream, dst[j], src[j], n);
  HIP_TRY(hipGetLastError());
  return BRAHMS_OK;
}

// One adjoint pass with an RK4 reverse sweep; its per-block phase
// derivatives go to slot (row, k == 0 ? 0 : 1) of the segment's partials.
brahms_status adj_pass(brahms_plan_s& p, const AdjLayout& L, int set, int row, int k,
                       float2* const* g, float2* const* y) {
  const int ax = brahms::detail::pass_axis(p, k);
  const int per_field = p.nx + p.ny + p.nt;
  const int trow = set * kSetRows + row;
  const float2* r = brahms::detail::table_row(p, trow);
  AdjArgs a{};
  for (int j = 0; j < 3; ++j) {
    a.g[j] = j < p.nf ? g[j] : nullptr;
    a.y[j] = j < p.nf ? y[j] : nullptr;
  }
  a.axis_off = ax == AX_X ? 0 : p.nx + p.ny;
  a.tw = r + p.nf * per_field + a.axis_off;
  a.consts = reinterpret_cast<const DftConsts*>(r + (p.nf + 1) * per_field);
  a.prop = r;
  a.field_stride = per_field;
  a.nl = brahms::detail::nl_coefficients(p, trow, k == 0 ? 0 : 1);
  a.nx = p.nx; a.ny = p.ny; a.nt = p.nt;
  double* parts = reinterpret_cast<double*>(p.adj_ws + L.parts[set]);
  a.dphi_out = parts + (size_t(row) * 2 + (k == 0 ? 0 : 1)) * size_t(L.max_blocks) * 3;
  // exp(-i Phi) on the sum-frequency field, exp(+i Phi) on the others
  if (p.nf == 3) {
    a.sigma[0] = -1.f; a.sigma[1] = 1.f; a.sigma[2] = 1.f;
  } else {
    a.sigma[0] = 1.f; a.sigma[1] = -1.f; a.sigma[2] = 0.f;
  }
  HIP_TRY(dispatch_adj(ax, k == 0 ? VJP_LAST : VJP_FIRST, p, a));
  return BRAHMS_OK;
}

// Run steps s0 .. s0+cnt-1 (table rows of the set) out of place through the
// set's segment slots, keeping every step's input (slot i) and the input of
// its second RK4 half-step; the last step writes `last_out` when given.
brahms_status record_segment(brahms_plan_s& p, const AdjLayout& L, int set, int cnt,
                             float2* const* last_out) {
  for (int i = 0; i < cnt; ++i) {
    brahms::detail::StepIO io{};
    for (int j = 0; j < p.nf; ++j) {
      io.in[j] = state_field(p.adj_ws + L.seg[set], L, p, i, j);
      io.out[j] = (i == cnt - 1 && last_out != nullptr)
                      ? last_out[j]
                      : state_field(p.adj_ws + L.seg[set], L, p, i + 1, j);
      io.pre[j] = state_field(p.adj_ws + L.pre[set], L, p, i, j);
    }
    if (brahms_status st = brahms::detail::launch_step(p, set * kSetRows + i, io)) return st;
  }
  return BRAHMS_OK;
}

// Recompute segment c (steps s0 .. s0+cnt-1) from its checkpoint into a set.
brahms_status recompute_segment(brahms_plan_s& p, const AdjLayout& L, int c, int set) {
  const long long s0 = p.adj_n0 + (long long)c * p.adj_every;
  const int cnt = int(std::min<long long>(p.adj_every, p.adj_n0 + p.adj_nsteps - s0));
  if (brahms_status st = brahms::detail::refresh_tables(p, s0, cnt, set * kSetRows)) return st;
  float2* slot0[3] = {nullptr, nullptr, nullptr};
  float2* ck[3] = {nullptr, nullptr, nullptr};
  for (int j = 0; j < p.nf; ++j) {
    slot0[j] = state_field(p.adj_ws + L.seg[set], L, p, 0, j);
    ck[j] = state_field(p.adj_ws + L.ckpt, L, p, c, j);
  }
  if (brahms_status st = copy_state(p, slot0, ck)) return st;
  return record_segment(p, L, set, cnt, nullptr);
}

// Reverse sweep over segment c held in a set, then its dJ/dPhi reduction.
brahms_status reverse_segment(brahms_plan_s& p, const AdjLayout& L, int c, int set, float2* const* g,
                              double* dphi) {
  const long long s0 = p.adj_n0 + (long long)c * p.adj_every;
  const int cnt = int(std::min<long long>(p.adj_every, p.adj_n0 + p.adj_nsteps - s0));
  for (int i = cnt - 1; i >= 0; --i) {
    float2* y2[3] = {nullptr, nullptr, nullptr};
    float2* y0[3] = {nullptr, nullptr, nullptr};
    for (int j = 0; j < p.nf; ++j) {
      y2[j] = state_field(p.adj_ws + L.pre[set], L, p, i, j);
      y0[j] = state_field(p.adj_ws + L.seg[set], L, p, i, j);
    }
    if (brahms_status st = adj_pass(p, L, set, i, 2, g, y2)) return st;
    if (brahms_status st = brahms::detail::launch_linear_pass(p, set * kSetRows + i, AX_Y, g, true))
      return st;
    if (brahms_status st = adj_pass(p, L, set, i, 0, g, y0)) return st;
  }
  // dJ/dPhi of the segment's steps, in a fixed order
  const int nb_first = pass_blocks(brahms::detail::pass_axis(p, 0), p);
  const int nb_last = pass_blocks(brahms::detail::pass_axis(p, 2), p);
  hipLaunchKernelGGL(reduce_dphi_segment, dim3(unsigned(cnt), 2), dim3(256), 0, p.stream,
                     reinterpret_cast<const double*>(p.adj_ws + L.parts[set]), nb_first, nb_last,
                     L.max_blocks, dphi + 6 * (s0 - p.adj_n0));
  HIP_TRY(hipGetLastError());
  return BRAHMS_OK;
}

brahms_status side_stream(brahms_plan_s& p) {
  if (!p.adj_side) HIP_TRY(hipStreamCreateWithFlags(&p.adj_side, hipStreamNonBlocking));
  for (hipEvent_t& e : p.adj_ev)
    if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return BRAHMS_OK;
}

}  // namespace

extern "C" {

brahms_status brahms_adjoint_workspace_size(brahms_plan plan, int nsteps, int checkpoint_every,
                                            size_t* bytes) {
  if (brahms_status st = check_plan(plan)) return st;
  if (bytes == nullptr) return fail(BRAHMS_E_INVALID_ARG, "bytes is NULL");
  if (!plan->dk_map.empty()) return fail(BRAHMS_E_UNSUPPORTED, "no adjoint with a transverse dk map");
  if (brahms::detail::long_tau(*plan)) return fail(BRAHMS_E_UNSUPPORTED, "no adjoint with nt > 256");
  if (plan->order > 1) return fail(BRAHMS_E_UNSUPPORTED, "the adjoint runs with pass order 0 or 1");
  if (nsteps < 1 || checkpoint_every < 1 || checkpoint_every > kChunk)
    return fail(BRAHMS_E_INVALID_ARG, "need nsteps >= 1 and 1 <= checkpoint_every <= 64");
  *bytes = adj_layout(*plan, nsteps, checkpoint_every).total;
  return BRAHMS_OK;
}

brahms_status brahms_adjoint_forward(brahms_plan plan, int nsteps, int checkpoint_every,
                                     void* adj_workspace) {
  if (brahms_status st = check_plan(plan)) return st;
  brahms_plan_s& p = *plan;
  if (!p.bound) return fail(BRAHMS_E_STATE, "brahms_adjoint_forward before brahms_plan_bind");
  if (!p.dk_map.empty()) return fail(BRAHMS_E_UNSUPPORTED, "no adjoint with a transverse dk map");
  if (brahms::detail::long_tau(p)) return fail(BRAHMS_E_UNSUPPORTED, "no adjoint with nt > 256");
  if (p.order > 1) return fail(BRAHMS_E_UNSUPPORTED, "the adjoint runs with pass order 0 or 1");
  if (adj_workspace == nullptr || reinterpret_cast<uintptr_t>(adj_workspace) % 256 != 0)
    return fail(BRAHMS_E_INVALID_ARG, "adjoint workspace must be a 256-byte aligned device pointer");
  if (nsteps < 1 || checkpoint_every < 1 || checkpoint_every > kChunk)
    return fail(BRAHMS_E_INVALID_ARG, "need nsteps >= 1 and 1 <= checkpoint_every <= 64");
  if (!p.dk.empty() && p.step + nsteps > (long long)p.dk.size())
    return fail(BRAHMS_E_INVALID_ARG, "steps beyond the end of the dk profile");
  p.adj_ready = false;
  p.adj_ws = static_cast<char*>(adj_workspace);
  const AdjLayout L = adj_layout(p, nsteps, checkpoint_every);
  p.adj_n0 = p.step;
  p.adj_nsteps = nsteps;
  p.adj_every = checkpoint_every;
  float2* fields[3] = {p.fields[0], p.fields[1], p.fields[2]};
  for (int c = 0; c < L.nckpt - 1; ++c) {
    float2* ck[3] = {nullptr, nullptr, nullptr};
    for (int j = 0; j < p.nf; ++j) ck[j] = state_field(p.adj_ws + L.ckpt, L, p, c, j);
    if (brahms_status st = copy_state(p, ck, fields)) return st;
    if (brahms_status st = brahms_step(plan, checkpoint_every)) return st;
  }
  // the last segment is recorded as the backward sweep needs it, so that
  // sweep starts without recomputing it
  const int cnt = nsteps - (L.nckpt - 1) * checkpoint_every;
  float2* slot0[3] = {nullptr, nullptr, nullptr};
  for (int j = 0; j < p.nf; ++j) slot0[j] = state_field(p.adj_ws + L.seg[0], L, p, 0, j);
  if (brahms_status st = copy_state(p, slot0, fields)) return st;
  if (brahms_status st = brahms::detail::refresh_tables(p, p.step, cnt)) return st;
  if (brahms_status st = record_segment(p, L, 0, cnt, fields)) return st;
  p.step += cnt;
  p.adj_last_recorded = true;
  p.adj_ready = true;
  return BRAHMS_OK;
}

brahms_status brahms_adjoint(brahms_plan plan, int nsteps, int checkpoint_every, const void* const* fields_in,
                             const void* const* grad_out, void* const* grad_in, double* grad_dk,
                             void* adj_workspace) {
  if (brahms_status st = check_plan(plan)) return st;
  brahms_plan_s& p = *plan;
  if (!p.bound) return fail(BRAHMS_E_STATE, "brahms_adjoint before brahms_plan_bind");
  if (fields_in == nullptr || grad_out == nullptr || grad_in == nullptr)
    return fail(BRAHMS_E_INVALID_ARG, "fields_in, grad_out and grad_in must not be NULL");
  for (int j = 0; j < p.nf; ++j)
    if (fields_in[j] == nullptr || grad_out[j] == nullptr || grad_in[j] == nullptr)
      return fail(BRAHMS_E_INVALID_ARG, "NULL field or cotangent pointer");
  // the forward runs in the plan's bound fields, from fields_in
  float2* dst[3] = {nullptr, nullptr, nullptr};
  float2* src[3] = {nullptr, nullptr, nullptr};
  bool copy = false;
  for (int j = 0; j < p.nf; ++j) {
    dst[j] = p.fields[j];
    src[j] = static_cast<float2*>(const_cast<void*>(fields_in[j]));
    copy = copy || dst[j] != src[j];
  }
  if (copy)
    if (brahms_status st = copy_state(p, dst, src)) return st;
  if (brahms_status st = brahms_adjoint_forward(plan, nsteps, checkpoint_every, adj_workspace)) return st;
  // the reverse sweep works in place in grad_in, from grad_out
  copy = false;
  for (int j = 0; j < p.nf; ++j) {
    dst[j] = static_cast<float2*>(grad_in[j]);
    src[j] = static_cast<float2*>(const_cast<void*>(grad_out[j]));
    copy = copy || dst[j] != src[j];
  }
  if (copy)
    if (brahms_status st = copy_state(p, dst, src)) return st;
  return brahms_adjoint_backward(plan, grad_in, grad_dk);
}

brahms_status brahms_adjoint_backward(brahms_plan plan, void* const* grad, double* grad_dk) {
  if (brahms_status st = check_plan(plan)) return st;
  brahms_plan_s& p = *plan;
  if (!p.adj_ready) return fail(BRAHMS_E_STATE, "brahms_adjoint_backward before brahms_adjoint_forward");
  if (grad == nullptr) return fail(BRAHMS_E_INVALID_ARG, "grad is NULL");
  for (int j = 0; j < p.nf; ++j)
    if (grad[j] == nullptr || reinterpret_cast<uintptr_t>(grad[j]) % 8 != 0)
      return fail(BRAHMS_E_INVALID_ARG, "grad pointers must be non-NULL and 8-byte aligned");
  const AdjLayout L = adj_layout(p, p.adj_nsteps, p.adj_every);
  float2* g[3] = {nullptr, nullptr, nullptr};
  for (int j = 0; j < p.nf; ++j) g[j] = static_cast<float2*>(grad[j]);
  double* dphi = reinterpret_cast<double*>(p.adj_ws + L.dphi);
  hipLaunchKernelGGL(zero_doubles, dim3(64), dim3(256), 0, p.stream, dphi, long(6) * p.adj_nsteps);
  HIP_TRY(hipGetLastError());
  const long long saved_step = p.step;
  const int last = L.nckpt - 1;
  if (L.nsets == 1) {
    for (int c = last; c >= 0; --c) {
      if (c != last || !p.adj_last_recorded)
        if (brahms_status st = recompute_segment(p, L, c, 0)) return st;
      if (brahms_status st = reverse_segment(p, L, c, 0, g, dphi)) return st;
    }
  } else {
    // Segment c lives in set (last - c) % 2.  While the caller's stream
    // sweeps segment c backwards, the side stream recomputes segment c - 1
    // into the other set, once the sweep of segment c + 1 has released it.
    if (brahms_status st = side_stream(p)) return st;
    hipEvent_t ev_start = p.adj_ev[0], *ev_ready = p.adj_ev + 1, *ev_free = p.adj_ev + 3;
    const hipStream_t main = p.stream;
    if (!p.adj_last_recorded)
      if (brahms_status st = recompute_segment(p, L, last, 0)) return st;
    HIP_TRY(hipEventRecord(ev_start, main));
    HIP_TRY(hipStreamWaitEvent(p.adj_side, ev_start, 0));
    brahms_status st = BRAHMS_OK;
    for (int c = last; c >= 0 && st == BRAHMS_OK; --c) {
      const int set = (last - c) % 2, other = 1 - set;
      if (c > 0) {
        if (c < last) HIP_TRY(hipStreamWaitEvent(p.adj_side, ev_free[other], 0));
        p.stream = p.adj_side;
        st = recompute_segment(p, L, c - 1, other);
        p.stream = main;
        if (st != BRAHMS_OK) break;
        HIP_TRY(hipEventRecord(ev_ready[other], p.adj_side));
      }
      if (c < last) HIP_TRY(hipStreamWaitEvent(main, ev_ready[set], 0));
      st = reverse_segment(p, L, c, set, g, dphi);
      if (st != BRAHMS_OK) break;
      HIP_TRY(hipEventRecord(ev_free[set], main));
    }
    p.stream = main;
    if (st != BRAHMS_OK) return st;
  }
  p.adj_last_recorded = false;
  p.step = saved_step;
  if (grad_dk != nullptr) {
    std::vector<double> G(size_t(6) * p.adj_nsteps);
    HIP_TRY(hipMemcpyAsync(G.data(), dphi, sizeof(double) * G.size(), hipMemcpyDeviceToHost, p.stream));
    HIP_TRY(hipStreamSynchronize(p.stream));
    // stage offsets z - z_n of the six dJ/dPhi entries of a step
    const double off[6] = {0.0, 0.25 * p.dz, 0.5 * p.dz, 0.5 * p.dz, 0.75 * p.dz, p.dz};
    if (p.dk.empty()) {
      // Phi = dk z: dJ/ddk = sum over stages of z_s dJ/dPhi(z_s)
      double acc = 0.0;
      for (int r = 0; r < p.adj_nsteps; ++r)
        for (int k = 0; k < 6; ++k)
          acc += (double(p.adj_n0 + r) * p.dz + off[k]) * G[size_t(6) * r + k];
      grad_dk[0] = acc;
    } else {
      const long long ndk = (long long)p.dk.size();
      for (long long m = 0; m < ndk; ++m) grad_dk[m] = 0.0;
      double later = 0.0;  // sum of dJ/dPhi over stages of steps after the current one
      for (int r = p.adj_nsteps - 1; r >= 0; --r) {
        double own = 0.0, tot = 0.0;
        for (int k = 0; k < 6; ++k) {
          own += off[k] * G[size_t(6) * r + k];
          tot += G[size_t(6) * r + k];
        }
        grad_dk[p.adj_n0 + r] = own + p.dz * later;
        later += tot;
      }
      for (long long m = 0; m < p.adj_n0; ++m) grad_dk[m] = p.dz * later;
    }
  }
  return BRAHMS_OK;
}

}  // extern "C"
