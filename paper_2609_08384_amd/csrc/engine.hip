// Host engine and C ABI of the chi(2) split-step z-loop (see include/brahms.h).
//
// A plan holds only host-side state.  Device state lives in caller memory:
// the fields, and one workspace holding the axis twiddles, the integrated
// mismatch profile, and a ring of per-step tables (propagators and RK4
// coefficients) that a small kernel refills every kChunk steps.  A z-step is
// three launches on the caller's stream, one per axis in the schedule's pass
// order (e.g. X pass: RK4 half-step + x line transforms, Y pass: y line
// transforms, T pass: tau line transforms + RK4 half-step); five launches
// when the tau axis is longer than 256.  With merged half-steps one RK4 step
// of size dz joins consecutive steps; with fused step pairs the steps
// alternate their axis order and one launch ends a step and begins the next
// (two launches per step, four with a long tau axis).  With the graph
// schedule whole chunks are replayed from a hipGraph.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/brahms.h"
#include "kernels.hpp"
#include "launch.hpp"
#include "plan.hpp"

using namespace brahms;
using brahms::detail::fail;
using brahms::detail::kAlign;
using brahms::detail::kChunk;
using brahms::detail::kTableRows;
using brahms::detail::kDiagChunks;
using brahms::detail::align_up;

namespace brahms {
namespace detail {

thread_local std::string g_last_error;

brahms_status fail(brahms_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

brahms_status check_plan(brahms_plan p) {
  if (p == nullptr) return fail(BRAHMS_E_INVALID_ARG, "plan is NULL");
  return BRAHMS_OK;
}

}  // namespace detail
}  // namespace brahms

using brahms::detail::check_plan;

namespace {

// tau axes longer than one line transform: nt = A B, transformed in three
// passes (b transforms, a transforms with the propagator, inverse b)
bool supported_long_tau(int n) { return n == 512 || n == 1024 || n == 2048 || n == 4096; }

// One pass along an axis of length n (a supported line length), with the
// second split of that length when alt is set and it has one.
hipError_t dispatch_axis(int n, bool alt, int axis, int nl, int nf, const brahms_plan_s& p, PassArgs a) {
  if (alt) {
    switch (n) {
#define BRAHMS_CASE_(N, N1, N2) \
  case N: return brahms::detail::launch_axis<N1, N2>(axis, nl, nf, p, a);
      BRAHMS_ALT_LENGTHS(BRAHMS_CASE_)
#undef BRAHMS_CASE_
      default: break;
    }
  }
  switch (n) {
#define BRAHMS_CASE_(N, N1, N2) \
  case N: return brahms::detail::launch_axis<N1, N2>(axis, nl, nf, p, a);
    BRAHMS_LENGTHS(BRAHMS_CASE_)
#undef BRAHMS_CASE_
    default: return hipErrorInvalidValue;
  }
}

template <int AX>
hipError_t dispatch_long_len(int len, int nl, int nf, const brahms_plan_s& p, const PassArgs& a) {
  switch (len) {
#define BRAHMS_CASE_(N, N1, N2) \
  case N: return brahms::detail::launch_long<N1, N2, AX>(nl, nf, p, a);
    BRAHMS_LONG_SUBLENGTHS(BRAHMS_CASE_)
#undef BRAHMS_CASE_
    default: return hipErrorInvalidValue;
  }
}

hipError_t dispatch_long(int axis, int nl, int nf, const brahms_plan_s& p, const PassArgs& a) {
  const int na = brahms::detail::long_tau_a(p.nt);
  const int nb = p.nt / na;
  if (axis == AX_TAF) return dispatch_long_len<AX_TAF>(nb, nl, nf, p, a);
  if (axis == AX_TB) return dispatch_long_len<AX_TB>(na, nl, nf, p, a);
  return dispatch_long_len<AX_TAI>(nb, nl, nf, p, a);
}

bool finite_params(const brahms_params* pr, int nf) {
  if (!std::isfinite(pr->dz) || !std::isfinite(pr->dk_const) || !std::isfinite(pr->dx) ||
      !std::isfinite(pr->dy) || !std::isfinite(pr->dt))
    return false;
  for (int j = 0; j < nf; ++j) {
    const brahms_field_params& f = pr->field[j];
    const double v[7] = {f.kappa, f.diffraction, f.tan_rho, f.delay, f.k2, f.k3, f.alpha};
    for (double x : v)
      if (!std::isfinite(x)) return false;
  }
  return true;
}

void layout(brahms_plan_s& p) {
  size_t off = 0;
  p.off_phi0 = off;
  off = align_up(off + sizeof(double) * (p.dk.size() + 1));
  p.off_dk = off;
  off = align_up(off + sizeof(double) * (p.dk.size() + 1));
  p.off_prop = off;
  off = align_up(off + sizeof(float2) * size_t(kTableRows) * table_row_stride(p.nf, p.nx, p.ny, p.nt));
  p.off_nl = off;
  off = align_up(off + sizeof(float2) * size_t(kTableRows) * 2 * p.nf * kNlCoef);
  p.off_flag = off;
  off = align_up(off + sizeof(int));
  p.off_diag = off;
  off = align_up(off + sizeof(double) * size_t(kDiagChunks) * p.nf * p.nt);
  p.off_n0 = off;
  off = align_up(off + 2 * sizeof(long long));
  if (!p.dk_map.empty()) {
    // phase tables of a whole 64-step chunk when they take at most 64 MB,
    // else one step at a time
    const size_t row = sizeof(float2) * 5 * p.dk_map.size();
    p.map_rows = row * kChunk <= (size_t(64) << 20) ? kChunk : 1;
    p.off_map = off;
    off = align_up(off + sizeof(double) * p.dk_map.size());
    p.off_maptab = off;
    off = align_up(off + row * size_t(p.map_rows));
    p.off_psi0 = off;
    off = align_up(off + sizeof(double) * (p.map_scale.size() + 1));
    p.off_scale = off;
    off = align_up(off + sizeof(double) * (p.map_scale.size() + 1));
  }
  p.ws_size = off;
}

__global__ void clear_flag(int* flag) { *flag = 0; }

constexpr size_t kMaxTimed = 65536;

brahms_status take_event(brahms_plan_s& p, hipEvent_t* ev) {
  if (!p.pool.empty()) {
    *ev = p.pool.back();
    p.pool.pop_back();
    return BRAHMS_OK;
  }
  HIP_TRY(hipEventCreate(ev));
  return BRAHMS_OK;
}

// Record a start event before a launch of the given kind (when timing).
brahms_status timing_start(brahms_plan_s& p, int kind) {
  if (!p.timing || p.timed.size() >= kMaxTimed) return BRAHMS_OK;
  brahms_plan_s::Timed t{kind, nullptr, nullptr};
  if (brahms_status st = take_event(p, &t.start)) return st;
  if (brahms_status st = take_event(p, &t.stop)) return st;
  HIP_TRY(hipEventRecord(t.start, p.stream));
  p.timed.push_back(t);
  return BRAHMS_OK;
}

// Record the stop event of the launch opened by the last timing_start.
brahms_status timing_stop(brahms_plan_s& p) {
  if (!p.timing || p.timed.empty() || p.timed.size() > kMaxTimed) return BRAHMS_OK;
  HIP_TRY(hipEventRecord(p.timed.back().stop, p.stream));
  return BRAHMS_OK;
}

}  // namespace

namespace brahms {
namespace detail {

const float2* table_row(const brahms_plan_s& p, int row) {
  return reinterpret_cast<const float2*>(p.ws + p.off_prop) +
         size_t(row) * table_row_stride(p.nf, p.nx, p.ny, p.nt);
}

const float2* nl_coefficients(const brahms_plan_s& p, int row, int half) {
  return reinterpret_cast<const float2*>(p.ws + p.off_nl) + (size_t(row) * 2 + half) * p.nf * kNlCoef;
}

int pass_axis(const brahms_plan_s& p, int k) {
  // orders 0: x y tau, 1: tau y x, 2: x tau y, 3: y tau x
  static const int axes[4][3] = {{AX_X, AX_Y, AX_T}, {AX_T, AX_Y, AX_X},
                                 {AX_X, AX_T, AX_Y}, {AX_Y, AX_T, AX_X}};
  // the transverse map runs only on x and tau passes: orders 2 and 3 fall
  // back to 0 and 1 for a plan with a map
  const int order = p.dk_map.empty() ? p.order : (p.order & 1);
  return axes[order][k];
}

StepPasses step_passes(const brahms_plan_s& p, bool batched) {
  StepPasses s{};
  if (long_tau(p)) {
    const int ax[5] = {AX_X, AX_Y, AX_TAF, AX_TB, AX_TAI};
    s.n = 5;
    for (int k = 0; k < 5; ++k) {
      s.ax[k] = ax[k];
      s.nl[k] = k == 0 ? NL_BEFORE : (k == 4 ? NL_AFTER : NL_NONE);
    }
    return s;
  }
  // A length-1 axis pass is the identity transform times that axis's
  // propagator entry at zero frequency: exactly 1 along x and y, and along
  // tau unless a field has loss (exp(-alpha dz / 2) sits in the tau table).
  const bool no_map = p.dk_map.empty();
  bool lossless = true;
  for (int j = 0; j < p.nf; ++j) lossless = lossless && p.fp[j].alpha == 0.0;
  if (no_map && p.nx == 1 && p.ny == 1 && p.nt > 1) {
    s.n = 1;
    s.ax[0] = AX_T;
    s.nl[0] = NL_BOTH;
    return s;
  }
  if (batched && no_map && lossless && p.nt == 1 && p.nx > 1 && p.ny > 1) {
    s.n = 2;
    const bool x_first = p.order == 0 || p.order == 2;
    s.ax[0] = x_first ? int(AX_X) : int(AX_Y);
    s.ax[1] = x_first ? int(AX_Y) : int(AX_X);
    s.nl[0] = NL_BEFORE;
    s.nl[1] = NL_AFTER;
    return s;
  }
  s.n = 3;
  for (int k = 0; k < 3; ++k) {
    s.ax[k] = pass_axis(p, k);
    s.nl[k] = k == 0 ? NL_BEFORE : (k == 2 ? NL_AFTER : NL_NONE);
  }
  return s;
}

namespace {
brahms_status map_table(brahms_plan_s& p, long long n0, int count);
}  // namespace

bool merging(const brahms_plan_s& p) {
  return p.merge && p.dk.empty() && p.dk_map.empty() && p.mon_every == 0 && p.snap_steps.empty();
}

bool fusing(const brahms_plan_s& p) {
  return p.fuse && merging(p) && (long_tau(p) || step_passes(p, false).n == 3);
}

brahms_status refresh_tables(brahms_plan_s& p, long long n0, int count, int row0,
                             long long merge_last) {
  if (count < 0 || row0 < 0 || row0 + count > kTableRows ||
      (!p.dk_map.empty() && p.map_rows == kChunk && count > kChunk))
    return fail(BRAHMS_E_INVALID_ARG, "table rows out of range");
  const int per_field = p.nx + p.ny + p.nt;
  TableArgs ta{};
  ta.row_stride = table_row_stride(p.nf, p.nx, p.ny, p.nt);
  ta.rows = reinterpret_cast<float2*>(p.ws + p.off_prop) + size_t(row0) * ta.row_stride;
  ta.nl = reinterpret_cast<float2*>(p.ws + p.off_nl) + size_t(row0) * 2 * p.nf * kNlCoef;
  ta.phi0 = p.dk.empty() ? nullptr : reinterpret_cast<const double*>(p.ws + p.off_phi0);
  ta.dk = p.dk.empty() ? nullptr : reinterpret_cast<const double*>(p.ws + p.off_dk);
  ta.n0 = n0;
  ta.n0_dev = p.table_n0_dev;
  ta.merge_last = merge_last;
  ta.count = count;
  p.table_n0 = n0;
  ta.nx = p.nx; ta.ny = p.ny; ta.nt = p.nt; ta.nf = p.nf;
  ta.dz = p.dz; ta.dx = p.dx; ta.dy = p.dy; ta.dt = p.dt; ta.dk_const = p.dk_const;
  for (int j = 0; j < p.nf; ++j) {
    const brahms_field_params& f = p.fp[j];
    ta.fc[j] = FieldCoef{f.kappa, f.diffraction, f.tan_rho, f.delay, f.k2, f.k3, f.alpha};
  }
  const long total = long(count) * ((p.nf + 1) * per_field + 1) + long(count) * 2 * p.nf;
  const bool timed = p.timing && p.timed.size() < kMaxTimed;
  if (brahms_status st = timing_start(p, 3)) return st;
  hipLaunchKernelGGL(step_tables, dim3(unsigned((total + 255) / 256)), dim3(256), 0, p.stream, ta);
  HIP_TRY(hipGetLastError());
  if (!p.dk_map.empty() && p.map_rows == kChunk) {
    if (row0 != 0) return fail(BRAHMS_E_UNSUPPORTED, "map tables are filled from row 0");
    if (brahms_status st = map_table(p, n0, count)) return st;
  }
  if (timed)
    if (brahms_status st = timing_stop(p)) return st;
  return BRAHMS_OK;
}

namespace {

PassArgs pass_args(const brahms_plan_s& p, int row, int ax) {
  const int per_field = p.nx + p.ny + p.nt;
  const float2* r = table_row(p, row);
  PassArgs a{};
  a.axis_off = (ax == AX_X) ? 0 : (ax == AX_Y ? p.nx : p.nx + p.ny);
  a.tw = r + p.nf * per_field + a.axis_off;
  a.consts = reinterpret_cast<const DftConsts*>(r + (p.nf + 1) * per_field);
  a.nx = p.nx; a.ny = p.ny; a.nt = p.nt;
  a.prop = r;
  a.field_stride = per_field;
  return a;
}

brahms_status timed_dispatch(brahms_plan_s& p, int ax, int nlmode, const PassArgs& a) {
  const bool timed = p.timing && p.timed.size() < kMaxTimed;
  if (brahms_status st = timing_start(p, long_tau_kind(ax) ? int(AX_T) : ax)) return st;
  if (long_tau_kind(ax)) {
    HIP_TRY(dispatch_long(ax, nlmode, p.nf, p, a));
  } else {
    const int n[3] = {p.nx, p.ny, p.nt};
    HIP_TRY(dispatch_axis(n[ax], ((p.split >> ax) & 1) != 0, ax, nlmode, p.nf, p, a));
  }
  if (timed)
    if (brahms_status st = timing_stop(p)) return st;
  return BRAHMS_OK;
}

// The transverse phase factors of steps n0 .. n0 + count - 1 at their five
// stage offsets, into table rows 0 .. count - 1.
brahms_status map_table(brahms_plan_s& p, long long n0, int count) {
  MapArgs m{};
  m.map = reinterpret_cast<const double*>(p.ws + p.off_map);
  m.psi0 = p.map_scale.empty() ? nullptr : reinterpret_cast<const double*>(p.ws + p.off_psi0);
  m.scale = p.map_scale.empty() ? nullptr : reinterpret_cast<const double*>(p.ws + p.off_scale);
  m.out = reinterpret_cast<float2*>(p.ws + p.off_maptab);
  m.plane = unsigned(p.dk_map.size());
  m.n0 = n0;
  m.n0_dev = p.table_n0_dev;
  m.dz = p.dz;
  hipLaunchKernelGGL(map_phase_table, dim3((m.plane + 255) / 256, unsigned(count)), dim3(256), 0,
                     p.stream, m);
  HIP_TRY(hipGetLastError());
  return BRAHMS_OK;
}

}  // namespace

brahms_status launch_step(brahms_plan_s& p, int row, const StepIO& io, bool continued) {
  const bool map = !p.dk_map.empty();
  if (map && p.map_rows == 1)
    if (brahms_status st = map_table(p, p.table_n0 + row, 1)) return st;
  const size_t map_row = map ? size_t(p.map_rows == 1 ? 0 : row) * 5 * p.dk_map.size() : 0;
  // the first pass carries the first RK4 half-step, the last pass the second
  // one (the axis operators commute)
  const StepPasses sp = step_passes(p, false);
  if (continued && map) return fail(BRAHMS_E_UNSUPPORTED, "merged half-steps with a map");
  for (int k = 0; k < sp.n; ++k) {
    const int ax = sp.ax[k];
    const bool first = k == 0, last = k == sp.n - 1;
    int nlmode = first && continued ? (sp.nl[k] & ~NL_BEFORE) : sp.nl[k];
    PassArgs a = pass_args(p, row, ax);
    if (map && nlmode != NL_NONE) {
      nlmode |= NL_MAP;
      a.map = reinterpret_cast<const float2*>(p.ws + p.off_maptab) + map_row +
              (first ? 0 : 2) * p.dk_map.size();
    }
    for (int j = 0; j < 3; ++j) {
      a.f[j] = first ? io.in[j] : io.out[j];
      a.fo[j] = io.out[j];
      a.pre[j] = last ? io.pre[j] : nullptr;
    }
    a.nl = nl_coefficients(p, row, 0);
    a.nl2 = nl_coefficients(p, row, 1);
    if (brahms_status st = timed_dispatch(p, ax, nlmode, a)) return st;
  }
  return BRAHMS_OK;
}

brahms_status launch_fused_step(brahms_plan_s& p, int row, bool first, bool last, bool odd) {
  // axes a, m, b of the schedule; odd steps run them as b, m, a.  A long
  // tau axis is the middle one (its three passes), with x and y at the ends.
  const bool lt = long_tau(p);
  int a0 = pass_axis(p, 0), b0 = pass_axis(p, 2);
  if (lt) {
    a0 = (p.order & 1) ? int(AX_Y) : int(AX_X);
    b0 = (p.order & 1) ? int(AX_X) : int(AX_Y);
  }
  const int mids[3] = {lt ? int(AX_TAF) : pass_axis(p, 1), int(AX_TB), int(AX_TAI)};
  const int nmid = lt ? 3 : 1;
  const int lead = odd ? b0 : a0, tail = odd ? a0 : b0;
  auto in_place = [&](PassArgs& a) {
    for (int j = 0; j < 3; ++j) {
      a.f[j] = p.fields[j];
      a.fo[j] = p.fields[j];
    }
    a.nl = nl_coefficients(p, row, 0);
    a.nl2 = nl_coefficients(p, row, 1);
  };
  if (first) {
    // the call's first step: its own first half-step, then its first axis
    PassArgs a = pass_args(p, row, lead);
    in_place(a);
    if (brahms_status st = timed_dispatch(p, lead, NL_BEFORE, a)) return st;
  }
  for (int k = 0; k < nmid; ++k) {
    PassArgs a = pass_args(p, row, mids[k]);
    in_place(a);
    if (brahms_status st = timed_dispatch(p, mids[k], NL_NONE, a)) return st;
  }
  PassArgs a = pass_args(p, row, tail);
  in_place(a);
  if (last) return timed_dispatch(p, tail, NL_AFTER, a);   // its own second half-step
  // the RK4 step of size dz from z_n + dz/2, then step n+1's first axis
  const PassArgs next = pass_args(p, row + 1, tail);
  a.tw2 = next.tw;
  a.prop2 = next.prop;
  a.consts2 = next.consts;
  return timed_dispatch(p, tail, NL_AFTER | NL_FUSE, a);
}

brahms_status launch_linear_pass(brahms_plan_s& p, int row, int axis, float2* const* fields,
                                 bool conj) {
  if (axis != AX_Y) return fail(BRAHMS_E_INVALID_ARG, "linear-only passes run along y");
  PassArgs a = pass_args(p, row, axis);
  for (int j = 0; j < 3; ++j) {
    a.f[j] = fields[j];
    a.fo[j] = fields[j];
  }
  a.conj = conj ? 1 : 0;
  return timed_dispatch(p, axis, NL_NONE, a);
}

}  // namespace detail
}  // namespace brahms

namespace {

detail::StepIO plain_io(const brahms_plan_s& p) {
  detail::StepIO io{};
  for (int j = 0; j < 3; ++j) {
    io.in[j] = p.fields[j];
    io.out[j] = p.fields[j];
  }
  return io;
}

// A whole 64-step chunk can be replayed from the plan's graph: no per-step
// host work (timing, monitors, snapshots, one-step map tables) is wanted.
bool graph_chunk_ok(const brahms_plan_s& p) {
  return p.use_graph && p.bound && !p.timing && p.mon_every == 0 && p.snap_steps.empty() &&
         (p.dk_map.empty() || p.map_rows == kChunk);
}

void drop_chunk_graph(brahms_plan_s& p) {
  if (p.chunk_exec) (void)hipGraphExecDestroy(p.chunk_exec);
  if (p.chunk_graph) (void)hipGraphDestroy(p.chunk_graph);
  p.chunk_exec = nullptr;
  p.chunk_graph = nullptr;
}

// Capture the tables and the 64 steps of one chunk on a private stream; the
// tables read the chunk's first step (and, with merged halves, the run's last
// step) from the workspace, set before each replay; everything else is the
// same for every chunk.  With merged halves the captured chunk continues a
// run: none of its steps has a first half-step of its own.
brahms_status build_chunk_graph(brahms_plan_s& p) {
  drop_chunk_graph(p);
  if (!p.capture_stream) HIP_TRY(hipStreamCreateWithFlags(&p.capture_stream, hipStreamNonBlocking));
  const hipStream_t user = p.stream;
  const long long saved_n0 = p.table_n0;
  p.stream = p.capture_stream;
  p.table_n0_dev = reinterpret_cast<const long long*>(p.ws + p.off_n0);
  brahms_status st = BRAHMS_OK;
  hipError_t e = hipStreamBeginCapture(p.capture_stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const detail::StepIO io = plain_io(p);
    if (detail::fusing(p)) {
      // an inner chunk of a call with fused step pairs (it starts on an
      // even step of the call and does not hold the call's last step)
      st = detail::refresh_tables(p, 0, kChunk + 1);
      for (int s = 0; s < kChunk && st == BRAHMS_OK; ++s)
        st = detail::launch_fused_step(p, s, false, false, (s & 1) != 0);
    } else {
      const bool continued = detail::merging(p);
      st = detail::refresh_tables(p, 0, kChunk);
      for (int s = 0; s < kChunk && st == BRAHMS_OK; ++s) st = detail::launch_step(p, s, io, continued);
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p.capture_stream, &g);
    if (st == BRAHMS_OK && e == hipSuccess) {
      p.chunk_graph = g;
      hipGraphExec_t exec = nullptr;
      e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      if (e == hipSuccess) p.chunk_exec = exec;   // drop_chunk_graph releases only what exists
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
  }
  p.stream = user;
  p.table_n0_dev = nullptr;
  p.table_n0 = saved_n0;
  if (st != BRAHMS_OK) {
    drop_chunk_graph(p);
    return st;
  }
  if (e != hipSuccess) {
    drop_chunk_graph(p);
    return fail(BRAHMS_E_DEVICE, std::string("chunk graph capture: ") + hipGetErrorString(e));
  }
  return BRAHMS_OK;
}

// nsteps z-steps from p.step.  With merged halves, the first step of the call
// keeps its first half-step, every step but the last ends with one RK4 step
// of size dz that also covers the next step's first half, and the last ends
// on its own second half-step, so the fields after the call are those at a
// step boundary.
// Fused step pairs: the call's steps alternate their axis order (even steps
// relative to the call's first take the schedule's order, odd ones its
// reverse), so each step but the last ends with one pass that holds its last
// transform, the merged RK4 step and the next step's first transform.  The
// tables of a chunk hold one more row, the next step's.  Graph replays take
// the inner chunks (from an even step, not holding the call's last step).
brahms_status run_fused(brahms_plan_s& p, int nsteps) {
  const long long merge_last = p.step + nsteps - 1;
  int done = 0;
  while (done < nsteps) {
    const int count = std::min(kChunk, nsteps - done);
    if (count == kChunk && graph_chunk_ok(p) && done > 0 && done + kChunk < nsteps) {
      if (!p.chunk_exec)
        if (brahms_status st = build_chunk_graph(p)) return st;
      hipLaunchKernelGGL(set_step_index, dim3(1), dim3(1), 0, p.stream,
                         reinterpret_cast<long long*>(p.ws + p.off_n0), p.step, merge_last);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipGraphLaunch(p.chunk_exec, p.stream));
      p.table_n0 = p.step;
      p.step += count;
      done += count;
      continue;
    }
    if (brahms_status st = detail::refresh_tables(p, p.step, count + 1, 0, merge_last)) return st;
    for (int s = 0; s < count; ++s) {
      const int g = done + s;
      if (brahms_status st = detail::launch_fused_step(p, s, g == 0, g == nsteps - 1, (g & 1) != 0))
        return st;
    }
    p.step += count;
    done += count;
  }
  return BRAHMS_OK;
}

brahms_status run_steps(brahms_plan_s& p, int nsteps) {
  if (detail::fusing(p)) return run_fused(p, nsteps);
  const detail::StepIO io = plain_io(p);
  const bool merge = detail::merging(p);
  const long long merge_last = merge ? p.step + nsteps - 1 : -1;
  int done = 0;
  while (done < nsteps) {
    const int count = std::min(kChunk, nsteps - done);
    // a captured chunk has no leading half-step when merging, so the call's
    // first chunk runs eagerly
    if (count == kChunk && graph_chunk_ok(p) && !(merge && done == 0)) {
      if (!p.chunk_exec)
        if (brahms_status st = build_chunk_graph(p)) return st;
      hipLaunchKernelGGL(set_step_index, dim3(1), dim3(1), 0, p.stream,
                         reinterpret_cast<long long*>(p.ws + p.off_n0), p.step, merge_last);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipGraphLaunch(p.chunk_exec, p.stream));
      p.table_n0 = p.step;
      p.step += count;
      done += count;
      continue;
    }
    if (brahms_status st = detail::refresh_tables(p, p.step, count, 0, merge_last)) return st;
    const bool watch = p.mon_every > 0 || !p.snap_steps.empty();
    for (int s = 0; s < count; ++s) {
      const bool continued = merge && (done > 0 || s > 0);
      if (brahms_status st = detail::launch_step(p, s, io, continued)) return st;
      if (watch)
        if (brahms_status st = detail::after_step(p, p.step + s + 1)) return st;
    }
    p.step += count;
    done += count;
  }
  return BRAHMS_OK;
}

}  // namespace

extern "C" {

const char* brahms_last_error(void) { return brahms::detail::g_last_error.c_str(); }

brahms_status brahms_plan_create(int nx, int ny, int nt, int nfields, const brahms_params* params,
                                 void* hip_stream, brahms_plan* out) {
  brahms::detail::g_last_error.clear();
  if (out == nullptr) return fail(BRAHMS_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (params == nullptr) return fail(BRAHMS_E_INVALID_ARG, "params is NULL");
  if (nx < 1 || ny < 1 || nt < 1) return fail(BRAHMS_E_INVALID_ARG, "axis length < 1");
  if (nfields != 2 && nfields != 3) return fail(BRAHMS_E_INVALID_ARG, "nfields must be 2 or 3");
  if (!finite_params(params, nfields)) return fail(BRAHMS_E_INVALID_ARG, "non-finite parameter");
  if (!(params->dz > 0.0)) return fail(BRAHMS_E_INVALID_ARG, "dz must be > 0");
  if (params->dx < 0.0 || params->dy < 0.0 || params->dt < 0.0)
    return fail(BRAHMS_E_INVALID_ARG, "negative grid spacing");
  if (params->dk != nullptr && params->n_dk < 1)
    return fail(BRAHMS_E_INVALID_ARG, "dk profile given with n_dk < 1");
  if (params->dk_map_scale != nullptr && (params->dk_map == nullptr || params->n_dk_map_scale < 1))
    return fail(BRAHMS_E_INVALID_ARG, "dk_map_scale needs dk_map and n_dk_map_scale >= 1");
  if (!brahms::line_length(nx) || !brahms::line_length(ny) ||
      !(brahms::line_length(nt) || supported_long_tau(nt)))
    return fail(BRAHMS_E_UNSUPPORTED,
                "axis lengths must be 2^a, 3 * 2^a or 9 * 2^a up to 256 (1, 2, 3, 4, 6, 8, 9, 12, 16, "
                "18, 24, 32, 36, 48, 64, 72, 96, 128, 144, 192, 256; tau also 512, 1024, 2048, 4096)");
  auto* p = new brahms_plan_s();
  p->nx = nx; p->ny = ny; p->nt = nt; p->nf = nfields;
  p->dz = params->dz;
  p->dx = params->dx > 0 ? params->dx : 1.0;
  p->dy = params->dy > 0 ? params->dy : 1.0;
  p->dt = params->dt > 0 ? params->dt : 1.0;
  p->dk_const = params->dk_const;
  if (params->dk != nullptr) {
    p->dk.assign(params->dk, params->dk + params->n_dk);
    for (double v : p->dk)
      if (!std::isfinite(v)) {
        delete p;
        return fail(BRAHMS_E_INVALID_ARG, "non-finite dk entry");
      }
    p->phi0.resize(p->dk.size() + 1);
    p->phi0[0] = 0.0;
    for (size_t k = 0; k < p->dk.size(); ++k) p->phi0[k + 1] = p->phi0[k] + p->dk[k] * p->dz;
  }
  if (params->dk_map != nullptr) {
    p->dk_map.assign(params->dk_map, params->dk_map + size_t(nx) * ny);
    bool ok = true;
    for (double v : p->dk_map) ok = ok && std::isfinite(v);
    if (params->dk_map_scale != nullptr) {
      p->map_scale.assign(params->dk_map_scale, params->dk_map_scale + params->n_dk_map_scale);
      for (double v : p->map_scale) ok = ok && std::isfinite(v);
      p->psi0.resize(p->map_scale.size() + 1);
      p->psi0[0] = 0.0;
      for (size_t k = 0; k < p->map_scale.size(); ++k) p->psi0[k + 1] = p->psi0[k] + p->map_scale[k] * p->dz;
    }
    if (!ok) {
      delete p;
      return fail(BRAHMS_E_INVALID_ARG, "non-finite dk_map or dk_map_scale entry");
    }
  }
  for (int j = 0; j < nfields; ++j) p->fp[j] = params->field[j];
  p->flags = params->flags;
  p->stream = reinterpret_cast<hipStream_t>(hip_stream);
  layout(*p);
  *out = p;
  return BRAHMS_OK;
}

brahms_status brahms_plan_workspace_size(brahms_plan plan, size_t* bytes) {
  if (brahms_status st = check_plan(plan)) return st;
  if (bytes == nullptr) return fail(BRAHMS_E_INVALID_ARG, "bytes is NULL");
  *bytes = plan->ws_size;
  return BRAHMS_OK;
}

brahms_status brahms_plan_bind(brahms_plan plan, void* const* fields, void* workspace) {
  if (brahms_status st = check_plan(plan)) return st;
  if (fields == nullptr || workspace == nullptr)
    return fail(BRAHMS_E_INVALID_ARG, "fields or workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(BRAHMS_E_INVALID_ARG, "workspace must be 256-byte aligned");
  for (int j = 0; j < plan->nf; ++j) {
    if (fields[j] == nullptr) return fail(BRAHMS_E_INVALID_ARG, "field pointer is NULL");
    if (reinterpret_cast<uintptr_t>(fields[j]) % 8 != 0)
      return fail(BRAHMS_E_INVALID_ARG, "field pointer must be 8-byte aligned");
  }
  plan->bound = false;
  plan->adj_ready = false;
  drop_chunk_graph(*plan);   // it holds the old pointers
  for (int j = 0; j < 3; ++j) plan->fields[j] = j < plan->nf ? static_cast<float2*>(fields[j]) : nullptr;
  plan->ws = static_cast<char*>(workspace);
  if (!plan->dk.empty()) {
    HIP_TRY(hipMemcpyAsync(plan->ws + plan->off_phi0, plan->phi0.data(),
                           sizeof(double) * plan->phi0.size(), hipMemcpyHostToDevice, plan->stream));
    HIP_TRY(hipMemcpyAsync(plan->ws + plan->off_dk, plan->dk.data(), sizeof(double) * plan->dk.size(),
                           hipMemcpyHostToDevice, plan->stream));
    HIP_TRY(hipStreamSynchronize(plan->stream));
  }
  if (!plan->dk_map.empty()) {
    HIP_TRY(hipMemcpyAsync(plan->ws + plan->off_map, plan->dk_map.data(),
                           sizeof(double) * plan->dk_map.size(), hipMemcpyHostToDevice, plan->stream));
    if (!plan->map_scale.empty()) {
      HIP_TRY(hipMemcpyAsync(plan->ws + plan->off_psi0, plan->psi0.data(),
                             sizeof(double) * plan->psi0.size(), hipMemcpyHostToDevice, plan->stream));
      HIP_TRY(hipMemcpyAsync(plan->ws + plan->off_scale, plan->map_scale.data(),
                             sizeof(double) * plan->map_scale.size(), hipMemcpyHostToDevice,
                             plan->stream));
    }
    HIP_TRY(hipStreamSynchronize(plan->stream));
  }
  plan->bound = true;
  if (graph_chunk_ok(*plan)) return build_chunk_graph(*plan);
  return BRAHMS_OK;
}

brahms_status brahms_step(brahms_plan plan, int nsteps) {
  if (brahms_status st = check_plan(plan)) return st;
  if (!plan->bound) return fail(BRAHMS_E_STATE, "brahms_step before brahms_plan_bind");
  if (nsteps < 0) return fail(BRAHMS_E_INVALID_ARG, "nsteps < 0");
  if (nsteps == 0) return BRAHMS_OK;
  plan->adj_ready = false;  // a recorded adjoint forward no longer matches
  if (!plan->dk.empty() && plan->step + nsteps > (long long)plan->dk.size())
    return fail(BRAHMS_E_INVALID_ARG, "steps beyond the end of the dk profile");
  if (!plan->map_scale.empty() && plan->step + nsteps > (long long)plan->map_scale.size())
    return fail(BRAHMS_E_INVALID_ARG, "steps beyond the end of the dk_map_scale profile");
  if (brahms_status st = run_steps(*plan, nsteps)) return st;
  if (plan->flags & BRAHMS_CHECK_FINITE) {
    int* flag = reinterpret_cast<int*>(plan->ws + plan->off_flag);
    hipLaunchKernelGGL(clear_flag, dim3(1), dim3(1), 0, plan->stream, flag);
    const long n = long(plan->nx) * plan->ny * plan->nt;
    for (int j = 0; j < plan->nf; ++j)
      hipLaunchKernelGGL(finite_check, dim3(1024), dim3(256), 0, plan->stream, plan->fields[j], n, flag);
    HIP_TRY(hipGetLastError());
    int host_flag = 0;
    HIP_TRY(hipMemcpyAsync(&host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, plan->stream));
    HIP_TRY(hipStreamSynchronize(plan->stream));
    if (host_flag) return fail(BRAHMS_E_NONFINITE, "a field holds NaN or Inf (dz too large?)");
  }
  return BRAHMS_OK;
}

static bool steps_to(double z_from_steps_dz, double z_end, double dz, long long* n_out) {
  const double r = z_end / dz;
  const double n = std::nearbyint(r);
  const double tol = 1e-9 * std::max(1.0, std::fabs(z_end));
  if (std::fabs(n * dz - z_end) > tol) return false;
  (void)z_from_steps_dz;
  *n_out = (long long)n;
  return true;
}

brahms_status brahms_propagate(brahms_plan plan, double z_end) {
  if (brahms_status st = check_plan(plan)) return st;
  if (!std::isfinite(z_end)) return fail(BRAHMS_E_INVALID_ARG, "z_end not finite");
  long long target = 0;
  if (!steps_to(0.0, z_end, plan->dz, &target))
    return fail(BRAHMS_E_INVALID_ARG, "z_end is not a multiple of dz");
  if (target < plan->step) return fail(BRAHMS_E_INVALID_ARG, "z_end lies before the current z");
  if (target - plan->step > 0x7fffffffLL) return fail(BRAHMS_E_INVALID_ARG, "too many steps");
  return brahms_step(plan, int(target - plan->step));
}

brahms_status brahms_get_z(brahms_plan plan, double* z) {
  if (brahms_status st = check_plan(plan)) return st;
  if (z == nullptr) return fail(BRAHMS_E_INVALID_ARG, "z is NULL");
  *z = double(plan->step) * plan->dz;
  return BRAHMS_OK;
}

brahms_status brahms_set_z(brahms_plan plan, double z) {
  if (brahms_status st = check_plan(plan)) return st;
  long long n = 0;
  if (!std::isfinite(z) || z < 0.0 || !steps_to(0.0, z, plan->dz, &n))
    return fail(BRAHMS_E_INVALID_ARG, "z must be a non-negative multiple of dz");
  plan->step = n;
  plan->adj_ready = false;
  return BRAHMS_OK;
}

brahms_status brahms_plan_set_schedule(brahms_plan plan, const brahms_schedule* sched) {
  if (brahms_status st = check_plan(plan)) return st;
  if (sched == nullptr) return fail(BRAHMS_E_INVALID_ARG, "schedule is NULL");
  if (sched->pass_order < 0 || sched->pass_order > 3)
    return fail(BRAHMS_E_INVALID_ARG, "pass_order must be 0, 1, 2 or 3");
  if (sched->graph != 0 && sched->graph != 1) return fail(BRAHMS_E_INVALID_ARG, "graph must be 0 or 1");
  if (sched->merge_halves != 0 && sched->merge_halves != 1)
    return fail(BRAHMS_E_INVALID_ARG, "merge_halves must be 0 or 1");
  if (sched->merge_halves && (!plan->dk.empty() || !plan->dk_map.empty()))
    return fail(BRAHMS_E_UNSUPPORTED, "merge_halves needs a constant dk and no transverse map");
  if (sched->fuse_steps != 0 && sched->fuse_steps != 1)
    return fail(BRAHMS_E_INVALID_ARG, "fuse_steps must be 0 or 1");
  if (sched->fuse_steps && !sched->merge_halves)
    return fail(BRAHMS_E_INVALID_ARG, "fuse_steps needs merge_halves");
  if (sched->fuse_steps && !detail::long_tau(*plan) && detail::step_passes(*plan, false).n != 3)
    return fail(BRAHMS_E_UNSUPPORTED, "fuse_steps needs an x and a y pass (not nx = ny = 1 with tau <= 256)");
  if (sched->split < 0 || sched->split > 7) return fail(BRAHMS_E_INVALID_ARG, "split must be 0 .. 7");
  if (sched->wide < 0 || sched->wide > 7) return fail(BRAHMS_E_INVALID_ARG, "wide must be 0 .. 7");
  if (plan->order != sched->pass_order || plan->use_graph != (sched->graph != 0) ||
      plan->merge != (sched->merge_halves != 0) || plan->fuse != (sched->fuse_steps != 0) ||
      plan->split != sched->split || plan->wide != sched->wide)
    drop_chunk_graph(*plan);
  plan->order = sched->pass_order;
  plan->split = sched->split;
  plan->wide = sched->wide;
  plan->use_graph = sched->graph != 0;
  plan->merge = sched->merge_halves != 0;
  plan->fuse = sched->fuse_steps != 0;
  // capture now rather than in the first call that replays it
  if (graph_chunk_ok(*plan) && !plan->chunk_exec) return build_chunk_graph(*plan);
  return BRAHMS_OK;
}

brahms_status brahms_plan_get_schedule(brahms_plan plan, brahms_schedule* sched) {
  if (brahms_status st = check_plan(plan)) return st;
  if (sched == nullptr) return fail(BRAHMS_E_INVALID_ARG, "schedule is NULL");
  *sched = brahms_schedule{};
  sched->pass_order = plan->order;
  sched->graph = plan->use_graph ? 1 : 0;
  sched->merge_halves = plan->merge ? 1 : 0;
  sched->fuse_steps = plan->fuse ? 1 : 0;
  sched->split = plan->split;
  sched->wide = plan->wide;
  return BRAHMS_OK;
}

brahms_status brahms_timing_enable(brahms_plan plan, int enable) {
  if (brahms_status st = check_plan(plan)) return st;
  plan->timing = enable != 0;
  return BRAHMS_OK;
}

brahms_status brahms_timing_read(brahms_plan plan, double* ms, long long* launches) {
  if (brahms_status st = check_plan(plan)) return st;
  if (ms == nullptr || launches == nullptr) return fail(BRAHMS_E_INVALID_ARG, "NULL output");
  for (int k = 0; k < BRAHMS_TIMING_KINDS; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  HIP_TRY(hipStreamSynchronize(plan->stream));
  for (const auto& t : plan->timed) {
    float el = 0.f;
    HIP_TRY(hipEventElapsedTime(&el, t.start, t.stop));
    ms[t.kind] += el;
    launches[t.kind] += 1;
  }
  for (const auto& t : plan->timed) {
    plan->pool.push_back(t.start);
    plan->pool.push_back(t.stop);
  }
  plan->timed.clear();
  return BRAHMS_OK;
}

brahms_status brahms_plan_destroy(brahms_plan plan) {
  if (plan == nullptr) return fail(BRAHMS_E_INVALID_ARG, "plan is NULL");
  for (const auto& t : plan->timed) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (hipEvent_t e : plan->pool) (void)hipEventDestroy(e);
  drop_chunk_graph(*plan);
  if (plan->capture_stream) (void)hipStreamDestroy(plan->capture_stream);
  for (hipEvent_t e : plan->adj_ev)
    if (e) (void)hipEventDestroy(e);
  if (plan->adj_side) (void)hipStreamDestroy(plan->adj_side);
  delete plan;
  return BRAHMS_OK;
}

}  // extern "C"
