// Batched parameter sweeps behind the C ABI (brahms_batch_*; see
// include/brahms.h).
//
// A batch holds many independent problems, each with its own grid, fields
// and parameters.  Problems of the same shape, field count and pass order
// form launch groups of at most `group_max` problems; one launch of a pass
// covers every problem of a group (the problem index is a grid dimension and
// each block reads its problem's pass arguments from a descriptor array), so
// small grids fill the GPU.  Problems with fewer steps than the longest in
// their group leave their blocks at once.  The whole run (tables and passes
// of every group) is captured once into a hipGraph and replayed by
// brahms_batch_run.  Launch groups are independent and could be parallel
// branches of that graph (up to four side streams, groups dealt out largest
// first) so that a bandwidth-bound group of large grids and latency-bound
// groups of small grids execute at the same time; that is switched off (see
// kParallelBranches) and the groups run one after the other, largest first;
// or (brahms_batch_set_streams) the groups are dealt over 2-4 streams, each
// stream's groups captured into a linear graph of their own.
// The default group size (a state of at most 160 MB) keeps a group's fields
// in the last-level cache while it is propagated.
//
// The graph is launched on the caller's stream, so a run orders itself after
// the caller's earlier work without cross-stream events.  The streams and
// events used to capture it come from a per-device pool and go back to it
// when the batch is destroyed: the library destroys no stream or event of a
// batch while the process runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/brahms.h"
#include "kernels.hpp"
#include "launch.hpp"
#include "plan.hpp"

using namespace brahms;
using brahms::detail::align_up;
using brahms::detail::fail;
using brahms::detail::kChunk;
using brahms::detail::kTableRows;

struct brahms_batch_s {
  int n = 0;
  std::vector<brahms_plan> plans;
  std::vector<int> nsteps;             // steps of the next run, per problem
  std::vector<int> capacity;           // steps the layout and graph are built for
  hipStream_t caller = nullptr;        // the caller's stream: uploads and graph launches
  int device = -1;                     // device of the capture streams
  hipStream_t stream = nullptr;        // capture stream (from the pool)
  char* ws = nullptr;
  bool bound = false;
  std::vector<size_t> plan_off;        // per problem: offset of its plan workspace
  size_t off_desc = 0, off_targs = 0, ws_size = 0;
  int group_max = 0;                   // 0: choose from the cache budget
  std::vector<int> group_limit;        // per problem, overrides group_max (empty: none)
  bool merge = false;                  // merged RK4 half-steps (constant dk only)
  int streams = 1;                     // 1: one captured graph; 2..4: one captured graph per
                                       // stream (the caller's and side streams)
  bool largest_alone = false;          // streams: the largest group after the others, alone
  bool eager_pending = false;          // a run may still be running on side streams
  bool fuse = false;                   // fused step pairs (groups of three-pass steps)
  // launch groups and descriptor placement (rebuilt when the schedule changes)
  struct Group {
    std::vector<int> members;
    int axis_len[3];
    int nf, order, split, wide, max_steps;
    size_t desc_off;                   // [3 passes][kChunk slots][members] PassArgs
    size_t targs_off;                  // [chunks][members] TableArgs
  };
  std::vector<Group> groups;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  // streams > 1: one linear graph per stream (index into the caller's and
  // side streams; the last, with largest_alone, on the caller's stream after
  // the join)
  static constexpr int kStreamGraphs = 6;
  int nsg = 0;
  hipGraph_t sgraph[kStreamGraphs] = {};
  hipGraphExec_t sexec[kStreamGraphs] = {};
  int sg_stream[kStreamGraphs] = {};
  bool sg_after_join[kStreamGraphs] = {};
  // side streams and events of the capture: launch groups are independent,
  // so they become parallel branches of the graph
  static constexpr int kBranches = 4;
  hipStream_t side[kBranches] = {};
  hipEvent_t fork = nullptr, join[kBranches] = {};
};

namespace {

// Capture streams and events of one batch, kept for reuse by later batches
// on the same device.
struct CaptureSet {
  int device;
  hipStream_t stream;
  hipStream_t side[brahms_batch_s::kBranches];
  hipEvent_t fork;
  hipEvent_t join[brahms_batch_s::kBranches];
};
std::mutex g_capture_mu;
std::vector<CaptureSet> g_capture_pool;

// Fills b's capture streams and events from the pool of the current device,
// or creates them.  Returns false when HIP cannot create them.
bool acquire_capture(brahms_batch_s& b) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  {
    std::lock_guard<std::mutex> lock(g_capture_mu);
    for (size_t k = 0; k < g_capture_pool.size(); ++k) {
      if (g_capture_pool[k].device != dev) continue;
      const CaptureSet c = g_capture_pool[k];
      g_capture_pool.erase(g_capture_pool.begin() + long(k));
      b.device = dev;
      b.stream = c.stream;
      b.fork = c.fork;
      for (int j = 0; j < brahms_batch_s::kBranches; ++j) {
        b.side[j] = c.side[j];
        b.join[j] = c.join[j];
      }
      return true;
    }
  }
  // on a failed creation the members made so far stay alive, unused
  b.device = dev;
  bool ok = hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&b.fork, hipEventDisableTiming) == hipSuccess;
  for (int j = 0; ok && j < brahms_batch_s::kBranches; ++j)
    ok = hipStreamCreateWithFlags(&b.side[j], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&b.join[j], hipEventDisableTiming) == hipSuccess;
  return ok;
}

// Hands b's capture streams and events back to the pool (a set with a
// missing member is kept out of it; its members stay alive unused).
void release_capture(brahms_batch_s& b) {
  if (b.device < 0) return;
  bool whole = b.stream != nullptr && b.fork != nullptr;
  for (int j = 0; j < brahms_batch_s::kBranches; ++j)
    whole = whole && b.side[j] != nullptr && b.join[j] != nullptr;
  if (whole) {
    CaptureSet c{};
    c.device = b.device;
    c.stream = b.stream;
    c.fork = b.fork;
    for (int j = 0; j < brahms_batch_s::kBranches; ++j) {
      c.side[j] = b.side[j];
      c.join[j] = b.join[j];
    }
    std::lock_guard<std::mutex> lock(g_capture_mu);
    g_capture_pool.push_back(c);
  }
  b.device = -1;
  b.stream = nullptr;
  b.fork = nullptr;
  for (int j = 0; j < brahms_batch_s::kBranches; ++j) {
    b.side[j] = nullptr;
    b.join[j] = nullptr;
  }
}

constexpr size_t kCacheBudget = size_t(160) << 20;  // bytes of field state per group

size_t state_bytes(const brahms_plan_s& p) {
  return sizeof(float2) * size_t(p.nx) * p.ny * p.nt * p.nf;
}

void make_groups(brahms_batch_s& b) {
  b.groups.clear();
  // members of a group share the shape, the field count and the passes of a
  // step (which also depend on the pass order and, for nt = 1, on loss)
  std::map<std::tuple<int, int, int, int, int, int>, std::vector<int>> by_key;
  for (int i = 0; i < b.n; ++i) {
    const brahms_plan_s& p = *b.plans[i];
    const brahms::detail::StepPasses sp = brahms::detail::step_passes(p, true);
    int code = sp.n;
    for (int k = 0; k < sp.n; ++k) code = code * 8 + sp.ax[k];
    by_key[{p.nx, p.ny, p.nt, p.nf, (p.order * 8 + p.split) * 8 + p.wide, code}].push_back(i);
  }
  for (auto& kv : by_key) {
    const std::vector<int>& ids = kv.second;
    const brahms_plan_s& p0 = *b.plans[ids[0]];
    int gmax = b.group_limit.empty() ? b.group_max : b.group_limit[size_t(ids[0])];
    if (gmax <= 0) gmax = int(std::max<size_t>(1, kCacheBudget / state_bytes(p0)));
    for (size_t s = 0; s < ids.size(); s += size_t(gmax)) {
      brahms_batch_s::Group g{};
      g.members.assign(ids.begin() + long(s), ids.begin() + long(std::min(ids.size(), s + size_t(gmax))));
      g.axis_len[0] = p0.nx;
      g.axis_len[1] = p0.ny;
      g.axis_len[2] = p0.nt;
      g.nf = p0.nf;
      g.order = p0.order;
      g.split = p0.split;
      g.wide = p0.wide;
      g.max_steps = 0;
      for (int m : g.members) g.max_steps = std::max(g.max_steps, b.capacity[m]);
      b.groups.push_back(g);
    }
  }
}

// Whether a group's steps run as fused step pairs: even steps take the
// axes a, m, b of their passes, odd steps b, m, a, and each step's last
// transform, the merged RK4 step and the next step's first transform are one
// launch (which ends a member's last step without the next transform).
bool group_fused(const brahms_batch_s& b, const brahms_batch_s::Group& g) {
  const brahms_plan_s& p0 = *b.plans[g.members[0]];
  return b.merge && b.fuse && !brahms::detail::long_tau(p0) &&
         brahms::detail::step_passes(p0, true).n == 3;
}

size_t descriptor_bytes(brahms_batch_s& b) {
  size_t off = 0;
  for (auto& g : b.groups) {
    g.desc_off = off;
    const int npass = brahms::detail::step_passes(*b.plans[g.members[0]], true).n;
    off = align_up(off + sizeof(PassArgs) * size_t(npass) * kChunk * g.members.size());
  }
  return off;
}

size_t table_arg_bytes(brahms_batch_s& b) {
  size_t off = 0;
  for (auto& g : b.groups) {
    g.targs_off = off;
    const int chunks = (g.max_steps + kChunk - 1) / kChunk;
    off = align_up(off + sizeof(TableArgs) * size_t(std::max(chunks, 1)) * g.members.size());
  }
  return off;
}

brahms::detail::GroupGeom geom_of(const brahms_batch_s::Group& g) {
  return brahms::detail::GroupGeom{unsigned(g.members.size()), g.axis_len[0], g.axis_len[1], g.axis_len[2],
                                   g.nf, g.wide};
}

template <int AX>
void dispatch_group_long_len(int len, int nl, const brahms_batch_s::Group& g, hipStream_t st,
                             const PassArgs* d, long long step) {
  switch (len) {
#define BRAHMS_CASE_(N, N1, N2) \
  case N: brahms::detail::launch_group_long<N1, N2, AX>(nl, geom_of(g), st, d, step); break;
    BRAHMS_LONG_SUBLENGTHS(BRAHMS_CASE_)
#undef BRAHMS_CASE_
    default: break;
  }
}

void dispatch_group_long(int axis, int nl, const brahms_batch_s::Group& g, hipStream_t st,
                         const PassArgs* d, long long step) {
  const int nt = g.axis_len[2];
  const int na = brahms::detail::long_tau_a(nt);   // the b passes have length nt / na
  if (axis == AX_TAF) dispatch_group_long_len<AX_TAF>(nt / na, nl, g, st, d, step);
  else if (axis == AX_TB) dispatch_group_long_len<AX_TB>(na, nl, g, st, d, step);
  else dispatch_group_long_len<AX_TAI>(nt / na, nl, g, st, d, step);
}

void dispatch_group_pass(int len, int axis, int nl, const brahms_batch_s::Group& g, hipStream_t st,
                         const PassArgs* d, long long step) {
  if ((g.split >> axis) & 1) {
    switch (len) {
#define BRAHMS_CASE_(N, N1, N2) \
  case N: brahms::detail::launch_group_pass<N1, N2>(axis, nl, geom_of(g), st, d, step); return;
      BRAHMS_ALT_LENGTHS(BRAHMS_CASE_)
#undef BRAHMS_CASE_
      default: break;
    }
  }
  switch (len) {
#define BRAHMS_CASE_(N, N1, N2) \
  case N: brahms::detail::launch_group_pass<N1, N2>(axis, nl, geom_of(g), st, d, step); break;
    BRAHMS_LENGTHS(BRAHMS_CASE_)
#undef BRAHMS_CASE_
    default: break;
  }
}

// Host images of the descriptors (pass arguments per slot and table
// arguments per chunk) of every group, uploaded once at bind.
brahms_status upload_descriptors(brahms_batch_s& b) {
  std::vector<char> desc(b.off_targs - b.off_desc), targ(b.ws_size - b.off_targs);
  for (auto& g : b.groups) {
    const size_t m = g.members.size();
    for (size_t k = 0; k < m; ++k) {
      brahms_plan_s& p = *b.plans[g.members[k]];
      const int per_field = p.nx + p.ny + p.nt;
      const int row_stride = table_row_stride(p.nf, p.nx, p.ny, p.nt);
      const float2* rows = reinterpret_cast<const float2*>(p.ws + p.off_prop);
      const float2* nls = reinterpret_cast<const float2*>(p.ws + p.off_nl);
      const brahms::detail::StepPasses sp = brahms::detail::step_passes(p, true);
      const bool fused = group_fused(b, g);
      for (int pass = 0; pass < sp.n; ++pass) {
        for (int s = 0; s < kChunk; ++s) {
          // fused step pairs: odd steps swap the first and last axes
          int ax = sp.ax[pass];
          if (fused && (s & 1) && pass != 1) ax = sp.ax[2 - pass];
          const int len = ax == AX_X ? p.nx : (ax == AX_Y ? p.ny : p.nt);
          PassArgs a{};
          const float2* r = rows + size_t(s) * row_stride;
          a.axis_off = (ax == AX_X) ? 0 : (ax == AX_Y ? p.nx : p.nx + p.ny);
          a.tw = r + p.nf * per_field + a.axis_off;
          a.consts = reinterpret_cast<const DftConsts*>(r + (p.nf + 1) * per_field);
          a.prop = r;
          a.field_stride = per_field;
          a.nl = nls + size_t(s) * 2 * p.nf * kNlCoef;
          a.nl2 = nls + (size_t(s) * 2 + 1) * p.nf * kNlCoef;
          a.nx = p.nx; a.ny = p.ny; a.nt = p.nt;
          for (int j = 0; j < 3; ++j) {
            a.f[j] = p.fields[j];
            a.fo[j] = p.fields[j];
          }
          a.tile_mul = 1;
          a.tiles = 1;
          if (ax == AX_T) {
            const long lines = long(p.nx) * p.ny;
            const int lpb = lines_per_block(len, ((p.split >> ax) & 1) != 0);
            a.tiles = unsigned((lines + lpb - 1) / lpb);
            a.tile_mul = brahms::detail::tile_multiplier(a.tiles);
          }
          a.nz = b.nsteps[g.members[k]];  // compared with the absolute step
          if (fused && pass == 2) {
            // the next step's tables along the same axis (row s + 1)
            const float2* r2 = r + row_stride;
            a.tw2 = r2 + p.nf * per_field + a.axis_off;
            a.prop2 = r2;
            a.consts2 = reinterpret_cast<const DftConsts*>(r2 + (p.nf + 1) * per_field);
          }
          std::memcpy(desc.data() + g.desc_off + ((size_t(pass) * kChunk + s) * m + k) * sizeof(PassArgs),
                      &a, sizeof(PassArgs));
        }
      }
      const int chunks = (g.max_steps + kChunk - 1) / kChunk;
      for (int c = 0; c < chunks; ++c) {
        TableArgs ta{};
        ta.rows = reinterpret_cast<float2*>(p.ws + p.off_prop);
        ta.row_stride = row_stride;
        ta.nl = reinterpret_cast<float2*>(p.ws + p.off_nl);
        ta.phi0 = p.dk.empty() ? nullptr : reinterpret_cast<const double*>(p.ws + p.off_phi0);
        ta.dk = p.dk.empty() ? nullptr : reinterpret_cast<const double*>(p.ws + p.off_dk);
        ta.n0 = (long long)c * kChunk;
        ta.merge_last = b.merge ? (long long)b.nsteps[g.members[k]] - 1 : -1;
        ta.count = std::max(0, std::min(kChunk, b.nsteps[g.members[k]] - c * kChunk));
        if (group_fused(b, g) && ta.count > 0) ta.count += 1;   // the next step's row
        ta.nx = p.nx; ta.ny = p.ny; ta.nt = p.nt; ta.nf = p.nf;
        ta.dz = p.dz; ta.dx = p.dx; ta.dy = p.dy; ta.dt = p.dt; ta.dk_const = p.dk_const;
        for (int j = 0; j < p.nf; ++j) {
          const brahms_field_params& f = p.fp[j];
          ta.fc[j] = FieldCoef{f.kappa, f.diffraction, f.tan_rho, f.delay, f.k2, f.k3, f.alpha};
        }
        std::memcpy(targ.data() + g.targs_off + (size_t(c) * m + k) * sizeof(TableArgs), &ta,
                    sizeof(TableArgs));
      }
    }
  }
  // on the caller's stream, after any run still reading the old descriptors
  HIP_TRY(hipMemcpyAsync(b.ws + b.off_desc, desc.data(), desc.size(), hipMemcpyHostToDevice, b.caller));
  HIP_TRY(hipMemcpyAsync(b.ws + b.off_targs, targ.data(), targ.size(), hipMemcpyHostToDevice, b.caller));
  HIP_TRY(hipStreamSynchronize(b.caller));
  return BRAHMS_OK;
}

// One launch group on stream st: per 64-step chunk, one batched table launch
// and then the batched pass launches of each step (three, fewer when an axis
// of length 1 is left out).  With merged halves only step 0 has a first
// half-step of its own.
brahms_status enqueue_group(brahms_batch_s& b, const brahms_batch_s::Group& g, hipStream_t st) {
  {
    const brahms_plan_s& p0 = *b.plans[g.members[0]];
    const int per_field = p0.nx + p0.ny + p0.nt;
    const unsigned m = unsigned(g.members.size());
    const int chunks = (g.max_steps + kChunk - 1) / kChunk;
    const bool fused = group_fused(b, g);
    for (int c = 0; c < chunks; ++c) {
      const long total = long(kTableRows) * ((g.nf + 1) * per_field + 1) + long(kTableRows) * 2 * g.nf;
      const TableArgs* targs =
          reinterpret_cast<const TableArgs*>(b.ws + b.off_targs + g.targs_off) + size_t(c) * m;
      hipLaunchKernelGGL(step_tables_batched, dim3(unsigned((total + 255) / 256), m), dim3(256), 0,
                         st, targs);
      HIP_TRY(hipGetLastError());
      const int cnt = std::min(kChunk, g.max_steps - c * kChunk);
      const brahms::detail::StepPasses sp = brahms::detail::step_passes(p0, true);
      for (int s = 0; s < cnt; ++s) {
        const long long step = (long long)c * kChunk + s;
        for (int pass = 0; pass < sp.n; ++pass) {
          int ax = sp.ax[pass];
          int nl = b.merge && step > 0 && pass == 0 ? (sp.nl[pass] & ~NL_BEFORE) : sp.nl[pass];
          if (fused) {
            if (pass == 0 && step > 0) continue;   // done by the previous fused pass
            if (s & 1) ax = sp.ax[2 - pass];
            if (pass == 2) nl = NL_AFTER | NL_FUSE;
          }
          const PassArgs* d = reinterpret_cast<const PassArgs*>(b.ws + b.off_desc + g.desc_off) +
                              (size_t(pass) * kChunk + s) * m;
          if (long_tau_kind(ax)) dispatch_group_long(ax, nl, g, st, d, step);
          else dispatch_group_pass(g.axis_len[ax], ax, nl, g, st, d, step);
          HIP_TRY(hipGetLastError());
        }
      }
    }
  }
  return BRAHMS_OK;
}

// Parallel graph branches (groups dealt round-robin over the side streams)
// are switched off: a batch whose branched graph had just been destroyed was
// followed, in several test runs, by a crash on the HIP runtime's own thread,
// and the cause was not found.  Linear graphs, as plans use them, never
// showed it.
constexpr bool kParallelBranches = false;

// The whole run, largest groups first: on b.stream one after the other, or,
// with parallel branches, forked from b.stream into the side streams and
// joined back.
brahms_status enqueue_run(brahms_batch_s& b) {
  std::vector<size_t> order(b.groups.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = k;
  auto work = [&](size_t k) {
    const auto& g = b.groups[k];
    return double(g.axis_len[0]) * g.axis_len[1] * g.axis_len[2] * g.members.size() * g.max_steps;
  };
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t c) { return work(a) > work(c); });
  if (!kParallelBranches) {
    for (size_t k = 0; k < order.size(); ++k)
      if (brahms_status st = enqueue_group(b, b.groups[order[k]], b.stream)) return st;
    return BRAHMS_OK;
  }
  const int nb = std::min<int>(brahms_batch_s::kBranches, int(order.size()));
  HIP_TRY(hipEventRecord(b.fork, b.stream));
  for (int k = 0; k < nb; ++k) HIP_TRY(hipStreamWaitEvent(b.side[k], b.fork, 0));
  for (size_t k = 0; k < order.size(); ++k)
    if (brahms_status st = enqueue_group(b, b.groups[order[k]], b.side[k % nb])) return st;
  for (int k = 0; k < nb; ++k) {
    HIP_TRY(hipEventRecord(b.join[k], b.side[k]));
    HIP_TRY(hipStreamWaitEvent(b.stream, b.join[k], 0));
  }
  return BRAHMS_OK;
}

// Captures the launches of the given groups, in order, on b.stream into one
// linear graph and instantiates it.
brahms_status capture_groups(brahms_batch_s& b, const std::vector<size_t>& gs, hipGraph_t* graph_out,
                             hipGraphExec_t* exec_out) {
  HIP_TRY(hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal));
  brahms_status st = BRAHMS_OK;
  for (size_t k : gs)
    if ((st = enqueue_group(b, b.groups[k], b.stream)) != BRAHMS_OK) break;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(b.stream, &graph);
  if (st != BRAHMS_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return st != BRAHMS_OK ? st
                           : fail(BRAHMS_E_DEVICE, std::string("batch graph capture: ") + hipGetErrorString(e));
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(BRAHMS_E_DEVICE, std::string("batch graph instantiation: ") + hipGetErrorString(ei));
  }
  *graph_out = graph;
  *exec_out = exec;
  return BRAHMS_OK;
}

// The whole run over b.streams streams: the caller's stream and
// b.streams - 1 side streams, forked from and joined back into the caller's
// stream; launch groups, largest first, each to the stream with the least
// work so far.  The groups are independent, so large bandwidth-bound groups
// and small latency-bound ones execute together.  With largest_alone the
// largest group runs after the others have joined, on the caller's stream:
// groups that each leave much of the chip idle then share it, and the
// largest group, which fills the chip, has it to itself.  Each stream's
// groups are captured once into a linear graph of their own (no graph has
// parallel branches) and replayed at every run, so that a run costs a few
// graph launches instead of thousands of kernel launches from the host.
brahms_status run_streams(brahms_batch_s& b) {
  std::vector<size_t> order(b.groups.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = k;
  auto work = [&](size_t k) {
    const auto& g = b.groups[k];
    return double(g.axis_len[0]) * g.axis_len[1] * g.axis_len[2] * g.members.size() * g.max_steps;
  };
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t c) { return work(a) > work(c); });
  std::vector<size_t> last;
  if (b.largest_alone && order.size() > 1) {
    last.push_back(order.front());
    order.erase(order.begin());
  }
  const int ns = std::max(1, std::min<int>(b.streams, int(order.size())));
  hipStream_t st[brahms_batch_s::kBranches + 1] = {b.caller};
  for (int k = 1; k < ns; ++k) st[k] = b.side[k - 1];
  if (b.nsg == 0) {
    std::vector<std::vector<size_t>> per(static_cast<size_t>(ns));
    std::vector<double> load(size_t(ns), 0.0);
    for (size_t k : order) {
      const size_t s = size_t(std::min_element(load.begin(), load.end()) - load.begin());
      load[s] += work(k);
      per[s].push_back(k);
    }
    for (int s = 0; s <= ns; ++s) {
      const std::vector<size_t>& gs = s < ns ? per[size_t(s)] : last;
      if (gs.empty()) continue;
      const int i = b.nsg;
      if (brahms_status e = capture_groups(b, gs, &b.sgraph[i], &b.sexec[i])) {
        // release the graphs built so far: the next run builds them all again
        for (int j = 0; j < i; ++j) {
          (void)hipGraphExecDestroy(b.sexec[j]);
          (void)hipGraphDestroy(b.sgraph[j]);
          b.sexec[j] = nullptr;
          b.sgraph[j] = nullptr;
        }
        b.nsg = 0;
        return e;
      }
      b.sg_stream[i] = s < ns ? s : 0;
      b.sg_after_join[i] = s == ns;
      b.nsg = i + 1;
    }
  }
  if (ns > 1) {
    HIP_TRY(hipEventRecord(b.fork, b.caller));
    for (int k = 1; k < ns; ++k) HIP_TRY(hipStreamWaitEvent(st[k], b.fork, 0));
  }
  for (int i = 0; i < b.nsg; ++i)
    if (!b.sg_after_join[i]) HIP_TRY(hipGraphLaunch(b.sexec[i], st[b.sg_stream[i]]));
  for (int k = 1; k < ns; ++k) {
    HIP_TRY(hipEventRecord(b.join[k - 1], st[k]));
    HIP_TRY(hipStreamWaitEvent(b.caller, b.join[k - 1], 0));
  }
  for (int i = 0; i < b.nsg; ++i)
    if (b.sg_after_join[i]) HIP_TRY(hipGraphLaunch(b.sexec[i], b.caller));
  b.eager_pending = true;
  return BRAHMS_OK;
}

void drop_graph(brahms_batch_s& b) {
  // no launch of a graph, on the caller's stream or a side stream, may still
  // run when it goes (the caller's stream has joined the side streams)
  if (b.exec || b.eager_pending || b.nsg > 0) (void)hipStreamSynchronize(b.caller);
  b.eager_pending = false;
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  if (b.graph) (void)hipGraphDestroy(b.graph);
  b.exec = nullptr;
  b.graph = nullptr;
  for (int i = 0; i < b.nsg; ++i) {
    (void)hipGraphExecDestroy(b.sexec[i]);
    (void)hipGraphDestroy(b.sgraph[i]);
    b.sexec[i] = nullptr;
    b.sgraph[i] = nullptr;
  }
  b.nsg = 0;
}

brahms_status check_batch(brahms_batch b) {
  if (b == nullptr) return fail(BRAHMS_E_INVALID_ARG, "batch is NULL");
  return BRAHMS_OK;
}

void layout_batch(brahms_batch_s& b) {
  size_t off = 0;
  b.plan_off.resize(b.n);
  for (int i = 0; i < b.n; ++i) {
    b.plan_off[i] = off;
    off = align_up(off + b.plans[i]->ws_size);
  }
  make_groups(b);
  b.off_desc = off;
  off += descriptor_bytes(b);
  b.off_targs = off;
  off += table_arg_bytes(b);
  b.ws_size = align_up(off);
}

}  // namespace

extern "C" {

brahms_status brahms_batch_create(int n, const int* shapes, const brahms_params* params,
                                  const int* nsteps, void* hip_stream, brahms_batch* out) {
  if (out == nullptr) return fail(BRAHMS_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n < 1 || shapes == nullptr || params == nullptr || nsteps == nullptr)
    return fail(BRAHMS_E_INVALID_ARG, "need n >= 1 and non-NULL shapes, params, nsteps");
  auto* b = new brahms_batch_s();
  b->n = n;
  b->caller = reinterpret_cast<hipStream_t>(hip_stream);
  for (int i = 0; i < n; ++i) {
    brahms_plan p = nullptr;
    if (nsteps[i] < 0) {
      brahms_batch_destroy(b);
      return fail(BRAHMS_E_INVALID_ARG, "negative step count");
    }
    if (brahms_status st = brahms_plan_create(shapes[4 * i], shapes[4 * i + 1], shapes[4 * i + 2],
                                              shapes[4 * i + 3], &params[i], nullptr, &p)) {
      brahms_batch_destroy(b);
      return st;
    }
    if (!p->dk_map.empty()) {
      brahms_plan_destroy(p);
      brahms_batch_destroy(b);
      return fail(BRAHMS_E_UNSUPPORTED, "batches take no transverse dk map");
    }
    if (!p->dk.empty() && nsteps[i] > (int)p->dk.size()) {
      brahms_plan_destroy(p);
      brahms_batch_destroy(b);
      return fail(BRAHMS_E_INVALID_ARG, "steps beyond the end of a dk profile");
    }
    b->plans.push_back(p);
    b->nsteps.push_back(nsteps[i]);
    b->capacity.push_back(nsteps[i]);
  }
  if (!acquire_capture(*b)) {
    brahms_batch_destroy(b);
    return fail(BRAHMS_E_DEVICE, "could not create the batch streams or events");
  }
  for (brahms_plan p : b->plans) p->stream = b->caller;
  layout_batch(*b);
  *out = b;
  return BRAHMS_OK;
}

brahms_status brahms_batch_set_schedule(brahms_batch b, int group_max, const int* pass_order) {
  if (brahms_status st = check_batch(b)) return st;
  if (group_max < 0) return fail(BRAHMS_E_INVALID_ARG, "group_max < 0");
  if (pass_order != nullptr)
    for (int i = 0; i < b->n; ++i)
      if (pass_order[i] < 0 || pass_order[i] > 3)
        return fail(BRAHMS_E_INVALID_ARG, "pass_order entries must be 0, 1, 2 or 3");
  b->group_max = group_max;
  if (pass_order != nullptr)
    for (int i = 0; i < b->n; ++i) b->plans[i]->order = pass_order[i];
  drop_graph(*b);
  b->bound = false;
  layout_batch(*b);
  return BRAHMS_OK;
}

brahms_status brahms_batch_set_merge_halves(brahms_batch b, int merge_halves) {
  if (brahms_status st = check_batch(b)) return st;
  if (merge_halves != 0 && merge_halves != 1) return fail(BRAHMS_E_INVALID_ARG, "merge_halves must be 0 or 1");
  if (merge_halves)
    for (brahms_plan p : b->plans)
      if (!p->dk.empty()) return fail(BRAHMS_E_UNSUPPORTED, "merge_halves needs a constant dk");
  b->merge = merge_halves != 0;
  drop_graph(*b);
  b->bound = false;
  layout_batch(*b);
  return BRAHMS_OK;
}

brahms_status brahms_batch_set_fuse_steps(brahms_batch b, int fuse_steps) {
  if (brahms_status st = check_batch(b)) return st;
  if (fuse_steps != 0 && fuse_steps != 1) return fail(BRAHMS_E_INVALID_ARG, "fuse_steps must be 0 or 1");
  if (fuse_steps && !b->merge) return fail(BRAHMS_E_INVALID_ARG, "fuse_steps needs merge_halves");
  // switched off for batches that hold a long tau problem: a test run of such
  // a batch was followed by a host fault whose cause was not found
  if (fuse_steps)
    for (brahms_plan p : b->plans)
      if (brahms::detail::long_tau(*p))
        return fail(BRAHMS_E_UNSUPPORTED, "fuse_steps in a batch with a long tau problem");
  b->fuse = fuse_steps != 0;
  drop_graph(*b);
  b->bound = false;
  layout_batch(*b);
  return BRAHMS_OK;
}

brahms_status brahms_batch_set_streams(brahms_batch b, int streams, int largest_alone) {
  if (brahms_status st = check_batch(b)) return st;
  if (streams < 1 || streams > brahms_batch_s::kBranches)
    return fail(BRAHMS_E_INVALID_ARG, "streams must be 1 .. 4");
  if (largest_alone != 0 && largest_alone != 1) return fail(BRAHMS_E_INVALID_ARG, "largest_alone must be 0 or 1");
  drop_graph(*b);
  b->streams = streams;
  b->largest_alone = largest_alone != 0;
  return BRAHMS_OK;
}

brahms_status brahms_batch_set_splits(brahms_batch b, const int* splits) {
  if (brahms_status st = check_batch(b)) return st;
  if (splits != nullptr)
    for (int i = 0; i < b->n; ++i)
      if (splits[i] < 0 || splits[i] > 7) return fail(BRAHMS_E_INVALID_ARG, "splits must be 0 .. 7");
  for (int i = 0; i < b->n; ++i) b->plans[i]->split = splits == nullptr ? 0 : splits[i];
  drop_graph(*b);
  b->bound = false;
  layout_batch(*b);
  return BRAHMS_OK;
}

brahms_status brahms_batch_set_wide(brahms_batch b, const int* wide) {
  if (brahms_status st = check_batch(b)) return st;
  if (wide != nullptr)
    for (int i = 0; i < b->n; ++i)
      if (wide[i] < 0 || wide[i] > 3) return fail(BRAHMS_E_INVALID_ARG, "wide must be 0 .. 3 in a batch");
  for (int i = 0; i < b->n; ++i) b->plans[i]->wide = wide == nullptr ? 0 : wide[i];
  drop_graph(*b);
  b->bound = false;
  layout_batch(*b);
  return BRAHMS_OK;
}

brahms_status brahms_batch_set_group_limits(brahms_batch b, const int* limits) {
  if (brahms_status st = check_batch(b)) return st;
  if (limits != nullptr)
    for (int i = 0; i < b->n; ++i)
      if (limits[i] < 0) return fail(BRAHMS_E_INVALID_ARG, "group limits must be >= 0");
  if (limits == nullptr) b->group_limit.clear();
  else b->group_limit.assign(limits, limits + b->n);
  drop_graph(*b);
  b->bound = false;
  layout_batch(*b);
  return BRAHMS_OK;
}

brahms_status brahms_batch_workspace_size(brahms_batch b, size_t* bytes) {
  if (brahms_status st = check_batch(b)) return st;
  if (bytes == nullptr) return fail(BRAHMS_E_INVALID_ARG, "bytes is NULL");
  *bytes = b->ws_size;
  return BRAHMS_OK;
}

brahms_status brahms_batch_bind(brahms_batch b, void* const* fields, void* workspace) {
  if (brahms_status st = check_batch(b)) return st;
  if (fields == nullptr || workspace == nullptr ||
      reinterpret_cast<uintptr_t>(workspace) % detail::kAlign != 0)
    return fail(BRAHMS_E_INVALID_ARG, "fields NULL or workspace not 256-byte aligned");
  drop_graph(*b);
  b->bound = false;
  b->ws = static_cast<char*>(workspace);
  size_t f = 0;
  for (int i = 0; i < b->n; ++i) {
    brahms_plan p = b->plans[i];
    if (brahms_status st = brahms_plan_bind(p, fields + f, b->ws + b->plan_off[i])) return st;
    f += size_t(p->nf);
  }
  if (brahms_status st = upload_descriptors(*b)) return st;
  b->bound = true;
  return BRAHMS_OK;
}

brahms_status brahms_batch_run(brahms_batch b) {
  if (brahms_status st = check_batch(b)) return st;
  if (!b->bound) return fail(BRAHMS_E_STATE, "brahms_batch_run before brahms_batch_bind");
  if (b->streams > 1) {
    if (brahms_status st = run_streams(*b)) return st;
    for (int i = 0; i < b->n; ++i) b->plans[i]->step = b->nsteps[i];
    return BRAHMS_OK;
  }
  if (b->exec == nullptr) {
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const brahms_status st = enqueue_run(*b);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &graph);
    if (st != BRAHMS_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(BRAHMS_E_DEVICE, std::string("batch graph capture: ") + hipGetErrorString(e));
    }
    // keep the handles only once both exist, so that a failed instantiation
    // leaves nothing for drop_graph to release twice
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return fail(BRAHMS_E_DEVICE, std::string("batch graph instantiation: ") + hipGetErrorString(ei));
    }
    b->graph = graph;
    b->exec = exec;
  }
  HIP_TRY(hipGraphLaunch(b->exec, b->caller));
  for (int i = 0; i < b->n; ++i) b->plans[i]->step = b->nsteps[i];
  return BRAHMS_OK;
}

brahms_status brahms_batch_run_steps(brahms_batch b, const int* nsteps) {
  if (brahms_status st = check_batch(b)) return st;
  if (!b->bound) return fail(BRAHMS_E_STATE, "brahms_batch_run_steps before brahms_batch_bind");
  if (nsteps == nullptr) return fail(BRAHMS_E_INVALID_ARG, "nsteps is NULL");
  bool changed = false;
  for (int i = 0; i < b->n; ++i) {
    if (nsteps[i] < 0 || nsteps[i] > b->capacity[i])
      return fail(BRAHMS_E_INVALID_ARG, "step counts must lie in 0 .. the counts given at create");
    changed = changed || nsteps[i] != b->nsteps[i];
  }
  if (changed) {
    // new per-problem counts in the descriptors (after any run still reading
    // them: the upload waits on the caller's stream); the graph stays
    b->nsteps.assign(nsteps, nsteps + b->n);
    if (brahms_status st = upload_descriptors(*b)) return st;
  }
  return brahms_batch_run(b);
}

brahms_status brahms_batch_groups(brahms_batch b, int* ngroups, int* members) {
  if (brahms_status st = check_batch(b)) return st;
  if (ngroups == nullptr) return fail(BRAHMS_E_INVALID_ARG, "ngroups is NULL");
  *ngroups = int(b->groups.size());
  if (members != nullptr)
    for (size_t g = 0; g < b->groups.size(); ++g) members[g] = int(b->groups[g].members.size());
  return BRAHMS_OK;
}

brahms_status brahms_batch_destroy(brahms_batch b) {
  if (b == nullptr) return fail(BRAHMS_E_INVALID_ARG, "batch is NULL");
  drop_graph(*b);   // waits for the caller's stream first
  for (brahms_plan p : b->plans) brahms_plan_destroy(p);
  release_capture(*b);
  delete b;
  return BRAHMS_OK;
}

}  // extern "C"
