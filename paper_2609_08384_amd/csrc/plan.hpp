// Internal host-side state of a plan, shared by the engine's translation
// units (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/brahms.h"

struct brahms_plan_s {
  int nx = 0, ny = 0, nt = 0, nf = 0;
  double dz = 0, dx = 1, dy = 1, dt = 1, dk_const = 0;
  std::vector<double> dk;      // per-step profile (empty: constant)
  std::vector<double> phi0;    // Phi_n prefix of the profile
  std::vector<double> dk_map;     // transverse mismatch map m(x, y), [ny][nx] (empty: none)
  std::vector<double> map_scale;  // s_n per step (empty: all 1)
  std::vector<double> psi0;       // Psi_n = dz sum_{l<n} s_l (when map_scale is given)
  long long table_n0 = 0;         // step index of table row 0
  brahms_field_params fp[3] = {};
  unsigned flags = 0;
  hipStream_t stream = nullptr;
  float2* fields[3] = {nullptr, nullptr, nullptr};
  char* ws = nullptr;
  bool bound = false;
  long long step = 0;          // z = step * dz
  int order = 0;               // 0: x, y, tau passes; 1: tau, y, x
  // schedule field merge_halves: adjacent RK4 half-steps of one call run as
  // one RK4 step of size dz (constant dk, no map, no monitor or snapshots)
  bool merge = false;
  // schedule field fuse_steps (with merged halves): steps alternate their
  // axis order so that step n's last transform, the RK4 step and step n+1's
  // first transform run as one pass
  bool fuse = false;
  // schedule field split: bit a (x = 1, y = 2, tau = 4) runs that axis's line
  // transforms with the second split of its length (lengths.hpp), if any
  int split = 0;
  // schedule field wide: bit a (x = 1, y = 2, tau = 4) runs that axis's
  // linear passes (one field per block) with kWideBlock threads per block
  int wide = 0;
  // hipGraph replay of whole 64-step chunks (schedule field `graph`)
  bool use_graph = false;
  hipGraph_t chunk_graph = nullptr;
  hipGraphExec_t chunk_exec = nullptr;
  hipStream_t capture_stream = nullptr;   // private stream the chunk is captured on
  const long long* table_n0_dev = nullptr;  // while capturing: tables read n0
                                            // and merge_last here
  // workspace offsets (bytes)
  size_t off_phi0 = 0, off_dk = 0, off_prop = 0, off_nl = 0, off_flag = 0, ws_size = 0;
  size_t off_map = 0, off_maptab = 0;   // map (FP64) and its per-step phase tables
  size_t off_psi0 = 0, off_scale = 0;   // Psi_n prefix and s_n (with a scale profile)
  int map_rows = 0;                     // steps per phase-table fill (kChunk or 1)
  size_t off_diag = 0;                  // partial sums of the diagnostics
  size_t off_n0 = 0;                    // first step of the chunk a graph replays
  // launch timing (diagnostics)
  bool timing = false;
  struct Timed { int kind; hipEvent_t start, stop; };
  std::vector<Timed> timed;             // one entry per timed launch
  std::vector<hipEvent_t> pool;         // reusable events
  // adjoint record (set by brahms_adjoint_forward)
  bool adj_ready = false;
  long long adj_n0 = 0;
  int adj_nsteps = 0, adj_every = 0;
  bool adj_last_recorded = false;   // segment slots hold the last segment
  char* adj_ws = nullptr;
  // reverse sweep: a second stream recomputes the next segment meanwhile
  hipStream_t adj_side = nullptr;
  hipEvent_t adj_ev[5] = {};          // start, ready[2], free[2]
  // diagnostics (brahms_set_monitor / brahms_set_snapshots)
  int mon_every = 0;                    // record when the step index is a multiple
  double* mon_records = nullptr;        // device, capacity x record doubles
  int mon_capacity = 0, mon_count = 0;
  std::vector<long long> snap_steps;    // step indices of the snapshots
  std::vector<float2*> snap_buffers;    // [snapshot * nf + field], device
};

namespace brahms {
namespace detail {

constexpr int kChunk = 64;     // steps per table refill
constexpr int kTableRows = kChunk + 1;  // table rows in the workspace: a chunk and
                                        // the next step (fused step pairs)
constexpr size_t kAlign = 256;
constexpr int kDiagChunks = 64;  // chunks per (tau, field) slice in diagnostics

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// A tau axis longer than one line transform (three passes per step).
inline bool long_tau(const brahms_plan_s& p) { return p.nt > 256; }
// Its split nt = A B (the a transforms have length A, the b transforms B):
// 512 = 32 x 16, 1024 = 32 x 32, 2048 = 64 x 32, 4096 = 64 x 64.
inline int long_tau_a(int nt) { return nt >= 2048 ? 64 : 32; }

brahms_status fail(brahms_status st, const std::string& msg);

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return ::brahms::detail::fail(BRAHMS_E_DEVICE,                                           \
                                    std::string(#expr) + ": " + hipGetErrorString(e_));        \
  } while (0)

brahms_status check_plan(brahms_plan p);

// Multiplier of the block -> tile permutation of the tau pass: coprime with
// the tile count (so the map is a bijection) and about tiles/64, so that
// consecutive blocks land about 1/64 of the plane apart.
inline unsigned tile_multiplier(unsigned tiles) {
  if (tiles < 128) return 1;
  unsigned m = tiles / 64 + 1;
  for (;; ++m) {
    unsigned a = m, b = tiles;
    while (b) {
      const unsigned r = a % b;
      a = b;
      b = r;
    }
    if (a == 1) return m;
  }
}

// Where one z-step reads and writes: the first pass reads `in` and writes
// `out`, the other two passes work in place on `out`; when `pre` is given the
// last pass also stores the input of the second RK4 half-step there.
struct StepIO {
  float2* in[3];
  float2* out[3];
  float2* pre[3];
};

// Fill table rows row0..row0+count-1 for steps n0..n0+count-1; steps
// n < merge_last get the merged second half-step (see merging()).
brahms_status refresh_tables(brahms_plan_s& p, long long n0, int count, int row0 = 0,
                             long long merge_last = -1);
// Whether a call of brahms_propagate merges adjacent half-steps: only for a
// constant dk (Phi linear in z across a step boundary) with no transverse
// map, and not while monitor records or snapshots are due (every step they
// look at must end on its own second half-step).
bool merging(const brahms_plan_s& p);
// Whether a call fuses step pairs: merging, and x and y passes at the ends
// of a step (three passes, or a long tau axis in the middle).
bool fusing(const brahms_plan_s& p);
// The passes of one z-step in order: axis (AX_*) and RK4 mode (NL_*) of
// each.  Three passes in general; passes along an axis of length 1 are left
// out when they would multiply by exactly 1 (so the result is unchanged bit
// for bit): nx = ny = 1 takes one tau pass with both half-steps; in a batch,
// nt = 1 with no loss and no transverse map takes x and y passes (a single
// CW problem keeps its tau pass, whose many short lines are its parallelism);
// a long tau axis takes five passes.
struct StepPasses {
  int n;
  int ax[5];
  int nl[5];
};
StepPasses step_passes(const brahms_plan_s& p, bool batched);
// One z-step with the tables of `row`; with continued = true the step's first
// half-step is left out (it was merged into the previous step's second one).
brahms_status launch_step(brahms_plan_s& p, int row, const StepIO& io, bool continued = false);
// One step of a call with fused step pairs (tables of `row`, and of row + 1
// unless `last`): the call's first step adds its first half-step and first
// axis, every step runs its middle axis, then either its own second
// half-step on its last axis (the call's last step) or the fused pass of its
// last axis, the merged RK4 step and step n+1's first axis.  Steps with `odd`
// set run the schedule's axes in reverse order.
brahms_status launch_fused_step(brahms_plan_s& p, int row, bool first, bool last, bool odd);
// The axis of the k-th pass of a step (k = 0, 1, 2) under the plan's order.
int pass_axis(const brahms_plan_s& p, int k);
// A linear-only pass (FFT . P . IFFT, or with conj(P)) along `axis`, in place.
brahms_status launch_linear_pass(brahms_plan_s& p, int row, int axis, float2* const* fields,
                                 bool conj);
const float2* table_row(const brahms_plan_s& p, int row);
// Monitor records and snapshots due once `step_done` steps are complete.
brahms_status after_step(brahms_plan_s& p, long long step_done);
const float2* nl_coefficients(const brahms_plan_s& p, int row, int half);

}  // namespace detail
}  // namespace brahms
