/* brahms.h -- C ABI of the MI355X (gfx950) engine for the chi(2)
 * split-step Fourier z-loop of BRAHMS (arXiv 2609.08384).
 *
 * The engine propagates nf = 2 (SHG) or nf = 3 (SFG / OPG) complex envelopes
 * A_j(x, y, tau) through a crystal along z by the symmetric split-step
 * scheme N/2 - L - N/2 (Sec. 3.1, eq. expon): each z-step is a fourth-order
 * Runge-Kutta half-step of the chi(2) coupling, the linear step (dispersion
 * eq. dispOp, diffraction and walk-off eq. diffOp) applied in Fourier space,
 * and a second Runge-Kutta half-step.  The equations solved, in the units of
 * brahms_field_params (x, y, tau in grid cells scaled by dx, dy, dt; z in
 * crystal lengths), are
 *
 *   nf = 3 (0 = p with w_p = w_s + w_i, 1 = s, 2 = i), eqs. CEp/CEs/CEi:
 *     dA_p/dz = L_p A_p + i kappa_p A_s A_i   exp(-i Phi(z))
 *     dA_s/dz = L_s A_s + i kappa_s A_p A_i^* exp(+i Phi(z))
 *     dA_i/dz = L_i A_i + i kappa_i A_p A_s^* exp(+i Phi(z))
 *   nf = 2 (0 = fundamental F, 1 = second harmonic S), the degenerate case:
 *     dF/dz = L_F F + i kappa_F S F^* exp(+i Phi(z))
 *     dS/dz = L_S S + i kappa_S F^2   exp(-i Phi(z))
 *   L_j = i D_j (d2/dx2 + d2/dy2) - tan(rho_j) d/dx - delta_j d/dtau
 *         - i (k''_j / 2) d2/dtau2 + (k'''_j / 6) d3/dtau3 - alpha_j / 2
 *   Phi(z) = integral_0^z dk(z') dz', dk piecewise constant per z-step,
 *
 * with periodic boundaries in x, y and tau.
 *
 * Data layout: every field is a caller-owned device buffer of nx*ny*nt
 * complex64 values (interleaved float re, im), x fastest, then y, then tau
 * (the x -> y -> tau index hierarchy of Sec. 4.3), at least 256-byte
 * aligned.  The engine updates the fields in place.
 *
 * Ownership: the library never allocates device memory.  The caller passes
 * the fields and one workspace buffer of brahms_plan_workspace_size() bytes
 * (256-byte aligned); the plan borrows both until it is destroyed or bound
 * again.  Every call after brahms_plan_create is asynchronous on the stream
 * given at creation (a hipStream_t, NULL = the legacy default stream), except
 * when BRAHMS_CHECK_FINITE is set, which synchronises that stream at the end
 * of each call.  A plan is not thread-safe; distinct plans are independent.
 *
 * Errors: every call returns a brahms_status and never throws;
 * brahms_last_error() returns a thread-local description of the last failure.
 */
#ifndef BRAHMS_H_
#define BRAHMS_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BRAHMS_OK = 0,
  BRAHMS_E_INVALID_ARG = 1,  /* bad size, pointer, parameter or step count   */
  BRAHMS_E_UNSUPPORTED = 2,  /* an axis length the transforms do not handle, or
                                a feature combination that is not provided  */
  BRAHMS_E_DEVICE = 3,       /* a HIP runtime error                          */
  BRAHMS_E_NONFINITE = 4,    /* a field became NaN/Inf (dz too large, Sec. 3.2) */
  BRAHMS_E_STATE = 5         /* call out of order (e.g. step before bind)    */
} brahms_status;

/* Flags of brahms_params.flags */
#define BRAHMS_CHECK_FINITE 1u  /* test fields for NaN/Inf after each call */

typedef struct brahms_plan_s* brahms_plan;

/* Coefficients of one field (eqs. dispOp, diffOp and the coupling of
 * eqs. CEp/CEs/CEi), in normalised units. */
typedef struct {
  double kappa;        /* nonlinear coupling kappa_j = 2 pi d_eff / (n_j lambda_j) */
  double diffraction;  /* D_j = 1 / (2 k_j)                                  */
  double tan_rho;      /* spatial walk-off tan(rho_j)                        */
  double delay;        /* group-delay coefficient delta_j (frame mismatch)   */
  double k2;           /* group-velocity dispersion k''_j                    */
  double k3;           /* third-order dispersion k'''_j                      */
  double alpha;        /* linear power attenuation alpha_j                   */
} brahms_field_params;

typedef struct {
  double dz;                    /* z-step (> 0); step n spans [n dz, (n+1) dz]    */
  double dk_const;              /* phase mismatch dk (eq. mismatch) when dk==NULL */
  const double* dk;             /* host array: per-step dk_n, copied at create    */
  int n_dk;                     /* length of dk (number of steps it covers)       */
  double dx, dy, dt;            /* grid spacings; 0 means 1                       */
  brahms_field_params field[3]; /* first nf entries used                          */
  unsigned flags;               /* BRAHMS_CHECK_FINITE                            */
  /* Transverse phase-mismatch map (the spatially varying dk(x, y, z) of the
   * phase-matching module, Sec. 4.1): in step n,
   *   dk(x, y, z) = dk_n + s_n m(x, y),
   * so Phi(x, y, z) = Phi(z) + m(x, y) Psi(z), Psi(z) = int_0^z s dz'.
   * dk_map: host array m[y][x] (nx * ny doubles, 1/L) or NULL (no map);
   * dk_map_scale: host array s_n (n_dk_map_scale steps) or NULL (s = 1).
   * Both are copied at create.  Plans only: batches and the adjoint reject a
   * map (BRAHMS_E_UNSUPPORTED). */
  const double* dk_map;
  const double* dk_map_scale;
  int n_dk_map_scale;
} brahms_params;

/* Create a plan for an nx x ny x nt grid with nfields in {2, 3}.
 * Axis lengths must be 2^a, 3 * 2^a or 9 * 2^a up to 256 (1, 2, 3, 4, 6, 8,
 * 9, 12, 16, 18, 24, 32, 36, 48, 64, 72, 96, 128, 144, 192, 256); tau may
 * also be 512, 1024, 2048 or 4096.  BRAHMS_E_UNSUPPORTED otherwise: a prime
 * factor other than 2 and 3, a factor 3^3 (27, 54, 81, 108, 162, 216, 243:
 * no register split of the line transform), x or y above 256.
 * The parameters are copied.
 * Errors: BRAHMS_E_INVALID_ARG for a non-positive size, nf outside {2, 3},
 * NULL params/out, dz <= 0, a non-finite coefficient, dk != NULL with
 * n_dk < 1, or dk_map_scale without dk_map or with n_dk_map_scale < 1. */
brahms_status brahms_plan_create(int nx, int ny, int nt, int nfields,
                                 const brahms_params* params, void* hip_stream,
                                 brahms_plan* out);

/* Bytes of device workspace the plan needs (tables and per-step
 * propagators). */
brahms_status brahms_plan_workspace_size(brahms_plan plan, size_t* bytes);

/* Attach nfields field buffers and the workspace (device pointers, see the
 * layout and ownership notes above) and upload the plan's tables.  Resets
 * nothing else: z keeps its value.  Errors: BRAHMS_E_INVALID_ARG for NULL or
 * misaligned pointers, BRAHMS_E_DEVICE for a failed upload. */
brahms_status brahms_plan_bind(brahms_plan plan, void* const* fields, void* workspace);

/* Advance nsteps z-steps (Sec. 3.1: N/2 - L - N/2 per step) from the current
 * step index; nsteps = 0 is a no-op.  Errors: BRAHMS_E_STATE before bind,
 * BRAHMS_E_INVALID_ARG for nsteps < 0 or steps beyond the dk profile,
 * BRAHMS_E_NONFINITE (with BRAHMS_CHECK_FINITE) when a field holds NaN/Inf
 * afterwards; the step index then counts the completed steps and the field
 * contents are unspecified. */
brahms_status brahms_step(brahms_plan plan, int nsteps);

/* Propagate to z_end: n = round((z_end - z) / dz) steps.  z_end must lie
 * within 1e-9 max(1, |z_end|) of a multiple of dz and not before z. */
brahms_status brahms_propagate(brahms_plan plan, double z_end);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): brahms_propagate
 * with the plan's workspace taken from a static device array of the library
 * (BRAHMS_NOALLOC_SCRATCH_BYTES bytes, one per GPU, held until the process
 * ends) instead of a caller buffer.  It binds `fields` (nfields device
 * pointers, the layout of brahms_plan_bind) and that array to the plan, then
 * propagates to z_end as brahms_propagate does, with the same kernels: the
 * result is bitwise the one brahms_plan_bind + brahms_propagate give.  The
 * plan stays bound to the fields and the array afterwards.  The call
 * allocates and frees no device memory (no hipMalloc, hipFree, graph capture
 * or event creation; kernel timing is skipped during the call).
 * Every call on one GPU shares that GPU's array and leaves its tables there:
 * calls that overlap on one GPU (two plans on different streams, or another
 * thread) race and give undefined results; serialise them.  Nothing in the
 * array needs to start at zero (every table is written before it is read).
 * Errors: BRAHMS_E_INVALID_ARG for NULL pointers, a z_end as for
 * brahms_propagate, or a plan whose workspace (brahms_plan_workspace_size)
 * exceeds BRAHMS_NOALLOC_SCRATCH_BYTES (checked before any device work);
 * BRAHMS_E_STATE for a plan with the graph schedule; BRAHMS_E_DEVICE. */
#define BRAHMS_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
brahms_status brahms_propagate_noalloc(brahms_plan plan, void* const* fields, double z_end);

/* Current z = (step index) * dz. */
brahms_status brahms_get_z(brahms_plan plan, double* z);

/* Set the step index to round(z / dz) (resume from saved fields); z must be
 * a non-negative multiple of dz within the tolerance of brahms_propagate. */
brahms_status brahms_set_z(brahms_plan plan, double z);

brahms_status brahms_plan_destroy(brahms_plan plan);

/* Execution schedule of a plan (pass order, graph replay and fused step
 * pairs change only how the method is computed; merge_halves changes the
 * integrator of the nonlinear part by O(h^5) per step; results of different
 * schedules agree to rounding).  The linear step is
 * applied as three commuting one-axis operators (Sec. 3.1: the dispersion
 * and diffraction operators commute), each a pass over the fields; the first
 * pass of a z-step also performs the first Runge-Kutta half-step and the last
 * pass the second one.
 *   pass_order 0: x pass, y pass, tau pass (default)
 *   pass_order 1: tau pass, y pass, x pass
 *   pass_order 2: x pass, tau pass, y pass (tau linear, one field per block)
 *   pass_order 3: y pass, tau pass, x pass
 *   (orders 2 and 3 act as 0 and 1 for a plan with a transverse dk map; the
 *   adjoint runs with orders 0 and 1 only; a tau axis longer than 256 always
 *   takes x, y and its three tau passes)
 *   graph 1: brahms_step replays whole 64-step chunks (tables and passes) from
 *     a hipGraph captured once per binding and schedule (bitwise the same
 *     result; removes the per-launch host cost).  Chunks that record timing,
 *     monitors or snapshots, partial chunks, and plans whose transverse map
 *     tables are filled per step run launch by launch.  The graph is captured
 *     by brahms_plan_set_schedule or brahms_plan_bind, whichever comes last.
 *   merge_halves 1: within one brahms_step call, the second RK4 half-step of
 *     step n and the first of step n + 1 (Eq. expon: N/2 - L - N/2 repeated)
 *     run as one classical RK4 step of size dz from z_n + dz/2.  The exact
 *     nonlinear flows over the two halves compose to the flow over dz, so
 *     only the RK4 truncation term changes (O(dz^5) per step); the call's
 *     first step keeps its first half-step and its last step its second one,
 *     so the fields returned are those at a step boundary.  One RK4 update
 *     per step instead of two.  Needs a constant dk (no profile) and no
 *     transverse map (BRAHMS_E_UNSUPPORTED otherwise); calls run with literal
 *     half-steps while monitor records or snapshots are set; the adjoint
 *     always differentiates the literal half-steps.
 *   fuse_steps 1 (needs merge_halves 1; not for nx = ny = 1 with tau <= 256,
 *     whose steps are one pass): within one call, even steps (counted from
 *     the call's first) take the axes in pass_order's order a, m, b and odd
 *     steps in the order b, m, a (a long tau axis is m, its three passes in
 *     the middle; x and y are a and b, y first for odd pass orders).  The axis operators commute (Sec. 3.1), so this
 *     is the same linear step; and each step's last transform, the merged RK4
 *     step and the next step's first transform are along one axis and run
 *     as one pass: two reads and writes of the fields per step instead of
 *     three.  Calls run without it while merge_halves is suspended.
 *     BRAHMS_E_INVALID_ARG without merge_halves, BRAHMS_E_UNSUPPORTED for
 *     other step structures.
 *   split (bits 1 = x, 2 = y, 4 = tau): a line of length N = N1 N2 is
 *     transformed by N2 lanes of N1 values each (a register DFT, one exchange
 *     through LDS, a second register DFT); lengths 8, 12, 16, 24, 32, 48 and
 *     64 also have a second split with half the lanes per line (or one lane)
 *     and so twice the lines per block: 8 = 8 x 1, 12 = 12 x 1, 16 = 8 x 2,
 *     24 = 24 x 1, 32 = 16 x 2, 48 = 24 x 2, 64 = 16 x 4 (the first splits
 *     are 4 x 2, 6 x 2, 4 x 4, 12 x 2, 8 x 4, 12 x 4, 8 x 8).  A set bit takes
 *     the second split on that axis where its length has one (other axes,
 *     the adjoint passes and long tau axes keep the first).  The result
 *     agrees to rounding.  BRAHMS_E_INVALID_ARG outside 0 .. 7.
 *   wide (bits 1 = x, 2 = y, 4 = tau): the linear passes along a set axis
 *     (one field per block, no RK4 step: the middle axis of fused step
 *     pairs, the first axis of merged steps) run blocks of 512 threads
 *     instead of 256, twice the lines per block; y and tau lines are then
 *     read and written in row segments twice as long (32 columns for a
 *     256-point axis).  Every line is transformed as before: bitwise the same
 *     result.  Axes of length 72 or 144 (36 values per lane, whose 512-lane
 *     exchange rows would not fit the LDS) ignore their bit.  Plans only
 *     (batches and the adjoint keep 256).  BRAHMS_E_INVALID_ARG outside
 *     0 .. 7.
 * The autotuner in the Python package times the candidates per grid shape. */
typedef struct {
  int pass_order;
  int graph;
  int merge_halves;
  int fuse_steps;
  int split;        /* bit a (x = 1, y = 2, tau = 4): second register/lane split of that axis */
  int wide;         /* bit a: that axis's linear passes with 512-thread blocks */
  int reserved[2];
} brahms_schedule;

brahms_status brahms_plan_set_schedule(brahms_plan plan, const brahms_schedule* sched);
brahms_status brahms_plan_get_schedule(brahms_plan plan, brahms_schedule* sched);

/* Kernel timing (diagnostics, not part of the method).  While enabled, every
 * kernel launch of brahms_step is bracketed by HIP events recorded on the
 * plan's stream (at most 65536 launches are timed between two reads).
 * brahms_timing_read synchronises that stream, then writes, per launch kind
 * (0 = X pass, 1 = Y pass, 2 = tau pass, 3 = per-step table kernel), the summed
 * duration in milliseconds and the number of timed launches, and clears the
 * record.  Errors: BRAHMS_E_INVALID_ARG for NULL outputs, BRAHMS_E_DEVICE. */
#define BRAHMS_TIMING_KINDS 4
brahms_status brahms_timing_enable(brahms_plan plan, int enable);
brahms_status brahms_timing_read(brahms_plan plan, double* ms, long long* launches);

/* Diagnostics: the output quantities of Sec. 6 (pulse power per time slice,
 * field energies) and the Manley-Rowe combinations of the coupled equations
 * (Sec. 2), taken on the device from the bound fields.
 *
 * A record is brahms_record_size() doubles describing the fields at step
 * index n (z = n dz):
 *   [0]                      n
 *   [1, 1 + nf nt)           P_j(tau) = sum_{x,y} |A_j|^2 dx dy, field-major
 *   [1 + nf nt, + nf)        E_j = sum_tau P_j(tau) dtau
 *   [1 + nf (nt + 1), + 3)   nf = 3: E_p/k_p + E_s/k_s, E_p/k_p + E_i/k_i,
 *                            E_s/k_s - E_i/k_i (kappa_j of the plan);
 *                            nf = 2: E_F/k_F + E_S/k_S, NaN, NaN;
 *                            NaN wherever a kappa is 0.
 * Sums run in FP64 in a fixed order: records are reproducible bit for bit.
 * Records and snapshot buffers are caller-owned device memory; the calls
 * below only store the pointers, which must stay valid while the plan steps.
 *
 * brahms_record_size: doubles per record.
 * brahms_diagnose: one record of the fields as they are now (asynchronous
 *   on the plan's stream).  Errors: BRAHMS_E_STATE before bind.
 * brahms_set_monitor: from now on, whenever brahms_step completes a step
 *   whose index is a multiple of `every`, append a record to `records`
 *   (room for `capacity` records; later ones are dropped).  every = 0
 *   switches the monitor off.  Resets the record count.
 * brahms_get_monitor_count: records written since brahms_set_monitor.
 * brahms_set_snapshots: n snapshots; when brahms_step completes step index
 *   steps[i] (>= 1) it copies field j to buffers[i * nf + j] (field layout of
 *   brahms_plan_bind).  n = 0 removes them.  Replaces earlier snapshots.
 * Errors: BRAHMS_E_INVALID_ARG for NULL pointers, negative sizes or steps
 * below 1. */
brahms_status brahms_record_size(brahms_plan plan, int* ndoubles);
brahms_status brahms_diagnose(brahms_plan plan, double* record);
brahms_status brahms_set_monitor(brahms_plan plan, int every, double* records, int capacity);
brahms_status brahms_get_monitor_count(brahms_plan plan, int* count);
brahms_status brahms_set_snapshots(brahms_plan plan, int n, const long long* steps,
                                   void* const* buffers);

/* Adjoint (reverse-mode gradient) of the z-loop, for inverse design.  Not in
 * the paper; it differentiates exactly the discrete map that brahms_step
 * computes (Sec. 3.1: RK4 half-steps and the Fourier-space linear step).
 * Cotangents follow the convention g = dJ/dRe(A) + i dJ/dIm(A) of a real loss
 * J, the layout of the fields.
 *
 * brahms_adjoint_workspace_size: device bytes needed for nsteps steps with a
 *   checkpoint every checkpoint_every (1..64) steps: ceil(nsteps/K) + 2K + 1
 *   states of nf fields plus small reduction buffers.
 * brahms_adjoint_forward: from the current step index n0, advance the bound
 *   fields nsteps steps exactly as brahms_step does, storing checkpoints in
 *   adj_workspace (caller-owned, 256-byte aligned, kept until the backward
 *   call).  The fields end at z = (n0 + nsteps) dz.
 * brahms_adjoint_backward: grad holds nf device buffers (field layout) with
 *   dJ/dA(z_end) on entry and dJ/dA(z0) on exit.  grad_dk (host, may be NULL)
 *   receives dJ/ddk: n_dk entries (entries past the window are zero) when a
 *   per-step profile was given at create, else one entry dJ/d(dk_const).
 *   The z counter is left at z_end.  Synchronises the plan's stream when
 *   grad_dk is not NULL.  brahms_step, brahms_set_z or brahms_plan_bind
 *   between the two calls discard the forward record (BRAHMS_E_STATE).
 * Errors: BRAHMS_E_STATE (not bound / no forward record), BRAHMS_E_INVALID_ARG
 * (sizes, pointers, steps beyond the dk profile), BRAHMS_E_DEVICE. */
brahms_status brahms_adjoint_workspace_size(brahms_plan plan, int nsteps, int checkpoint_every,
                                            size_t* bytes);
brahms_status brahms_adjoint_forward(brahms_plan plan, int nsteps, int checkpoint_every,
                                     void* adj_workspace);
brahms_status brahms_adjoint_backward(brahms_plan plan, void* const* grad, double* grad_dk);

/* The adjoint in one call: the vector-Jacobian product of nsteps steps from
 * the plan's current step n0 for a given cotangent.  fields_in (nf device
 * buffers) is copied into the plan's bound fields, which are advanced as by
 * brahms_adjoint_forward (they end at z = (n0 + nsteps) dz, the forward
 * output); grad_out (dJ/dA at z_end) is copied into grad_in, which then
 * receives dJ/dA at z0 as by brahms_adjoint_backward, and grad_dk as there.
 * Buffers may alias (fields_in = the bound fields, grad_in = grad_out).
 * The split calls above serve the usual case where the cotangent depends on
 * the forward output (a loss of the fields at z_end): there one forward with
 * checkpoints serves both the loss and the reverse sweep, where this call
 * would repeat it.  adj_workspace as for brahms_adjoint_forward.  Errors as
 * for the two calls it combines. */
brahms_status brahms_adjoint(brahms_plan plan, int nsteps, int checkpoint_every, const void* const* fields_in,
                             const void* const* grad_out, void* const* grad_in, double* grad_dk,
                             void* adj_workspace);

/* Batched sweeps: many independent problems (each its own grid, fields and
 * parameters, e.g. a scan of dk or of the focusing, as the parameter-sweep
 * tab of Sec. 4.4 runs them one after another) propagated together.
 * Problems of equal shape, field count and pass order share launches, in
 * groups of at most group_max problems (0 = sized so that a group's fields
 * fit a 160 MB cache budget); the whole run is captured once into a hipGraph
 * (on a capture stream of the library's) and replayed on the caller's stream
 * hip_stream, so it is ordered after work already queued there and before
 * work queued there afterwards.
 *
 * brahms_batch_create: n problems; shapes holds n x 4 ints (nx, ny, nt, nf),
 *   params n brahms_params, nsteps n step counts (each problem is propagated
 *   nsteps[i] steps from z = 0 by every run).  Per-problem errors as for
 *   brahms_plan_create.
 * brahms_batch_set_schedule: launch-group size and (optional, n entries)
 *   pass orders; invalidates the binding (bind again).
 * brahms_batch_set_merge_halves: 1 runs every problem with merged RK4
 *   half-steps (as the plan schedule field merge_halves: each run's first
 *   step keeps its first half-step, each problem's last step its second
 *   one); 0 (default) keeps the literal N/2 - L - N/2.  Invalidates the
 *   binding.  Errors: BRAHMS_E_INVALID_ARG for another value,
 *   BRAHMS_E_UNSUPPORTED if a problem has a dk profile.
 * brahms_batch_set_fuse_steps: 1 runs the launch groups whose steps take
 *   three passes as fused step pairs (as the plan schedule field fuse_steps;
 *   a problem's last step ends on its own second half-step inside the fused
 *   launch).  Needs merged half-steps (BRAHMS_E_INVALID_ARG otherwise);
 *   BRAHMS_E_UNSUPPORTED for a batch that holds a problem with a tau axis
 *   longer than 256.  Invalidates the binding.
 * brahms_batch_set_splits: per-problem register/lane splits (n entries, the
 *   schedule field split of plans: bits x = 1, y = 2, tau = 4), or NULL for
 *   the first split everywhere; problems of one shape with different splits
 *   go to different launch groups.  Invalidates the binding.  Errors:
 *   BRAHMS_E_INVALID_ARG outside 0 .. 7.
 * brahms_batch_set_wide: per-problem 512-thread blocks for the linear x and
 *   y passes (n entries, the schedule field wide of plans restricted to the
 *   bits x = 1 and y = 2: a batch's linear tau passes share their block-to-
 *   tile map with the tau launches that carry a half-step, and keep 256
 *   threads), or NULL for none; bitwise the same result.  Problems of one
 *   shape with different values go to different launch groups.  Invalidates
 *   the binding.  Errors: BRAHMS_E_INVALID_ARG outside 0 .. 3.
 * brahms_batch_set_streams: 1 (default) captures the run into one hipGraph
 *   whose launch groups run one after the other (largest first); 2 .. 4
 *   runs on that many streams, the caller's stream hip_stream and
 *   streams - 1 side streams of the batch, forked from hip_stream and joined
 *   back into it with events: launch groups, largest first, each go to the
 *   stream with the least work so far, so groups of large and of small grids
 *   execute at the same time.  Each stream's groups are captured into a
 *   linear hipGraph of their own at the first run and replayed after that.
 *   With largest_alone = 1 the largest group instead runs after the others
 *   have finished, on hip_stream (the smaller groups share the chip, the
 *   largest fills it alone).  Same kernels and tables, bitwise the same
 *   result.  Errors:
 *   BRAHMS_E_INVALID_ARG for streams outside 1 .. 4 or largest_alone
 *   outside {0, 1}.
 * brahms_batch_set_group_limits: per-problem launch-group sizes (n entries,
 *   0 = from the cache budget) that replace group_max; a group takes the
 *   limit of its first problem, so give problems of one shape the same one.
 *   NULL goes back to group_max.  Invalidates the binding.  Errors:
 *   BRAHMS_E_INVALID_ARG for a negative limit.
 * brahms_batch_bind: fields holds sum(nf_i) device pointers, problem-major,
 *   each in the field layout of brahms_plan_bind; workspace as for plans.
 * brahms_batch_run: propagate every problem nsteps[i] steps from z = 0
 *   (asynchronous: one graph launch on hip_stream, or one per stream; the
 *   first run also builds the graphs).  Descriptor uploads at bind also go on hip_stream and
 *   wait for it.
 * brahms_batch_run_steps: a run with per-problem step counts nsteps[i] (n
 *   entries, each between 0 and the count given at create): the counts go
 *   into the descriptors (uploaded on hip_stream, after any run still reading
 *   them) and the same graph is replayed; problems past their count leave
 *   their launches at once.  Errors: BRAHMS_E_INVALID_ARG for a count out of
 *   range, BRAHMS_E_STATE before bind.
 * brahms_batch_groups: number of launch groups and their sizes (members may
 *   be NULL or hold one int per group).
 * brahms_batch_destroy: waits for hip_stream, then frees the batch; the
 *   streams and events that captured its graph are kept for later batches on
 *   the same device, not destroyed. */
typedef struct brahms_batch_s* brahms_batch;
brahms_status brahms_batch_create(int n, const int* shapes, const brahms_params* params,
                                  const int* nsteps, void* hip_stream, brahms_batch* out);
brahms_status brahms_batch_set_schedule(brahms_batch batch, int group_max, const int* pass_order);
brahms_status brahms_batch_set_group_limits(brahms_batch batch, const int* limits);
brahms_status brahms_batch_set_streams(brahms_batch batch, int streams, int largest_alone);
brahms_status brahms_batch_set_splits(brahms_batch batch, const int* splits);
brahms_status brahms_batch_set_wide(brahms_batch batch, const int* wide);
brahms_status brahms_batch_set_merge_halves(brahms_batch batch, int merge_halves);
brahms_status brahms_batch_set_fuse_steps(brahms_batch batch, int fuse_steps);
brahms_status brahms_batch_workspace_size(brahms_batch batch, size_t* bytes);
brahms_status brahms_batch_bind(brahms_batch batch, void* const* fields, void* workspace);
brahms_status brahms_batch_run(brahms_batch batch);
brahms_status brahms_batch_run_steps(brahms_batch batch, const int* nsteps);
brahms_status brahms_batch_groups(brahms_batch batch, int* ngroups, int* members);
brahms_status brahms_batch_destroy(brahms_batch batch);

/* Thread-local message for the last failing call (empty if none). */
const char* brahms_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BRAHMS_H_ */
