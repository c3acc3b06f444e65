// Device kernels of the chi(2) split-step z-loop (gfx950).
//
// One z-step (symmetric splitting N/2 - L - N/2, Sec. 3.1 eq. expon) is three
// HBM passes over the fields, each a batch of independent 1D lines:
//
//   X pass : RK4 half-step of the coupled chi(2) equations (eqs. CEp/CEs/CEi),
//            then FFT_x . P_x . IFFT_x                    (all fields together)
//   Y pass : FFT_y . P_y . IFFT_y                          (one field per block)
//   T pass : FFT_tau . P_tau . IFFT_tau, then the second RK4 half-step
//
// The linear step exp(L dz) is separable, L = L_x + L_y + L_tau with the
// three parts acting on different axes, so its Fourier-space form is the
// product of three commuting 1D transform-multiply-inverse operators; this is
// the paper's own split into a tau step and an xy step (Sec. 4.3), taken one
// axis further.  Fields stay x-fastest, [nt][ny][nx] complex64, in place:
// the y and tau passes read their lines with a stride instead of
// materialising the paper's reordered copy.  The passes may run in either
// order (x, y, tau or tau, y, x); a tau axis longer than 256 takes three
// passes (a four-step transform, AX_TAF / AX_TB / AX_TAI below).
#pragma once

#include <hip/hip_runtime.h>

#include "dft.hpp"

namespace brahms {

constexpr int kBlock = 256;        // threads per block in every pass but the wide linear ones
constexpr int kNlCoef = 6;         // RK4 coefficients per field per half-step

enum Axis { AX_X = 0, AX_Y = 1, AX_T = 2,
            // a tau axis longer than one line transform, nt = A B, tau = a + A b
            // (a four-step transform over three passes):
            AX_TAF = 3,   // B-point transforms over b, times exp(-2 pi i a k_b / nt)
            AX_TB = 4,    // A-point transforms over a, propagator, inverse transforms
            AX_TAI = 5 }; // times exp(+2 pi i a k_b / nt), inverse B-point transforms
constexpr int kMaxLongT = 4096;   // longest tau axis (entries of the staged table)

__host__ __device__ constexpr bool long_tau_kind(int ax) { return ax >= AX_TAF; }
enum NlMode { NL_NONE = 0, NL_BEFORE = 1, NL_AFTER = 2,
              NL_BOTH = 3 };   // both half-steps in one pass (the only pass of a step)
// Added to NL_BEFORE / NL_AFTER: the mismatch phase also has a transverse
// part (a per-(x, y) table of exp(i m(x, y) Psi(z)) for each RK4 stage).
constexpr int NL_MAP = 4;
// Added to NL_AFTER (fused step pair): after the RK4 step the pass applies
// the next z-step's transform along the same axis, with that step's tables
// (tw2, prop2, consts2), so the last axis of step n and the first axis of
// step n + 1 cost one read and one write of the fields.
constexpr int NL_FUSE = 8;

struct PassArgs {
  float2* f[3];          // fields read (complex64, [nt][ny][nx])
  float2* fo[3];         // fields written (== f for an in-place pass)
  float2* pre[3];        // if pre[0]: the last pass also stores its values
                         // just before the RK4 half-step here
  int conj;              // multiply by conj(P) (adjoint linear step)
  const float2* tw;      // this step's forward twiddles exp(-2 pi i m / N), m < N
  const float2* prop;    // this step's propagators, field j's table of this
                         // axis at prop + j * field_stride + axis_off
  const float2* nl;      // RK4 coefficients of the step's first half-step, [nf][6]
  const float2* nl2;     // those of its second half-step (or, when adjacent
                         // halves are merged, of one RK4 step of size dz
                         // from z_n + dz/2)
  const DftConsts* consts;  // this step's register-DFT constants
  int nx, ny, nt;
  int axis_off, field_stride;
  unsigned tile_mul;     // block -> tile map: tile = (block * tile_mul) mod tiles
  unsigned tiles;        // number of tiles (blocks along x of the launch)
  long long nz;          // batched launches: the instance is done once step >= nz
  const float2* map;     // NL_MAP: exp(i m(x,y) Psi) at this half-step's three
                         // stage positions, [3][ny][nx]
  const float2* tw2;     // NL_FUSE: the next step's twiddles, propagators and
  const float2* prop2;   // DFT constants along the same axis
  const DftConsts* consts2;
};

// ---------------------------------------------------------------------------
// chi(2) RK4 point update.  With c_j(z) = i kappa_j exp(sigma_j i Phi(z)) and
// the bilinear products Q_j (p: s i, s: p i*, i: p s*; SHG F: S F*, S: F F)
// one classical RK4 step of size h from z_a is
//   y2 = y + a1 Q(y),  y3 = y + a2 Q(y2),  y4 = y + a3 Q(y3),
//   y' = y + b1 Q(y) + b2 Q(y2) + b2 Q(y3) + b4 Q(y4)
// with a1 = h/2 c(z_a), a2 = h/2 c(z_m), a3 = h c(z_m), b1 = h/6 c(z_a),
// b2 = h/3 c(z_m), b4 = h/6 c(z_a + h), z_m = z_a + h/2.  The coefficients
// are formed in double precision per half-step by the table kernel.
// Adjacent halves (the second half of step n and the first of step n + 1)
// may be merged into one RK4 step of size h = dz from z_n + dz/2: the exact
// flows compose, and the two integrators differ by O(h^5) per step.
// ---------------------------------------------------------------------------
template <int NF>
__device__ inline void chi2_products(const float2* y, float2* q) {
  if constexpr (NF == 3) {
    q[0] = cmul(y[1], y[2]);
    q[1] = cmulc(y[0], y[2]);
    q[2] = cmulc(y[0], y[1]);
  } else {
    q[0] = cmulc(y[1], y[0]);
    q[1] = cmul(y[0], y[0]);
  }
}

__device__ inline float2 cfma(float2 acc, float2 c, float2 q) {  // acc + c q
  return make_float2(fmaf(c.x, q.x, fmaf(-c.y, q.y, acc.x)),
                     fmaf(c.x, q.y, fmaf(c.y, q.x, acc.y)));
}

// A value that is the same in every lane, moved into scalar registers.
__device__ inline float2 wave_uniform(float2 v) {
  return make_float2(__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v.x))),
                     __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v.y))));
}

// Transverse part of the mismatch phase at one stage: Q_j times
// exp(i sigma_j m Psi) = w (sigma = +1) or conj(w) (sigma = -1, the
// sum-frequency field: p of three fields, S of SHG).
template <int NF>
__device__ inline void rotate_products(float2* q, float2 w) {
  constexpr int neg = NF == 3 ? 0 : 1;
#pragma unroll
  for (int j = 0; j < NF; ++j) q[j] = j == neg ? cmulc(q[j], w) : cmul(q[j], w);
}

// MAP: w[0], w[1], w[2] are the transverse phase factors at z_a, z_a + h/2
// and z_a + h (unused otherwise).
//
// The update sums stage values rather than increments: a1 = 3 b1, a2 = 3 b2 / 2
// and a3 = 3 b2, so b1 Q(y) = (y2 - y) / 3, b2 Q(y2) = 2 (y3 - y) / 3 and
// b2 Q(y3) = (y4 - y) / 3, and
//   y' = y + (y2 + 2 y3 + y4 - 4 y) / 3 + b4 Q(y4).
// Two operations per stage and field replace the complex multiply-add of
// each increment.  The factor 1/3 (rounded to FP32) scales only the O(h)
// bracket, so its rounding biases the nonlinear increment by ~3e-8 of itself
// and never the field; the bracket's rounding errors are of the size of the
// increment sums' (about one ulp of y per step) and independent from step to
// step.
template <int NF, bool MAP = false>
__device__ inline void rk4_point(float2* y, const float2 (*co)[kNlCoef], const float2* w = nullptr) {
  constexpr float kThird = 1.0f / 3.0f;
  float2 q[NF], s[NF], ys[NF];
  chi2_products<NF>(y, q);
  if constexpr (MAP) rotate_products<NF>(q, w[0]);
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    ys[j] = cfma(y[j], co[j][0], q[j]);   // y2
    s[j] = ys[j];
  }
  chi2_products<NF>(ys, q);
  if constexpr (MAP) rotate_products<NF>(q, w[1]);
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    ys[j] = cfma(y[j], co[j][1], q[j]);   // y3
    s[j] = make_float2(fmaf(2.0f, ys[j].x, s[j].x), fmaf(2.0f, ys[j].y, s[j].y));
  }
  chi2_products<NF>(ys, q);
  if constexpr (MAP) rotate_products<NF>(q, w[1]);
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    ys[j] = cfma(y[j], co[j][2], q[j]);   // y4
    s[j] = cadd(s[j], ys[j]);
  }
  chi2_products<NF>(ys, q);
  if constexpr (MAP) rotate_products<NF>(q, w[2]);
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    const float2 d = make_float2(fmaf(-4.0f, y[j].x, s[j].x), fmaf(-4.0f, y[j].y, s[j].y));
    const float2 u = make_float2(fmaf(kThird, d.x, y[j].x), fmaf(kThird, d.y, y[j].y));
    y[j] = cfma(u, co[j][5], q[j]);
  }
}

// ---------------------------------------------------------------------------
// One line transform of length N = N1 N2 (N2 divides N1) by N2 threads.
// Thread t holds x[t + N2 e] in slot e (e < N1).  Stage 1: an N1-point DFT in
// registers over e, times exp(-+2 pi i t k1 / N).  Exchange through LDS.
// Stage 2: for each k1 = t + N2 a, an N2-point DFT over the N2 threads' values.
// The result X[k1 + N1 k2] lands in slot a + (N1/N2) k2, i.e. thread t again
// holds index t + N2 e in slot e, so the inverse transform starts from the
// same layout without another exchange.
// ---------------------------------------------------------------------------
template <int N1, int N2, int BLOCK = kBlock>
struct LineGeom {
  static constexpr int N = N1 * N2;
  static constexpr int LPB = BLOCK / N2;                   // lines per block
  static constexpr int ROW = (N2 > 1) ? N2 + 1 : 1;        // padded LDS row
  static constexpr int LS0 = N1 * ROW;
  static constexpr int LSTRIDE = (N2 > 1) ? (LS0 | 1) : LS0;  // odd stride
  static constexpr int LDS_ELEMS = (N2 > 1) ? LPB * LSTRIDE : 1;
};

// Synchronisation of a line's lanes around its LDS exchange: the block's
// barrier, or, when every line lies within one wavefront (WAVE), only an
// ordering fence (a wave's LDS instructions complete in issue order).
template <bool WAVE>
__device__ __forceinline__ void line_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  } else {
    __syncthreads();
  }
}

template <int N1, int N2, bool INV, bool WAVE = false>
__device__ inline void line_fft(float2 (&v)[N1], int t, float2* lbuf, const float2* tw,
                                const DftConsts& K) {
  using G = LineGeom<N1, N2>;
  dft<N1, INV>(v, K);
  if constexpr (N2 > 1) {
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) {
      float2 w = tw[t * k1];
      if (INV) w.y = -w.y;
      v[k1] = cmul(v[k1], w);
    }
    line_sync<WAVE>();  // earlier readers of this line's LDS row are done
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) lbuf[k1 * G::ROW + t] = v[k1];
    line_sync<WAVE>();
    constexpr int R = N1 / N2;
#pragma unroll
    for (int a = 0; a < R; ++a) {
      float2 u[N2];
      const int k1 = t + N2 * a;
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) u[n2] = lbuf[k1 * G::ROW + n2];
      dft<N2, INV>(u, K);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) v[a + R * k2] = u[k2];
    }
  }
}

// ---------------------------------------------------------------------------
// Field access.  Field values are streamed once per pass; the addresses are a
// uniform base (scalar registers) plus a 32-bit element offset.
// ---------------------------------------------------------------------------
#ifndef BRAHMS_NT_X
#define BRAHMS_NT_X 1
#endif
#ifndef BRAHMS_NT_YT
#define BRAHMS_NT_YT 0
#endif
// Blocks of kBlock threads per CU the pass kernels are compiled for: 3 is
// 3 waves per SIMD, a budget of 168 VGPRs (granules of 8 out of 512).  The
// three-field passes that carry an RK4 step take 132-148 and the fused
// step-pair pass's LDS allows 3 blocks as well; without the bound the
// compiler may take more registers and leave room for 2 waves only, which
// cost the fused pass ~15 % of its speed.  Kernels whose LDS already limits
// them to fewer blocks keep their register count.  Lines of 36 values per
// lane (lengths 72 and 144) need 216 VGPRs for three fields and an LDS row
// block that leaves room for one block per CU, so they are compiled for one.
#ifndef BRAHMS_MIN_BLOCKS
#define BRAHMS_MIN_BLOCKS 3
#endif

typedef float f32x2 __attribute__((ext_vector_type(2)));

// Tie a point's RK4 inputs to the previous point's results with an empty asm
// (no instructions): the points of a thread are then updated one after the
// other instead of all interleaved, which would run out of registers.
template <int NF, int N1>
__device__ __forceinline__ void point_link(float2* y, float2 (&v)[NF][N1], int prev) {
#pragma unroll
  for (int j = 0; j < NF; ++j)
    asm volatile("" : "+v"(y[j].x), "+v"(y[j].y), "+v"(v[j][prev].x), "+v"(v[j][prev].y));
}

// The fields of a pass are read and written through buffer resources: the
// field's base and byte size sit in scalar registers, a lane's slot e at the
// lane's byte offset plus the uniform offset 8 e estep, which the scalar unit
// forms, so the slots' addresses take no vector instructions (global
// addressing takes a 64-bit add per slot).  The byte offsets fit 32 bits:
// a field holds at most 2^28 values.  Accesses past the size read zero and
// store nothing.
constexpr int kRsrcWord3 = 0x00020000;   // raw, untyped 32-bit buffer

__device__ inline __amdgpu_buffer_rsrc_t field_rsrc(const float2* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(base), short(0), int(bytes), kRsrcWord3);
}

template <bool NT>
__device__ inline float2 load_slot(__amdgpu_buffer_rsrc_t r, unsigned lane_bytes, unsigned slot_bytes) {
  const f32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, lane_bytes, slot_bytes, NT ? 2 : 0);
  return make_float2(v.x, v.y);
}

template <bool NT>
__device__ inline void store_slot(__amdgpu_buffer_rsrc_t r, unsigned lane_bytes, unsigned slot_bytes,
                                  float2 v) {
  f32x2 w;
  w.x = v.x;
  w.y = v.y;
  __builtin_amdgcn_raw_buffer_store_b64(w, r, lane_bytes, slot_bytes, NT ? 2 : 0);
}

template <bool NT>
__device__ inline float2 load_field(const float2* base, unsigned idx) {
  if constexpr (NT) {
    const f32x2 v = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(base) + idx);
    return make_float2(v.x, v.y);
  } else {
    return base[idx];
  }
}

template <bool NT>
__device__ inline void store_field(float2* base, unsigned idx, float2 v) {
  if constexpr (NT) {
    f32x2 w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<f32x2*>(base) + idx);
  } else {
    base[idx] = v;
  }
}

// Transverse phase factors of slot e at the half-step's three stage
// positions: read per slot along x, the column's values along tau.
template <int AX, int N2>
__device__ __forceinline__ void map_factors(const float2* map, unsigned plane, unsigned xy0, int e,
                                            const float2* wt, float2* w) {
  if constexpr (AX == AX_T || long_tau_kind(AX)) {
#pragma unroll
    for (int k = 0; k < 3; ++k) w[k] = wt[k];
  } else {
    const unsigned xy = xy0 + unsigned(N2 * e);
#pragma unroll
    for (int k = 0; k < 3; ++k) w[k] = map[k * plane + xy];
  }
}

// ---------------------------------------------------------------------------
// The fused axis pass.  AX selects the line family:
//   X: line = (y, tau), element stride 1, lanes t-fastest (contiguous loads)
//   Y: line = (x, tau), element stride nx, lanes x-fastest (coalesced rows)
//   T: line = (x, y),   element stride nx*ny, lanes (x,y)-fastest
// NF is the number of fields held by one thread (Y: 1, one field per block).
// FULL: every line of every block exists (no bounds masks).
// ---------------------------------------------------------------------------
// bx: tile index along the launch's x dimension; field0: first field
// handled (y pass: the block's field); next: a fused pass also applies the
// next step's transform (false: the problem's last step, which ends on its
// own second half-step).
template <int N1, int N2, int AX, int NF, int NL, bool FULL, int BLOCK = kBlock>
__device__ __forceinline__ void axis_pass_body(const PassArgs& args, unsigned bx, int field0,
                                               bool next = true) {
  using G = LineGeom<N1, N2, BLOCK>;
  constexpr int N = G::N;
  constexpr int NLM = NL & 3;                  // where the RK4 half-step goes
  constexpr bool MAP = (NL & NL_MAP) != 0;     // transverse mismatch map
  constexpr bool NT = (AX == AX_X) ? bool(BRAHMS_NT_X) : bool(BRAHMS_NT_YT);
  constexpr bool LONG = long_tau_kind(AX);
  constexpr bool FUSE = (NL & NL_FUSE) != 0;   // and the next step's transform
  // x lines: a line's N2 lanes are consecutive threads, within one wavefront
  constexpr bool WL = AX == AX_X && N2 <= 64 && 64 % N2 == 0;
  static_assert(!(MAP && (NLM == NL_BOTH || AX == AX_Y)),
                "the transverse map runs only with a half-step per pass on x or tau");
  static_assert(!FUSE || (NLM == NL_AFTER && !MAP && !LONG),
                "a fused step pair ends one step and begins the next on one short axis");
  __shared__ float2 lds[G::LDS_ELEMS];
  __shared__ float2 s_tw[N];
  __shared__ float2 s_prop[LONG ? 1 : NF * N];
  __shared__ float2 s_tw2[FUSE ? N : 1];
  __shared__ float2 s_prop2[FUSE ? NF * N : 1];
  // long tau axis: the nt-point twiddles (a and b passes) or the tau
  // propagator (transform pass) of the whole axis
  __shared__ float2 s_long[LONG ? kMaxLongT : 1];

  const int tid = threadIdx.x;
  // RK4 coefficients of the half-step: the same for every thread, read
  // before any store and kept in scalar registers
  float2 co[NF][kNlCoef];
  if constexpr (NLM != NL_NONE) {
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
      for (int c = 0; c < kNlCoef; ++c)
        co[j][c] = wave_uniform(((NLM & NL_BEFORE) != 0 ? args.nl : args.nl2)[j * kNlCoef + c]);
  }
  // this step's twiddles and this block's propagators, staged once
  if constexpr (LONG) {
    // args.tw is the nt-point row exp(-2 pi i m / nt); the line transforms
    // of length N take every (nt / N)-th entry
    const int nt = args.nt;
    const int stride = nt / N;
    for (int i = tid; i < N; i += BLOCK) s_tw[i] = args.tw[i * stride];
    if constexpr (AX == AX_TB) {
      const float2* pr = args.prop + field0 * args.field_stride + args.axis_off;
      for (int i = tid; i < nt; i += BLOCK) {
        float2 pv = pr[i];
        if (args.conj) pv.y = -pv.y;
        s_long[i] = pv;
      }
    } else {
      for (int i = tid; i < nt; i += BLOCK) s_long[i] = args.tw[i];
    }
  } else {
    for (int i = tid; i < N; i += BLOCK) s_tw[i] = args.tw[i];
    for (int i = tid; i < NF * N; i += BLOCK) {
      float2 pv = args.prop[(field0 + i / N) * args.field_stride + args.axis_off + i % N];
      if (args.conj) pv.y = -pv.y;
      s_prop[i] = pv;
    }
    if constexpr (FUSE) {
      for (int i = tid; i < N; i += BLOCK) s_tw2[i] = args.tw2[i];
      for (int i = tid; i < NF * N; i += BLOCK)
        s_prop2[i] = args.prop2[(field0 + i / N) * args.field_stride + args.axis_off + i % N];
    }
  }

  int t, li;
  unsigned base, estride;
  unsigned lidx = 0;     // long tau axis: a (b passes) or k_b (a pass) of the line
  bool valid = true;
  const float2* fin[NF];
  float2* fout[NF];
  if constexpr (AX == AX_X) {
    t = tid % N2;
    li = tid / N2;
    const unsigned line = bx * unsigned(G::LPB) + li;
    if constexpr (!FULL) valid = line < unsigned(args.ny) * unsigned(args.nt);
    base = line * unsigned(args.nx);
    estride = 1;
  } else if constexpr (AX == AX_Y) {
    // lines (x, tau) numbered x-fastest, so that a block's LPB lines are
    // consecutive x (coalesced rows) and only the last block can be partial
    li = tid % G::LPB;
    t = tid / G::LPB;
    const unsigned line = bx * unsigned(G::LPB) + li;
    if constexpr (!FULL) valid = line < unsigned(args.nx) * unsigned(args.nt);
    const unsigned xx = line % unsigned(args.nx);
    const unsigned tt = line / unsigned(args.nx);
    base = xx + unsigned(args.nx) * unsigned(args.ny) * tt;
    estride = args.nx;
  } else if constexpr (LONG) {
    // lines (column, a) of the b transforms or (column, k_b) of the a
    // transforms, column-fastest: a block's lines are consecutive columns
    li = tid % G::LPB;
    t = tid / G::LPB;
    const unsigned plane_xy = unsigned(args.nx) * unsigned(args.ny);
    const unsigned nsub = unsigned(args.nt) / unsigned(N);     // A (b passes) or B (a pass)
    const unsigned line = bx * unsigned(G::LPB) + li;
    if constexpr (!FULL) valid = line < plane_xy * nsub;
    const unsigned col = line % plane_xy;
    // the other index: a (b passes) or k_b (a pass); clamped on padding lines
    lidx = min(line / plane_xy, nsub - 1u);
    if constexpr (AX == AX_TB) {
      base = col + plane_xy * unsigned(N) * lidx;   // elements a at tau = a + A k_b
      estride = plane_xy;
    } else {
      base = col + plane_xy * lidx;                 // elements b at tau = a + A b
      estride = plane_xy * nsub;
    }
  } else {
    li = tid % G::LPB;
    t = tid / G::LPB;
    // tiles of consecutive (x, y) columns; concurrently running blocks are
    // spread over the whole plane so that their strided rows fall into many
    // memory channels rather than one narrow address window
    const unsigned tile = unsigned((unsigned long long)bx * args.tile_mul % args.tiles);
    const unsigned q = tile * unsigned(G::LPB) + li;
    if constexpr (!FULL) valid = q < unsigned(args.nx) * unsigned(args.ny);
    base = q;
    estride = unsigned(args.nx) * unsigned(args.ny);
  }
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    fin[j] = args.f[field0 + j];
    fout[j] = args.fo[field0 + j];
  }
  const unsigned idx0 = base + unsigned(t) * estride;
  const unsigned estep = unsigned(N2) * estride;
  // transverse-map index of slot 0 (x pass: slot e adds N2 e; tau pass: the
  // same column for every slot, so its three factors are read once here)
  unsigned plane = 0, xy0 = 0;
  float2 wt[3];
  if constexpr (MAP) {
    plane = unsigned(args.nx) * unsigned(args.ny);
    xy0 = idx0 % plane;
    if constexpr (AX == AX_T || LONG) {
#pragma unroll
      for (int k = 0; k < 3; ++k) wt[k] = args.map[k * plane + xy0];
    }
  }
  // a line's LDS row (lines of one lane exchange nothing: no row)
  float2* lbuf = (N2 > 1) ? lds + li * G::LSTRIDE : lds;
  const DftConsts K = *args.consts;

  const unsigned field_bytes = unsigned(args.nx) * unsigned(args.ny) * unsigned(args.nt) * 8u;
  const unsigned lane_bytes = idx0 * 8u;
  const unsigned slot_bytes = estep * 8u;
  __amdgpu_buffer_rsrc_t rin[NF], rout[NF];
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    rin[j] = field_rsrc(fin[j], field_bytes);
    rout[j] = field_rsrc(fout[j], field_bytes);
  }
  float2 v[NF][N1];
#pragma unroll
  for (int j = 0; j < NF; ++j) {
#pragma unroll
    for (int e = 0; e < N1; ++e)
      v[j][e] = valid ? load_slot<NT>(rin[j], lane_bytes, unsigned(e) * slot_bytes) : make_float2(0.f, 0.f);
  }
  __syncthreads();  // s_tw, s_prop staged

  if constexpr ((NLM & NL_BEFORE) != 0) {
#pragma unroll
    for (int e = 0; e < N1; ++e) {
      float2 y[NF];
#pragma unroll
      for (int j = 0; j < NF; ++j) y[j] = v[j][e];
      if (e > 0) point_link<NF>(y, v, e - 1);
      if constexpr (MAP) {
        float2 w[3];
        map_factors<AX, N2>(args.map, plane, xy0, e, wt, w);
        rk4_point<NF, true>(y, co, w);
      } else {
        rk4_point<NF>(y, co);
      }
#pragma unroll
      for (int j = 0; j < NF; ++j) v[j][e] = y[j];
    }
  }

#pragma unroll
  for (int j = 0; j < NF; ++j) {
    if constexpr (AX == AX_TAF) {
      // B-point transform, then exp(-2 pi i a k_b / nt) on output k_b
      line_fft<N1, N2, false, WL>(v[j], t, lbuf, s_tw, K);
#pragma unroll
      for (int e = 0; e < N1; ++e)
        v[j][e] = cmul(v[j][e], s_long[(lidx * unsigned(t + N2 * e)) & unsigned(args.nt - 1)]);
    } else if constexpr (AX == AX_TAI) {
      // conjugate twiddle, then the inverse B-point transform
#pragma unroll
      for (int e = 0; e < N1; ++e)
        v[j][e] = cmulc(v[j][e], s_long[(lidx * unsigned(t + N2 * e)) & unsigned(args.nt - 1)]);
      line_fft<N1, N2, true, WL>(v[j], t, lbuf, s_tw, K);
    } else if constexpr (AX == AX_TB) {
      // A-point transform over a gives frequency k = k_b + B k_a in slot k_a
      line_fft<N1, N2, false, WL>(v[j], t, lbuf, s_tw, K);
      const unsigned nb = unsigned(args.nt) / unsigned(N);
#pragma unroll
      for (int e = 0; e < N1; ++e) v[j][e] = cmul(v[j][e], s_long[lidx + nb * unsigned(t + N2 * e)]);
      line_fft<N1, N2, true, WL>(v[j], t, lbuf, s_tw, K);
    } else {
      line_fft<N1, N2, false, WL>(v[j], t, lbuf, s_tw, K);
#pragma unroll
      for (int e = 0; e < N1; ++e) v[j][e] = cmul(v[j][e], s_prop[j * N + t + N2 * e]);
      line_fft<N1, N2, true, WL>(v[j], t, lbuf, s_tw, K);
    }
    if constexpr ((NLM & NL_AFTER) == 0) {
      if (valid) {
#pragma unroll
        for (int e = 0; e < N1; ++e) store_slot<NT>(rout[j], lane_bytes, unsigned(e) * slot_bytes, v[j][e]);
      }
    }
  }

  if constexpr ((NLM & NL_AFTER) != 0) {
    if constexpr (NLM == NL_BOTH) {
#pragma unroll
      for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int c = 0; c < kNlCoef; ++c) co[j][c] = wave_uniform(args.nl2[j * kNlCoef + c]);
    }
    if (args.pre[0] != nullptr && valid) {
#pragma unroll
      for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int e = 0; e < N1; ++e) store_field<NT>(args.pre[j], idx0 + unsigned(e) * estep, v[j][e]);
    }
#pragma unroll
    for (int e = 0; e < N1; ++e) {
      float2 y[NF];
#pragma unroll
      for (int j = 0; j < NF; ++j) y[j] = v[j][e];
      // (after the transforms a schedule barrier between points keeps
      // fewer registers live than the link above)
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (MAP) {
        float2 w[3];
        map_factors<AX, N2>(args.map, plane, xy0, e, wt, w);
        rk4_point<NF, true>(y, co, w);
      } else {
        rk4_point<NF>(y, co);
      }
#pragma unroll
      for (int j = 0; j < NF; ++j) v[j][e] = y[j];
    }
    if constexpr (FUSE) if (next) {
      // the next step's first transform along this axis
      const DftConsts K2 = *args.consts2;
#pragma unroll
      for (int j = 0; j < NF; ++j) {
        line_fft<N1, N2, false, WL>(v[j], t, lbuf, s_tw2, K2);
#pragma unroll
        for (int e = 0; e < N1; ++e) v[j][e] = cmul(v[j][e], s_prop2[j * N + t + N2 * e]);
        line_fft<N1, N2, true, WL>(v[j], t, lbuf, s_tw2, K2);
      }
    }
    if (valid) {
#pragma unroll
      for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int e = 0; e < N1; ++e) store_slot<NT>(rout[j], lane_bytes, unsigned(e) * slot_bytes, v[j][e]);
    }
  }
}

// Threads per block of the wide linear passes (schedule field `wide`): twice
// the lines of a kBlock block, so y and tau rows are read in segments twice
// as long; their LDS allows two blocks per CU.
constexpr int kWideBlock = 2 * kBlock;

// Blocks per CU a pass kernel of N1 values per lane and BLOCK threads is
// compiled for (the second argument of its launch bounds).
template <int N1, int BLOCK>
constexpr int pass_min_blocks() {
  return BLOCK != kBlock ? 2 : (N1 > 24 ? 1 : BRAHMS_MIN_BLOCKS);
}

// Whether the wide linear passes of a split fit the LDS of one CU (160 KB):
// not for 36 values per lane, whose rows of 512 lanes would take 185-223 KB.
// Such axes run their linear passes with kBlock threads whatever the
// schedule's `wide` bit says (the results are the same either way).
template <int N1>
constexpr bool wide_split() {
  return N1 <= 24;
}

// One pass of one problem; BLOCK threads per block (kBlock, or kWideBlock
// for the wide linear passes of the schedule field `wide`).
template <int N1, int N2, int AX, int NF, int NL, bool FULL, int BLOCK = kBlock>
__global__ __launch_bounds__(BLOCK, (pass_min_blocks<N1, BLOCK>())) void axis_pass(PassArgs args) {
  // passes with one field per block take it from blockIdx.z
  constexpr bool per_field = NF == 1;
  axis_pass_body<N1, N2, AX, NF, NL, FULL, BLOCK>(args, blockIdx.x, per_field ? int(blockIdx.z) : 0);
}

// One pass over a group of problems of the same shape (a batch): descs[i]
// describes problem i at this step; passes over all fields take the problem
// from blockIdx.y, passes with one field per block from blockIdx.z / nf.  Problems whose own step count
// is reached (step >= nz) leave at once.
template <int N1, int N2, int AX, int NF, int NL, bool FULL, int BLOCK = kBlock>
__global__ __launch_bounds__(BLOCK, (pass_min_blocks<N1, BLOCK>())) void axis_pass_batched(
    const PassArgs* descs, long long step, int nf) {
  // linear y and long-tau passes take one field per block: problem and field
  // from blockIdx.z
  constexpr bool per_field = NF == 1;
  const unsigned inst = per_field ? blockIdx.z / unsigned(nf) : blockIdx.y;
  const PassArgs& a = descs[inst];
  if (step >= a.nz) return;
  // a fused pass ends the problem's last step without the next transform
  axis_pass_body<N1, N2, AX, NF, NL, FULL, BLOCK>(a, blockIdx.x, per_field ? int(blockIdx.z % unsigned(nf)) : 0,
                                                  step + 1 < a.nz);
}

// ---------------------------------------------------------------------------
// Per-step tables, formed in double precision.
//
// Propagator of field j along one axis for step n (z_n = n dz):
//   P_n(k) = s * U(z_{n+1}, k) * conj(U(z_n, k)),   U(z, k) = fl32(exp(i phi(k) z))
// with phi the imaginary part of that axis's share of the symbol Lambda_j,
// the phase reduced mod 2 pi in double before the sine and cosine, and s the
// 1/N normalisation (times exp(-alpha dz/2) on the tau axis).  Because U is
// rounded at every z_n separately, the phase rounding errors of consecutive
// steps cancel (a telescoping product) instead of accumulating coherently.
//
// The propagator entries themselves, the transform twiddles, the register-DFT
// constants and the RK4 coefficients (see rk4_point; Phi(z) = Phi_n +
// dk_n (z - z_n) is the integrated mismatch) are rounded to float
// stochastically, with a
// counter-based hash of (step, entry) as the random source, so that their
// rounding errors are independent from one z-step to the next; a fixed
// rounding would repeat the same error every step and add up linearly.
//
// Row layout of one step (float2 units): [nf][nx | ny | nt] propagators,
// [nx | ny | nt] twiddles, 8 float2 of DftConsts.
// ---------------------------------------------------------------------------
struct FieldCoef {
  double kappa, diffraction, tan_rho, delay, k2, k3, alpha;
};

struct TableArgs {
  float2* rows;          // [count][row_stride]
  float2* nl;            // [count][2][nf][6]
  const double* phi0;    // Phi_n prefix (profile) or null
  const double* dk;      // dk_n (profile) or null
  long n0;               // first step of the rows (unless n0_dev is set)
  const long long* n0_dev;  // device copies of n0 and merge_last (graph
                            // replays), or null
  long long merge_last;  // steps n < merge_last get the merged second
                         // half-step coefficients; -1: none (constant dk only)
  int count;
  int nx, ny, nt, nf;
  int row_stride;
  double dz, dx, dy, dt, dk_const;
  FieldCoef fc[3];
};

__device__ inline long table_n0(const TableArgs& a) {
  return a.n0_dev != nullptr ? long(a.n0_dev[0]) : a.n0;
}

__device__ inline long long table_merge_last(const TableArgs& a) {
  return a.n0_dev != nullptr ? a.n0_dev[1] : a.merge_last;
}

__host__ __device__ inline int table_row_stride(int nf, int nx, int ny, int nt) {
  return (nf + 1) * (nx + ny + nt) + int(sizeof(DftConsts) / sizeof(float2));
}

__device__ inline double reduce_2pi(double a) {
  const double two_pi = 6.283185307179586476925286766559;
  double r = fmod(a, two_pi);
  return r < 0.0 ? r + two_pi : r;
}

__device__ inline double ang_freq(int m, int n, double d) {
  const int mm = (m >= (n + 1) / 2) ? m - n : m;
  return 6.283185307179586476925286766559 * double(mm) / (double(n) * d);
}

__device__ inline double2 rounded_unit(double theta) {
  double s, c;
  sincos(reduce_2pi(theta), &s, &c);
  return make_double2(double(float(c)), double(float(s)));
}

// 32-bit integer hash (xorshift-multiply finaliser).
__device__ inline unsigned mix32(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__device__ inline unsigned entry_bits(long n, unsigned slot) {
  return mix32(mix32(unsigned(n) * 0x9e3779b1u ^ unsigned(n >> 32)) ^ (slot * 0x85ebca6bu + 0x632be5abu));
}

// Round v to one of its two float neighbours, up with probability equal to
// the distance from the lower one (unbiased), using 24 random bits.
__device__ inline float stochastic_round(double v, unsigned bits) {
  const float f = float(v);
  const double d = double(f);
  if (d == v) return f;
  float lo, hi;
  if (d < v) {
    lo = f;
    hi = nextafterf(f, HUGE_VALF);
  } else {
    hi = f;
    lo = nextafterf(f, -HUGE_VALF);
  }
  const double p = (v - double(lo)) / (double(hi) - double(lo));
  const double u = double(bits >> 8) * (1.0 / 16777216.0);
  return (u < p) ? hi : lo;
}

__device__ __forceinline__ void step_tables_body(const TableArgs& a, long gid) {
  const int per_field = a.nx + a.ny + a.nt;
  const int per_step = (a.nf + 1) * per_field + 1;  // + one thread for DftConsts
  const long nrow = long(a.count) * per_step;
  if (gid < nrow) {
    const int s = int(gid / per_step);
    const int r = int(gid % per_step);
    const long n = table_n0(a) + s;
    float2* row = a.rows + long(s) * a.row_stride;
    if (r == per_step - 1) {
      // register-DFT constants of this step
      const double v[6] = {0.70710678118654752440, 0.92387953251128675613, 0.38268343236508977173,
                           0.86602540378443864676, 0.96592582628906828675, 0.25881904510252076235};
      float* out = reinterpret_cast<float*>(row + (a.nf + 1) * per_field);
      for (int k = 0; k < 6; ++k) out[k] = stochastic_round(v[k], entry_bits(n, 0x40000000u + k));
      out[6] = stochastic_round(0.41421356237309504880, entry_bits(n, 0x40000006u));   // tan(pi/8)
      out[7] = 0.f;
      // cos and sin of 10, 20 and 40 degrees (radices with a factor 9)
      const double w[6] = {0.98480775301220805937, 0.17364817766693034885, 0.93969262078590838405,
                           0.34202014332566873304, 0.76604444311897803520, 0.64278760968653932632};
      for (int k = 0; k < 6; ++k) out[8 + k] = stochastic_round(w[k], entry_bits(n, 0x40000008u + k));
      out[14] = 0.f;
      out[15] = 0.f;
      return;
    }
    int m = r % per_field;
    int nax, axis;
    double d;
    if (m < a.nx) {
      axis = 0; nax = a.nx; d = a.dx;
    } else if (m < a.nx + a.ny) {
      axis = 1; nax = a.ny; d = a.dy; m -= a.nx;
    } else {
      axis = 2; nax = a.nt; d = a.dt; m -= a.nx + a.ny;
    }
    if (r >= a.nf * per_field) {
      // forward twiddle exp(-2 pi i m / nax) of this axis
      double sn, cs;
      sincospi(2.0 * double(m) / double(nax), &sn, &cs);
      const unsigned slot = 2u * unsigned(r);
      row[r] = make_float2(stochastic_round(cs, entry_bits(n, slot)),
                           stochastic_round(-sn, entry_bits(n, slot + 1)));
      return;
    }
    const int j = r / per_field;
    const FieldCoef& f = a.fc[j];
    const double k = ang_freq(m, nax, d);
    double phi, scale;
    if (axis == 0) {
      phi = -f.diffraction * k * k - f.tan_rho * k;
      scale = 1.0 / a.nx;
    } else if (axis == 1) {
      phi = -f.diffraction * k * k;
      scale = 1.0 / a.ny;
    } else {
      phi = -f.delay * k + 0.5 * f.k2 * k * k - (f.k3 / 6.0) * k * k * k;
      scale = exp(-0.5 * f.alpha * a.dz) / a.nt;
    }
    const double2 u1 = rounded_unit(phi * (double(n + 1) * a.dz));
    const double2 u0 = rounded_unit(phi * (double(n) * a.dz));
    const double re = (u1.x * u0.x + u1.y * u0.y) * scale;
    const double im = (u1.y * u0.x - u1.x * u0.y) * scale;
    // stochastic, like the other per-step constants: an entry that is the
    // same at every step (zero frequency, where it is the 1/n scale, which is
    // inexact for n = 96) would otherwise be rounded the same way every step
    // and its error would grow linearly with the number of steps
    const unsigned slot = 2u * unsigned(r);
    row[r] = make_float2(stochastic_round(re, entry_bits(n, slot)),
                         stochastic_round(im, entry_bits(n, slot + 1)));
    return;
  }
  const long g2 = gid - nrow;
  const long nco = long(a.count) * 2 * a.nf;
  if (g2 >= nco) return;
  const int s = int(g2 / (2 * a.nf));
  const int half = int((g2 / a.nf) % 2);
  const int j = int(g2 % a.nf);
  const long n = table_n0(a) + s;
  double phi_n, dkn;
  if (a.dk != nullptr) {
    phi_n = a.phi0[n];
    dkn = a.dk[n];
  } else {
    dkn = a.dk_const;
    phi_n = dkn * (double(n) * a.dz);
  }
  // sigma_j: exp(-i Phi) on the sum-frequency field, exp(+i Phi) on the others
  double sigma;
  if (a.nf == 3) sigma = (j == 0) ? -1.0 : 1.0;
  else sigma = (j == 0) ? 1.0 : -1.0;
  // merged: one step of size dz from z_n + dz/2 (stages at dz/2, dz, 3 dz/2
  // past z_n; only for a constant dk, so Phi stays linear across z_{n+1})
  const bool merged = half == 1 && n < table_merge_last(a);
  const double h = merged ? a.dz : 0.5 * a.dz;
  const double kap = a.fc[j].kappa;
  double2 c[3];  // c_j at z_a, z_a + h/2, z_a + h
  for (int k = 0; k < 3; ++k) {
    const double off = merged ? (0.5 + 0.5 * double(k)) * a.dz                   // z - z_n
                              : (double(half) * 2.0 + double(k)) * 0.25 * a.dz;
    const double ph = reduce_2pi(phi_n + dkn * off);
    double sn, cs;
    sincos(ph, &sn, &cs);
    // i kappa (cos + i sigma sin) = kappa (-sigma sin + i cos)
    c[k] = make_double2(-kap * sigma * sn, kap * cs);
  }
  const double w[6] = {h / 2, h / 2, h, h / 6, h / 3, h / 6};
  const int which[6] = {0, 1, 1, 0, 1, 2};
  float2* out = a.nl + g2 * kNlCoef;
  for (int k = 0; k < 6; ++k) {
    const unsigned slot = 0x50000000u + unsigned((half * a.nf + j) * kNlCoef + k) * 2u;
    out[k] = make_float2(stochastic_round(w[k] * c[which[k]].x, entry_bits(n, slot)),
                         stochastic_round(w[k] * c[which[k]].y, entry_bits(n, slot + 1)));
  }
}

static __global__ void step_tables(TableArgs a) {
  step_tables_body(a, long(blockIdx.x) * blockDim.x + threadIdx.x);
}

// Tables of several problems: problem blockIdx.y uses targs[blockIdx.y].
static __global__ void step_tables_batched(const TableArgs* targs) {
  step_tables_body(targs[blockIdx.y], long(blockIdx.x) * blockDim.x + threadIdx.x);
}

// Set a flag when any field value is not finite (the step-size hazard of
// Sec. 3.2: a too-large dz makes the nonlinear increment blow up).
// exp(i m(x, y) Psi(z_n + o dz)) for the five distinct stage offsets
// o = 0, 1/4, 1/2, 3/4, 1 of steps n0 .. n0 + count - 1 (the first half-step
// uses offsets 0..2, the second 2..4), from the FP64 map and Psi reduced
// mod 2 pi in FP64.  Psi(z_n + o dz) = Psi_n + s_n o dz with Psi_n = psi0[n]
// and s_n = scale[n], or n dz and 1 without a scale profile.
struct MapArgs {
  const double* map;    // [ny][nx]
  const double* psi0;   // Psi_n prefix (NULL: no scale profile)
  const double* scale;  // s_n (NULL: no scale profile)
  float2* out;          // [count][5][ny][nx]
  unsigned plane;
  long long n0;              // first step (unless n0_dev is set)
  const long long* n0_dev;   // device copy of n0 (graph replays), or null
  double dz;
};

static __global__ void map_phase_table(MapArgs a) {
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.plane) return;
  const long long n = (a.n0_dev != nullptr ? *a.n0_dev : a.n0) + blockIdx.y;
  const double psi_n = a.psi0 != nullptr ? a.psi0[n] : double(n) * a.dz;
  const double s_n = a.scale != nullptr ? a.scale[n] : 1.0;
  const double m = a.map[i];
  float2* out = a.out + size_t(blockIdx.y) * 5 * a.plane;
  for (int k = 0; k < 5; ++k) {
    double sn, cs;
    sincos(reduce_2pi(m * (psi_n + s_n * (0.25 * k) * a.dz)), &sn, &cs);
    out[k * a.plane + i] = make_float2(float(cs), float(sn));
  }
}

// First step index of a chunk and the last step of the run (merged halves),
// for tables read by a replayed graph.
static __global__ void set_step_index(long long* dst, long long n0, long long merge_last) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    dst[0] = n0;
    dst[1] = merge_last;
  }
}

static __global__ void finite_check(const float2* f, long n, int* flag) {
  long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  const long stride = long(gridDim.x) * blockDim.x;
  int bad = 0;
  for (; i < n; i += stride) {
    const float2 v = f[i];
    bad |= !(isfinite(v.x) && isfinite(v.y));
  }
  if (bad) atomicOr(flag, 1);
}

}  // namespace brahms
