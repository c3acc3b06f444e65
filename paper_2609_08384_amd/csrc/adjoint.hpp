// Adjoint (reverse-mode) kernels of the chi(2) split-step z-loop (gfx950).
//
// Cotangents follow the convention g = dJ/dRe(A) + i dJ/dIm(A) for a real
// loss J, so that dJ = sum Re(conj(g) dA).  For a pointwise map
// A' = f(A, conj A) with dA' = M dA + B conj(dA) the cotangent of the input
// is g = M^H g' + B^T conj(g') (the transpose of the map seen as a real-linear
// map on (Re A, Im A)).
//
// * Linear step (Sec. 3.1): exp(L dz) = F^-1 diag(P) F is complex-linear, its
//   adjoint is F^-1 diag(conj P) F: the same axis passes with conjugated
//   propagators.
// * RK4 half-step (Sec. 3.1, coefficients as in rk4_point): reverse sweep over
//   the four stages, with the stage values recomputed in registers from the
//   half-step's input.  Every coefficient is w c_j(z) with
//   c_j = i kappa_j exp(i sigma_j Phi(z)), so d/dPhi of a term w c q is
//   i sigma_j w c q; the per-stage sums of Re(conj(g_term) i sigma_j term) over
//   the grid are dJ/dPhi at the stage positions z_a, z_a + h/2, z_a + h.
#pragma once

#include "kernels.hpp"

namespace brahms {

__device__ inline float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// g_y of the products Q (see chi2_products) for cotangent gq of Q.
template <int NF>
__device__ inline void chi2_products_vjp(const float2* y, const float2* gq, float2* gy) {
  if constexpr (NF == 3) {
    // Q_p = s i, Q_s = p conj(i), Q_i = p conj(s)
    gy[0] = cadd(cmul(y[2], gq[1]), cmul(y[1], gq[2]));
    gy[1] = cadd(cmulc(gq[0], y[2]), cmulc(y[0], gq[2]));
    gy[2] = cadd(cmulc(gq[0], y[1]), cmulc(y[0], gq[1]));
  } else {
    // Q_F = S conj(F), Q_S = F F
    const float2 t = cmulc(gq[1], y[0]);  // gS conj(F)
    gy[0] = cadd(cmulc(y[1], gq[0]), make_float2(2.f * t.x, 2.f * t.y));
    gy[1] = cmul(y[0], gq[0]);
  }
}

// sum_j sigma_j Re(conj(g_j) i w_j) with w_j = c_j q_j
template <int NF>
__device__ inline float phase_term(const float2* g, const float2 (*co)[kNlCoef], int k,
                                   const float2* q, const float* sigma) {
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    const float2 w = cmul(co[j][k], q[j]);
    // Re(conj(g) i w) = g.x * (-w.y) + g.y * w.x
    s += sigma[j] * (g[j].y * w.x - g[j].x * w.y);
  }
  return s;
}

// Reverse sweep of one RK4 half-step at one grid point: y is the half-step's
// input, g holds the cotangent of its output on entry and of its input on
// exit; dphi[0..2] accumulate dJ/dPhi at z_a, z_a + h/2, z_a + h.
template <int NF>
__device__ inline void rk4_vjp_point(const float2* y, float2* g, const float2 (*co)[kNlCoef],
                                     const float* sigma, double* dphi) {
  float2 q1[NF], q2[NF], q3[NF], q4[NF], ys1[NF], ys2[NF], ys3[NF];
  chi2_products<NF>(y, q1);
#pragma unroll
  for (int j = 0; j < NF; ++j) ys1[j] = cfma(y[j], co[j][0], q1[j]);
  chi2_products<NF>(ys1, q2);
#pragma unroll
  for (int j = 0; j < NF; ++j) ys2[j] = cfma(y[j], co[j][1], q2[j]);
  chi2_products<NF>(ys2, q3);
#pragma unroll
  for (int j = 0; j < NF; ++j) ys3[j] = cfma(y[j], co[j][2], q3[j]);
  chi2_products<NF>(ys3, q4);

  float2 gout[NF], gq[NF], gys[NF], gy[NF];
#pragma unroll
  for (int j = 0; j < NF; ++j) gout[j] = g[j];
  // y' = y + b1 q1 + b2 q2 + b2 q3 + b4 q4, ys_k = y + a_k q_k
  float pa = phase_term<NF>(gout, co, 3, q1, sigma);
  float pm = phase_term<NF>(gout, co, 4, q2, sigma) + phase_term<NF>(gout, co, 4, q3, sigma);
  const float pe = phase_term<NF>(gout, co, 5, q4, sigma);
#pragma unroll
  for (int j = 0; j < NF; ++j) gq[j] = cmulc(gout[j], co[j][5]);        // conj(b4) g'
  chi2_products_vjp<NF>(ys3, gq, gys);                                   // g of ys3
  pm += phase_term<NF>(gys, co, 2, q3, sigma);
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    gy[j] = cadd(gout[j], gys[j]);
    gq[j] = cadd(cmulc(gys[j], co[j][2]), cmulc(gout[j], co[j][4]));  // conj(a3) g_ys3 + conj(b2) g'
  }
  chi2_products_vjp<NF>(ys2, gq, gys);                                   // g of ys2
  pm += phase_term<NF>(gys, co, 1, q2, sigma);
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    gy[j] = cadd(gy[j], gys[j]);
    gq[j] = cadd(cmulc(gys[j], co[j][1]), cmulc(gout[j], co[j][4]));  // conj(a2) g_ys2 + conj(b2) g'
  }
  chi2_products_vjp<NF>(ys1, gq, gys);                                   // g of ys1
  pa += phase_term<NF>(gys, co, 0, q1, sigma);
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    gy[j] = cadd(gy[j], gys[j]);
    gq[j] = cadd(cmulc(gys[j], co[j][0]), cmulc(gout[j], co[j][3]));  // conj(a1) g_ys1 + conj(b1) g'
  }
  chi2_products_vjp<NF>(y, gq, gys);
#pragma unroll
  for (int j = 0; j < NF; ++j) g[j] = cadd(gy[j], gys[j]);
  dphi[0] += double(pa);
  dphi[1] += double(pm);
  dphi[2] += double(pe);
}

// ---------------------------------------------------------------------------
// Adjoint axis pass.  AT selects where the RK4 reverse sweep goes:
//   VJP_FIRST: the pass undoes the last pass of a forward step (whose RK4
//              half-step came after its transforms): reverse RK4 with the
//              saved half-step input, then FFT . conj(P) . IFFT;
//   VJP_LAST:  the pass undoes the first pass of a forward step: FFT .
//              conj(P) . IFFT, then reverse RK4 with the step's input.
// g is updated in place; the block's three dJ/dPhi partial sums (fixed-order
// tree reduction in double) go to dphi_out[block].
// ---------------------------------------------------------------------------
enum VjpWhere { VJP_FIRST = 1, VJP_LAST = 2 };

struct AdjArgs {
  float2* g[3];             // cotangent fields, in place
  const float2* y[3];       // saved input of the RK4 half-step
  const float2* tw;
  const float2* prop;
  const float2* nl;
  const DftConsts* consts;
  double* dphi_out;         // [gridDim.x][3]
  int nx, ny, nt;
  int axis_off, field_stride;
  unsigned tile_mul;
  float sigma[3];
};

template <int N1, int N2, int AX, int NF, int AT, bool FULL>
__global__ __launch_bounds__(kBlock) void adjoint_pass(AdjArgs args) {
  using G = LineGeom<N1, N2>;
  constexpr int N = G::N;
  __shared__ float2 lds[G::LDS_ELEMS];
  __shared__ float2 s_tw[N];
  __shared__ float2 s_prop[NF * N];
  __shared__ double s_red[kBlock];

  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += kBlock) s_tw[i] = args.tw[i];
  for (int i = tid; i < NF * N; i += kBlock)
    s_prop[i] = args.prop[(i / N) * args.field_stride + args.axis_off + i % N];

  int t, li;
  unsigned base, estride;
  bool valid = true;
  if constexpr (AX == AX_X) {
    t = tid % N2;
    li = tid / N2;
    const unsigned line = blockIdx.x * unsigned(G::LPB) + li;
    if constexpr (!FULL) valid = line < unsigned(args.ny) * unsigned(args.nt);
    base = line * unsigned(args.nx);
    estride = 1;
  } else {
    static_assert(AX == AX_T, "RK4 reverse sweeps live in the x or tau pass");
    li = tid % G::LPB;
    t = tid / G::LPB;
    const unsigned tile = unsigned((unsigned long long)blockIdx.x * args.tile_mul % gridDim.x);
    const unsigned q = tile * unsigned(G::LPB) + li;
    if constexpr (!FULL) valid = q < unsigned(args.nx) * unsigned(args.ny);
    base = q;
    estride = unsigned(args.nx) * unsigned(args.ny);
  }
  const unsigned idx0 = base + unsigned(t) * estride;
  const unsigned estep = unsigned(N2) * estride;
  // x lines: a line's N2 lanes are consecutive threads, within one wavefront
  constexpr bool WL = AX == AX_X && N2 <= 64 && 64 % N2 == 0;
  // a line's LDS row (lines of one lane exchange nothing: no row)
  float2* lbuf = (N2 > 1) ? lds + li * G::LSTRIDE : lds;
  const DftConsts K = *args.consts;
  // fields through buffer resources, as in the forward passes
  const unsigned field_bytes = unsigned(args.nx) * unsigned(args.ny) * unsigned(args.nt) * 8u;
  const unsigned lane_bytes = idx0 * 8u;
  const unsigned slot_bytes = estep * 8u;
  __amdgpu_buffer_rsrc_t rg[NF], ry[NF];
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    rg[j] = field_rsrc(args.g[j], field_bytes);
    ry[j] = field_rsrc(args.y[j], field_bytes);
  }
  // RK4 coefficients: the same for every thread, in scalar registers
  float2 co[NF][kNlCoef];
#pragma unroll
  for (int j = 0; j < NF; ++j)
#pragma unroll
    for (int c = 0; c < kNlCoef; ++c) co[j][c] = wave_uniform(args.nl[j * kNlCoef + c]);
  float sigma[NF];
#pragma unroll
  for (int j = 0; j < NF; ++j) sigma[j] = args.sigma[j];
  double dphi[3] = {0.0, 0.0, 0.0};

  float2 v[NF][N1];
#pragma unroll
  for (int j = 0; j < NF; ++j)
#pragma unroll
    for (int e = 0; e < N1; ++e)
      v[j][e] = valid ? load_slot<false>(rg[j], lane_bytes, unsigned(e) * slot_bytes) : make_float2(0.f, 0.f);
  __syncthreads();  // s_tw, s_prop staged

  auto reverse_rk4 = [&]() {
#pragma unroll
    for (int e = 0; e < N1; ++e) {
      float2 yy[NF], gg[NF];
#pragma unroll
      for (int j = 0; j < NF; ++j) {
        yy[j] = valid ? load_slot<false>(ry[j], lane_bytes, unsigned(e) * slot_bytes) : make_float2(0.f, 0.f);
        gg[j] = v[j][e];
      }
      // One point at a time: tie this point's inputs to the phase sums of the
      // previous points (an empty asm, no instructions), so the compiler
      // cannot interleave all points and run out of registers.
#pragma unroll
      for (int j = 0; j < NF; ++j)
        asm volatile("" : "+v"(yy[j].x), "+v"(yy[j].y), "+v"(gg[j].x), "+v"(gg[j].y), "+v"(dphi[0]),
                          "+v"(dphi[1]), "+v"(dphi[2]));
      rk4_vjp_point<NF>(yy, gg, co, sigma, dphi);
#pragma unroll
      for (int j = 0; j < NF; ++j) v[j][e] = gg[j];
    }
  };

  if constexpr (AT == VJP_FIRST) reverse_rk4();
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    line_fft<N1, N2, false, WL>(v[j], t, lbuf, s_tw, K);
#pragma unroll
    for (int e = 0; e < N1; ++e) v[j][e] = cmulc(v[j][e], s_prop[j * N + t + N2 * e]);
    line_fft<N1, N2, true, WL>(v[j], t, lbuf, s_tw, K);
  }
  if constexpr (AT == VJP_LAST) reverse_rk4();
  if (valid) {
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
      for (int e = 0; e < N1; ++e) store_slot<false>(rg[j], lane_bytes, unsigned(e) * slot_bytes, v[j][e]);
  }

  // block reduction of the three phase derivatives, fixed order
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    __syncthreads();
    s_red[tid] = dphi[k];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if (tid < w) s_red[tid] += s_red[tid + w];
      __syncthreads();
    }
    if (tid == 0) args.dphi_out[blockIdx.x * 3 + k] = s_red[0];
  }
}

// Sum the per-block phase derivatives of a segment's adjoint passes (fixed
// order).  Block (i, w) handles step i of the segment and pass w (0: the
// reverse first half-step, 1: the reverse second half-step), whose launch had
// nblocks[w] blocks and wrote parts[((i * 2 + w) * stride + b) * 3 + k];
// out[6 i + 3 w + k] receives the sum over b (block size 256).
static __global__ void reduce_dphi_segment(const double* parts, int nblocks0, int nblocks1,
                                           int stride, double* out) {
  __shared__ double s[256];
  const int i = blockIdx.x, w = blockIdx.y;
  const int nb = w == 0 ? nblocks0 : nblocks1;
  const double* src = parts + (size_t(i) * 2 + w) * size_t(stride) * 3;
  for (int k = 0; k < 3; ++k) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += src[b * 3 + k];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
      if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[6 * i + 3 * w + k] = s[0];
    __syncthreads();
  }
}

// dst = src over n complex values (checkpoint copies)
static __global__ void copy_field(float2* dst, const float2* src, long n) {
  long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  const long stride = long(gridDim.x) * blockDim.x;
  for (; i < n; i += stride) dst[i] = src[i];
}

static __global__ void zero_doubles(double* p, long n) {
  long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  const long stride = long(gridDim.x) * blockDim.x;
  for (; i < n; i += stride) p[i] = 0.0;
}

}  // namespace brahms
