// Register-resident DFT building blocks (gfx950).
//
// dft<N, INV>(v) transforms v[0..N-1] in place, natural order in and out:
//   forward  V[k] = sum_n v[n] exp(-2 pi i n k / N)
//   inverse  V[k] = sum_n v[n] exp(+2 pi i n k / N)   (unnormalised)
// N is a compile-time divisor of 144 (a product of 2s and 3s).  Every loop
// is fully unrolled and every index is a compile-time constant, so the arrays
// live in registers and the choice of each twiddle operation folds at compile
// time; the irrational constants are uniform run-time values (DftConsts).
// unit_root evaluates roots of unity in double precision (exact quadrant
// symmetry plus a Taylor series on at most a half quadrant) for the
// host-side tables.
#pragma once

#include <hip/hip_runtime.h>

namespace brahms {

constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 16; ++k) {
    term *= -x2 / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}

constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 16; ++k) {
    term *= -x2 / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}

// cos and sin of 2 pi m / n for integers m, n > 0.
constexpr void unit_root(long m, long n, double& c, double& s) {
  long r = ((m % n) + n) % n;
  long q = (4 * r) / n;        // quadrant
  long num = 4 * r - q * n;    // remaining angle = (pi/2) num / n, num in [0, n)
  double cd = 0.0, sd = 0.0;
  if (2 * num <= n) {
    double d = (kPi / 2.0) * double(num) / double(n);
    cd = taylor_cos(d);
    sd = taylor_sin(d);
  } else {
    double d = (kPi / 2.0) * double(n - num) / double(n);
    cd = taylor_sin(d);
    sd = taylor_cos(d);
  }
  switch (q) {
    case 0: c = cd; s = sd; break;
    case 1: c = -sd; s = cd; break;
    case 2: c = -cd; s = -sd; break;
    default: c = sd; s = -cd; break;
  }
}

__host__ __device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__host__ __device__ inline float2 rot_quarter(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// The irrational constants the register DFTs need.  The radices 2, 3, 4, 6,
// 8, 9, 12, 16, 18, 24 and 36 all divide 144, so every root is a multiple of
// 2 pi / 144 and reduces by exact quadrant symmetry to a first-quadrant
// value; the ones that occur are the multiples of 7.5 degrees (the radices
// dividing 48) and of 10 degrees (those with a factor 9).  They are run-time
// values supplied per z-step: rounding them afresh at every step
// (stochastically, from a double-precision value) keeps their rounding errors
// independent from step to step, so the errors of repeated transform round
// trips grow like sqrt(steps) instead of linearly.
struct DftConsts {
  float h;         // cos(pi/4) = sin(pi/4)
  float c8, s8;    // cos(pi/8), sin(pi/8)
  float r3;        // cos(pi/6) = sin(pi/3)
  float c12, s12;  // cos(pi/12), sin(pi/12)
  float t8;        // tan(pi/8) (the folded twiddles of the 16-point DFT)
  float pad;
  float c36, s36;  // cos(pi/18), sin(pi/18)   (10 degrees)
  float c18, s18;  // cos(pi/9), sin(pi/9)     (20 degrees)
  float c9, s9;    // cos(2pi/9), sin(2pi/9)   (40 degrees)
  float pad2[2];
};

// a * exp(-+ 2 pi i m / N) with m a compile-time constant after unrolling
// (every branch below folds away); quarter turns cost no multiplies.
template <int N, bool INV>
__host__ __device__ inline float2 twiddle_const(float2 a, int m, const DftConsts& K) {
  static_assert(144 % N == 0, "register DFT radices must divide 144");
  m %= N;
  if (m == 0) return a;
  const int r = m * (144 / N);  // angle in units of 2 pi / 144 (2.5 degrees)
  const int q = r / 36;         // quarter turns
  const int rem = r % 36;       // remaining angle
  float2 b = a;
  if (rem != 0) {
    float c = 0.f, s = 0.f;
    if (rem == 18) {
      // exp(-+i pi/4) = h (1 -+ i)
      b = INV ? make_float2(K.h * (a.x - a.y), K.h * (a.x + a.y))
              : make_float2(K.h * (a.x + a.y), K.h * (a.y - a.x));
    } else if (rem % 4 == 0 && rem % 12 != 0) {
      // multiples of 10 degrees (radices with a factor 9), the product's
      // multiply-adds written out so that every kernel rounds them alike
      switch (rem) {
        case 4: c = K.c36; s = K.s36; break;
        case 8: c = K.c18; s = K.s18; break;
        case 16: c = K.c9; s = K.s9; break;
        case 20: c = K.s9; s = K.c9; break;
        case 28: c = K.s18; s = K.c18; break;
        default: c = K.s36; s = K.c36; break;  // rem == 32
      }
      if (!INV) s = -s;
      b = make_float2(fmaf(a.x, c, -(a.y * s)), fmaf(a.x, s, a.y * c));
    } else {
      switch (rem) {
        case 6: c = K.c12; s = K.s12; break;
        case 9: c = K.c8; s = K.s8; break;
        case 12: c = K.r3; s = 0.5f; break;
        case 24: c = 0.5f; s = K.r3; break;
        case 27: c = K.s8; s = K.c8; break;
        default: c = K.s12; s = K.c12; break;  // rem == 30
      }
      if (!INV) s = -s;
      b = make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
    }
  }
  if (q == 1) return rot_quarter<INV>(b);
  if (q == 2) return make_float2(-b.x, -b.y);
  if (q == 3) return rot_quarter<!INV>(b);
  return b;
}

template <int N, bool INV>
struct Dft {
  static constexpr int P = (N % 4 == 0 && N > 4) ? 4 : ((N % 2 == 0) ? 2 : 3);
  static constexpr int Q = N / P;
  __host__ __device__ static inline void run(float2* v, const DftConsts& K) {
    // n = Q n1 + n2, k = k1 + P k2
    float2 y[N];
#pragma unroll
    for (int n2 = 0; n2 < Q; ++n2) {
      float2 u[P];
#pragma unroll
      for (int n1 = 0; n1 < P; ++n1) u[n1] = v[Q * n1 + n2];
      Dft<P, INV>::run(u, K);
#pragma unroll
      for (int k1 = 0; k1 < P; ++k1) y[n2 * P + k1] = twiddle_const<N, INV>(u[k1], n2 * k1, K);
    }
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) {
      float2 w[Q];
#pragma unroll
      for (int n2 = 0; n2 < Q; ++n2) w[n2] = y[n2 * P + k1];
      Dft<Q, INV>::run(w, K);
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) v[k1 + P * k2] = w[k2];
    }
  }
};

template <bool INV>
struct Dft<1, INV> {
  __host__ __device__ static inline void run(float2*, const DftConsts&) {}
};

template <bool INV>
struct Dft<2, INV> {
  __host__ __device__ static inline void run(float2* v, const DftConsts&) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<3, INV> {
  __host__ __device__ static inline void run(float2* v, const DftConsts& K) {
    const float h = K.r3;  // sin(2 pi/3)
    float2 a = v[0];
    float2 t1 = cadd(v[1], v[2]);
    float2 t2 = csub(v[1], v[2]);
    float2 m = make_float2(a.x - 0.5f * t1.x, a.y - 0.5f * t1.y);
    // forward: X1 = m - i h t2, X2 = m + i h t2
    float2 r = make_float2(-h * t2.y, h * t2.x);  // i h t2
    v[0] = cadd(a, t1);
    if (INV) {
      v[1] = cadd(m, r);
      v[2] = csub(m, r);
    } else {
      v[1] = csub(m, r);
      v[2] = cadd(m, r);
    }
  }
};

template <bool INV>
struct Dft<4, INV> {
  __host__ __device__ static inline void run(float2* v, const DftConsts&) {
    float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    float2 s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
    float2 r = rot_quarter<INV>(d13);  // -i d13 forward, +i d13 inverse
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, r);
    v[3] = csub(d02, r);
  }
};

// Helpers of the 16-point DFT below: u times the unit-free factor of a
// twiddle, (1 -+ i t), (t -+ i), (1 -+ i) or (-1 -+ i) (forward / inverse).
template <bool INV>
__host__ __device__ inline float2 mul_one_it(float2 u, float t) {
  return INV ? make_float2(fmaf(-t, u.y, u.x), fmaf(t, u.x, u.y))
             : make_float2(fmaf(t, u.y, u.x), fmaf(-t, u.x, u.y));
}
template <bool INV>
__host__ __device__ inline float2 mul_t_i(float2 u, float t) {
  return INV ? make_float2(fmaf(t, u.x, -u.y), fmaf(t, u.y, u.x))
             : make_float2(fmaf(t, u.x, u.y), fmaf(t, u.y, -u.x));
}
template <bool INV>
__host__ __device__ inline float2 mul_one_i(float2 u) {
  return INV ? make_float2(u.x - u.y, u.y + u.x) : make_float2(u.x + u.y, u.y - u.x);
}
template <bool INV>
__host__ __device__ inline float2 mul_mone_i(float2 u) {
  return INV ? make_float2(-u.x - u.y, u.x - u.y) : make_float2(u.y - u.x, -u.y - u.x);
}

// Radix-4 butterfly of the inputs a0, a2 = s b2, a1 = r b1 and a3 = r b3
// (s, r real), the scalings taken into fused multiply-adds; x[k] =
// sum_n a_n exp(-+ 2 pi i n k / 4).
template <bool INV>
__host__ __device__ inline void radix4_scaled(float2 a0, float s, float2 b2, float r, float2 b1, float2 b3,
                                              float2* x) {
  const float2 s02 = make_float2(fmaf(s, b2.x, a0.x), fmaf(s, b2.y, a0.y));
  const float2 d02 = make_float2(fmaf(-s, b2.x, a0.x), fmaf(-s, b2.y, a0.y));
  const float2 e = cadd(b1, b3);
  const float2 f = rot_quarter<INV>(csub(b1, b3));
  x[0] = make_float2(fmaf(r, e.x, s02.x), fmaf(r, e.y, s02.y));
  x[2] = make_float2(fmaf(-r, e.x, s02.x), fmaf(-r, e.y, s02.y));
  x[1] = make_float2(fmaf(r, f.x, d02.x), fmaf(r, f.y, d02.y));
  x[3] = make_float2(fmaf(-r, f.x, d02.x), fmaf(-r, f.y, d02.y));
}

// N = 16 as 4 x 4 (n = 4 n1 + n2, k = k1 + 4 k2).  The twiddles
// exp(-+ 2 pi i n2 k1 / 16) between the two layers are c (1 -+ i t),
// c (t -+ i), h (1 -+ i), h (-1 -+ i), -c (1 -+ i t) or a quarter turn, with
// c = cos(pi/8), t = tan(pi/8), h = cos(pi/4).  The unit-free factor costs
// two operations, and the real factor is shared by the pair of inputs it
// meets in a second-layer butterfly, where it goes into that butterfly's
// fused multiply-adds (the factorisation of Linzer and Feig for
// multiply-add machines): 144 operations instead of the 160 of the generic
// split with full twiddle products.
template <bool INV>
struct Dft<16, INV> {
  __host__ __device__ static inline void run(float2* v, const DftConsts& K) {
    float2 u[4][4];   // [n2][k1]
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      float2 w[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
      Dft<4, INV>::run(w, K);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) u[n2][k1] = w[k1];
    }
    const float c = K.c8, t = K.t8, h = K.h;
    float2 x[4];
    // k1 = 0: no twiddles
    float2 col[4] = {u[0][0], u[1][0], u[2][0], u[3][0]};
    Dft<4, INV>::run(col, K);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[4 * k2] = col[k2];
    // k1 = 1: twiddles 1, c (1 -+ i t), h (1 -+ i), c (t -+ i)
    radix4_scaled<INV>(u[0][1], h, mul_one_i<INV>(u[2][1]), c, mul_one_it<INV>(u[1][1], t),
                       mul_t_i<INV>(u[3][1], t), x);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[1 + 4 * k2] = x[k2];
    // k1 = 2: twiddles 1, h (1 -+ i), -+i, h (-1 -+ i)
    radix4_scaled<INV>(u[0][2], 1.0f, rot_quarter<INV>(u[2][2]), h, mul_one_i<INV>(u[1][2]),
                       mul_mone_i<INV>(u[3][2]), x);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[2 + 4 * k2] = x[k2];
    // k1 = 3: twiddles 1, c (t -+ i), h (-1 -+ i), -c (1 -+ i t)
    const float2 m = mul_one_it<INV>(u[3][3], t);
    radix4_scaled<INV>(u[0][3], h, mul_mone_i<INV>(u[2][3]), c, mul_t_i<INV>(u[1][3], t),
                       make_float2(-m.x, -m.y), x);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[3 + 4 * k2] = x[k2];
  }
};

template <int N, bool INV>
__host__ __device__ inline void dft(float2* v, const DftConsts& K) { Dft<N, INV>::run(v, K); }

}  // namespace brahms
