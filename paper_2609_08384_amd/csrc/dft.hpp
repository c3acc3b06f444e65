// Register-resident DFT building blocks (gfx950).
//
// dft<N, INV>(v) transforms v[0..N-1] in place, natural order in and out:
//   forward  V[k] = sum_n v[n] exp(-2 pi i n k / N)
//   inverse  V[k] = sum_n v[n] exp(+2 pi i n k / N)   (unnormalised)
// N is a compile-time product of 2s and 3s.  Every loop is fully unrolled and
// every index is a compile-time constant, so the arrays live in registers and
// the twiddle constants fold into literals.  The roots of unity are evaluated
// at compile time in double precision (exact quadrant symmetry plus a Taylor
// series on at most a half quadrant) and rounded once to float.
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

template <int N>
struct RootTable {
  float c[N];
  float s[N];
  constexpr RootTable() : c(), s() {
    for (int m = 0; m < N; ++m) {
      double cc = 0.0, ss = 0.0;
      unit_root(m, N, cc, ss);
      c[m] = float(cc);
      s[m] = float(ss);
    }
  }
};

template <int N>
struct Roots {
  static constexpr RootTable<N> table{};
};

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

// a * exp(-+ 2 pi i m / N) with m a compile-time constant after unrolling;
// trivial rotations cost no multiplies.
template <int N, bool INV>
__host__ __device__ inline float2 twiddle_const(float2 a, int m) {
  m %= N;
  if (m == 0) return a;
  if ((4 * m) % N == 0) {
    int q = (4 * m) / N;  // exp(-i q pi/2)
    if (q == 2) return make_float2(-a.x, -a.y);
    if (q == 1) return rot_quarter<INV>(a);
    return rot_quarter<!INV>(a);
  }
  if ((8 * m) % N == 0) {
    // odd multiple of pi/4: exp(-+i o pi/4) = (+-1 +- i) / sqrt(2)
    const float h = 0.70710678118654752440f;
    int o = (8 * m) / N;  // 1, 3, 5, 7
    float c = (o == 1 || o == 7) ? h : -h;
    float s = (o == 1 || o == 3) ? h : -h;  // sin(o pi/4)
    if (!INV) s = -s;
    // (a.x + i a.y)(c + i s) with |c| = |s| = h
    float p = a.x * c, q = a.y * s, r = a.x * s, u = a.y * c;
    return make_float2(p - q, r + u);
  }
  const float c = Roots<N>::table.c[m];
  const float s = INV ? Roots<N>::table.s[m] : -Roots<N>::table.s[m];
  return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
}

template <int N, bool INV>
struct Dft {
  static constexpr int P = (N % 4 == 0 && N > 4) ? 4 : ((N % 2 == 0) ? 2 : 3);
  static constexpr int Q = N / P;
  __host__ __device__ static inline void run(float2* v) {
    // n = Q n1 + n2, k = k1 + P k2
    float2 y[N];
#pragma unroll
    for (int n2 = 0; n2 < Q; ++n2) {
      float2 u[P];
#pragma unroll
      for (int n1 = 0; n1 < P; ++n1) u[n1] = v[Q * n1 + n2];
      Dft<P, INV>::run(u);
#pragma unroll
      for (int k1 = 0; k1 < P; ++k1) y[n2 * P + k1] = twiddle_const<N, INV>(u[k1], n2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) {
      float2 w[Q];
#pragma unroll
      for (int n2 = 0; n2 < Q; ++n2) w[n2] = y[n2 * P + k1];
      Dft<Q, INV>::run(w);
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) v[k1 + P * k2] = w[k2];
    }
  }
};

template <bool INV>
struct Dft<1, INV> {
  __host__ __device__ static inline void run(float2*) {}
};

template <bool INV>
struct Dft<2, INV> {
  __host__ __device__ static inline void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<3, INV> {
  __host__ __device__ static inline void run(float2* v) {
    const float h = 0.86602540378443864676f;  // sin(2 pi/3)
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
  __host__ __device__ static inline void run(float2* v) {
    float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    float2 s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
    float2 r = rot_quarter<INV>(d13);  // -i d13 forward, +i d13 inverse
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, r);
    v[3] = csub(d02, r);
  }
};

template <int N, bool INV>
__host__ __device__ inline void dft(float2* v) { Dft<N, INV>::run(v); }

}  // namespace brahms
