// Register-resident mixed-radix FFT building blocks for gfx950.
//
// One thread owns one length-N line in registers: the Stockham autosort
// recursion (radices 2, 3, 4, 5, 8) is fully unrolled at compile time, so every
// index and every twiddle factor is a compile-time constant and the line never
// leaves the VGPR file.  The Poisson solves of the exchange operator apply
// these lines along the three grid axes (Section 2, the O(N_g log N_g) cost per
// pair charge).
//
// Sign convention: SIGN = -1 computes X[k] = sum_n x[n] exp(-2 pi i n k / N)
// (forward, unnormalised); SIGN = +1 the unnormalised inverse.
#pragma once

#include <hip/hip_runtime.h>

namespace ace {

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// conj(a) * b
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by s*i (s = +1 or -1)
template <int S, typename T>
__device__ __forceinline__ cx<T> mul_si(cx<T> a) {
  return S > 0 ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
}

// ---------------------------------------------------------------------------
// Compile-time twiddles exp(2 pi i t / N).  The angle is reduced exactly in
// integer arithmetic to |r| <= pi/4 around a multiple of pi/2, then a Taylor
// series (terms far below double rounding) evaluates cos and sin.
struct cs_pair {
  double c, s;
};

constexpr double kPi = 3.14159265358979323846;

constexpr double ce_sin_small(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr double ce_cos_small(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
constexpr cs_pair ce_unit_root(long t, long N) {
  t %= N;
  if (t < 0) t += N;
  // quadrant k = round(4 t / N); remainder r = (pi / (2N)) * (4t - kN), |r| <= pi/4
  long k = (8 * t + N) / (2 * N);
  double r = (kPi / (2.0 * double(N))) * double(4 * t - k * N);
  double c = ce_cos_small(r), s = ce_sin_small(r);
  switch (k & 3) {
    case 0: return {c, s};
    case 1: return {-s, c};
    case 2: return {-c, -s};
    default: return {s, -c};
  }
}

template <int N>
struct UnitRoots {
  double c[N];
  double s[N];
  constexpr UnitRoots() : c(), s() {
    for (int t = 0; t < N; ++t) {
      cs_pair p = ce_unit_root(t, N);
      c[t] = p.c;
      s[t] = p.s;
    }
  }
};

template <int N>
__constant__ constexpr UnitRoots<N> kRoots{};

// exp(SIGN * 2 pi i q / N)
template <int N, int SIGN, typename T>
__device__ __forceinline__ cx<T> root(int q) {
  return {T(kRoots<N>.c[q]), T(SIGN * kRoots<N>.s[q])};
}

// ---------------------------------------------------------------------------
// Small DFTs on registers: v[k] <- sum_r v[r] exp(SIGN 2 pi i r k / R).
template <int R, int S, typename T>
struct SmallDft;

template <int S, typename T>
struct SmallDft<2, S, T> {
  __device__ __forceinline__ static void run(cx<T>* v) {
    cx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int S, typename T>
struct SmallDft<3, S, T> {
  __device__ __forceinline__ static void run(cx<T>* v) {
    const T h = T(0.86602540378443864676);  // sqrt(3)/2
    cx<T> t = cadd(v[1], v[2]);
    cx<T> d = csub(v[1], v[2]);
    cx<T> m = {v[0].x - T(0.5) * t.x, v[0].y - T(0.5) * t.y};
    cx<T> q = mul_si<S>(cscale(d, h));
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, q);
    v[2] = csub(m, q);
  }
};

template <int S, typename T>
struct SmallDft<4, S, T> {
  __device__ __forceinline__ static void run(cx<T>* v) {
    cx<T> t0 = cadd(v[0], v[2]);
    cx<T> t1 = csub(v[0], v[2]);
    cx<T> t2 = cadd(v[1], v[3]);
    cx<T> t3 = mul_si<S>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <int S, typename T>
struct SmallDft<5, S, T> {
  __device__ __forceinline__ static void run(cx<T>* v) {
    const T c1 = T(0.30901699437494742410);   // cos(2 pi / 5)
    const T c2 = T(-0.80901699437494742410);  // cos(4 pi / 5)
    const T s1 = T(0.95105651629515357212);   // sin(2 pi / 5)
    const T s2 = T(0.58778525229247312917);   // sin(4 pi / 5)
    cx<T> a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    cx<T> a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    cx<T> x0 = v[0];
    cx<T> p1 = {x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y};
    cx<T> p2 = {x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y};
    cx<T> q1 = mul_si<S>(cx<T>{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y});
    cx<T> q2 = mul_si<S>(cx<T>{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y});
    v[0] = cadd(x0, cadd(a1, a2));
    v[1] = cadd(p1, q1);
    v[4] = csub(p1, q1);
    v[2] = cadd(p2, q2);
    v[3] = csub(p2, q2);
  }
};

template <int S, typename T>
struct SmallDft<8, S, T> {
  // one radix-2 split (decimation in frequency), then two length-4 DFTs
  __device__ __forceinline__ static void run(cx<T>* v) {
    const T r = T(0.70710678118654752440);
    cx<T> a[4], b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k] = cadd(v[k], v[k + 4]);
      b[k] = csub(v[k], v[k + 4]);
    }
    // b[k] *= exp(S 2 pi i k / 8)
    b[1] = cscale(cadd(b[1], mul_si<S>(b[1])), r);
    b[2] = mul_si<S>(b[2]);
    b[3] = cscale(csub(mul_si<S>(b[3]), b[3]), r);
    SmallDft<4, S, T>::run(a);
    SmallDft<4, S, T>::run(b);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[2 * k] = a[k];
      v[2 * k + 1] = b[k];
    }
  }
};

// ---------------------------------------------------------------------------
// Radix plans.  Product of the list must equal N.
template <int N>
struct Plan;
template <> struct Plan<8>   { template <template <int...> class F> using apply = F<8>; };
template <> struct Plan<12>  { template <template <int...> class F> using apply = F<4, 3>; };
template <> struct Plan<16>  { template <template <int...> class F> using apply = F<4, 4>; };
template <> struct Plan<20>  { template <template <int...> class F> using apply = F<5, 4>; };
template <> struct Plan<24>  { template <template <int...> class F> using apply = F<8, 3>; };
template <> struct Plan<32>  { template <template <int...> class F> using apply = F<8, 4>; };
template <> struct Plan<36>  { template <template <int...> class F> using apply = F<4, 3, 3>; };
template <> struct Plan<40>  { template <template <int...> class F> using apply = F<8, 5>; };
template <> struct Plan<48>  { template <template <int...> class F> using apply = F<4, 4, 3>; };
template <> struct Plan<60>  { template <template <int...> class F> using apply = F<5, 4, 3>; };
template <> struct Plan<64>  { template <template <int...> class F> using apply = F<8, 8>; };
template <> struct Plan<72>  { template <template <int...> class F> using apply = F<8, 3, 3>; };
template <> struct Plan<80>  { template <template <int...> class F> using apply = F<5, 4, 4>; };
template <> struct Plan<96>  { template <template <int...> class F> using apply = F<8, 4, 3>; };

// One Stockham stage of radix R when the sub-transforms already done have
// length Ns: butterflies read stride N/R, apply exp(SIGN 2 pi i (j mod Ns) r /
// (Ns R)), and scatter to (j / Ns) Ns R + (j mod Ns) + r Ns.
template <int N, int S, int Ns, int R, typename T>
__device__ __forceinline__ void stockham_stage(const cx<T>* in, cx<T>* out) {
#pragma unroll
  for (int j = 0; j < N / R; ++j) {
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[j + r * (N / R)];
    const int k = j % Ns;
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], root<N, S, T>((k * r * (N / (Ns * R))) % N));
    }
    SmallDft<R, S, T>::run(v);
    const int d = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[d + r * Ns] = v[r];
  }
}

template <int N, int S, typename T, int Ns, int R, int... Rest>
__device__ __forceinline__ void stockham_run(cx<T>* a, cx<T>* b) {
  stockham_stage<N, S, Ns, R, T>(a, b);
  if constexpr (sizeof...(Rest) > 0) {
    stockham_run<N, S, T, Ns * R, Rest...>(b, a);
  }
}

template <int... Rs>
struct RadixList {
  static constexpr int count = sizeof...(Rs);
  template <int N, int S, typename T>
  __device__ __forceinline__ static void run(cx<T>* v) {
    cx<T> tmp[N];
    stockham_run<N, S, T, 1, Rs...>(v, tmp);
    if constexpr (count % 2 == 1) {
#pragma unroll
      for (int q = 0; q < N; ++q) v[q] = tmp[q];
    }
  }
};

// In-place length-N DFT of a register array.
template <int N, int S, typename T>
__device__ __forceinline__ void fft_line(cx<T>* v) {
  Plan<N>::template apply<RadixList>::template run<N, S, T>(v);
}

}  // namespace ace
