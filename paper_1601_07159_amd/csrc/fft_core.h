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

// v * exp(SIGN 2 pi i q / N).  q is a constant once the stage loops are
// unrolled, so the branches fold away; the roots 1, +-i, -1 and the eighth
// roots (1 +- i)/sqrt(2) cost no multiply or two, not the four of a general
// complex product (a product by an exact 1 or 0 is not removed by the
// compiler, since x * 0 is not 0 for every x in IEEE arithmetic).
template <int N, int SIGN, typename T>
__device__ __forceinline__ cx<T> twiddle(cx<T> v, int q) {
  if (q == 0) return v;
  if (4 * q == N) return mul_si<SIGN>(v);
  if (2 * q == N) return cx<T>{-v.x, -v.y};
  if (4 * q == 3 * N) return mul_si<-SIGN>(v);
  if (8 * q == N || 8 * q == 3 * N || 8 * q == 5 * N || 8 * q == 7 * N) {
    // exp(SIGN i pi m / 4), m odd: ((+-1) + SIGN (+-1) i) / sqrt(2)
    const T r = T(0.70710678118654752440);
    const int m = 8 * q / N;
    const T cr = (m == 1 || m == 7) ? T(1) : T(-1);
    const T ci = (m == 1 || m == 3) ? T(SIGN) : T(-SIGN);
    // (cr + i ci)(x + i y) = (cr x - ci y) + i (cr y + ci x)
    return cx<T>{r * (cr * v.x - ci * v.y), r * (cr * v.y + ci * v.x)};
  }
  return cmul(v, root<N, SIGN, T>(q));
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
template <> struct Plan<2>   { template <template <int...> class F> using apply = F<2>; };
template <> struct Plan<3>   { template <template <int...> class F> using apply = F<3>; };
template <> struct Plan<4>   { template <template <int...> class F> using apply = F<4>; };
template <> struct Plan<5>   { template <template <int...> class F> using apply = F<5>; };
template <> struct Plan<6>   { template <template <int...> class F> using apply = F<3, 2>; };
template <> struct Plan<10>  { template <template <int...> class F> using apply = F<5, 2>; };
template <> struct Plan<9>   { template <template <int...> class F> using apply = F<3, 3>; };
template <> struct Plan<18>  { template <template <int...> class F> using apply = F<3, 3, 2>; };
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
      for (int r = 1; r < R; ++r) v[r] = twiddle<N, S, T>(v[r], (k * r * (N / (Ns * R))) % N);
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

// Prime-factor (Good-Thomas) split N = N1 N2 with gcd(N1, N2) = 1: input
// index n = (n1 N2 + n2 N1) mod N, output index k = CRT(k1 mod N1, k2 mod N2);
// then exp(2 pi i n k / N) = exp(2 pi i n1 k1 / N1) exp(2 pi i n2 k2 / N2), so
// the transform is N2 DFTs of length N1 and N1 of length N2 with no twiddle
// factors between them (the index maps are register renamings).
template <int N>
struct PfaSplit {
  static constexpr int n1 = 0, n2 = 0;
};
template <> struct PfaSplit<12> { static constexpr int n1 = 4, n2 = 3; };
template <> struct PfaSplit<18> { static constexpr int n1 = 2, n2 = 9; };
template <> struct PfaSplit<24> { static constexpr int n1 = 8, n2 = 3; };
template <> struct PfaSplit<40> { static constexpr int n1 = 8, n2 = 5; };
template <> struct PfaSplit<48> { static constexpr int n1 = 16, n2 = 3; };
template <> struct PfaSplit<72> { static constexpr int n1 = 8, n2 = 9; };

constexpr int inv_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 1;
}

template <int N, int S, typename T>
__device__ __forceinline__ void fft_line(cx<T>* v);

template <int N, int S, typename T>
__device__ __forceinline__ void fft_pfa(cx<T>* v) {
  constexpr int N1 = PfaSplit<N>::n1, N2 = PfaSplit<N>::n2;
  static_assert(N1 * N2 == N, "PFA split");
  constexpr int E1 = N2 * inv_mod(N2 % N1, N1);  // = 1 mod N1, 0 mod N2
  constexpr int E2 = N1 * inv_mod(N1 % N2, N2);  // = 0 mod N1, 1 mod N2
  cx<T> a[N2][N1];
#pragma unroll
  for (int n2 = 0; n2 < N2; ++n2)
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) a[n2][n1] = v[(n1 * N2 + n2 * N1) % N];
#pragma unroll
  for (int n2 = 0; n2 < N2; ++n2) fft_line<N1, S, T>(a[n2]);
  cx<T> b[N1][N2];
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1)
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) b[k1][n2] = a[n2][k1];
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) fft_line<N2, S, T>(b[k1]);
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) v[(k1 * E1 + k2 * E2) % N] = b[k1][k2];
}

// In-place length-N DFT of a register array.
template <int N, int S, typename T>
__device__ __forceinline__ void fft_line(cx<T>* v) {
  if constexpr (N == 1) {
    (void)v;
  } else if constexpr (PfaSplit<N>::n1 > 0) {
    fft_pfa<N, S, T>(v);
  } else {
    Plan<N>::template apply<RadixList>::template run<N, S, T>(v);
  }
}

// ---------------------------------------------------------------------------
// Lines split over the 4 lanes of a quad (N = 4 M).  Lane h of the quad holds
// M values.  Two layouts:
//   decimated  lane h holds x[h + 4 m],            m = 0..M-1
//   block      lane h holds X[k + M kp(h)],        k = 0..M-1,
//              kp(h) = (h >> 1) | ((h & 1) << 1)   (0, 2, 1, 3)
// fft_quad_d2b maps decimated input to block output, fft_quad_b2d block input
// to decimated output; both compute the unnormalised DFT of sign S.  The
// factorisation is N = 4 x M: an M-point DFT per lane, twiddles
// exp(S 2 pi i h k / N), and a 4-point DFT across the quad done as two
// radix-2 exchanges through DPP quad permutations (no LDS, no barrier).
constexpr int kQuadXor1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;  // quad_perm [2,3,0,1]

template <int CTRL>
__device__ __forceinline__ float quad_swap(float x) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double quad_swap(double x) {
  const long long u = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL, typename T>
__device__ __forceinline__ cx<T> quad_swap(cx<T> a) {
  return {quad_swap<CTRL>(a.x), quad_swap<CTRL>(a.y)};
}

// Value held by lane (l ^ D) of the wave: D = 1, 2 by DPP quad permutations;
// D = 16, 32 by the gfx950 permlane swaps, whose lane layout (measured with a
// probe): permlane16_swap(x, x) returns, in every pair of 16-lane rows, the
// even row's value in [0] and the odd row's in [1]; permlane32_swap(x, x)
// returns the lower 32 lanes' value in [0] and the upper 32 lanes' in [1].
template <int D>
__device__ __forceinline__ unsigned lane_xor_u32(unsigned u) {
  static_assert(D == 1 || D == 2 || D == 16 || D == 32, "lane distance");
  // (a quad permutation has a valid source for every lane, so the DPP move
  // needs no old value: mov_dpp leaves it undefined and saves a register copy)
  if constexpr (D == 1) {
    return (unsigned)__builtin_amdgcn_mov_dpp((int)u, kQuadXor1, 0xF, 0xF, false);
  } else if constexpr (D == 2) {
    return (unsigned)__builtin_amdgcn_mov_dpp((int)u, kQuadXor2, 0xF, 0xF, false);
  } else {
    const bool upper = (__lane_id() & D) != 0;
    if constexpr (D == 16) {
      const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
      return upper ? r[0] : r[1];
    } else {
      const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
      return upper ? r[0] : r[1];
    }
  }
}
template <int D>
__device__ __forceinline__ float lane_xor(float x) {
  return __builtin_bit_cast(float, lane_xor_u32<D>(__builtin_bit_cast(unsigned, x)));
}
template <int D>
__device__ __forceinline__ double lane_xor(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = lane_xor_u32<D>((unsigned)(u & 0xffffffffULL));
  const unsigned hi = lane_xor_u32<D>((unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | (unsigned long long)lo);
}
template <int D, typename T>
__device__ __forceinline__ cx<T> lane_xor(cx<T> a) {
  return {lane_xor<D>(a.x), lane_xor<D>(a.y)};
}

// Quad twiddles exp(S 2 pi i h k / N) (h = 0..3, k = 0..M-1, M = N / 4) in
// the working precision, stored [k][h] so that lane h reads entry (k, h) at a
// fixed per-lane base plus the compile-time offset 4 k: one load per value
// instead of choosing among four constants by lane.  Entries equal
// root<N, S, T>(h k) (h k < N), with exp(0) stored as 1 + 0i.
template <int N, typename T>
struct QuadRoots {
  cx<T> w[2][N];  // [0]: S = -1, [1]: S = +1
  constexpr QuadRoots() : w() {
    for (int k = 0; k < N / 4; ++k)
      for (int h = 0; h < 4; ++h) {
        const cs_pair p = ce_unit_root((long)h * k, N);
        const bool one = h * k == 0;
        w[0][4 * k + h] = one ? cx<T>{T(1), T(0)} : cx<T>{T(p.c), T(-1 * p.s)};
        w[1][4 * k + h] = one ? cx<T>{T(1), T(0)} : cx<T>{T(p.c), T(p.s)};
      }
  }
};

template <int N, typename T>
__constant__ constexpr QuadRoots<N, T> kQuadRoots{};

// Butterfly across lanes l and l ^ D: partner + sg * own, sg = +1 on the lane
// without bit D and -1 on the lane with it, i.e. (u + w, u - w) for u, w
// held by the lower and upper lane.  D = 1, 2: a DPP quad permutation brings
// the partner's value.  D = 16, 32: the permlane swap returns both halves in
// every lane ([0] the lower lane's value, [1] the upper's), so no per-lane
// choice is needed; r0 + sg r1 rounds exactly as partner + sg own.
template <int D>
__device__ __forceinline__ float xor_bfly(float own, float sg) {
  if constexpr (D == 1 || D == 2) {
    return fma(sg, own, lane_xor<D>(own));
  } else {
    static_assert(D == 16 || D == 32, "lane distance");
    const unsigned u = __builtin_bit_cast(unsigned, own);
    const auto r = D == 16 ? __builtin_amdgcn_permlane16_swap(u, u, false, false)
                           : __builtin_amdgcn_permlane32_swap(u, u, false, false);
    return fma(sg, __builtin_bit_cast(float, (unsigned)r[1]),
               __builtin_bit_cast(float, (unsigned)r[0]));
  }
}
template <int D>
__device__ __forceinline__ double xor_bfly(double own, double sg) {
  if constexpr (D == 1 || D == 2) {
    return fma(sg, own, lane_xor<D>(own));
  } else {
    static_assert(D == 16 || D == 32, "lane distance");
    const unsigned long long u = __builtin_bit_cast(unsigned long long, own);
    const unsigned lo = (unsigned)(u & 0xffffffffULL), hi = (unsigned)(u >> 32);
    const auto rl = D == 16 ? __builtin_amdgcn_permlane16_swap(lo, lo, false, false)
                            : __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto rh = D == 16 ? __builtin_amdgcn_permlane16_swap(hi, hi, false, false)
                            : __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    const double r0 = __builtin_bit_cast(
        double, ((unsigned long long)(unsigned)rh[0] << 32) | (unsigned long long)(unsigned)rl[0]);
    const double r1 = __builtin_bit_cast(
        double, ((unsigned long long)(unsigned)rh[1] << 32) | (unsigned long long)(unsigned)rl[1]);
    return fma(sg, r1, r0);
  }
}
template <int D, typename T>
__device__ __forceinline__ cx<T> xor_bfly(cx<T> own, T sg) {
  return {xor_bfly<D>(own.x, sg), xor_bfly<D>(own.y, sg)};
}

template <int N, int S, typename T>
__device__ __forceinline__ void quad_twiddle(cx<T>* v, int h) {
  constexpr int M = N / 4;
  const cx<T>* tw = kQuadRoots<N, T>.w[S > 0 ? 1 : 0] + h;
#pragma unroll
  for (int k = 1; k < M; ++k) v[k] = cmul(v[k], tw[4 * k]);
}

// The two radix-2 exchanges of the 4-point DFT across a quad, written without
// choosing operands by lane: with sigma = +-1 per lane, p + sigma v is exactly
// the rounded p - v or v + p of the butterfly, and the factor (S i) of the
// second stage is applied before the exchange by the lane whose value it
// multiplies (a product by +-i is exact), so every lane ends with
// received + sigma * own.
// D1: lane distance between the parts h and h ^ 1 of a line (1: the 4 lanes
// of a quad; 16: lanes l, l + 16, l + 32, l + 48, so that 16 consecutive
// lanes hold the same part of 16 lines, which keeps their global accesses
// contiguous); parts h and h ^ 2 are 2 D1 apart.
template <int N, int S, typename T, int D1 = 1>
__device__ __forceinline__ void fft_quad_d2b(cx<T>* v, int h) {
  constexpr int M = N / 4;
  static_assert(N % 4 == 0, "quad lines need N divisible by 4");
  fft_line<M, S, T>(v);
  quad_twiddle<N, S, T>(v, h);
  const bool hi = (h >> 1) != 0, odd = (h & 1) != 0;
  const T sg_hi = hi ? T(-1) : T(1), sg_odd = odd ? T(-1) : T(1);
  const bool rot = hi && odd;
#pragma unroll
  for (int k = 0; k < M; ++k)  // lanes h, h^2: (u, w) -> (u + w, u - w)
    v[k] = xor_bfly<2 * D1>(v[k], sg_hi);
#pragma unroll
  for (int k = 0; k < M; ++k)  // lanes h, h^1: (u, w) -> (u + t w, u - t w), t = (S i)^(h >> 1)
    v[k] = xor_bfly<D1>(rot ? mul_si<S>(v[k]) : v[k], sg_odd);  // the odd lane's w enters as t w
}

template <int N, int S, typename T, int D1 = 1>
__device__ __forceinline__ void fft_quad_b2d(cx<T>* v, int h) {
  constexpr int M = N / 4;
  static_assert(N % 4 == 0, "quad lines need N divisible by 4");
  const bool hi = (h >> 1) != 0, odd = (h & 1) != 0;
  const T sg_hi = hi ? T(-1) : T(1), sg_odd = odd ? T(-1) : T(1);
  const bool rot = hi && odd;
#pragma unroll
  for (int k = 0; k < M; ++k)  // lanes L, L^1 hold X[c], X[c + 2]: sum and difference
    v[k] = xor_bfly<D1>(v[k], sg_odd);
#pragma unroll
  for (int k = 0; k < M; ++k)  // lanes L, L^2: the odd pair carries the factor S i
    v[k] = xor_bfly<2 * D1>(rot ? mul_si<S>(v[k]) : v[k], sg_hi);  // the upper lane's q enters as w q
  quad_twiddle<N, S, T>(v, h);
  fft_line<M, S, T>(v);
}

// block position of value k on lane h
__device__ __forceinline__ int quad_block_index(int k, int M, int h) {
  return k + M * (((h >> 1) | ((h & 1) << 1)));
}

// ---------------------------------------------------------------------------
// Lines split over the 8 lanes of an octet (N = 8 M): at N = 72 a plane of
// 72 lines is nine full waves (a quad split leaves half a wave idle and
// carries 18 values per lane).  Layouts as for quads:
//   decimated  lane h holds x[h + 8 m],              m = 0..M-1
//   block      lane h holds X[k + M br3(h)],         k = 0..M-1,
//              br3(h) = the three bits of h reversed
// N = 8 x M: an M-point DFT per lane, twiddles exp(S 2 pi i h k / N), and an
// 8-point DFT across the octet as three radix-2 exchanges (decimation in
// frequency for d2b, in time for b2d): lanes h ^ 4 (DPP half-row mirror, then
// quad reversal), h ^ 2 and h ^ 1 (quad permutations).  The lane-dependent
// twiddles are read once per kernel (OctTw) for the forward sign; the inverse
// uses their conjugates.
constexpr int kDppHalfMirror = 0x141;  // row_half_mirror: lane i <- lane 7 - i of its 8
constexpr int kQuadRev = 0x1B;         // quad_perm [3,2,1,0]

template <typename T>
__device__ __forceinline__ cx<T> oct_swap4(cx<T> a) {  // value of lane h ^ 4
  return quad_swap<kQuadRev>(quad_swap<kDppHalfMirror>(a));
}

template <int N, typename T>
struct OctTw {
  cx<T> w[N / 8];  // w[k] = exp(-2 pi i h k / N), k = 1..M-1
  cx<T> w8;        // exp(-2 pi i (h & 3) / 8)
};

template <int N, typename T>
__device__ __forceinline__ OctTw<N, T> oct_twiddles(int h) {
  OctTw<N, T> t;
  t.w[0] = {T(1), T(0)};
#pragma unroll
  for (int k = 1; k < N / 8; ++k) t.w[k] = root<N, -1, T>((h * k) % N);
  t.w8 = root<8, -1, T>(h & 3);
  return t;
}

template <int S, typename T>
__device__ __forceinline__ cx<T> tw_sign(cx<T> w) {  // w for S = -1, conj(w) for S = +1
  return S < 0 ? w : cx<T>{w.x, -w.y};
}

template <int N, int S, typename T>
__device__ __forceinline__ void fft_oct_d2b(cx<T>* v, int h, const OctTw<N, T>& tw) {
  constexpr int M = N / 8;
  static_assert(N % 8 == 0, "octet lines need N divisible by 8");
  fft_line<M, S, T>(v);
#pragma unroll
  for (int k = 1; k < M; ++k) v[k] = cmul(v[k], tw_sign<S>(tw.w[k]));
  const cx<T> w8 = tw_sign<S>(tw.w8);
  const bool b2 = (h & 4) != 0, b1 = (h & 2) != 0, b0 = (h & 1) != 0;
#pragma unroll
  for (int k = 0; k < M; ++k) {  // lanes h, h^4: (u, w) -> (u + w, (u - w) w8^(h & 3))
    const cx<T> p = oct_swap4(v[k]);
    v[k] = b2 ? cmul(csub(p, v[k]), w8) : cadd(v[k], p);
  }
#pragma unroll
  for (int k = 0; k < M; ++k) {  // lanes h, h^2: (u, w) -> (u + w, (u - w) (S i)^(h & 1))
    const cx<T> p = quad_swap<kQuadXor2>(v[k]);
    const cx<T> d = csub(p, v[k]);
    v[k] = b1 ? (b0 ? mul_si<S>(d) : d) : cadd(v[k], p);
  }
#pragma unroll
  for (int k = 0; k < M; ++k) {  // lanes h, h^1: (u, w) -> (u + w, u - w)
    const cx<T> p = quad_swap<kQuadXor1>(v[k]);
    v[k] = b0 ? csub(p, v[k]) : cadd(v[k], p);
  }
}

template <int N, int S, typename T>
__device__ __forceinline__ void fft_oct_b2d(cx<T>* v, int h, const OctTw<N, T>& tw) {
  constexpr int M = N / 8;
  static_assert(N % 8 == 0, "octet lines need N divisible by 8");
  const bool b2 = (h & 4) != 0, b1 = (h & 2) != 0, b0 = (h & 1) != 0;
#pragma unroll
  for (int k = 0; k < M; ++k) {  // lanes h, h^1: sum and difference
    const cx<T> p = quad_swap<kQuadXor1>(v[k]);
    v[k] = b0 ? csub(p, v[k]) : cadd(v[k], p);
  }
#pragma unroll
  for (int k = 0; k < M; ++k) {  // lanes h, h^2: the value of the bit-1 lane carries (S i)^(h & 1)
    const cx<T> p = quad_swap<kQuadXor2>(v[k]);
    const cx<T> q = b1 ? v[k] : p, r = b1 ? p : v[k];
    const cx<T> wq = b0 ? mul_si<S>(q) : q;
    v[k] = b1 ? csub(r, wq) : cadd(r, wq);
  }
  const cx<T> w8 = tw_sign<S>(tw.w8);
#pragma unroll
  for (int k = 0; k < M; ++k) {  // lanes h, h^4: the value of the bit-2 lane carries w8^(h & 3)
    const cx<T> p = oct_swap4(v[k]);
    const cx<T> q = b2 ? v[k] : p, r = b2 ? p : v[k];
    const cx<T> wq = cmul(q, w8);
    v[k] = b2 ? csub(r, wq) : cadd(r, wq);
  }
#pragma unroll
  for (int k = 1; k < M; ++k) v[k] = cmul(v[k], tw_sign<S>(tw.w[k]));
  fft_line<M, S, T>(v);
}

// block position of value k on lane h of an octet
__device__ __forceinline__ int oct_block_index(int k, int M, int h) {
  return k + M * (((h & 1) << 2) | (h & 2) | ((h >> 2) & 1));
}

}  // namespace ace
