// Device bodies of the pair passes shared by the per-pass kernels
// (fft_passes.hip) and the persistent batched kernel (persist.hip): the kernel
// table, the pair indexing, the one-thread-per-line slab and plane passes and
// the two accumulate forms.  Each body processes one logical workgroup's work
// given its logical id, so a kernel can take that id from its grid position or
// from a work queue; the arithmetic is the same either way.
#pragma once

#include <cmath>

#include "ace_internal.h"

namespace ace {
namespace {

// Per-thread evaluator of the scaled kernel K'(G) (ace_kspec), in the
// precision T of the pass: |G|^2 = sum_a (2 pi / L_a)^2 m_a^2 with m_a the
// signed frequency of bin k_a (the Nyquist bin's sign does not matter:
// squared).  The plane passes form the (k1, k2) part once per line and add the
// k0 part per element, instead of reading an N_g table per pair.
template <typename T>
struct KEval {
  T t0, t1, t2, c, inv4mu2, g0c;
  int n, kind;
  __device__ __forceinline__ explicit KEval(const ace_kspec& ks)
      : t0(T(ks.t2[0])), t1(T(ks.t2[1])), t2(T(ks.t2[2])),
        c(T(ks.coef * (ks.dscale ? *ks.dscale : 1.0))), inv4mu2(T(ks.inv4mu2)),
        g0c(T(ks.coef * (ks.dscale ? *ks.dscale : 1.0) * ks.g0)), n(ks.n), kind(ks.kind) {}
  __device__ __forceinline__ T msq(int k) const {
    const int m = k <= n / 2 ? k : k - n;
    return T(m * m);
  }
  // sum of the axis-1 and axis-2 terms of |G|^2.  The sums are explicit fused
  // multiply-adds, so that every kernel (whatever the compiler would contract)
  // rounds K' the same way: the forms of a pass must agree bit for bit.
  __device__ __forceinline__ T part12(int k1, int k2) const {
    return fma(t1, msq(k1), t2 * msq(k2));
  }
  // 1 - exp(-x) for x >= 0.  FP32: the hardware exp2 above x = 0.1 (relative
  // error below 6e-7 there), the Taylor series to x^6 below (terms past it
  // under 2e-9); FP64: expm1.
  __device__ __forceinline__ static T one_minus_exp(T x) {
    if constexpr (sizeof(T) == 4) {
      const float e = __builtin_amdgcn_exp2f(-1.44269504088896341f * x);
      float tay = fma(x, -1.0f / 720.0f, 1.0f / 120.0f);
      tay = fma(x, tay, -1.0f / 24.0f);
      tay = fma(x, tay, 1.0f / 6.0f);
      tay = fma(x, tay, -0.5f);
      tay = fma(x, tay, 1.0f);
      return x > 0.1f ? 1.0f - e : x * tay;
    } else {
      return -expm1(-x);
    }
  }
  __device__ __forceinline__ T at(int k0, T s12) const {
    const T g2 = fma(t0, msq(k0), s12);
    if (kind == kKindKinetic) return c * (T(0.5) * g2);
    if (!(g2 > T(0))) return g0c;  // G = 0
    // FP32: hardware reciprocal (1 ulp); FP64: correctly rounded division
    T K;
    if constexpr (sizeof(T) == 4)
      K = c * (12.566370614359172954f * __builtin_amdgcn_rcpf(g2));
    else
      K = c * (T(12.566370614359172954) / g2);
    if (kind == ACE_ERFC) K *= one_minus_exp(g2 * inv4mu2);
    return K;
  }
};

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2:
// physical workgroup b runs on XCD b % 8.  The launches pad the grid to a
// multiple of 8 and map physical ids so that XCD x receives the contiguous
// logical range [x G/8, (x+1) G/8); logical ids >= count exit at once.  Logical
// order is chosen so that neighbours share inputs (the same x0 slab of phi and
// psi, the same pencil tile of phi), which then stay in one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ long xcd_logical(long bid, long padded) {
  return (bid % kXcds) * (padded / kXcds) + bid / kXcds;
}
inline unsigned xcd_pad(long count) { return (unsigned)((count + kXcds - 1) / kXcds * kXcds); }


// Streaming (non-temporal) store of one complex value.  The forward slab
// pass writes every pair spectrum once and re-reads the orbital slabs from
// L2; plain stores of the 2-3 GB stream evict those slabs (measured at
// 48^3: 0.88 -> 0.68 ms for the pass with streaming stores).
template <typename T>
__device__ __forceinline__ void store_nt(cx<T>* p, cx<T> v) {
  if constexpr (sizeof(T) == 4) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(f2{v.x, v.y}, reinterpret_cast<f2*>(p));
  } else {
    typedef double d2 __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(d2{v.x, v.y}, reinterpret_cast<d2*>(p));
  }
}

// Units of the packed real triangle before column c: sum over c' < c of
// (floor(c'/2) + 1).
__host__ __device__ __forceinline__ long real_tri_units(int c) {
  const long q = c / 2;
  return c + ((c & 1) ? q * q : q * (q - 1));
}
// Column c and row pair m of triangle unit p (p < real_tri_units(n)).
__device__ __forceinline__ void real_tri_of(long p, int* c, int* m) {
  int cc = (int)(2.0 * sqrt((double)p));  // close to the root of c^2/4 + c/2 = p
  while (cc > 0 && real_tri_units(cc) > p) --cc;
  while (real_tri_units(cc + 1) <= p) ++cc;
  *c = cc;
  *m = (int)(p - real_tri_units(cc));
}

// Pair of block-local index p.
//  mode 0: rectangle, i = i0 + p % A, j = j0 + p / A
//  mode 1: upper triangle i <= j of a diagonal block starting at i0 (= j0),
//          block triangle index p0 + p (row-major in j)
//  mode 3: the whole occupied triangle (A = n_occ orbitals, A(A+1)/2 pairs)
//          followed by the rectangle of orbitals x bands j0 = A ... in one chunk
__device__ __forceinline__ void pair_of(int mode, int i0, int A, int j0, long p0, long p, int* i,
                                        int* j) {
  if (mode == 3) {
    const long tri = (long)A * (A + 1) / 2;
    if (p >= tri) {
      *i = (int)((p - tri) % A);
      *j = j0 + (int)((p - tri) / A);
      return;
    }
    mode = 1;  // triangle of the occupied block, which starts at orbital i0
    j0 = i0;
  }
  if (mode == 0) {
    *i = i0 + (int)(p % A);
    *j = j0 + (int)(p / A);
  } else {
    const long g = p0 + p;
    long jj = (long)((sqrt(8.0 * (double)g + 1.0) - 1.0) * 0.5);
    while (jj * (jj + 1) / 2 > g) --jj;
    while ((jj + 1) * (jj + 2) / 2 <= g) ++jj;
    *j = j0 + (int)jj;
    *i = i0 + (int)(g - jj * (jj + 1) / 2);
  }
}

// One-thread-per-line variants of the slab and plane passes: each thread owns
// a whole row or column in registers.  A workgroup takes P slabs (planes) of
// N lines each, P chosen so that P N fills whole waves within an LDS budget
// (N = 48 planes: four in three full waves instead of one wave of 48 lanes).
// The slab pass gets the smaller budget: it issues two loads per value and
// measured slower at N = 48 with four slabs (fewer workgroups per CU).
template <int N, typename T>
constexpr int t1_group(long lds_budget) {
  int best = 1;
  double best_use = 0.0;
  for (int P = 1; P <= 16; ++P) {
    const long lds = (long)P * N * (N + 1) * (long)sizeof(cx<T>);
    if (P * N > 1024 || lds > lds_budget) break;
    const int waves = (P * N + 63) / 64;
    const double use = (double)(P * N) / (64.0 * waves);
    if (use > best_use + 1e-9) {
      best_use = use;
      best = P;
    }
  }
  return best;
}

// Forward slab pass, one group of N threads per unit (x0 slab, pair of the
// launch's npairs).  Group q of P takes unit lid0 + q; a group at or past `end`
// (only in the last workgroup of a launch or the last step of a task) redoes
// unit end - 1 and does not store.  `dead` threads (past the P groups of a
// larger persistent workgroup) take part in the barriers only.  s_all: P
// planes of N x (N + 1) values in LDS.  The slab is loaded LB rows at a time
// (LB = N: every load issued before the first use; smaller LB keeps fewer
// registers live, with the same arithmetic).
template <int N, typename T, int P, int LB = N>
__device__ __forceinline__ void slab_t1_body(cx<T>* s_all, int tid, bool dead, long lid0,
                                             long end, const cx<T>* __restrict__ phi, long ldphi,
                                             const cx<T>* __restrict__ psi, long ldpsi,
                                             cx<T>* __restrict__ buf, int mode, int i0, int A,
                                             int j0, long p0, int npairs) {
  constexpr int NN = N * N;
  constexpr int LD = N + 1;
  // group q of the workgroup (compile-time 0 when P = 1, keeping the LDS
  // addresses constant offsets)
  const int q = P == 1 ? 0 : tid / N;
  const int t = P == 1 ? tid : tid - q * N;
  cx<T>* s = s_all + q * N * LD;
  const bool live = P == 1 || lid0 + q < end;
  const long lid = live ? lid0 + q : end - 1;
  const int x0 = (int)(lid / npairs);
  const int p = (int)(lid - (long)x0 * npairs);
  if (!dead) {
    int i, j;
    pair_of(mode, i0, A, j0, p0, p, &i, &j);
    const cx<T>* a = phi + (size_t)i * ldphi + (size_t)x0 * NN;
    const cx<T>* b = psi + (size_t)j * ldpsi + (size_t)x0 * NN;
    static_assert(N % LB == 0, "load batch must divide N");
#pragma unroll
    for (int r0 = 0; r0 < N; r0 += LB) {
      cx<T> va[LB], vb[LB];
#pragma unroll
      for (int r = 0; r < LB; ++r) va[r] = a[(r0 + r) * N + t];
#pragma unroll
      for (int r = 0; r < LB; ++r) vb[r] = b[(r0 + r) * N + t];
#pragma unroll
      for (int r = 0; r < LB; ++r) s[(r0 + r) * LD + t] = cmulc(va[r], vb[r]);
    }
  }
  __syncthreads();
  cx<T> v[N];
  if (!dead) {
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = s[t * LD + k];
    fft_line<N, -1, T>(v);
#pragma unroll
    for (int k = 0; k < N; ++k) s[t * LD + k] = v[k];
  }
  __syncthreads();
  if (dead) return;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = s[k * LD + t];
  fft_line<N, -1, T>(v);
  if (!live) return;
  cx<T>* out = buf + (size_t)p * N * NN + (size_t)x0 * NN;
#pragma unroll
  for (int k = 0; k < N; ++k) store_nt(&out[k * N + t], v[k]);
}

// Plane pass, one group of N threads per unit (k1 plane, pair).  The plane
// buf[k0][k1][.] (N rows of N contiguous values, rows N^2 apart) goes through
// LDS: forward FFT along axis 0, multiply by K', inverse FFT along axis 0, then
// inverse FFT along axis 2.  Loads and stores are contiguous N-wide rows.
// Units, `end` and `dead` as in slab_t1_body.
template <int N, typename T, int P>
__device__ __forceinline__ void plane_t1_body(cx<T>* s_all, int tid, bool dead, long lid0,
                                              long end, cx<T>* __restrict__ buf,
                                              const ace_kspec& ks, int npairs) {
  constexpr int NN = N * N;
  constexpr int LD = N + 1;
  const int q = P == 1 ? 0 : tid / N;
  const int t = P == 1 ? tid : tid - q * N;
  cx<T>* s = s_all + q * N * LD;
  const bool live = P == 1 || lid0 + q < end;
  const long lid = live ? lid0 + q : end - 1;
  // pair-major: the planes of one pair on neighbouring units, so that the
  // rows read and written at every k0 form one contiguous run
  const int p = (int)(lid / N);
  const int k1 = (int)(lid - (long)p * N);
  cx<T>* plane = buf + (size_t)p * N * NN + (size_t)k1 * N;
  cx<T> v[N];
  if (!dead) {
    // axis 0 (column t of the plane, k2 = t): forward, kernel, inverse.  The
    // column is read straight from global memory (lanes on consecutive k2).
#pragma unroll
    for (int r = 0; r < N; ++r) v[r] = plane[(size_t)r * NN + t];
    fft_line<N, -1, T>(v);
    const KEval<T> ke(ks);
    const T s12 = ke.part12(k1, t);
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const T kk = ke.at(r, s12);
      v[r].x *= kk;
      v[r].y *= kk;
    }
    fft_line<N, +1, T>(v);
#pragma unroll
    for (int r = 0; r < N; ++r) s[r * LD + t] = v[r];
  }
  __syncthreads();
  if (!dead) {
    // axis 2 (row t of the plane, x0 = t): inverse
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = s[t * LD + k];
    fft_line<N, +1, T>(v);
#pragma unroll
    for (int k = 0; k < N; ++k) s[t * LD + k] = v[k];
  }
  __syncthreads();
  if (dead || !live) return;
#pragma unroll
  for (int r = 0; r < N; ++r) plane[(size_t)r * NN + t] = s[r * LD + t];
}

// Pencil pass with accumulation: one thread per (x0, x2) pencil along axis 1,
// 64 pencils per workgroup, one band per workgroup row of the grid.  Loops
// over the orbitals i of the block: inverse FFT along axis 1, multiply by
// phi_i, accumulate into a thread-private LDS column; the band is written once
// per block.  Lanes hold consecutive pencils, so every global access is a
// contiguous row; no barrier is needed anywhere.
// Band j = j0 + b, orbital i = i0 + a; the spectrum of the pair comes from
//  mode 0: a rectangle chunk (i0 + a, j0 + b) at index a + A b;
//  mode 1: the triangle chunk of a diagonal block (i0 = j0): pairs i <= j at
//          local index j'(j'+1)/2 + i', and u_ij = conj(u_ji) for i > j;
//  mode 2: a rectangle chunk stored the other way round, (j, i) at index
//          b + nbc a, read conjugated (u_ij = conj(u_ji));
//  mode 3: the single chunk of pair_of's mode 3 (i0 = j0 = 0, A = n_occ):
//          bands j < A as mode 1, bands j >= A from the rectangle after the
//          triangle.
// Body of one logical workgroup (lid < TILES nbc) on the 64 lanes of a wave;
// acc: the wave's N x 64 accumulator in LDS.
template <int N, typename T>
__device__ __forceinline__ void accum_lds_body(cx<T>* acc, int t, long lid,
                                               const cx<T>* __restrict__ phi, long ldphi,
                                               const cx<T>* __restrict__ buf,
                                               cx<T>* __restrict__ W, long ldW, int i0, int A,
                                               int j0, int nbc, int accumulate, int mode) {
  constexpr int NN = N * N;
  const int tile = (int)(lid / nbc);
  const int b = (int)(lid - (long)tile * nbc);
  const int q = tile * 64 + t;
  if (q >= NN) return;
  const int x0 = q / N, x2 = q - x0 * N;
  const size_t off = (size_t)x0 * NN + x2;
  // Branch-free body: the accumulator starts at zero, and all loads of an
  // iteration (the pencil of u_ij and of phi_i) are issued before any use.
#pragma unroll
  for (int k = 0; k < N; ++k) acc[k * 64 + t] = cx<T>{T(0), T(0)};
  const int j = j0 + b;
  // Bands of a triangle block take their orbitals in round-robin tournament
  // order (the circle method over the block's A bands, a bye when A is odd):
  // at step s band b meets partner p(s, b), and p(s, p(s, b)) = b, so the two
  // waves that need the spectrum of the pair {b, p} (one as u, one as conj u)
  // read it at the same step.  (The L2 does not keep it between the two
  // reads: a step's working set on one XCD exceeds it.)  The bands of a tile
  // are neighbouring workgroups, so the orbital pencils phi_i of the tile are
  // shared in L2; band-major order (a band's tiles adjacent) measured slower
  // (48^3: 0.93 -> 1.26 ms per build).
  const bool tri = mode == 1 || (mode == 3 && b < A);
  const int rounds = A - 1 + (A & 1);  // players A (+1 bye when odd), fixed player m
  for (int s = 0; s < A; ++s) {
    int a = s;
    if (tri) {
      const int m = rounds;
      if (s >= rounds) {
        a = b;  // even A: the band's own pair last
      } else if (b == m) {
        a = s;
      } else {
        int q = (2 * s - b) % m;
        q = q < 0 ? q + m : q;
        a = q == b ? m : q;
        if (a == A) a = b;  // odd A: the bye is the band's own pair
      }
    }
    const int i = i0 + a;
    size_t pidx;
    bool conj_u;
    if (mode == 0) {
      pidx = (size_t)a + (size_t)A * b;
      conj_u = false;
    } else if (mode == 1 || (mode == 3 && b < A)) {
      const int il = a, jl = b;  // local indices in the diagonal block
      pidx = il <= jl ? (size_t)jl * (jl + 1) / 2 + il : (size_t)il * (il + 1) / 2 + jl;
      conj_u = il > jl;
    } else if (mode == 3) {
      pidx = (size_t)A * (A + 1) / 2 + (size_t)a + (size_t)A * (b - A);
      conj_u = false;
    } else {
      pidx = (size_t)b + (size_t)nbc * a;
      conj_u = true;
    }
    const cx<T>* src = buf + pidx * N * NN + off;
    const cx<T>* fp = phi + (size_t)i * ldphi + off;
    cx<T> v[N];
    cx<T> f[N];
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = src[k * N];
#pragma unroll
    for (int k = 0; k < N; ++k) f[k] = fp[k * N];
    fft_line<N, +1, T>(v);
    if (conj_u) {
#pragma unroll
      for (int k = 0; k < N; ++k) v[k].y = -v[k].y;
    }
#pragma unroll
    for (int k = 0; k < N; ++k) acc[k * 64 + t] = cadd(acc[k * 64 + t], cmul(f[k], v[k]));
  }
  cx<T>* w = W + (size_t)j * ldW + off;
  if (accumulate) {
    cx<T> old[N];
#pragma unroll
    for (int k = 0; k < N; ++k) old[k] = w[k * N];
#pragma unroll
    for (int k = 0; k < N; ++k) w[k * N] = cadd(old[k], acc[k * 64 + t]);
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) w[k * N] = acc[k * 64 + t];
  }
}

// Index of the orbital that band b of a triangle block (A bands) meets at step
// s: the round-robin tournament of k_pencil_accum (circle method, a bye when A
// is odd, the band's own pair at the bye or, for even A, at the last step).
__device__ __forceinline__ int tri_partner(int A, int b, int s) {
  const int m = A - 1 + (A & 1);
  if (s >= m) return b;
  if (b == m) return s;
  int q = (2 * s - b) % m;
  q = q < 0 ? q + m : q;
  const int a = q == b ? m : q;
  return a == A ? b : a;
}

// Accumulate pass on split lines: every (x0, x2) pencil along axis 1 is split
// over 4 lanes 16 apart (lane p + 16 h holds part h of pencil p: it loads rows
// h + 4 m and, after fft_quad_d2b, holds rows k + M kp(h)), 16 consecutive
// pencils per one-wave workgroup, so every load and store of 16 lanes is one
// contiguous row segment; one band per workgroup row of the grid.  The band's
// accumulator stays in registers (no LDS), so occupancy is set by registers
// alone.  Modes, pair indices and the tournament order of the triangle bands
// as in k_pencil_accum.
// Body of one logical workgroup (lid < (N^2 / 16) nbc) on lane `lane` of a
// full wave.
template <int N, typename T>
__device__ __forceinline__ void accum_q_body(int lane, long lid, const cx<T>* __restrict__ phi,
                                             long ldphi, const cx<T>* __restrict__ buf,
                                             cx<T>* __restrict__ W, long ldW, int i0, int A,
                                             int j0, int nbc, int accumulate, int mode) {
  constexpr int NN = N * N;
  constexpr int M = N / 4;
  static_assert(N % 4 == 0, "quad lines need N divisible by 4");
  const int tile = (int)(lid / nbc);
  const int b = (int)(lid - (long)tile * nbc);
  const int h = lane >> 4;
  const int q = tile * 16 + (lane & 15);
  const int x0 = q / N, x2 = q - x0 * N;
  const size_t off = (size_t)x0 * NN + x2;
  cx<T> acc[M];
#pragma unroll
  for (int k = 0; k < M; ++k) acc[k] = cx<T>{T(0), T(0)};
  const int j = j0 + b;
  const bool tri = mode == 1 || (mode == 3 && b < A);
  for (int s = 0; s < A; ++s) {
    const int a = tri ? tri_partner(A, b, s) : s;
    const int i = i0 + a;
    size_t pidx;
    bool conj_u;
    if (mode == 0) {
      pidx = (size_t)a + (size_t)A * b;
      conj_u = false;
    } else if (tri) {
      pidx = a <= b ? (size_t)b * (b + 1) / 2 + a : (size_t)a * (a + 1) / 2 + b;
      conj_u = a > b;
    } else if (mode == 3) {
      pidx = (size_t)A * (A + 1) / 2 + (size_t)a + (size_t)A * (b - A);
      conj_u = false;
    } else {
      pidx = (size_t)b + (size_t)nbc * a;
      conj_u = true;
    }
    const cx<T>* src = buf + pidx * N * NN + off;
    const cx<T>* fp = phi + (size_t)i * ldphi + off;
    cx<T> v[M], f[M];
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = src[(size_t)(h + 4 * m) * N];
#pragma unroll
    for (int k = 0; k < M; ++k) f[k] = fp[(size_t)quad_block_index(k, M, h) * N];
    fft_quad_d2b<N, +1, T, 16>(v, h);
    const T sg = conj_u ? T(-1) : T(1);
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const cx<T> u = {v[k].x, sg * v[k].y};
      acc[k] = cadd(acc[k], cmul(f[k], u));
    }
  }
  cx<T>* w = W + (size_t)j * ldW + off;
  if (accumulate) {
    cx<T> old[M];
#pragma unroll
    for (int k = 0; k < M; ++k) old[k] = w[(size_t)quad_block_index(k, M, h) * N];
#pragma unroll
    for (int k = 0; k < M; ++k) w[(size_t)quad_block_index(k, M, h) * N] = cadd(old[k], acc[k]);
  } else {
#pragma unroll
    for (int k = 0; k < M; ++k) w[(size_t)quad_block_index(k, M, h) * N] = acc[k];
  }
}

}  // namespace
}  // namespace ace
