// Matrix-core (MFMA) products of the ACE compression and apply (Section 3):
//   reduction   C = alpha * A^H B      (n_a x n_b, K = N_g grid points)
//               M = dV psi^H W, the Gram matrix dV X^H X, dV xi^H X
//   expansion   Y = A C                (N_g x n_b, K = n_a orbitals)
//               xi = W L^{-H}, V_ACE X = -xi (dV xi^H X)
//
// Complex arithmetic on real MFMAs.  For the reduction, a lane loads two
// consecutive complex grid values (re0, im0, re1, im1) of its row; every real
// becomes one K slot, so Re(conj(a) b) accumulates a_s b_s and Im(conj(a) b)
// accumulates a_s b''_s with b'' = (im0, -re0, im1, -re1).  For the expansion
// the K slots are orbitals: the streaming kernel forms Re y = ar cr - ai ci,
// Im y = ar ci + ai cr (four real products), the resident one three real
// products P1 = ar cr, P2 = ai ci, P3 = (ar + ai)(cr + ci) with Re y = P1 - P2,
// Im y = P3 - P1 - P2 (Gauss).
//
// MFMA operand layout (16x16xK blocks): lane l supplies A[row l%16][k group
// l/16] and B[k group l/16][col l%16]; the 16x16 result sits in 4 registers of
// column l%16: rows 4(l/16)+v for the FP32-result instructions, rows l/16+4v
// for the FP64 one (measured on gfx950).
#include <type_traits>

#include "ace_internal.h"

namespace ace {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <typename T>
struct Acc4;
template <>
struct Acc4<float> {
  typedef v4f type;
};
template <>
struct Acc4<double> {
  typedef v4d type;
};

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4d mfma4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Row of the 16x16 result held in register v of lane l.
template <typename TAcc>
__device__ __forceinline__ int mfma_row(int l, int v) {
  return std::is_same<TAcc, double>::value ? (l >> 4) + 4 * v : 4 * (l >> 4) + v;
}

typedef unsigned v4u __attribute__((ext_vector_type(4)));
// Third word of a raw buffer resource (32-bit data, no swizzle): loads past
// num_records return zero.
constexpr int kBufferFlags = 0x00020000;

// (v1, -v0, v3, -v2, ...) of eight BF16 values, on the 32-bit words.
__device__ __forceinline__ v8bf partner_neg(v8bf v) {
  typedef unsigned v4u __attribute__((ext_vector_type(4)));
  v4u w = __builtin_bit_cast(v4u, v);
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = ((w[i] >> 16) | (w[i] << 16)) ^ 0x80000000u;
  return __builtin_bit_cast(v8bf, w);
}

// ---------------------------------------------------------------------------
// Reduction products.  A workgroup of TA x TB waves (blockDim = (64 TA, TB))
// covers up to 32 TA x 32 TB outputs, one wave per 32 x 32 complex tile (2 x 2
// MFMA blocks), every wave walking the same K chunk: rows shared by the waves
// of a workgroup come from HBM once and are served to the others by the CU's
// caches.  K is split over blockIdx.z; each wave writes its FP32 (or FP64)
// accumulators unchanged as one partial, and the partials are summed in FP64
// in a fixed order afterwards.  16 x 16 blocks that lie wholly outside the
// output are skipped (a wave-uniform test), so an 80 x 80 product costs 25
// blocks of MFMA work, not 36.
template <typename T>
struct TileRows {
  const cx<T>* pa[2];
  const cx<T>* pb[2];
  bool va[2], vb[2];  // this lane's row inside the output
  bool ba[2], bb[2];  // any row of the 16-block inside (wave-uniform)
  int a0, b0;
};

// Tile of wave w of the workgroup.  The workgroup's tiles are taken in the
// order: tiles wholly inside the output first, then the cut ones, each group
// row by row; waves go to SIMDs round robin, so the heavy tiles spread over
// all four SIMDs instead of piling on one.
template <typename T>
__device__ __forceinline__ TileRows<T> tile_rows(const cx<T>* A, long lda, int na, const cx<T>* B,
                                                 long ldb, int nb, int r16) {
  TileRows<T> t;
  const int ta = blockDim.x >> 6, tb = blockDim.y;
  const int w = (threadIdx.y * blockDim.x + threadIdx.x) >> 6;
  const int gx0 = blockIdx.x * ta, gy0 = blockIdx.y * tb;
  int n_full_a = (na / 32) - gx0, n_full_b = (nb / 32) - gy0;
  n_full_a = n_full_a < 0 ? 0 : n_full_a > ta ? ta : n_full_a;
  n_full_b = n_full_b < 0 ? 0 : n_full_b > tb ? tb : n_full_b;
  int tx, ty;
  if (w < n_full_a * n_full_b) {
    tx = w % n_full_a;
    ty = w / n_full_a;
  } else {
    int m = w - n_full_a * n_full_b;  // m-th cut tile, row by row
    tx = 0;
    ty = 0;
    for (int q = 0; q < ta * tb; ++q) {
      const int qx = q % ta, qy = q / ta;
      if (qx < n_full_a && qy < n_full_b) continue;
      if (m-- == 0) {
        tx = qx;
        ty = qy;
        break;
      }
    }
  }
  t.a0 = (gx0 + tx) * 32;
  t.b0 = (gy0 + ty) * 32;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int ra = t.a0 + 16 * h + r16, rb = t.b0 + 16 * h + r16;
    t.va[h] = ra < na;
    t.vb[h] = rb < nb;
    t.ba[h] = t.a0 + 16 * h < na;
    t.bb[h] = t.b0 + 16 * h < nb;
    t.pa[h] = A + (size_t)(t.va[h] ? ra : 0) * lda;
    t.pb[h] = B + (size_t)(t.vb[h] ? rb : 0) * ldb;
  }
  return t;
}

// Hermitian mode (C = A^H A-like products whose lower triangle is the
// conjugate of the upper one): workgroups are rows of waves, wave w of
// workgroup x taking tile number x * (waves per workgroup) + w on or above the
// diagonal, in the order (0,0), (0,1), (1,1), (0,2), ... (column-major over
// the upper triangle of tiles); a wave past the last tile has none.
template <typename T>
__device__ __forceinline__ TileRows<T> tile_rows_herm(const cx<T>* A, long lda, int na,
                                                      const cx<T>* B, long ldb, int nb, int r16) {
  TileRows<T> t;
  int ty = 0, tx = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  while (tx > ty) {
    tx -= ty + 1;
    ++ty;
  }
  t.a0 = tx * 32;
  t.b0 = ty * 32;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int ra = t.a0 + 16 * h + r16, rb = t.b0 + 16 * h + r16;
    t.va[h] = ra < na;
    t.vb[h] = rb < nb;
    t.ba[h] = t.a0 + 16 * h < na;
    t.bb[h] = t.b0 + 16 * h < nb;
    t.pa[h] = A + (size_t)(t.va[h] ? ra : 0) * lda;
    t.pb[h] = B + (size_t)(t.vb[h] ? rb : 0) * ldb;
  }
  return t;
}

// T: the data type; TAcc: the MFMA and accumulation type (T, or double for
// FP64 products of complex64 data).
template <typename T, typename TAcc>
__global__ __launch_bounds__(sizeof(TAcc) == 8 ? 512 : 1024) void k_cn_mfma(
    const cx<T>* __restrict__ A, long lda, int na, const cx<T>* __restrict__ B, long ldb, int nb,
    long K, long kchunk, cx<TAcc>* __restrict__ partial, int herm) {
  typedef typename Acc4<TAcc>::type acc_t;
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  const TileRows<T> t = herm ? tile_rows_herm<T>(A, lda, na, B, ldb, nb, r16)
                             : tile_rows<T>(A, lda, na, B, ldb, nb, r16);
  if (!t.ba[0] || !t.bb[0]) return;  // whole wave outside the output
  const long kbeg = (long)blockIdx.z * kchunk;
  const long kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  acc_t cre[2][2], cim[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      cre[x][y] = acc_t{0, 0, 0, 0};
      cim[x][y] = acc_t{0, 0, 0, 0};
    }
  // Rolling pipeline over 8-point steps: the loads of step i + R - 1 are
  // issued before the MFMAs of step i, so R - 1 steps are always in flight.
  constexpr int R = sizeof(T) == 8 ? 2 : 4;
  // Loads are unconditional (a conditional load makes the compiler wait for
  // every load in flight at the join, which serialises the pipeline): a row
  // outside the output reads row 0 (pa/pb are clamped) and is never stored; a
  // point past the chunk reads the chunk's first point and is zeroed when
  // used (kin).  K and kchunk are even, so k + 1 is in range with k.
  T a[R][2][4], b[R][2][4];
  bool kin[R];
  auto load = [&](T (&ar)[2][4], T (&br)[2][4], bool& in, long k) {
    in = k < kend;
    const long kc = in ? k : kbeg;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const cx<T> x0 = t.pa[h][kc], x1 = t.pa[h][kc + 1];
      const cx<T> y0 = t.pb[h][kc], y1 = t.pb[h][kc + 1];
      ar[h][0] = x0.x; ar[h][1] = x0.y; ar[h][2] = x1.x; ar[h][3] = x1.y;
      br[h][0] = y0.x; br[h][1] = y0.y; br[h][2] = y1.x; br[h][3] = y1.y;
    }
  };
#pragma unroll
  for (int j = 0; j < R - 1; ++j) load(a[j], b[j], kin[j], kbeg + 8 * j + 2 * kq);
  // Tiles with all four 16-blocks inside the output (wave-uniform) take a
  // branch-free loop that interleaves the eight accumulator chains; cut tiles
  // skip the blocks outside.
  auto run = [&](auto full) {
    constexpr bool F = decltype(full)::value;
    for (long k0 = kbeg; k0 < kend; k0 += 8 * R) {
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int nx = (j + R - 1) % R;
        load(a[nx], b[nx], kin[nx], k0 + 8 * (j + R - 1) + 2 * kq);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
              if (!F && (!t.ba[x] || !t.bb[y])) continue;
              const TAcc av = kin[j] ? (TAcc)a[j][x][s] : TAcc(0);
              const TAcc bv = (TAcc)b[j][y][s];
              const TAcc bpp = (TAcc)((s & 1) ? -b[j][y][s ^ 1] : b[j][y][s ^ 1]);
              cre[x][y] = mfma4(av, bv, cre[x][y]);
              cim[x][y] = mfma4(av, bpp, cim[x][y]);
            }
      }
    }
  };
  if (t.ba[1] && t.bb[1])
    run(std::true_type{});
  else
    run(std::false_type{});
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ra = t.a0 + 16 * x + mfma_row<TAcc>(lane, v);
        const int rb = t.b0 + 16 * y + r16;
        if (ra < na && rb < nb)
          partial[((size_t)blockIdx.z * nb + rb) * na + ra] = {cre[x][y][v], cim[x][y][v]};
      }
}

// ---------------------------------------------------------------------------
// Reduction product in BF16-split precision: every FP32 operand x = hi + lo
// with hi = bf16(x), lo = bf16(x - hi); products hi*hi + hi*lo + lo*hi on the
// 16x16x32 BF16 MFMA with FP32 accumulation (the lo*lo term, ~2^-16 relative,
// is dropped).  A lane's 8 K slots are 4 consecutive complex grid values.
// Same partials as k_cn_mfma; at most kBf16Waves waves per workgroup.
constexpr int kBf16Stages = 4;
constexpr int kBf16Waves = 8;
__global__ __launch_bounds__(64 * kBf16Waves) void k_cn_mfma_bf16x3(const cx<float>* __restrict__ A, long lda,
                                                         int na, const cx<float>* __restrict__ B,
                                                         long ldb, int nb, long K, long kchunk,
                                                         cx<float>* __restrict__ partial,
                                                         int herm) {
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  const TileRows<float> t = herm ? tile_rows_herm<float>(A, lda, na, B, ldb, nb, r16)
                                 : tile_rows<float>(A, lda, na, B, ldb, nb, r16);
  if (!t.ba[0] || !t.bb[0]) return;
  const long kbeg = (long)blockIdx.z * kchunk;
  const long kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  v4f cre[2][2], cim[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      cre[x][y] = v4f{0, 0, 0, 0};
      cim[x][y] = v4f{0, 0, 0, 0};
    }
  // Rolling pipeline over 16-point steps: the raw loads of step i + R - 1 are
  // issued before step i is split into BF16 halves and multiplied, so R - 1
  // steps are in flight (two slots left the waves waiting on memory: the
  // kernel ran at 8% MFMA use and a third of its HBM rate at cfg 2).  Loads go
  // through per-wave buffer resources spanning the tile's rows inside the
  // output: rows outside it fall past the resource and read zero without a
  // memory access, so no load is conditional (a conditional load makes the
  // compiler wait for every load in flight).  Points past the chunk are
  // zeroed when used (kin bits).
  const int nva = na - t.a0 < 32 ? na - t.a0 : 32, nvb = nb - t.b0 < 32 ? nb - t.b0 : 32;
  const __amdgpu_buffer_rsrc_t rsa = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(A + (size_t)t.a0 * lda), (short)0, (int)((long)nva * lda * 8), kBufferFlags);
  const __amdgpu_buffer_rsrc_t rsb = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(B + (size_t)t.b0 * ldb), (short)0, (int)((long)nvb * ldb * 8), kBufferFlags);
  constexpr int R = kBf16Stages;
  float a[R][2][8], b[R][2][8];
  unsigned kin[R];
  auto load = [&](float (&ar)[2][8], float (&br)[2][8], unsigned& in, long k) {
    in = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) in |= (k + q < kend ? 1u : 0u) << q;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const long ea = (long)(16 * h + r16) * lda + k, eb = (long)(16 * h + r16) * ldb + k;
#pragma unroll
      for (int q = 0; q < 4; q += 2) {
        const v4u va = __builtin_amdgcn_raw_buffer_load_b128(rsa, (int)((ea + q) * 8), 0, 0);
        const v4u vb = __builtin_amdgcn_raw_buffer_load_b128(rsb, (int)((eb + q) * 8), 0, 0);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          ar[h][2 * q + c] = __uint_as_float(va[c]);
          br[h][2 * q + c] = __uint_as_float(vb[c]);
        }
      }
    }
  };
#pragma unroll
  for (int j = 0; j < R - 1; ++j) load(a[j], b[j], kin[j], kbeg + 16 * j + 4 * kq);
  for (long k0 = kbeg; k0 < kend; k0 += 16 * R) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int nx = (j + R - 1) % R;
      load(a[nx], b[nx], kin[nx], k0 + 16 * (j + R - 1) + 4 * kq);
      v8bf ahi[2], alo[2], bhi[2], blo[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const float av = (kin[j] >> (s >> 1)) & 1u ? a[j][h][s] : 0.f;
          // round-to-nearest-even conversions (v_cvt_pk_bf16_f32)
          const __bf16 ah = (__bf16)av, bh = (__bf16)b[j][h][s];
          ahi[h][s] = ah;
          alo[h][s] = (__bf16)(av - (float)ah);
          bhi[h][s] = bh;
          blo[h][s] = (__bf16)(b[j][h][s] - (float)bh);
        }
      }
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        // b'' = (im0, -re0, im1, -re1, ...): swap the two halves of every
        // 32-bit word and flip the sign of the upper one
        const v8bf phi_ = partner_neg(bhi[y]), plo = partner_neg(blo[y]);
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          if (!t.ba[x] || !t.bb[y]) continue;
          cre[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[x], bhi[y], cre[x][y], 0, 0, 0);
          cre[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[x], blo[y], cre[x][y], 0, 0, 0);
          cre[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[x], bhi[y], cre[x][y], 0, 0, 0);
          cim[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[x], phi_, cim[x][y], 0, 0, 0);
          cim[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[x], plo, cim[x][y], 0, 0, 0);
          cim[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[x], phi_, cim[x][y], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ra = t.a0 + 16 * x + mfma_row<float>(lane, v);
        const int rb = t.b0 + 16 * y + r16;
        if (ra < na && rb < nb)
          partial[((size_t)blockIdx.z * nb + rb) * na + ra] = {cre[x][y][v], cim[x][y][v]};
      }
}

// C[a + b ldc] = alpha * sum_k partial[k][b][a] in FP64: a workgroup takes
// 64 consecutive elements (one per lane, coalesced), its 16 waves sum every
// 16th partial each and are combined in a fixed-order tree (deterministic).
template <typename P>
__global__ __launch_bounds__(1024) void k_reduce_partials2(const cx<P>* __restrict__ partial,
                                                           int ks, int na, int nb, double alpha,
                                                           cx<double>* __restrict__ C, int ldc,
                                                           int real_part, int herm) {
  __shared__ double red[2][16][64];
  const int el = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int idx = blockIdx.x * 64 + el;
  const int a = idx % na, b = idx / na;
  // Hermitian mode: tiles below the diagonal were not computed; the entries
  // of the tiles above it are written twice, the second time conjugated
  const bool live = idx < na * nb && !(herm && a / 32 > b / 32);
  double sr = 0.0, si = 0.0;
  if (live) {
    const cx<P>* p = partial + idx;
    const size_t step = (size_t)na * nb;
    int k = g;
    for (; k + 48 < ks; k += 64) {  // four partials in flight
      const cx<P> v0 = p[k * step], v1 = p[(k + 16) * step];
      const cx<P> v2 = p[(k + 32) * step], v3 = p[(k + 48) * step];
      sr += (double)v0.x;
      si += (double)v0.y;
      sr += (double)v1.x;
      si += (double)v1.y;
      sr += (double)v2.x;
      si += (double)v2.y;
      sr += (double)v3.x;
      si += (double)v3.y;
    }
    for (; k < ks; k += 16) {
      const cx<P> v = p[k * step];
      sr += (double)v.x;
      si += (double)v.y;
    }
  }
  red[0][g][el] = sr;
  red[1][g][el] = si;
  __syncthreads();
  for (int w = 8; w > 0; w >>= 1) {
    if (g < w) {
      red[0][g][el] += red[0][g + w][el];
      red[1][g][el] += red[1][g + w][el];
    }
    __syncthreads();
  }
  if (g == 0 && live) {
    const double re = alpha * red[0][0][el], im = real_part ? 0.0 : alpha * red[1][0][el];
    C[a + (size_t)b * ldc] = {re, im};
    if (herm && a / 32 < b / 32) C[b + (size_t)a * ldc] = {re, -im};
  }
}

// ---------------------------------------------------------------------------
// Expansion product Y_b[r] = sum_a A_a[r] C[a + b ldc].  A workgroup of 4
// waves covers 4 x 16 XB grid rows (16 XB per wave: XB MFMA row blocks) and
// 16 NBB columns; C is staged in LDS KC orbitals at a time in the
// accumulation type.  With FP64 accumulation (64-cycle MFMAs, 8 registers per
// 16 x 16 block) a wave keeps one row block and the chunk is 32 orbitals, so
// that two or more waves fit on each SIMD to hide the grid-row loads.
template <typename TAcc>
struct NnShape {
  static constexpr int XB = sizeof(TAcc) == 8 ? 1 : 2;
  static constexpr int KC = sizeof(TAcc) == 8 ? 32 : 64;
  static constexpr int ROWS = 64 * XB;  // grid rows per workgroup
};

// upper: C is upper triangular, so chunks of orbitals past the workgroup's
// last column are not staged or read, and steps past the last column of a
// 16-column block skip its MFMAs.
template <typename TIn, typename TAcc, int NBB>
__global__ __launch_bounds__(256) void k_nn_mfma(const cx<TIn>* __restrict__ A, long lda, int na,
                                                 const cx<double>* __restrict__ C, int ldc, int nb,
                                                 cx<TIn>* __restrict__ Y, long ldy, long K,
                                                 int upper) {
  typedef typename Acc4<TAcc>::type acc_t;
  constexpr int XB = NnShape<TAcc>::XB, KC = NnShape<TAcc>::KC;
  constexpr int NBC = 16 * NBB;
  __shared__ TAcc cs_re[KC][NBC];
  __shared__ TAcc cs_im[KC][NBC];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const long rt0 = (long)blockIdx.x * NnShape<TAcc>::ROWS + 16 * XB * wave;
  const int b0 = blockIdx.y * NBC;
  acc_t yre[XB][NBB], yim[XB][NBB];
#pragma unroll
  for (int x = 0; x < XB; ++x)
#pragma unroll
    for (int y = 0; y < NBB; ++y) {
      yre[x][y] = acc_t{0, 0, 0, 0};
      yim[x][y] = acc_t{0, 0, 0, 0};
    }
  const int na_used = upper && b0 + NBC < na ? b0 + NBC : na;
  for (int ac = 0; ac < na_used; ac += KC) {
    for (int e = threadIdx.x; e < KC * NBC; e += 256) {
      const int aa = e / NBC, bb = e - aa * NBC;
      TAcc vr = 0, vi = 0;
      if (ac + aa < na && b0 + bb < nb) {
        const cx<double> cv = C[(ac + aa) + (size_t)(b0 + bb) * ldc];
        vr = (TAcc)cv.x;
        vi = (TAcc)cv.y;
      }
      cs_re[aa][bb] = vr;
      cs_im[aa][bb] = vi;
    }
    __syncthreads();
    const int steps = (na - ac) < KC ? (na - ac + 3) / 4 : KC / 4;
    const int ngroups = (steps + 3) / 4;
    // Groups of four 4-orbital steps, double-buffered: the A loads of group
    // g + 1 are in flight while group g is multiplied.  Loads are
    // unconditional from clamped addresses (an orbital past n_a meets zero
    // rows of C, a grid row past K is not stored, a group past the last
    // re-reads it), so the compiler keeps them in flight.
    auto loadg = [&](cx<TIn> (&v)[4][XB], int grp) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int a = ac + 4 * (4 * grp + u) + kq;
        const int ac_ = a < na ? a : na - 1;
#pragma unroll
        for (int x = 0; x < XB; ++x) {
          const long r = rt0 + 16 * x + r16;
          v[u][x] = A[(size_t)ac_ * lda + (r < K ? r : K - 1)];
        }
      }
    };
    auto mulg = [&](const cx<TIn> (&v)[4][XB], int grp) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int st = 4 * grp + u;
        if (st >= steps) break;
#pragma unroll
        for (int y = 0; y < NBB; ++y) {
          if (upper && ac + 4 * st > b0 + 16 * y + 15) continue;  // wave-uniform
          const TAcc cr = cs_re[4 * st + kq][16 * y + r16];
          const TAcc ci = cs_im[4 * st + kq][16 * y + r16];
#pragma unroll
          for (int x = 0; x < XB; ++x) {
            const TAcc xr = (TAcc)v[u][x].x, xi = (TAcc)v[u][x].y;
            yre[x][y] = mfma4(xr, cr, yre[x][y]);
            yre[x][y] = mfma4(xi, -ci, yre[x][y]);
            yim[x][y] = mfma4(xr, ci, yim[x][y]);
            yim[x][y] = mfma4(xi, cr, yim[x][y]);
          }
        }
      }
    };
    cx<TIn> xa[4][XB], xb[4][XB];
    loadg(xa, 0);
    for (int grp = 0; grp < ngroups; grp += 2) {
      loadg(xb, grp + 1 < ngroups ? grp + 1 : grp);
      mulg(xa, grp);
      loadg(xa, grp + 2 < ngroups ? grp + 2 : ngroups - 1);
      if (grp + 1 < ngroups) mulg(xb, grp + 1);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < XB; ++x)
#pragma unroll
    for (int y = 0; y < NBB; ++y) {
      const int b = b0 + 16 * y + r16;
      if (b >= nb) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long r = rt0 + 16 * x + mfma_row<TAcc>(lane, v);
        if (r < K) Y[(size_t)b * ldy + r] = {(TIn)yre[x][y][v], (TIn)yim[x][y][v]};
      }
    }
}

// Expansion product with all of C resident in LDS (n_a <= ACAP): a
// persistent grid of one 8-wave workgroup per CU stages its 16 NBB columns of
// C once, then every wave walks 16 XB-row tiles of Y with a stride of the
// whole grid, so the staging is paid once per CU instead of once per tile.
// The grid-row loads run R - 1 steps (4 orbitals each) ahead of the MFMAs.
constexpr int kNnResA = 80;
// Larger resident capacity for FP32 accumulation with up to 64 columns per
// workgroup: 256 orbitals x 64 columns x 8 bytes = 128 KiB of LDS.
constexpr int kNnResA2 = 256;

// upper: C is upper triangular (C[a][b] = 0 for a > b), so a step of four
// orbitals past the last column of a 16-column block adds nothing to it and
// its MFMAs are skipped (the triangular products xi = W L^{-H} and the
// orthonormalisation's X R^{-1} do about 60% of the full work).
template <typename TIn, typename TAcc, int NBB, int ACAP>
__global__ __launch_bounds__(512) void k_nn_mfma_res(const cx<TIn>* __restrict__ A, long lda,
                                                     int na, const cx<double>* __restrict__ C,
                                                     int ldc, int nb, cx<TIn>* __restrict__ Y,
                                                     long ldy, long K, int upper) {
  typedef typename Acc4<TAcc>::type acc_t;
  constexpr int XB = NnShape<TAcc>::XB;
  constexpr int NBC = 16 * NBB;
  constexpr int R = sizeof(TIn) == 8 ? 4 : 8;  // grid-row loads in flight
  // With 3 or 4 column blocks the skip branches make the register allocator
  // spill the accumulators (hundreds of spills); there the zero blocks of an
  // upper-triangular C are multiplied instead.
  constexpr bool kSkip = NBB != 3 && NBB != 4;
  __shared__ TAcc cs_re[ACAP][NBC];
  __shared__ TAcc cs_im[ACAP][NBC];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int b0 = blockIdx.y * NBC;
  const int na4 = (na + 3) & ~3;
  for (int e = threadIdx.x; e < na4 * NBC; e += blockDim.x) {
    const int aa = e / NBC, bb = e - aa * NBC;
    TAcc vr = 0, vi = 0;
    if (aa < na && b0 + bb < nb) {
      const cx<double> cv = C[aa + (size_t)(b0 + bb) * ldc];
      vr = (TAcc)cv.x;
      vi = (TAcc)cv.y;
    }
    cs_re[aa][bb] = vr;
    cs_im[aa][bb] = vi;
  }
  __syncthreads();
  const int nsteps = na4 / 4;
  const long ntiles = (K + 16 * XB - 1) / (16 * XB);
  const int nwaves = blockDim.x >> 6;
  for (long tile = (long)blockIdx.x * nwaves + wave; tile < ntiles;
       tile += (long)gridDim.x * nwaves) {
    const long rt0 = tile * 16 * XB;
    acc_t yre[XB][NBB], yim[XB][NBB], ys[XB][NBB];
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
      for (int y = 0; y < NBB; ++y) {
        yre[x][y] = acc_t{0, 0, 0, 0};
        yim[x][y] = acc_t{0, 0, 0, 0};
        ys[x][y] = acc_t{0, 0, 0, 0};
      }
    cx<TIn> buf[R][XB];
    // Unconditional loads from clamped addresses: an orbital past n_a meets
    // zero rows of C, a grid row past K is not stored, a step past the last
    // is not used.  (A conditional load makes the compiler wait for it at
    // once, which serialises the pipeline.)
    auto load = [&](cx<TIn> (&v)[XB], int st) {
      const int a = 4 * st + kq < na ? 4 * st + kq : na - 1;
#pragma unroll
      for (int x = 0; x < XB; ++x) {
        const long r = rt0 + 16 * x + r16;
        v[x] = A[(size_t)a * lda + (r < K ? r : K - 1)];
      }
    };
    // C entries of a step, read from LDS one step ahead of their use (the
    // step past the last one re-reads the last: rows stay inside cs_*)
    TAcc cb[2][NBB][2];
    auto loadc = [&](TAcc (&cv)[NBB][2], int st) {
      const int a = 4 * (st < nsteps ? st : nsteps - 1) + kq;
#pragma unroll
      for (int y = 0; y < NBB; ++y) {
        cv[y][0] = cs_re[a][16 * y + r16];
        cv[y][1] = cs_im[a][16 * y + r16];
      }
    };
#pragma unroll
    for (int j = 0; j < R - 1; ++j) load(buf[j], j);
    loadc(cb[0], 0);
    for (int st0 = 0; st0 < nsteps; st0 += R) {
#pragma unroll
      for (int j = 0; j < R; ++j) {
        load(buf[(j + R - 1) % R], st0 + j + R - 1);
        const int st = st0 + j;  // st0 is a multiple of R (even): step st uses cb[j & 1]
        loadc(cb[(j + 1) & 1], st + 1);
        if (st < nsteps) {
#pragma unroll
          for (int y = 0; y < NBB; ++y) {
            if (kSkip && upper && 4 * st > b0 + 16 * y + 15) continue;  // wave-uniform
            const TAcc cr = cb[j & 1][y][0], ci = cb[j & 1][y][1];
#pragma unroll
            for (int x = 0; x < XB; ++x) {
              const TAcc xr = (TAcc)buf[j][x].x, xi = (TAcc)buf[j][x].y;
              // three real products (Gauss): yre = P1 (x_re c_re), yim = P2
              // (x_im c_im), ys = P3 ((x_re + x_im)(c_re + c_im));
              // Re = P1 - P2, Im = P3 - P1 - P2 at the end
              yre[x][y] = mfma4(xr, cr, yre[x][y]);
              yim[x][y] = mfma4(xi, ci, yim[x][y]);
              ys[x][y] = mfma4(xr + xi, cr + ci, ys[x][y]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
      for (int y = 0; y < NBB; ++y) {
        const acc_t p1 = yre[x][y], p2 = yim[x][y];
        yre[x][y] = p1 - p2;
        yim[x][y] = ys[x][y] - p1 - p2;
      }
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
      for (int y = 0; y < NBB; ++y) {
        const int b = b0 + 16 * y + r16;
        if (b >= nb) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const long r = rt0 + 16 * x + mfma_row<TAcc>(lane, v);
          if (r < K) Y[(size_t)b * ldy + r] = {(TIn)yre[x][y][v], (TIn)yim[x][y][v]};
        }
      }
  }
}

}  // namespace

// Workgroup shape and K split of a reduction product: TA x TB waves per
// workgroup, at most max_waves (16 for the FP32 kernel, 12 for the BF16-split
// one, 8 for FP64).  The K chunks are sized so that all workgroups run in one
// round on the 256 CUs (as many per CU as its cu_waves resident waves allow):
// a second, partial round would double the time.  Each chunk is a whole
// number of unrolled steps (a multiple of 64 points).
struct CnShape {
  int ta, tb, gx, gy;
  long ks, kchunk;
};

static CnShape cn_shape(int na, int nb, long K, int max_waves, int cu_waves) {
  CnShape s;
  const int wa = (na + 31) / 32, wb = (nb + 31) / 32;
  s.ta = wa < 4 ? wa : 4;
  s.tb = wb < max_waves / s.ta ? wb : max_waves / s.ta;
  s.gx = (wa + s.ta - 1) / s.ta;
  s.gy = (wb + s.tb - 1) / s.tb;
  int per_cu = cu_waves / (s.ta * s.tb);
  if (per_cu < 1) per_cu = 1;
  long ks = 256L * per_cu / ((long)s.gx * s.gy);
  if (ks < 1) ks = 1;
  long kchunk = (K + ks - 1) / ks;
  kchunk = (kchunk + 63) / 64 * 64;
  if (kchunk < 64) kchunk = 64;
  ks = (K + kchunk - 1) / kchunk;
  s.ks = ks < 1 ? 1 : ks;
  s.kchunk = kchunk;
  return s;
}

// Hermitian mode: the n_up = T(T+1)/2 upper tiles (T tiles of 32 per side)
// over gx workgroup rows of at most max_waves waves each, as many workgroups
// per CU as cu_waves allows, one round.
static bool herm_shape(int n, long K, int max_waves, int cu_waves, CnShape* s) {
  const int T = (n + 31) / 32, nup = T * (T + 1) / 2;
  const int gx = (nup + max_waves - 1) / max_waves;
  const int w = (nup + gx - 1) / gx;
  s->ta = w;
  s->tb = 1;
  s->gx = gx;
  s->gy = 1;
  int per_cu = cu_waves / w;
  if (per_cu < 1) per_cu = 1;
  long kchunk = (K * gx + 256L * per_cu - 1) / (256L * per_cu);
  kchunk = (kchunk + 63) / 64 * 64;
  if (kchunk < 64) kchunk = 64;
  s->kchunk = kchunk;
  s->ks = (K + kchunk - 1) / kchunk;
  if (s->ks < 1) s->ks = 1;
  return true;
}

size_t gemm_cn_scratch_bytes(int na, int nb, long K) {
  CnShape s32 = cn_shape(na, nb, K, 16, 16), s16 = cn_shape(na, nb, K, kBf16Waves, kBf16Waves);
  CnShape s64 = cn_shape(na, nb, K, 8, 12);
  long k32 = s32.ks > s16.ks ? s32.ks : s16.ks, k64 = s64.ks;
  if (na == nb) {
    CnShape h;
    if (herm_shape(na, K, 16, 16, &h) && h.ks > k32) k32 = h.ks;
    if (herm_shape(na, K, kBf16Waves, kBf16Waves, &h) && h.ks > k32) k32 = h.ks;
    if (herm_shape(na, K, 8, 12, &h) && h.ks > k64) k64 = h.ks;
  }
  const size_t b32 = (size_t)k32 * na * nb * sizeof(cx<float>);
  const size_t b64 = (size_t)k64 * na * nb * sizeof(cx<double>);
  return align_up(b32 > b64 ? b32 : b64, 256);
}

size_t gemm_cn_partial_bytes(int na, int nb, long K, size_t data_bytes, CnMode mode, bool herm) {
  const bool bf16_split = data_bytes == sizeof(cx<float>) && mode == kBf16Split;
  const bool f64 = data_bytes == sizeof(cx<double>) || mode == kFp64;
  const int max_waves = f64 ? 8 : bf16_split ? kBf16Waves : 16;
  const int cu_waves = f64 ? 12 : bf16_split ? kBf16Waves : 16;
  CnShape s = cn_shape(na, nb, K, max_waves, cu_waves);
  if (herm && na == nb) herm_shape(na, K, max_waves, cu_waves, &s);
  const size_t part_eb = f64 ? sizeof(cx<double>) : sizeof(cx<float>);
  return align_up((size_t)s.ks * na * nb * part_eb, 256);
}

template <typename T>
ace_status gemm_cn(ace_ctx c, const cx<T>* A, long lda, int na, const cx<T>* B, long ldb, int nb,
                   long K, double alpha, cx<double>* C, int ldc, CnMode mode,
                   bool real_part, bool herm) {
  const bool bf16_split = std::is_same<T, float>::value && mode == kBf16Split;
  const bool f64 = sizeof(T) == 8 || mode == kFp64;
  // the BF16-split kernel addresses a tile's 32 rows through a buffer
  // resource with 32-bit byte offsets
  if (bf16_split && (lda > (1L << 31) / 256 || ldb > (1L << 31) / 256))
    return fail(c, ACE_E_UNSUPPORTED, "leading dimension too large for the BF16-split product");
  const int max_waves = f64 ? 8 : bf16_split ? kBf16Waves : 16;
  const int cu_waves = f64 ? 12 : bf16_split ? kBf16Waves : 16;
  CnShape s = cn_shape(na, nb, K, max_waves, cu_waves);
  herm = herm && na == nb && herm_shape(na, K, max_waves, cu_waves, &s);
  const int hm = herm ? 1 : 0;
  ace_status st;
  const size_t part_eb = f64 ? sizeof(cx<double>) : sizeof(cx<float>);
  void* partial = ws_take(c, (size_t)s.ks * na * nb * part_eb, &st);
  if (!partial) return st;
  const dim3 grid((unsigned)s.gx, (unsigned)s.gy, (unsigned)s.ks);
  const dim3 block(64 * s.ta, s.tb);
  if constexpr (std::is_same<T, float>::value) {
    if (bf16_split) {
      if ((st = launch(c, "cn_mfma_bf16x3", k_cn_mfma_bf16x3, grid, block, 0, A, lda, na, B, ldb,
                       nb, K, s.kchunk, (cx<float>*)partial, hm)) != ACE_OK)
        return st;
    } else if (f64) {
      if ((st = launch(c, "cn_mfma_f32in_f64", k_cn_mfma<float, double>, grid, block, 0, A, lda,
                       na, B, ldb, nb, K, s.kchunk, (cx<double>*)partial, hm)) != ACE_OK)
        return st;
    } else if ((st = launch(c, "cn_mfma_f32", k_cn_mfma<float, float>, grid, block, 0, A, lda, na,
                            B, ldb, nb, K, s.kchunk, (cx<float>*)partial, hm)) != ACE_OK) {
      return st;
    }
  } else {
    if ((st = launch(c, "cn_mfma_f64", k_cn_mfma<double, double>, grid, block, 0, A, lda, na, B,
                     ldb, nb, K, s.kchunk, (cx<double>*)partial, hm)) != ACE_OK)
      return st;
  }
  if (f64)
    return launch(c, "reduce_partials", k_reduce_partials2<double>, dim3((na * nb + 63) / 64),
                  dim3(1024), 0, (const cx<double>*)partial, (int)s.ks, na, nb, alpha, C, ldc,
                  real_part ? 1 : 0, hm);
  return launch(c, "reduce_partials", k_reduce_partials2<float>, dim3((na * nb + 63) / 64),
                dim3(1024), 0, (const cx<float>*)partial, (int)s.ks, na, nb, alpha, C, ldc,
                real_part ? 1 : 0, hm);
}

template <typename TIn, typename TAcc>
static ace_status nn_dispatch(ace_ctx c, const char* name, const cx<TIn>* A, long lda, int na,
                              const cx<double>* C, int ldc, int nb, cx<TIn>* Y, long ldy,
                              long K, bool c_upper) {
  const int nbb = nb <= 16 ? 1 : nb <= 32 ? 2 : nb <= 48 ? 3 : nb <= 80 && nb > 64 ? 5 : 4;
  const dim3 block(256);
  const bool resident = na <= kNnResA;
  const bool resident2 = !resident && na <= kNnResA2;
  const unsigned gy = (unsigned)((nb + 16 * nbb - 1) / (16 * nbb));
#define ACE_NN_RES(NBBV, CAP)                                                                  \
  {                                                                                            \
    const long tiles = (K + 16 * NnShape<TAcc>::XB - 1) / (16 * NnShape<TAcc>::XB);            \
    long gx = (tiles + 7) / 8;                                                                 \
    const long cap = (256 + gy - 1) / gy;                                                      \
    if (gx > cap) gx = cap;                                                                    \
    return launch(c, name, k_nn_mfma_res<TIn, TAcc, NBBV, CAP>, dim3((unsigned)gx, gy),        \
                  dim3(512), 0, A, lda, na, C, ldc, nb, Y, ldy, K, c_upper ? 1 : 0);           \
  }
#define ACE_NN(NBBV)                                                                           \
  case NBBV: {                                                                                 \
    if (resident) ACE_NN_RES(NBBV, kNnResA)                                                    \
    if constexpr (sizeof(TAcc) == 4 && NBBV <= 4)                                              \
      if (resident2) ACE_NN_RES(NBBV, kNnResA2)                                                \
    const long rows = NnShape<TAcc>::ROWS;                                                    \
    const dim3 grid((unsigned)((K + rows - 1) / rows), gy);                                    \
    return launch(c, name, k_nn_mfma<TIn, TAcc, NBBV>, grid, block, 0, A, lda, na, C, ldc, nb, Y, \
                  ldy, K, c_upper ? 1 : 0);                                                    \
  }
  switch (nbb) {
    ACE_NN(1)
    ACE_NN(2)
    ACE_NN(3)
    ACE_NN(4)
    ACE_NN(5)
  }
#undef ACE_NN
#undef ACE_NN_RES
  return fail(c, ACE_E_ARG, "internal: column block");
}

template <typename T>
ace_status gemm_nn(ace_ctx c, const cx<T>* A, long lda, int na, const cx<double>* C, int ldc,
                   int nb, cx<T>* Y, long ldy, long K, bool fp64_accumulate, bool c_upper) {
  if (fp64_accumulate || std::is_same<T, double>::value)
    return nn_dispatch<T, double>(c, "nn_mfma_f64", A, lda, na, C, ldc, nb, Y, ldy, K, c_upper);
  return nn_dispatch<T, float>(c, "nn_mfma_f32", A, lda, na, C, ldc, nb, Y, ldy, K, c_upper);
}

template ace_status gemm_cn<float>(ace_ctx, const cx<float>*, long, int, const cx<float>*, long,
                                   int, long, double, cx<double>*, int, CnMode, bool, bool);
template ace_status gemm_cn<double>(ace_ctx, const cx<double>*, long, int, const cx<double>*, long,
                                    int, long, double, cx<double>*, int, CnMode, bool, bool);
template ace_status gemm_nn<float>(ace_ctx, const cx<float>*, long, int, const cx<double>*, int,
                                   int, cx<float>*, long, long, bool, bool);
template ace_status gemm_nn<double>(ace_ctx, const cx<double>*, long, int, const cx<double>*, int,
                                    int, cx<double>*, long, long, bool, bool);

}  // namespace ace
