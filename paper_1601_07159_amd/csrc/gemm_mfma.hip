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
// the K slots are (orbital a, re/im): Re y = ar cr - ai ci, Im y = ar ci + ai cr.
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

// Round-to-nearest-even FP32 -> BF16 on the bit pattern (finite inputs).
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_float(unsigned short h) {
  return __uint_as_float((unsigned)h << 16);
}
__device__ __forceinline__ __bf16 as_bf16(unsigned short h) {
  return __builtin_bit_cast(__bf16, h);
}

// ---------------------------------------------------------------------------
// Reduction product, FP32 or FP64 MFMA.  A wave owns a 32 x 32 complex tile
// (2 x 2 MFMA blocks); the 4 waves of a workgroup take interleaved 8-point K
// steps of the same tile and are summed through LDS; one partial per
// workgroup (split K over blockIdx.z), combined later in FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_cn_mfma(const cx<T>* __restrict__ A, long lda, int na,
                                                 const cx<T>* __restrict__ B, long ldb, int nb,
                                                 long K, long kchunk,
                                                 cx<double>* __restrict__ partial) {
  typedef typename Acc4<T>::type acc_t;
  __shared__ double red[4][2][2][2][4][64];  // wave, alpha, beta, re/im, v, lane
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int a0 = blockIdx.x * 32, b0 = blockIdx.y * 32;
  const long kbeg = (long)blockIdx.z * kchunk;
  const long kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  const cx<T>* pa[2];
  const cx<T>* pb[2];
  bool va[2], vb[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int ra = a0 + 16 * h + r16, rb = b0 + 16 * h + r16;
    va[h] = ra < na;
    vb[h] = rb < nb;
    pa[h] = A + (size_t)(va[h] ? ra : 0) * lda;
    pb[h] = B + (size_t)(vb[h] ? rb : 0) * ldb;
  }
  acc_t cre[2][2], cim[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      cre[x][y] = acc_t{0, 0, 0, 0};
      cim[x][y] = acc_t{0, 0, 0, 0};
    }
  constexpr int U = 4;  // steps per iteration (loads issued together)
  for (long k0 = kbeg + 8 * wave; k0 < kend; k0 += 32 * U) {
    T a[U][2][4], b[U][2][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long k = k0 + 32 * u + 2 * kq;
      const bool kin = k < kend;  // N_g and kchunk are even: k + 1 is in range too
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        cx<T> x0 = {T(0), T(0)}, x1 = {T(0), T(0)}, y0 = {T(0), T(0)}, y1 = {T(0), T(0)};
        if (kin && va[h]) {
          x0 = pa[h][k];
          x1 = pa[h][k + 1];
        }
        if (kin && vb[h]) {
          y0 = pb[h][k];
          y1 = pb[h][k + 1];
        }
        a[u][h][0] = x0.x; a[u][h][1] = x0.y; a[u][h][2] = x1.x; a[u][h][3] = x1.y;
        b[u][h][0] = y0.x; b[u][h][1] = y0.y; b[u][h][2] = y1.x; b[u][h][3] = y1.y;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) {
            const T bs = b[u][y][s];
            const T bpp = (s & 1) ? -b[u][y][s ^ 1] : b[u][y][s ^ 1];
            cre[x][y] = mfma4(a[u][x][s], bs, cre[x][y]);
            cim[x][y] = mfma4(a[u][x][s], bpp, cim[x][y]);
          }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        red[wave][x][y][0][v][lane] = (double)cre[x][y][v];
        red[wave][x][y][1][v][lane] = (double)cim[x][y][v];
      }
  __syncthreads();
  // 256 threads write the 32 x 32 tile: thread -> (x, y, v, lane) over 2*2*4*64/4
  for (int e = threadIdx.x; e < 2 * 2 * 4 * 64; e += 256) {
    const int l = e & 63, v = (e >> 6) & 3, y = (e >> 8) & 1, x = (e >> 9) & 1;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      sr += red[w][x][y][0][v][l];
      si += red[w][x][y][1][v][l];
    }
    const int ra = a0 + 16 * x + mfma_row<T>(l, v);
    const int rb = b0 + 16 * y + (l & 15);
    if (ra < na && rb < nb)
      partial[((size_t)blockIdx.z * nb + rb) * na + ra] = {sr, si};
  }
}

// ---------------------------------------------------------------------------
// Reduction product in BF16-split precision: every FP32 operand x = hi + lo
// with hi = bf16(x), lo = bf16(x - hi); products hi*hi + hi*lo + lo*hi on the
// 16x16x32 BF16 MFMA with FP32 accumulation (the lo*lo term, ~2^-16 relative,
// is dropped).  A lane's 8 K slots are 4 consecutive complex grid values.
__global__ __launch_bounds__(256) void k_cn_mfma_bf16x3(const cx<float>* __restrict__ A, long lda,
                                                        int na, const cx<float>* __restrict__ B,
                                                        long ldb, int nb, long K, long kchunk,
                                                        cx<double>* __restrict__ partial) {
  __shared__ double red[4][2][2][2][4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int a0 = blockIdx.x * 32, b0 = blockIdx.y * 32;
  const long kbeg = (long)blockIdx.z * kchunk;
  const long kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  const cx<float>* pa[2];
  const cx<float>* pb[2];
  bool va[2], vb[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int ra = a0 + 16 * h + r16, rb = b0 + 16 * h + r16;
    va[h] = ra < na;
    vb[h] = rb < nb;
    pa[h] = A + (size_t)(va[h] ? ra : 0) * lda;
    pb[h] = B + (size_t)(vb[h] ? rb : 0) * ldb;
  }
  v4f cre[2][2], cim[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      cre[x][y] = v4f{0, 0, 0, 0};
      cim[x][y] = v4f{0, 0, 0, 0};
    }
  constexpr int U = 2;
  for (long k0 = kbeg + 16 * wave; k0 < kend; k0 += 64 * U) {
    float a[U][2][8], b[U][2][8];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long k = k0 + 64 * u + 4 * kq;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          cx<float> x = {0.f, 0.f}, y = {0.f, 0.f};
          if (k + q < kend && va[h]) x = pa[h][k + q];
          if (k + q < kend && vb[h]) y = pb[h][k + q];
          a[u][h][2 * q] = x.x; a[u][h][2 * q + 1] = x.y;
          b[u][h][2 * q] = y.x; b[u][h][2 * q + 1] = y.y;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v8bf ahi[2], alo[2], bhi[2], blo[2], phi_[2], plo[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const unsigned short ah = bf16_bits(a[u][h][s]);
          const unsigned short al = bf16_bits(a[u][h][s] - bf16_to_float(ah));
          const unsigned short bh = bf16_bits(b[u][h][s]);
          const unsigned short bl = bf16_bits(b[u][h][s] - bf16_to_float(bh));
          ahi[h][s] = as_bf16(ah);
          alo[h][s] = as_bf16(al);
          bhi[h][s] = as_bf16(bh);
          blo[h][s] = as_bf16(bl);
          // b'' = (im0, -re0, im1, -re1, ...): slot s takes the partner value,
          // negated (sign bit flipped) in the odd slots
          const int d = s ^ 1;
          const unsigned short sign = (d & 1) ? 0x8000 : 0;
          phi_[h][d] = as_bf16((unsigned short)(bh ^ sign));
          plo[h][d] = as_bf16((unsigned short)(bl ^ sign));
        }
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          cre[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[x], bhi[y], cre[x][y], 0, 0, 0);
          cre[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[x], blo[y], cre[x][y], 0, 0, 0);
          cre[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[x], bhi[y], cre[x][y], 0, 0, 0);
          cim[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[x], phi_[y], cim[x][y], 0, 0, 0);
          cim[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[x], plo[y], cim[x][y], 0, 0, 0);
          cim[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[x], phi_[y], cim[x][y], 0, 0, 0);
        }
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        red[wave][x][y][0][v][lane] = (double)cre[x][y][v];
        red[wave][x][y][1][v][lane] = (double)cim[x][y][v];
      }
  __syncthreads();
  for (int e = threadIdx.x; e < 2 * 2 * 4 * 64; e += 256) {
    const int l = e & 63, v = (e >> 6) & 3, y = (e >> 8) & 1, x = (e >> 9) & 1;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      sr += red[w][x][y][0][v][l];
      si += red[w][x][y][1][v][l];
    }
    const int ra = a0 + 16 * x + mfma_row<float>(l, v);
    const int rb = b0 + 16 * y + (l & 15);
    if (ra < na && rb < nb)
      partial[((size_t)blockIdx.z * nb + rb) * na + ra] = {sr, si};
  }
}

// C[a + b ldc] = alpha * sum_k partial[k][b][a]: 16 threads per element, each
// summing every 16th partial, combined in a fixed-order tree (deterministic).
__global__ __launch_bounds__(256) void k_reduce_partials2(const cx<double>* __restrict__ partial,
                                                          int ks, int na, int nb, double alpha,
                                                          cx<double>* __restrict__ C, int ldc) {
  __shared__ double red[2][16][16];
  const int g = threadIdx.x & 15, el = threadIdx.x >> 4;
  const int idx = blockIdx.x * 16 + el;
  double sr = 0.0, si = 0.0;
  if (idx < na * nb) {
    for (int k = g; k < ks; k += 16) {
      const cx<double> v = partial[(size_t)k * na * nb + idx];
      sr += v.x;
      si += v.y;
    }
  }
  red[0][el][g] = sr;
  red[1][el][g] = si;
  __syncthreads();
  for (int w = 8; w > 0; w >>= 1) {
    if (g < w) {
      red[0][el][g] += red[0][el][g + w];
      red[1][el][g] += red[1][el][g + w];
    }
    __syncthreads();
  }
  if (g == 0 && idx < na * nb) {
    const int a = idx % na, b = idx / na;
    C[a + (size_t)b * ldc] = {alpha * red[0][el][0], alpha * red[1][el][0]};
  }
}

// ---------------------------------------------------------------------------
// Expansion product Y_b[r] = sum_a A_a[r] C[a + b ldc].  A workgroup of 4 waves
// covers 128 grid rows (32 per wave, 2 MFMA row blocks) and 16 NBB columns;
// C is staged in LDS 64 orbitals at a time in the accumulation type.
template <typename TIn, typename TAcc, int NBB>
__global__ __launch_bounds__(256) void k_nn_mfma(const cx<TIn>* __restrict__ A, long lda, int na,
                                                 const cx<double>* __restrict__ C, int ldc, int nb,
                                                 cx<TIn>* __restrict__ Y, long ldy, long K) {
  typedef typename Acc4<TAcc>::type acc_t;
  constexpr int NBC = 16 * NBB;
  __shared__ TAcc cs_re[64][NBC];
  __shared__ TAcc cs_im[64][NBC];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const long rt0 = (long)blockIdx.x * 128 + 32 * wave;
  const int b0 = blockIdx.y * NBC;
  acc_t yre[2][NBB], yim[2][NBB];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < NBB; ++y) {
      yre[x][y] = acc_t{0, 0, 0, 0};
      yim[x][y] = acc_t{0, 0, 0, 0};
    }
  for (int ac = 0; ac < na; ac += 64) {
    for (int e = threadIdx.x; e < 64 * NBC; e += 256) {
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
    const int steps = (na - ac) < 64 ? (na - ac + 3) / 4 : 16;
    // four 4-orbital steps per group: all their A loads are issued first
    for (int st0 = 0; st0 < steps; st0 += 4) {
      TAcc xr[4][2], xi[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int a = ac + 4 * (st0 + u) + kq;
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          const long r = rt0 + 16 * x + r16;
          cx<TIn> v = {TIn(0), TIn(0)};
          if (st0 + u < steps && a < na && r < K) v = A[(size_t)a * lda + r];
          xr[u][x] = (TAcc)v.x;
          xi[u][x] = (TAcc)v.y;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (st0 + u >= steps) break;
        const int st = st0 + u;
#pragma unroll
        for (int y = 0; y < NBB; ++y) {
          const TAcc cr = cs_re[4 * st + kq][16 * y + r16];
          const TAcc ci = cs_im[4 * st + kq][16 * y + r16];
#pragma unroll
          for (int x = 0; x < 2; ++x) {
            yre[x][y] = mfma4(xr[u][x], cr, yre[x][y]);
            yre[x][y] = mfma4(xi[u][x], -ci, yre[x][y]);
            yim[x][y] = mfma4(xr[u][x], ci, yim[x][y]);
            yim[x][y] = mfma4(xi[u][x], cr, yim[x][y]);
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
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

}  // namespace

static void cn_split2(int na, int nb, long K, long* ks_out, long* kchunk_out) {
  const long tiles = (long)((na + 31) / 32) * ((nb + 31) / 32);
  long ks = (1024 + tiles - 1) / tiles;  // about 1024 workgroups
  long kchunk = (K + ks - 1) / ks;
  kchunk = (kchunk + 255) / 256 * 256;  // whole unrolled iterations, even
  if (kchunk < 256) kchunk = 256;
  ks = (K + kchunk - 1) / kchunk;
  if (ks < 1) ks = 1;
  *ks_out = ks;
  *kchunk_out = kchunk;
}

size_t gemm_cn_scratch_bytes(int na, int nb, long K) {
  long ks, kchunk;
  cn_split2(na, nb, K, &ks, &kchunk);
  return align_up((size_t)ks * na * nb * sizeof(cx<double>), 256);
}

template <typename T>
ace_status gemm_cn(ace_ctx c, const cx<T>* A, long lda, int na, const cx<T>* B, long ldb, int nb,
                   long K, double alpha, cx<double>* C, int ldc, bool bf16_split) {
  long ks, kchunk;
  cn_split2(na, nb, K, &ks, &kchunk);
  ace_status st;
  cx<double>* partial = (cx<double>*)ws_take(c, (size_t)ks * na * nb * sizeof(cx<double>), &st);
  if (!partial) return st;
  const dim3 grid((na + 31) / 32, (nb + 31) / 32, (unsigned)ks);
  if constexpr (std::is_same<T, float>::value) {
    if (bf16_split) {
      if ((st = launch(c, "cn_mfma_bf16x3", k_cn_mfma_bf16x3, grid, dim3(256), 0, A, lda, na, B,
                       ldb, nb, K, kchunk, partial)) != ACE_OK)
        return st;
    } else if ((st = launch(c, "cn_mfma_f32", k_cn_mfma<float>, grid, dim3(256), 0, A, lda, na,
                            B, ldb, nb, K, kchunk, partial)) != ACE_OK) {
      return st;
    }
  } else {
    if ((st = launch(c, "cn_mfma_f64", k_cn_mfma<double>, grid, dim3(256), 0, A, lda, na, B, ldb,
                     nb, K, kchunk, partial)) != ACE_OK)
      return st;
  }
  return launch(c, "reduce_partials", k_reduce_partials2, dim3((na * nb + 15) / 16), dim3(256), 0,
                (const cx<double>*)partial, (int)ks, na, nb, alpha, C, ldc);
}

template <typename TIn, typename TAcc>
static ace_status nn_dispatch(ace_ctx c, const char* name, const cx<TIn>* A, long lda, int na,
                              const cx<double>* C, int ldc, int nb, cx<TIn>* Y, long ldy,
                              long K) {
  const int nbb = nb <= 16 ? 1 : nb <= 32 ? 2 : nb <= 48 ? 3 : nb <= 80 && nb > 64 ? 5 : 4;
  const dim3 block(256);
#define ACE_NN(NBBV)                                                                           \
  case NBBV: {                                                                                 \
    const dim3 grid((unsigned)((K + 127) / 128), (unsigned)((nb + 16 * NBBV - 1) / (16 * NBBV))); \
    return launch(c, name, k_nn_mfma<TIn, TAcc, NBBV>, grid, block, 0, A, lda, na, C, ldc, nb, Y, \
                  ldy, K);                                                                     \
  }
  switch (nbb) {
    ACE_NN(1)
    ACE_NN(2)
    ACE_NN(3)
    ACE_NN(4)
    ACE_NN(5)
  }
#undef ACE_NN
  return fail(c, ACE_E_ARG, "internal: column block");
}

template <typename T>
ace_status gemm_nn(ace_ctx c, const cx<T>* A, long lda, int na, const cx<double>* C, int ldc,
                   int nb, cx<T>* Y, long ldy, long K, bool fp64_accumulate) {
  if (fp64_accumulate || std::is_same<T, double>::value)
    return nn_dispatch<T, double>(c, "nn_mfma_f64", A, lda, na, C, ldc, nb, Y, ldy, K);
  return nn_dispatch<T, float>(c, "nn_mfma_f32", A, lda, na, C, ldc, nb, Y, ldy, K);
}

template ace_status gemm_cn<float>(ace_ctx, const cx<float>*, long, int, const cx<float>*, long,
                                   int, long, double, cx<double>*, int, bool);
template ace_status gemm_cn<double>(ace_ctx, const cx<double>*, long, int, const cx<double>*, long,
                                    int, long, double, cx<double>*, int, bool);
template ace_status gemm_nn<float>(ace_ctx, const cx<float>*, long, int, const cx<double>*, int,
                                   int, cx<float>*, long, long, bool);
template ace_status gemm_nn<double>(ace_ctx, const cx<double>*, long, int, const cx<double>*, int,
                                    int, cx<double>*, long, long, bool);

}  // namespace ace
