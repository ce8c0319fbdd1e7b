// Dense stages of the ACE build (Section 3): projected exchange matrix
// M = <psi, W>, Cholesky of -M, xi = W L^{-H}, the low-rank apply and the
// energy from the projection vectors.  Small matrices (n_band x n_band and
// n_band x n_x) live in FP64 complex, column-major.
#include <cmath>

#include "ace_internal.h"

namespace ace {

namespace {

template <typename T>
__device__ __forceinline__ cx<double> to_d(cx<T> a) {
  return {(double)a.x, (double)a.y};
}

// ---------------------------------------------------------------------------
// Long-K reduction product, split over K:
//   partial[ks][b][a] = sum_{r in split ks} conj(A_a[r]) B_b[r]
// 16 x 16 output tile per workgroup, K staged through LDS in 64-wide slices
// loaded as contiguous rows of each vector.
template <typename T, typename ACC>
__global__ __launch_bounds__(256) void k_gemm_cn_partial(const cx<T>* __restrict__ A, long lda,
                                                         int na, const cx<T>* __restrict__ B,
                                                         long ldb, int nb, long K, long kchunk,
                                                         cx<double>* __restrict__ partial) {
  constexpr int TK = 64;
  __shared__ cx<T> As[16][TK + 1];
  __shared__ cx<T> Bs[16][TK + 1];
  const int t = threadIdx.x;
  const int ta = t & 15, tb = t >> 4;
  const int a0 = blockIdx.x * 16, b0 = blockIdx.y * 16;
  const long rbeg = (long)blockIdx.z * kchunk;
  const long rend = rbeg + kchunk < K ? rbeg + kchunk : K;
  cx<double> acc = {0.0, 0.0};
  const cx<T> zero = {T(0), T(0)};
  for (long r0 = rbeg; r0 < rend; r0 += TK) {
    for (int e = t; e < 16 * TK; e += 256) {
      const int row = e / TK, col = e - row * TK;
      const long r = r0 + col;
      As[row][col] = (a0 + row < na && r < rend) ? A[(size_t)(a0 + row) * lda + r] : zero;
      Bs[row][col] = (b0 + row < nb && r < rend) ? B[(size_t)(b0 + row) * ldb + r] : zero;
    }
    __syncthreads();
    cx<ACC> part = {ACC(0), ACC(0)};
#pragma unroll 8
    for (int k = 0; k < TK; ++k) {
      const cx<T> x = As[ta][k], y = Bs[tb][k];
      part.x += (ACC)x.x * (ACC)y.x + (ACC)x.y * (ACC)y.y;
      part.y += (ACC)x.x * (ACC)y.y - (ACC)x.y * (ACC)y.x;
    }
    acc.x += (double)part.x;
    acc.y += (double)part.y;
    __syncthreads();
  }
  if (a0 + ta < na && b0 + tb < nb)
    partial[((size_t)blockIdx.z * nb + (b0 + tb)) * na + (a0 + ta)] = acc;
}

__global__ __launch_bounds__(256) void k_reduce_partials(const cx<double>* __restrict__ partial,
                                                         int ks, int na, int nb, double alpha,
                                                         cx<double>* __restrict__ C, int ldc) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= na * nb) return;
  const int a = idx % na, b = idx / na;
  cx<double> s = {0.0, 0.0};
  for (int k = 0; k < ks; ++k) {
    const cx<double> v = partial[(size_t)k * na * nb + idx];
    s.x += v.x;
    s.y += v.y;
  }
  C[a + (size_t)b * ldc] = {alpha * s.x, alpha * s.y};
}

// ---------------------------------------------------------------------------
// Long-M expansion product Y_b[r] = sum_a A_a[r] C[a + b ldc]: one grid point r
// per thread, NBT output columns per workgroup, C staged through LDS.
template <typename T, typename ACC, int NBT>
__global__ __launch_bounds__(256) void k_gemm_nn(const cx<T>* __restrict__ A, long lda, int na,
                                                 const cx<double>* __restrict__ C, int ldc, int nb,
                                                 cx<T>* __restrict__ Y, long ldy, long K) {
  __shared__ cx<ACC> Cs[64][NBT];
  const long r = (long)blockIdx.x * 256 + threadIdx.x;
  const int b0 = blockIdx.y * NBT;
  cx<ACC> acc[NBT];
#pragma unroll
  for (int bb = 0; bb < NBT; ++bb) acc[bb] = {ACC(0), ACC(0)};
  for (int a0 = 0; a0 < na; a0 += 64) {
    for (int e = threadIdx.x; e < 64 * NBT; e += 256) {
      const int aa = e / NBT, bb = e - aa * NBT;
      cx<ACC> v = {ACC(0), ACC(0)};
      if (a0 + aa < na && b0 + bb < nb) {
        const cx<double> cv = C[(a0 + aa) + (size_t)(b0 + bb) * ldc];
        v = {(ACC)cv.x, (ACC)cv.y};
      }
      Cs[aa][bb] = v;
    }
    __syncthreads();
    if (r < K) {
      const int amax = na - a0 < 64 ? na - a0 : 64;
      for (int aa = 0; aa < amax; ++aa) {
        const cx<T> xv = A[(size_t)(a0 + aa) * lda + r];
        const ACC xr = (ACC)xv.x, xi = (ACC)xv.y;
#pragma unroll
        for (int bb = 0; bb < NBT; ++bb) {
          const cx<ACC> cv = Cs[aa][bb];
          acc[bb].x += xr * cv.x - xi * cv.y;
          acc[bb].y += xr * cv.y + xi * cv.x;
        }
      }
    }
    __syncthreads();
  }
  if (r < K) {
#pragma unroll
    for (int bb = 0; bb < NBT; ++bb)
      if (b0 + bb < nb) Y[(size_t)(b0 + bb) * ldy + r] = {(T)acc[bb].x, (T)acc[bb].y};
  }
}

// ---------------------------------------------------------------------------
// A <- s (A + A^H) / 2, in place (one thread per unordered pair).
__global__ __launch_bounds__(256) void k_hermitize(cx<double>* A, int n, double s) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)n * n) return;
  const int i = (int)(idx % n), j = (int)(idx / n);
  if (i < j) return;
  const cx<double> a = A[i + (size_t)j * n], b = A[j + (size_t)i * n];
  if (i == j) {
    A[i + (size_t)j * n] = {s * a.x, 0.0};
  } else {
    const cx<double> v = {0.5 * s * (a.x + b.x), 0.5 * s * (a.y - b.y)};
    A[i + (size_t)j * n] = v;
    A[j + (size_t)i * n] = {v.x, -v.y};
  }
}

// Right-looking Cholesky of a Hermitian positive definite matrix by one
// workgroup: column k is scaled by 1/sqrt(pivot), then the trailing lower
// triangle gets the rank-1 update.  The strict upper triangle is zeroed.
// A failure recorded in *prior (an earlier factorisation of the same chain) is
// propagated to *info without touching A.
__global__ __launch_bounds__(1024) void k_cholesky(cx<double>* A, int n, int* info,
                                                   const int* prior) {
  __shared__ double piv;
  __shared__ int failed;
  const int t = threadIdx.x;
  if (prior && *prior != 0) {
    if (t == 0) *info = *prior;
    return;
  }
  if (t == 0) failed = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (t == 0) {
      const double d = A[k + (size_t)k * n].x;
      if (!(d > 0.0) || !isfinite(d)) {
        failed = k + 1;
      } else {
        piv = sqrt(d);
        A[k + (size_t)k * n] = {piv, 0.0};
      }
    }
    __syncthreads();
    if (failed) break;
    const double inv = 1.0 / piv;
    for (int i = k + 1 + t; i < n; i += 1024) {
      cx<double> v = A[i + (size_t)k * n];
      A[i + (size_t)k * n] = {v.x * inv, v.y * inv};
    }
    __syncthreads();
    const int m = n - k - 1;
    for (long e = t; e < (long)m * m; e += 1024) {
      const int i = k + 1 + (int)(e % m), j = k + 1 + (int)(e / m);
      if (i < j) continue;
      const cx<double> lik = A[i + (size_t)k * n], ljk = A[j + (size_t)k * n];
      cx<double> v = A[i + (size_t)j * n];
      v.x -= lik.x * ljk.x + lik.y * ljk.y;  // lik * conj(ljk)
      v.y -= lik.y * ljk.x - lik.x * ljk.y;
      A[i + (size_t)j * n] = v;
    }
    __syncthreads();
  }
  for (long e = t; e < (long)n * n; e += 1024) {
    const int i = (int)(e % n), j = (int)(e / n);
    if (i < j) A[e] = {0.0, 0.0};
  }
  if (t == 0) *info = failed;
}

// X = L^{-1} by forward substitution, one column per thread; then
// C = X^H (upper triangular).  Skipped when the factorisation failed.
__global__ __launch_bounds__(1024) void k_tri_inv_herm(const cx<double>* __restrict__ L, int n,
                                                       cx<double>* __restrict__ X,
                                                       cx<double>* __restrict__ C,
                                                       const int* __restrict__ info) {
  if (*info != 0) return;
  for (int j = threadIdx.x; j < n; j += 1024) {
    for (int i = 0; i < n; ++i) {
      if (i < j) {
        X[i + (size_t)j * n] = {0.0, 0.0};
        continue;
      }
      cx<double> s = {i == j ? 1.0 : 0.0, 0.0};
      for (int k = j; k < i; ++k) {
        const cx<double> l = L[i + (size_t)k * n], x = X[k + (size_t)j * n];
        s.x -= l.x * x.x - l.y * x.y;
        s.y -= l.x * x.y + l.y * x.x;
      }
      const double d = 1.0 / L[i + (size_t)i * n].x;
      X[i + (size_t)j * n] = {s.x * d, s.y * d};
    }
  }
  __syncthreads();
  for (long e = threadIdx.x; e < (long)n * n; e += 1024) {
    const int a = (int)(e % n), b = (int)(e / n);
    const cx<double> x = X[b + (size_t)a * n];
    C[e] = {x.x, -x.y};
  }
}

__global__ __launch_bounds__(1024) void k_sumsq(const cx<double>* __restrict__ A, long count,
                                                double s, double* __restrict__ out) {
  __shared__ double red[1024];
  double acc = 0.0;
  for (long k = threadIdx.x; k < count; k += 1024) acc += A[k].x * A[k].x + A[k].y * A[k].y;
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s * red[0];
}

__global__ __launch_bounds__(256) void k_copy_c128(const cx<double>* __restrict__ src, long count,
                                                   cx<double>* __restrict__ dst) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx < count) dst[idx] = src[idx];
}

}  // namespace

static void cn_split(int na, int nb, long K, long* ks_out, long* kchunk_out) {
  const int ta = (na + 15) / 16, tb = (nb + 15) / 16;
  long ks = (2048 + (long)ta * tb - 1) / ((long)ta * tb);
  long kchunk = (K + ks - 1) / ks;
  kchunk = (kchunk + 63) / 64 * 64;
  if (kchunk < 64) kchunk = 64;
  ks = (K + kchunk - 1) / kchunk;
  if (ks < 1) ks = 1;
  *ks_out = ks;
  *kchunk_out = kchunk;
}

size_t gemm_cn_scratch_bytes(int na, int nb, long K) {
  long ks, kchunk;
  cn_split(na, nb, K, &ks, &kchunk);
  return align_up((size_t)ks * na * nb * sizeof(cx<double>), 256);
}

template <typename T>
ace_status gemm_cn(ace_ctx c, const cx<T>* A, long lda, int na, const cx<T>* B, long ldb, int nb,
                   long K, double alpha, cx<double>* C, int ldc, bool bf16_split) {
  (void)bf16_split;
  const int ta = (na + 15) / 16, tb = (nb + 15) / 16;
  long ks, kchunk;
  cn_split(na, nb, K, &ks, &kchunk);
  ace_status st;
  cx<double>* partial = (cx<double>*)ws_take(c, (size_t)ks * na * nb * sizeof(cx<double>), &st);
  if (!partial) return st;
  if ((st = launch(c, "gemm_cn_partial", k_gemm_cn_partial<T, T>, dim3(ta, tb, (unsigned)ks),
                   dim3(256), 0, A, lda, na, B, ldb, nb, K, kchunk, partial)) != ACE_OK)
    return st;
  return launch(c, "reduce_partials", k_reduce_partials, dim3((na * nb + 255) / 256), dim3(256), 0,
                (const cx<double>*)partial, (int)ks, na, nb, alpha, C, ldc);
}

template <typename T>
ace_status gemm_nn(ace_ctx c, const cx<T>* A, long lda, int na, const cx<double>* C, int ldc,
                   int nb, cx<T>* Y, long ldy, long K, bool fp64_accumulate) {
  constexpr int NBT = 16;
  const dim3 grid((unsigned)((K + 255) / 256), (unsigned)((nb + NBT - 1) / NBT));
  if (fp64_accumulate)
    return launch(c, "gemm_nn_f64acc", k_gemm_nn<T, double, NBT>, grid, dim3(256), 0, A, lda, na,
                  C, ldc, nb, Y, ldy, K);
  return launch(c, "gemm_nn", k_gemm_nn<T, T, NBT>, grid, dim3(256), 0, A, lda, na, C, ldc, nb, Y,
                ldy, K);
}

ace_status hermitize(ace_ctx c, cx<double>* A, int n, double s) {
  return launch(c, "hermitize", k_hermitize, dim3((unsigned)(((long)n * n + 255) / 256)),
                dim3(256), 0, A, n, s);
}

ace_status cholesky(ace_ctx c, cx<double>* A, int n, int* info_dev, const int* prior) {
  return launch(c, "cholesky", k_cholesky, dim3(1), dim3(1024), 0, A, n, info_dev, prior);
}

ace_status tri_inv_herm(ace_ctx c, const cx<double>* L, int n, cx<double>* C,
                        cx<double>* scratch, const int* info_dev) {
  return launch(c, "tri_inv_herm", k_tri_inv_herm, dim3(1), dim3(1024), 0, L, n, scratch, C,
                info_dev);
}

ace_status sumsq(ace_ctx c, const cx<double>* A, long count, double s, double* out) {
  return launch(c, "sumsq", k_sumsq, dim3(1), dim3(1024), 0, A, count, s, out);
}

ace_status copy_matrix(ace_ctx c, const cx<double>* src, int n, cx<double>* dst) {
  const long count = (long)n * n;
  return launch(c, "copy_c128", k_copy_c128, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                src, count, dst);
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
