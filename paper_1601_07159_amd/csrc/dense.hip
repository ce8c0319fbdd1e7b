// Dense FP64 stages of the ACE build (Section 3): the factorisation of the
// projected exchange matrix (Cholesky of -M and the inverse of L that gives
// xi = W L^{-H}) and the energy reduction.  Small matrices (n_band x n_band and
// n_band x n_x) live in FP64 complex, column-major.
#include <cmath>

#include "ace_internal.h"

namespace ace {

namespace {

// ---------------------------------------------------------------------------
// Fused factorisation of a small Hermitian matrix, one workgroup:
//   A = s (M + M^H)/2  (lower triangle),  A = L L^H  (Cholesky, right-looking),
//   optional copy of L,  X = L^{-1} in place,  C = X^H = L^{-H}.
// Cholesky step k updates the trailing lower triangle with the unscaled column
// k divided by the pivot, and in the same phase finishes column k-1 (scale by
// 1/sqrt(pivot)); columns touched in one phase are disjoint, so one barrier per
// step suffices.  The in-place inverse eliminates column by column:
//   x_kk = 1/l_kk, rows below k of the left block get the rank-1 update with
//   the column -l_ik x_kk, then column k and row k are scaled.
// `A` points to LDS (n <= kCholLdsMax) or to a global scratch matrix; lda >= n.
constexpr int kCholLdsMax = 88;

__device__ __forceinline__ void chol_inv_body(const cx<double>* __restrict__ M, int n, double s,
                                              cx<double>* A, int lda,
                                              cx<double>* __restrict__ Lout,
                                              cx<double>* __restrict__ C, int* __restrict__ info,
                                              const int* __restrict__ prior) {
  // Element loops: waves stride over columns, lanes over rows (consecutive
  // rows are consecutive in memory), so no integer division is needed.
  __shared__ int failed;
  const int t = threadIdx.x, nt = blockDim.x;
  const int lane = t & 63, wave = t >> 6, nw = nt >> 6;
  if (prior && *prior != 0) {
    if (t == 0) *info = *prior;
    return;
  }
  if (t == 0) failed = 0;
  for (int j = wave; j < n; j += nw)
    for (int i = j + lane; i < n; i += 64) {
      const cx<double> a = M[i + (size_t)j * n], b = M[j + (size_t)i * n];
      A[i + (size_t)j * lda] = (i == j) ? cx<double>{s * a.x, 0.0}
                                        : cx<double>{0.5 * s * (a.x + b.x), 0.5 * s * (a.y - b.y)};
    }
  __syncthreads();
  // Cholesky
  double prev_inv = 0.0;
  for (int k = 0; k < n; ++k) {
    const double d = A[k + (size_t)k * lda].x;
    if (!(d > 0.0) || !isfinite(d)) {
      if (t == 0) failed = k + 1;
      break;  // uniform: every thread read the same pivot
    }
    const double invd = 1.0 / d;
    // (i, j) pairs of the trailing lower triangle, four columns per pass so
    // that the LDS loads of a pass are independent and overlap
    for (int j0 = k + 1 + wave; j0 < n; j0 += 4 * nw) {
      for (int i0 = j0 + lane; i0 < n; i0 += 64) {
        cx<double> lik[4], ljk[4], v[4];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = j0 + u * nw, i = i0 + u * nw;
          ok[u] = j < n && i < n;
          const int jj = ok[u] ? j : k, ii = ok[u] ? i : k;
          ljk[u] = A[jj + (size_t)k * lda];
          lik[u] = A[ii + (size_t)k * lda];
          v[u] = A[ii + (size_t)jj * lda];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (!ok[u]) continue;
          v[u].x -= (lik[u].x * ljk[u].x + lik[u].y * ljk[u].y) * invd;
          v[u].y -= (lik[u].y * ljk[u].x - lik[u].x * ljk[u].y) * invd;
          A[(i0 + u * nw) + (size_t)(j0 + u * nw) * lda] = v[u];
        }
      }
    }
    if (k > 0) {  // finish column k-1
      for (int i = k - 1 + t; i < n; i += nt) {
        cx<double> v = A[i + (size_t)(k - 1) * lda];
        A[i + (size_t)(k - 1) * lda] =
            (i == k - 1) ? cx<double>{sqrt(v.x), 0.0} : cx<double>{v.x * prev_inv, v.y * prev_inv};
      }
    }
    prev_inv = 1.0 / sqrt(d);
    __syncthreads();
  }
  __syncthreads();
  const int fail_k = failed;
  if (fail_k == 0 && t == 0) {
    const cx<double> v = A[(n - 1) + (size_t)(n - 1) * lda];
    A[(n - 1) + (size_t)(n - 1) * lda] = {sqrt(v.x), 0.0};
  }
  __syncthreads();
  if (t == 0) *info = fail_k;
  if (fail_k != 0) return;
  if (Lout) {
    for (int j = wave; j < n; j += nw)
      for (int i = lane; i < n; i += 64)
        Lout[i + (size_t)j * n] = (i >= j) ? A[i + (size_t)j * lda] : cx<double>{0.0, 0.0};
  }
  // in-place inverse of the lower triangle
  for (int k = 0; k < n; ++k) {
    const double xkk = 1.0 / A[k + (size_t)k * lda].x;  // diagonal is real
    for (int i = k + 1 + lane; i < n; i += 64) {
      const cx<double> lik = A[i + (size_t)k * lda];
      for (int j0 = wave; j0 < k; j0 += 4 * nw) {
        cx<double> akj[4], v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = j0 + u * nw < k ? j0 + u * nw : j0;
          akj[u] = A[k + (size_t)j * lda];
          v[u] = A[i + (size_t)j * lda];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (j0 + u * nw >= k) continue;
          v[u].x -= (lik.x * akj[u].x - lik.y * akj[u].y) * xkk;
          v[u].y -= (lik.x * akj[u].y + lik.y * akj[u].x) * xkk;
          A[i + (size_t)(j0 + u * nw) * lda] = v[u];
        }
      }
    }
    __syncthreads();
    for (int i = k + 1 + t; i < n; i += nt) {
      const cx<double> v = A[i + (size_t)k * lda];
      A[i + (size_t)k * lda] = {-v.x * xkk, -v.y * xkk};
    }
    for (int j = t; j < k; j += nt) {
      const cx<double> v = A[k + (size_t)j * lda];
      A[k + (size_t)j * lda] = {v.x * xkk, v.y * xkk};
    }
    if (t == 0) A[k + (size_t)k * lda] = {xkk, 0.0};
    __syncthreads();
  }
  // C = X^H (upper triangular)
  for (int b = wave; b < n; b += nw)
    for (int a = lane; a < n; a += 64) {
      const cx<double> x = (b >= a) ? A[b + (size_t)a * lda] : cx<double>{0.0, 0.0};
      C[a + (size_t)b * n] = {x.x, -x.y};
    }
}

__global__ __launch_bounds__(1024) void k_chol_inv_lds(const cx<double>* __restrict__ M, int n,
                                                      double s, cx<double>* __restrict__ Lout,
                                                      cx<double>* __restrict__ C,
                                                      int* __restrict__ info,
                                                      const int* __restrict__ prior) {
  __shared__ cx<double> A[kCholLdsMax * (kCholLdsMax + 1)];
  chol_inv_body(M, n, s, A, n + 1, Lout, C, info, prior);
}

__global__ __launch_bounds__(1024) void k_chol_inv_global(const cx<double>* __restrict__ M, int n,
                                                          double s, cx<double>* __restrict__ A,
                                                          cx<double>* __restrict__ Lout,
                                                          cx<double>* __restrict__ C,
                                                          int* __restrict__ info,
                                                          const int* __restrict__ prior) {
  chol_inv_body(M, n, s, A, n, Lout, C, info, prior);
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

}  // namespace

ace_status chol_inv(ace_ctx c, const cx<double>* M, int n, double s, cx<double>* Lout,
                    cx<double>* C, cx<double>* scratch, int* info_dev, const int* prior) {
  if (n <= kCholLdsMax)
    return launch(c, "chol_inv_lds", k_chol_inv_lds, dim3(1), dim3(1024), 0, M, n, s, Lout, C,
                  info_dev, prior);
  return launch(c, "chol_inv_global", k_chol_inv_global, dim3(1), dim3(1024), 0, M, n, s, scratch,
                Lout, C, info_dev, prior);
}

ace_status sumsq(ace_ctx c, const cx<double>* A, long count, double s, double* out) {
  return launch(c, "sumsq", k_sumsq, dim3(1), dim3(1024), 0, A, count, s, out);
}

}  // namespace ace
