// Dense FP64 stages of the ACE build (Section 3): the factorisation of the
// projected exchange matrix (Cholesky of -M and the inverse of L that gives
// xi = W L^{-H}) and the energy reduction.  Small matrices (n_band x n_band and
// n_band x n_x) live in FP64 complex, column-major.
#include <cmath>

#include "ace_internal.h"

namespace ace {

namespace {

// ---------------------------------------------------------------------------
// Factorisation of a Hermitian matrix, one workgroup:
//   A = s (M + M^H)/2  (lower triangle),  A = L L^H  (Cholesky),
//   optional copy of L,  and with do_inverse C = L^{-H} (upper triangular).
// This form serves n above kCholRegMax (the register form below covers the
// smaller ones), with A in global scratch.  Blocked in panels of kCholNB
// columns so that only a few workgroup barriers are needed per panel:
//   Cholesky  the diagonal block is factored by wave 0 alone (lanes of one
//             wave stay ordered without barriers), the rows below solve
//             x L_kk^H = a one thread per row, the trailing lower triangle is
//             updated with kCholNB-term dot products.
//   inverse   (n > kCholPanelRows; below, k_tri_inv_wave follows instead)
//             X = L^{-1}: diagonal blocks inverted in place, one wave each;
//             then block row i: X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj, with the
//             finished blocks of X kept (conjugate-transposed) in C.
// lda >= n; T is scratch of kCholNB x n.
constexpr int kCholNB = 16;
// Up to this n the current panel (n x kCholNB) is staged in LDS.
constexpr int kCholPanelRows = 512;
__shared__ cx<double> chol_panel[kCholNB][kCholPanelRows];

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ cx<double> cmul_d(cx<double> a, cx<double> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
__device__ __forceinline__ cx<double> cmulcj_d(cx<double> a, cx<double> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}


// 1/sqrt(d) from the hardware estimate, refined by three Newton-Raphson steps
// y <- y (3/2 - d y^2 / 2).
__device__ __forceinline__ double rsq_refined(double d) {
  double y = __builtin_amdgcn_rsq(d);
  const double h = 0.5 * d;
#pragma unroll
  for (int it = 0; it < 3; ++it) {
    const double e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
  }
  return y;
}

__device__ __forceinline__ void chol_inv_body(const cx<double>* __restrict__ M, int n, double s,
                                              cx<double>* A, int lda, cx<double>* T,
                                              cx<double>* __restrict__ Lout,
                                              cx<double>* __restrict__ C, int* __restrict__ info,
                                              const int* __restrict__ prior, int real_only,
                                              int do_inverse) {
  constexpr int NB = kCholNB;
  __shared__ int failed;
  __shared__ double pinv[kCholNB];  // 1 / L_kk of the current diagonal block
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
      A[i + (size_t)j * lda] =
          (i == j)    ? cx<double>{s * a.x, 0.0}
          : real_only ? cx<double>{0.5 * s * (a.x + b.x), 0.0}
                      : cx<double>{0.5 * s * (a.x + b.x), 0.5 * s * (a.y - b.y)};
    }
  __syncthreads();

  // ---- Cholesky, right-looking by panels
  for (int kb = 0; kb < n; kb += NB) {
    const int nb = n - kb < NB ? n - kb : NB;
    if (n <= kCholPanelRows) {
      // the panel (rows kb.., columns kb..kb+nb-1) in LDS: P[c][r] = A[kb + r][kb + c]
      cx<double> (*P)[kCholPanelRows] = chol_panel;
      const int R = n - kb;
      for (int e = t; e < nb * R; e += nt) {
        const int c = e / R, r = e - c * R;
        P[c][r] = A[(kb + r) + (size_t)(kb + c) * lda];
      }
      __syncthreads();
      if (wave == 0) {
        for (int k = 0; k < nb; ++k) {
          const double d = P[k][k].x;
          if (!(d > 0.0) || !isfinite(d)) {
            if (lane == 0) failed = kb + k + 1;
            break;  // uniform across the wave
          }
          // 1/sqrt(d) and sqrt(d) from the refined reciprocal square root
          // (no divide on the serial path)
          const double inv = rsq_refined(d), r = d * inv;
          wave_sync();
          if (lane == 0) {
            P[k][k] = {r, 0.0};
            pinv[k] = inv;
          }
          const int i = k + 1 + lane;
          if (i < nb) {
            const cx<double> v = P[k][i];
            P[k][i] = {v.x * inv, v.y * inv};
          }
          wave_sync();
          // rank-1 update of the block's trailing triangle: lane -> (row
          // offset lane % 16, column offset lane / 16 + 4 t), no divisions
#pragma unroll
          for (int tq = 0; tq < 4; ++tq) {
            const int ii = k + 1 + (lane & 15), jj = k + 1 + (lane >> 4) + 4 * tq;
            if (ii < nb && jj < nb && ii >= jj) {
              const cx<double> u = cmulcj_d(P[k][ii], P[k][jj]);
              const cx<double> v = P[jj][ii];
              P[jj][ii] = {v.x - u.x, v.y - u.y};
            }
          }
          wave_sync();
        }
      }
      __syncthreads();
      if (failed) break;
      // rows below the diagonal block: x L_kk^H = a, one thread per row,
      // solved in place in the LDS panel (a register array indexed by the
      // loop counters went to scratch memory)
      for (int r = nb + t; r < R; r += nt) {
        for (int c = 0; c < nb; ++c) {
          cx<double> v = P[c][r];
          for (int d = 0; d < c; ++d) {
            const cx<double> u = cmulcj_d(P[d][r], P[d][c]);
            v.x -= u.x;
            v.y -= u.y;
          }
          const double inv = pinv[c];
          P[c][r] = {v.x * inv, v.y * inv};
        }
      }
      __syncthreads();
      // the finished panel back to A; the trailing lower triangle from the
      // LDS panel (disjoint columns of A)
      for (int e = t; e < nb * R; e += nt) {
        const int c = e / R, r = e - c * R;
        if (r >= c) A[(kb + r) + (size_t)(kb + c) * lda] = P[c][r];
      }
      // four columns jb..jb+3 per wave and lane row i: P[c][i] is read once for
      // the four (the P[c][j] are wave-uniform broadcasts).  Loads are
      // unconditional from clamped columns; entries above the diagonal or past
      // n are computed on scratch values and not stored.
      // Two row blocks (i and i + 64) per step with all eight loads issued
      // first, so that a thread waits for memory once per step.
      for (int jb = kb + nb + 4 * wave; jb < n; jb += 4 * nw) {
        int jq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) jq[q] = jb + q < n ? jb + q : n - 1;
        for (int i0 = jb + lane; i0 < n; i0 += 128) {
          int im[2];
          cx<double> acc[2][4];
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            im[m] = i0 + 64 * m < n ? i0 + 64 * m : n - 1;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[m][q] = A[im[m] + (size_t)jq[q] * lda];
          }
#pragma unroll
          for (int c = 0; c < NB; ++c) {
            if (c >= nb) break;
            cx<double> pj[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) pj[q] = P[c][jq[q] - kb];
#pragma unroll
            for (int m = 0; m < 2; ++m) {
              const cx<double> pi = P[c][im[m] - kb];
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const cx<double> u = cmulcj_d(pi, pj[q]);
                acc[m][q].x -= u.x;
                acc[m][q].y -= u.y;
              }
            }
          }
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            const int i = i0 + 64 * m;
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (i < n && jb + q < n && i >= jb + q) A[i + (size_t)(jb + q) * lda] = acc[m][q];
          }
        }
      }
      __syncthreads();
      continue;
    }
    // n > kCholPanelRows: the panel stays in global memory
    if (wave == 0) {
      for (int k = kb; k < kb + nb; ++k) {
        const double d = A[k + (size_t)k * lda].x;
        if (!(d > 0.0) || !isfinite(d)) {
          if (lane == 0) failed = k + 1;
          break;  // uniform across the wave
        }
        const double r = sqrt(d), inv = 1.0 / r;
        wave_sync();
        if (lane == 0) A[k + (size_t)k * lda] = {r, 0.0};
        const int i = k + 1 + lane;
        if (i < kb + nb) {
          const cx<double> v = A[i + (size_t)k * lda];
          A[i + (size_t)k * lda] = {v.x * inv, v.y * inv};
        }
        wave_sync();
        const int m = kb + nb - k - 1;
        for (int e = lane; e < m * m; e += 64) {
          const int ii = k + 1 + e % m, jj = k + 1 + e / m;
          if (ii < jj) continue;
          const cx<double> u = cmulcj_d(A[ii + (size_t)k * lda], A[jj + (size_t)k * lda]);
          cx<double> v = A[ii + (size_t)jj * lda];
          A[ii + (size_t)jj * lda] = {v.x - u.x, v.y - u.y};
        }
        wave_sync();
      }
    }
    __syncthreads();
    if (failed) break;
    // rows below the diagonal block: x L_kk^H = a, one thread per row
    for (int i = kb + nb + t; i < n; i += nt) {
      cx<double> x[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = c < nb ? A[i + (size_t)(kb + c) * lda] : cx<double>{0, 0};
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c >= nb) break;
        cx<double> v = x[c];
#pragma unroll
        for (int d = 0; d < c; ++d) {
          const cx<double> u = cmulcj_d(x[d], A[(kb + c) + (size_t)(kb + d) * lda]);
          v.x -= u.x;
          v.y -= u.y;
        }
        const double inv = 1.0 / A[(kb + c) + (size_t)(kb + c) * lda].x;
        x[c] = {v.x * inv, v.y * inv};
      }
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nb) A[i + (size_t)(kb + c) * lda] = x[c];
    }
    __syncthreads();
    // trailing lower triangle
    for (int j = kb + nb + wave; j < n; j += nw)
      for (int i = j + lane; i < n; i += 64) {
        cx<double> acc = A[i + (size_t)j * lda];
        for (int c = 0; c < nb; ++c) {
          const cx<double> u =
              cmulcj_d(A[i + (size_t)(kb + c) * lda], A[j + (size_t)(kb + c) * lda]);
          acc.x -= u.x;
          acc.y -= u.y;
        }
        A[i + (size_t)j * lda] = acc;
      }
    __syncthreads();
  }
  const int fail_k = failed;
  if (t == 0) *info = fail_k;
  if (fail_k != 0) return;
  if (Lout) {
    for (int j = wave; j < n; j += nw)
      for (int i = lane; i < n; i += 64)
        Lout[i + (size_t)j * n] = (i >= j) ? A[i + (size_t)j * lda] : cx<double>{0.0, 0.0};
  }
  if (!do_inverse) return;  // L stays in the lower triangle of A
  __syncthreads();  // Lout read A before the diagonal blocks are overwritten

  // ---- inverse: diagonal blocks in place (one wave each)
  const int nbk = (n + NB - 1) / NB;
  for (int b = wave; b < nbk; b += nw) {
    const int kb = b * NB, nb = n - kb < NB ? n - kb : NB;
    for (int k = kb; k < kb + nb; ++k) {
      const double xkk = 1.0 / A[k + (size_t)k * lda].x;
      wave_sync();
      const int mi = kb + nb - k - 1, mj = k - kb;
      for (int e = lane; e < mi * mj; e += 64) {
        const int i = k + 1 + e % mi, j = kb + e / mi;
        const cx<double> u = cmul_d(A[i + (size_t)k * lda], A[k + (size_t)j * lda]);
        cx<double> v = A[i + (size_t)j * lda];
        A[i + (size_t)j * lda] = {v.x - u.x * xkk, v.y - u.y * xkk};
      }
      wave_sync();
      for (int e = lane; e < mi; e += 64) {
        const cx<double> v = A[(k + 1 + e) + (size_t)k * lda];
        A[(k + 1 + e) + (size_t)k * lda] = {-v.x * xkk, -v.y * xkk};
      }
      for (int e = lane; e < mj; e += 64) {
        const cx<double> v = A[k + (size_t)(kb + e) * lda];
        A[k + (size_t)(kb + e) * lda] = {v.x * xkk, v.y * xkk};
      }
      if (lane == 0) A[k + (size_t)k * lda] = {xkk, 0.0};
      wave_sync();
    }
  }
  __syncthreads();
  // C = X^H: diagonal blocks now, zero strict lower part; the rest per block
  // row.  Finished off-diagonal blocks of X are also kept, conjugated, in the
  // unused strict upper triangle of A: X[k][j] sits at A[j + k lda] (j < k).
  for (int b = wave; b < n; b += nw)
    for (int a = lane; a < n; a += 64) {
      if (b < a) {
        C[a + (size_t)b * n] = {0.0, 0.0};
      } else if (a / NB == b / NB) {
        const cx<double> x = A[b + (size_t)a * lda];
        C[a + (size_t)b * n] = {x.x, -x.y};
      }
    }
  for (int ib = 1; ib < nbk; ++ib) {
    const int ri = ib * NB, ni = n - ri < NB ? n - ri : NB;
    // (the inverse runs here only above kCholPanelRows: from global memory)
    // T[r][col] = sum_{k = col}^{ri-1} L[ri + r][k] X[k][col]
    for (int col = wave; col < ri; col += nw)
      for (int r = lane; r < ni; r += 64) {
        const int cb_end = (col / NB + 1) * NB;  // X[k][col] for k < cb_end: diagonal block
        cx<double> acc = {0.0, 0.0};
        for (int k = col; k < cb_end; ++k) {
          const cx<double> u = cmul_d(A[(ri + r) + (size_t)k * lda], A[k + (size_t)col * lda]);
          acc.x += u.x;
          acc.y += u.y;
        }
#pragma unroll 4
        for (int k = cb_end; k < ri; ++k) {
          const cx<double> u =
              cmulcj_d(A[(ri + r) + (size_t)k * lda], A[col + (size_t)k * lda]);
          acc.x += u.x;
          acc.y += u.y;
        }
        T[r + (size_t)col * NB] = acc;
      }
    __syncthreads();
    // X[ri + r][col] = -sum_{q <= r} X_ii[r][q] T[q][col]
    for (int col = wave; col < ri; col += nw)
      for (int r = lane; r < ni; r += 64) {
        cx<double> acc = {0.0, 0.0};
        for (int q = 0; q <= r; ++q) {
          const cx<double> u = cmul_d(A[(ri + r) + (size_t)(ri + q) * lda], T[q + (size_t)col * NB]);
          acc.x += u.x;
          acc.y += u.y;
        }
        const cx<double> xc = {-acc.x, acc.y};  // conj(X[ri + r][col])
        A[col + (size_t)(ri + r) * lda] = xc;
        C[col + (size_t)(ri + r) * n] = xc;
      }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Factorisation for n <= kCholRegMax in two kernels.
// k_chol_reg: one workgroup, the entries of the lower triangle of A owned by
// threads in registers (up to kCholSlots each) for the whole kernel; one
// barrier per column k.  Right-looking on the unscaled Schur complement:
//   a_ij -= a_ik conj(a_jk) / a_kk  for i >= j > k,   L_ik = a_ik / sqrt(a_kk).
// Column k + 1 becomes final during step k; its owners publish it to LDS (two
// buffers, alternating with the parity of k), and after the barrier every
// thread reads what it needs.  A slot reads LDS only while active (the
// traffic of reading every slot at every step would dominate), but the reads
// of all slots are issued before the first is used.  The entries are numbered
// by column from the last one backwards, so the entries still active at step
// k form a prefix and fill whole waves; within a wave the column index is
// mostly uniform and its reads are broadcasts.
// k_tri_inv: C = L^{-H}, one wave per column of L^{-1} (forward substitution,
// many workgroups in parallel).  The fused single-workgroup form that also
// carried the inverse in the Cholesky sweep measured 101 us at n = 80, the
// two kernels 62 + 23 us (46 + 21 us with two columns per barrier).
constexpr int kCholRegMax = 88;
constexpr int kCholSlots = 4;  // ceil(88 * 89 / 2 / 1024)

__device__ __forceinline__ void tri_index_desc(int e, int n, int* i, int* j) {
  // e-th entry of the lower triangle (incl. diagonal), columns n-1, n-2, ...
  int jj = n - 1, len = 1;
  while (e >= len) {
    e -= len;
    --jj;
    ++len;
  }
  *j = jj;
  *i = jj + e;
}

// 1/sqrt(d) (rsq_refined); then 1/d = y^2 and sqrt(d) = d y.
__device__ __forceinline__ void pivot_terms(double d, double* invr, double* invd, double* r) {
  const double y = rsq_refined(d);
  *invr = y;
  *invd = y * y;
  *r = d * y;
}

// Pivot terms of d (1/sqrt(d), 1/d, sqrt(d)) and a failure flag, to LDS.
__device__ __forceinline__ void publish_pivot(double d, double* pv) {
  const bool ok = d > 0.0 && isfinite(d);
  double invr = 0.0, invd = 0.0, r = 0.0;
  if (ok) pivot_terms(d, &invr, &invd, &r);
  pv[0] = invr;
  pv[1] = invd;
  pv[2] = r;
  pv[3] = ok ? 0.0 : 1.0;
}

// Cholesky only (the inverse follows in k_tri_inv).  Two columns per barrier:
// at the start of step pair (k, k+1) LDS holds column k (final) and column
// k+1 as updated through column k-1; every thread forms the values of column
// k+1 it needs (and the pivot k+1) from those two exactly as their owners
// would, applies both updates to its entries, and the owners of columns k+2
// (final) and k+3 publish them for the next pair.  The operations on every
// entry are those of the one-column sweep, in the same order (the same L bit
// for bit), with half the barriers (measured at n = 80: 57 -> 46 us).  L is
// written once at the end (Lw and the optional Lout; upper triangle zero),
// not column by column inside the loop.
__global__ __launch_bounds__(1024) void k_chol_reg(const cx<double>* __restrict__ M, int n,
                                                   double s, cx<double>* __restrict__ Lw,
                                                   cx<double>* __restrict__ Lout,
                                                   int* __restrict__ info,
                                                   const int* __restrict__ prior, int real_only) {
  constexpr int SL = kCholSlots;
  __shared__ cx<double> colA[2][2][kCholRegMax];
  __shared__ double piv[2][4];
  __shared__ double lscale[kCholRegMax][2];  // per column: 1/sqrt(pivot), sqrt(pivot)
  const int t = threadIdx.x, nt = blockDim.x;
  if (prior && *prior != 0) {
    if (t == 0) *info = *prior;
    return;
  }
  const int tot_a = n * (n + 1) / 2;
  int ai[SL], aj[SL];
  cx<double> a[SL];
#pragma unroll
  for (int q = 0; q < SL; ++q) {
    const int e = t + q * nt;
    ai[q] = aj[q] = 0;  // column 0 is never updated
    if (e < tot_a) tri_index_desc(e, n, &ai[q], &aj[q]);
  }
  cx<double> m1[SL], m2[SL];
#pragma unroll
  for (int q = 0; q < SL; ++q) {
    m1[q] = m2[q] = {0.0, 0.0};
    if (t + q * nt < tot_a) {
      m1[q] = M[ai[q] + (size_t)aj[q] * n];
      m2[q] = M[aj[q] + (size_t)ai[q] * n];
    }
  }
#pragma unroll
  for (int q = 0; q < SL; ++q) {
    a[q] = ai[q] == aj[q] ? cx<double>{s * m1[q].x, 0.0}
           : real_only    ? cx<double>{0.5 * s * (m1[q].x + m2[q].x), 0.0}
                          : cx<double>{0.5 * s * (m1[q].x + m2[q].x), 0.5 * s * (m1[q].y - m2[q].y)};
    if (t + q * nt < tot_a) {
      if (aj[q] == 0) {
        colA[0][0][ai[q]] = a[q];
        if (ai[q] == 0) publish_pivot(a[q].x, piv[0]);
      }
      if (aj[q] == 1) colA[0][1][ai[q]] = a[q];
    }
  }
  __syncthreads();
  int fail_k = 0;
  for (int k = 0; k < n; k += 2) {
    const int p = (k >> 1) & 1;
    const bool two = k + 1 < n;
    const double invr0 = piv[p][0], invd0 = piv[p][1], r0 = piv[p][2], bad0 = piv[p][3];
    if (bad0 != 0.0) {
      fail_k = k + 1;
      break;
    }
    // column k + 1 after the column-k update, as its owners form it
    const cx<double> kk1 = colA[p][0][two ? k + 1 : k];
    auto col1 = [&](int x) {
      const cx<double> u = cmulcj_d(colA[p][0][x], kk1);
      cx<double> v = colA[p][1][x];
      v.x -= u.x * invd0;
      v.y -= u.y * invd0;
      return v;
    };
    double invr1 = 0.0, invd1 = 0.0, r1 = 0.0;
    if (two) {
      const double d1 = col1(k + 1).x;
      if (!(d1 > 0.0 && isfinite(d1))) {
        fail_k = k + 2;
        break;
      }
      pivot_terms(d1, &invr1, &invd1, &r1);
    }
    if (t == 0) {
      lscale[k][0] = invr0;
      lscale[k][1] = r0;
      if (two) {
        lscale[k + 1][0] = invr1;
        lscale[k + 1][1] = r1;
      }
    }
#pragma unroll
    for (int q = 0; q < SL; ++q)
      if (aj[q] > k) {
        {
          const cx<double> u = cmulcj_d(colA[p][0][ai[q]], colA[p][0][aj[q]]);
          a[q].x -= u.x * invd0;
          a[q].y -= u.y * invd0;
        }
        if (aj[q] > k + 1) {
          const cx<double> u = cmulcj_d(col1(ai[q]), col1(aj[q]));
          a[q].x -= u.x * invd1;
          a[q].y -= u.y * invd1;
        }
        if (aj[q] == k + 2) {
          colA[p ^ 1][0][ai[q]] = a[q];
          if (ai[q] == k + 2) publish_pivot(a[q].x, piv[p ^ 1]);
        }
        if (aj[q] == k + 3) colA[p ^ 1][1][ai[q]] = a[q];
      }
    __syncthreads();
  }
  if (t == 0) *info = fail_k;
  if (fail_k) return;
  // L_ij = a_ij / sqrt(pivot_j) below the diagonal, sqrt(pivot_j) on it
#pragma unroll
  for (int q = 0; q < SL; ++q)
    if (t + q * nt < tot_a) {
      const int i = ai[q], j = aj[q];
      const cx<double> l = i == j ? cx<double>{lscale[j][1], 0.0}
                                  : cx<double>{a[q].x * lscale[j][0], a[q].y * lscale[j][0]};
      Lw[i + (size_t)j * n] = l;
      if (Lout) Lout[i + (size_t)j * n] = l;
    }
  for (int e = t; e < n * n; e += nt)
    if (e % n < e / n) {
      Lw[e] = {0.0, 0.0};
      if (Lout) Lout[e] = {0.0, 0.0};
    }
}

__device__ __forceinline__ double bcast_lane(double v, int src) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// C = L^{-H} for n <= kCholRegMax: one wave per column j of X = L^{-1}, the
// lower triangle of L staged in LDS.  Column-oriented forward substitution:
// lane i holds rows i and i + 64 of y = e_j - sum_{m<k} L_:m x_m; at step k
// the owner of row k forms x_k = y_k / L_kk and broadcasts it, and every
// lane subtracts L_ik x_k.  Row j of C is conj(x).
__global__ __launch_bounds__(256) void k_tri_inv(const cx<double>* __restrict__ L, int n,
                                                 cx<double>* __restrict__ C,
                                                 const int* __restrict__ info) {
  __shared__ cx<double> Ls[kCholRegMax * kCholRegMax];
  if (*info != 0) return;
  const int j = blockIdx.x, t = threadIdx.x;
  // columns j .. n-1 (zeros above the diagonal included), staged by all four
  // waves with 32 loads in flight per lane; wave 0 alone then substitutes
  const int nn = n * n;
  for (int e0 = j * n; e0 < nn; e0 += 32 * 256) {
    cx<double> v[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int e = e0 + u * 256 + t;
      v[u] = e < nn ? L[e] : cx<double>{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int e = e0 + u * 256 + t;
      if (e < nn) Ls[e] = v[u];
    }
  }
  __syncthreads();
  if (t >= 64) return;
  const int lane = t;
  const int i0 = lane, i1 = lane + 64;
  cx<double> y0 = {i0 == j ? 1.0 : 0.0, 0.0}, y1 = {i1 == j ? 1.0 : 0.0, 0.0};
  const double inv0 = (i0 >= j && i0 < n) ? 1.0 / Ls[i0 + (size_t)i0 * n].x : 0.0;
  const double inv1 = (i1 >= j && i1 < n) ? 1.0 / Ls[i1 + (size_t)i1 * n].x : 0.0;
  for (int k = lane; k < j; k += 64) C[j + (size_t)k * n] = {0.0, 0.0};
  // rows beyond n and above k read zeros (the staged upper triangle is zero;
  // rows >= n are clamped), so the update needs no branch
  const int r0 = i0 < n ? i0 : n - 1, r1 = i1 < n ? i1 : n - 1;
  // column k of L is read one step ahead (unconditionally; the rows at or
  // above k are masked when used)
  cx<double> n0 = Ls[r0 + j * n], n1 = Ls[r1 + j * n];
  for (int k = j; k < n; ++k) {
    const cx<double> c0 = n0, c1 = n1;
    const int kn = k + 1 < n ? k + 1 : k;
    n0 = Ls[r0 + kn * n];
    n1 = Ls[r1 + kn * n];
    const cx<double> l0 = i0 > k ? c0 : cx<double>{0.0, 0.0};
    const cx<double> l1 = i1 > k && i1 < n ? c1 : cx<double>{0.0, 0.0};
    const cx<double> own = k < 64 ? cx<double>{y0.x * inv0, y0.y * inv0}
                                  : cx<double>{y1.x * inv1, y1.y * inv1};
    const int src = k & 63;  // the same in every lane: a scalar read of the owner's value
    const cx<double> xk = {bcast_lane(own.x, src), bcast_lane(own.y, src)};
    if (lane == src) C[j + (size_t)k * n] = {xk.x, -xk.y};
    const cx<double> u0 = cmul_d(l0, xk), u1 = cmul_d(l1, xk);
    y0.x -= u0.x;
    y0.y -= u0.y;
    y1.x -= u1.x;
    y1.y -= u1.y;
  }
}

__global__ __launch_bounds__(1024) void k_chol_inv_global(const cx<double>* __restrict__ M, int n,
                                                          double s, cx<double>* __restrict__ A,
                                                          cx<double>* __restrict__ Lout,
                                                          cx<double>* __restrict__ C,
                                                          int* __restrict__ info,
                                                          const int* __restrict__ prior,
                                                          int real_only, int do_inverse) {
  chol_inv_body(M, n, s, A, n, A + (size_t)n * n, Lout, C, info, prior, real_only, do_inverse);
}

// C = L^{-H} for kCholRegMax < n <= 64 R, L (lower triangle, column-major,
// leading dimension n) in global memory: one wave per column j of
// X = L^{-1}, many workgroups in parallel (the single-workgroup block inverse
// took most of the factorisation's time at n = 256).  Forward substitution
// y = e_j, x_k = y_k / L_kk, y_i -= L_ik x_k (i > k); lane l holds rows
// l + 64 r.  Column k of L is loaded kTriPrefetch steps ahead (coalesced:
// consecutive rows on consecutive lanes); rows at or above k read zero.  Row
// j of C is conj(x), its entries left of the diagonal zero.
constexpr int kTriPrefetch = 4;
template <int R>
__global__ __launch_bounds__(64) void k_tri_inv_wave(const cx<double>* __restrict__ L, int n,
                                                     cx<double>* __restrict__ C,
                                                     const int* __restrict__ info) {
  if (*info != 0) return;
  const int j = blockIdx.x, lane = threadIdx.x;
  cx<double> y[R];
  double inv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = lane + 64 * r;
    y[r] = {i == j ? 1.0 : 0.0, 0.0};
    inv[r] = (i >= j && i < n) ? 1.0 / L[i + (size_t)i * n].x : 0.0;
  }
  for (int k = lane; k < j; k += 64) C[j + (size_t)k * n] = {0.0, 0.0};
  constexpr int PD = kTriPrefetch;
  cx<double> lc[PD][R];
  // column k of L below the diagonal (zero elsewhere); unconditional loads
  // from a clamped address, masked when used
  auto load_col = [&](cx<double> (&dst)[R], int k) {
    const int kc = k < n ? k : n - 1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = lane + 64 * r;
      const int ic = i < n ? i : n - 1;
      const cx<double> v = L[ic + (size_t)kc * n];
      dst[r] = (i > k && i < n && k < n) ? v : cx<double>{0.0, 0.0};
    }
  };
#pragma unroll
  for (int p = 0; p < PD; ++p) load_col(lc[p], j + p);
  for (int k0 = j; k0 < n; k0 += PD) {
#pragma unroll
    for (int p = 0; p < PD; ++p) {
      const int k = k0 + p;
      if (k >= n) break;  // uniform
      // x_k from the owner of row k (slot k / 64, lane k % 64)
      const int slot = k >> 6;
      cx<double> own = y[0];
      double oinv = inv[0];
#pragma unroll
      for (int r = 1; r < R; ++r)
        if (slot == r) {
          own = y[r];
          oinv = inv[r];
        }
      const int src = k & 63;
      const cx<double> xk = {bcast_lane(own.x * oinv, src), bcast_lane(own.y * oinv, src)};
      if (lane == 0) C[j + (size_t)k * n] = {xk.x, -xk.y};
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const cx<double> u = cmul_d(lc[p][r], xk);
        y[r].x -= u.x;
        y[r].y -= u.y;
      }
      load_col(lc[p], k + PD);
    }
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

}  // namespace

ace_status chol_inv(ace_ctx c, const cx<double>* M, int n, double s, cx<double>* Lout,
                    cx<double>* C, cx<double>* scratch, int* info_dev, const int* prior,
                    bool real_only) {
  if (n <= kCholRegMax) {
    const int need = (n * (n + 1) / 2 + kCholSlots - 1) / kCholSlots;
    const int threads = need < 64 ? 64 : (need + 63) / 64 * 64;
    ace_status st = launch(c, "chol_reg", k_chol_reg, dim3(1), dim3(threads), 0, M, n, s,
                           scratch, Lout, info_dev, prior, real_only ? 1 : 0);
    if (st != ACE_OK) return st;
    return launch(c, "tri_inv", k_tri_inv, dim3(n), dim3(256), 0, (const cx<double>*)scratch, n,
                  C, (const int*)info_dev);
  }
  // up to 512: Cholesky in one workgroup, then C = L^{-H} one wave per column;
  // above: the fused single-workgroup form (the wave form's rows per lane grow
  // with n)
  const int wave_inverse = n <= 512 ? 1 : 0;
  ace_status st = launch(c, "chol_inv_global", k_chol_inv_global, dim3(1), dim3(1024), 0, M, n, s,
                         scratch, Lout, C, info_dev, prior, real_only ? 1 : 0, 1 - wave_inverse);
  if (st != ACE_OK || !wave_inverse) return st;
  const cx<double>* Lw = scratch;
  if (n <= 128)
    return launch(c, "tri_inv_wave", k_tri_inv_wave<2>, dim3(n), dim3(64), 0, Lw, n, C,
                  (const int*)info_dev);
  if (n <= 256)
    return launch(c, "tri_inv_wave", k_tri_inv_wave<4>, dim3(n), dim3(64), 0, Lw, n, C,
                  (const int*)info_dev);
  return launch(c, "tri_inv_wave", k_tri_inv_wave<8>, dim3(n), dim3(64), 0, Lw, n, C,
                (const int*)info_dev);
}

ace_status sumsq(ace_ctx c, const cx<double>* A, long count, double s, double* out) {
  return launch(c, "sumsq", k_sumsq, dim3(1), dim3(1024), 0, A, count, s, out);
}

}  // namespace ace
