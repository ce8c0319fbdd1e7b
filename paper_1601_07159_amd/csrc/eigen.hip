// Building blocks of the linear eigensolver inside the self-consistent loops
// of Section 2 (Alg. 1: the exchange operator applied as V_X[phi] by pair
// Poisson solves) and Section 3 (Alg. 2: the same loop with V_ACE), for a
// Hamiltonian H = -1/2 Laplacian + V_loc + V_ex of the form of Eq. HFlineig
// with a fixed local potential:
//   ace_apply_h        Y = H X, the exchange part V_ACE (from xi), V_X[phi]
//                      (pair solves) or absent;
//   ace_combine        D = a A + b B + c C on orbital blocks (the three-term
//                      recurrences of polynomial filters);
//   ace_rayleigh_ritz  S = dV X^H (HX), S = Q diag(e) Q^H by a parallel
//                      cyclic Jacobi method in one workgroup, X Q and (HX) Q.
// The kinetic term runs on the pair FFT passes: one "orbital" of ones and the
// kernel |G|^2 / 2 make them compute ifftn(|G|^2/2 fftn(x)) for every x.
#include <cmath>
#include <cstdio>

#include "ace_internal.h"

#define ACE_EXPORT extern "C" __attribute__((visibility("default")))

namespace ace {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_fill_ones(cx<T>* __restrict__ x, long ng) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < ng) x[i] = cx<T>{T(1), T(0)};
}

// Y_b[r] += V(r) X_b[r] for b < n (V real, one value per grid point).
template <typename T>
__global__ __launch_bounds__(256) void k_add_local(const cx<T>* __restrict__ X, long ldx,
                                                   const T* __restrict__ V, cx<T>* __restrict__ Y,
                                                   long ldy, long ng, int n) {
  const long total = ng * n;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long b = e / ng, r = e - b * ng;
    const cx<T> x = X[b * ldx + r];
    const T v = V[r];
    cx<T> y = Y[b * ldy + r];
    y.x += v * x.x;
    y.y += v * x.y;
    Y[b * ldy + r] = y;
  }
}

// D_b[r] = a A_b[r] + b B_b[r] + c C_b[r]  (B, C nullable: their term absent).
template <typename T>
__global__ __launch_bounds__(256) void k_combine(double a, const cx<T>* __restrict__ A, long lda,
                                                 double b, const cx<T>* __restrict__ B, long ldb,
                                                 double c, const cx<T>* __restrict__ C, long ldc,
                                                 cx<T>* __restrict__ D, long ldd, long ng, int n) {
  const long total = ng * n;
  const T ta = (T)a, tb = (T)b, tc = (T)c;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long k = e / ng, r = e - k * ng;
    const cx<T> x = A[k * lda + r];
    cx<T> y = {ta * x.x, ta * x.y};
    if (B) {
      const cx<T> u = B[k * ldb + r];
      y.x += tb * u.x;
      y.y += tb * u.y;
    }
    if (C) {
      const cx<T> u = C[k * ldc + r];
      y.x += tc * u.x;
      y.y += tc * u.y;
    }
    D[k * ldd + r] = y;
  }
}

inline unsigned stream_blocks(long total) {
  const long b = (total + 255) / 256;
  return (unsigned)(b < 8192 ? b : 8192);
}

// ---------------------------------------------------------------------------
// Hermitian eigensolver for n <= kJacobiMax, one workgroup of 1024 threads:
// the parallel cyclic Jacobi method (Brent-Luk order).  A sweep visits every
// pair (p, q) once in n - 1 steps (n even; a dummy index pads odd n) of n/2
// disjoint pairs, scheduled by the circle method (index m = n - 1 fixed, the
// others rotating).  Each step computes the n/2 rotations from A, then applies
// them to the rows of A (A <- J^H A), to the columns of A and of V
// (A <- A J, V <- V J); rotations of disjoint pairs commute.  For the pair
// (p, q) with a = A_pp, b = A_qq, A_pq = |c| e^{i phi}: the phase
// D = diag(1, e^{-i phi}) makes the pair block real, then the real rotation
// [[cs, sn], [-sn, cs]] with t = tan(theta) the smaller root of
// t^2 + 2 tau t - 1 = 0, tau = (b - a) / (2 |c|), annihilates it:
//   rows:    p <- cs p - sn e^{i phi} q,   q <- sn p + cs e^{i phi} q
//   columns: p <- cs p - sn e^{-i phi} q,  q <- sn p + cs e^{-i phi} q.
// Sweeps stop when the off-diagonal Frobenius norm falls below tol times the
// whole norm (or after max_sweeps).  The eigenvalues (real parts of the final
// diagonal) are sorted ascending, ties by index, and the columns of V follow.
// A is kept in LDS up to kJacobiLds rows, in global scratch beyond.
constexpr int kJacobiMax = 512;
constexpr int kJacobiLds = 88;  // 88^2 complex128 = 121 KiB of LDS

struct JacobiRot {
  int p, q;
  double cs, sn, er, ei;  // cosine, sine, e^{i phi}
};

template <bool LDS>
__global__ __launch_bounds__(1024) void k_jacobi_eigh(const cx<double>* __restrict__ S, int lds_,
                                                      int n, cx<double>* __restrict__ Ag,
                                                      cx<double>* __restrict__ V,
                                                      cx<double>* __restrict__ Vout, int ldv,
                                                      double* __restrict__ evals, int max_sweeps,
                                                      double tol) {
  __shared__ cx<double> a_lds[LDS ? kJacobiLds * kJacobiLds : 1];
  __shared__ JacobiRot rot[kJacobiMax / 2];
  __shared__ double red[1024];
  __shared__ int stop;
  const int t = threadIdx.x, nt = blockDim.x;
  const int lda = LDS ? kJacobiLds : n;
  cx<double>* A = LDS ? a_lds : Ag;
  // A = (S + S^H)/2, V = I
  for (int e = t; e < n * n; e += nt) {
    const int i = e % n, j = e / n;
    const cx<double> u = S[i + (size_t)j * lds_], w = S[j + (size_t)i * lds_];
    A[i + j * lda] = {0.5 * (u.x + w.x), 0.5 * (u.y - w.y)};
    V[i + (size_t)j * ldv] = {i == j ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  const int ne = n + (n & 1);  // players; index n is the dummy when n is odd
  const int m = ne - 1, np = ne / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // convergence: off-diagonal vs whole Frobenius norm
    double off = 0.0, all = 0.0;
    for (int e = t; e < n * n; e += nt) {
      const int i = e % n, j = e / n;
      const cx<double> u = A[i + j * lda];
      const double v = u.x * u.x + u.y * u.y;
      all += v;
      if (i != j) off += v;
    }
    red[t] = off;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if (t < w) red[t] += red[t + w];
      __syncthreads();
    }
    const double off_sum = red[0];
    __syncthreads();
    red[t] = all;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if (t < w) red[t] += red[t + w];
      __syncthreads();
    }
    if (t == 0) stop = !(off_sum > tol * tol * red[0]);
    __syncthreads();
    if (stop) break;
    for (int st = 0; st < m; ++st) {
      // the step's pairs: (st, m) and (st + k, st - k) mod m for k = 1 .. np - 1
      for (int k = t; k < np; k += nt) {
        int p, q;
        if (k == 0) {
          p = st;
          q = m;
        } else {
          p = (st + k) % m;
          q = (st - k + m) % m;
        }
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        JacobiRot r{p, q, 1.0, 0.0, 1.0, 0.0};
        if (q < n) {
          const double a = A[p + p * lda].x, b = A[q + q * lda].x;
          const cx<double> c = A[p + q * lda];
          const double ac = sqrt(c.x * c.x + c.y * c.y);
          if (ac > 1e-300 && ac > 1e-18 * sqrt(fabs(a * b))) {
            const double tau = (b - a) / (2.0 * ac);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            r.cs = 1.0 / sqrt(1.0 + tt * tt);
            r.sn = tt * r.cs;
            r.er = c.x / ac;
            r.ei = c.y / ac;
          }
        }
        rot[k] = r;
      }
      __syncthreads();
      // rows: A <- J^H A
      for (int e = t; e < np * n; e += nt) {
        const int k = e / n, col = e - k * n;
        const JacobiRot r = rot[k];
        if (r.q >= n || r.sn == 0.0) continue;
        const cx<double> ap = A[r.p + col * lda], aq = A[r.q + col * lda];
        // e^{i phi} aq
        const cx<double> eq = {r.er * aq.x - r.ei * aq.y, r.er * aq.y + r.ei * aq.x};
        A[r.p + col * lda] = {r.cs * ap.x - r.sn * eq.x, r.cs * ap.y - r.sn * eq.y};
        A[r.q + col * lda] = {r.sn * ap.x + r.cs * eq.x, r.sn * ap.y + r.cs * eq.y};
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int e = t; e < np * n; e += nt) {
        const int k = e / n, row = e - k * n;
        const JacobiRot r = rot[k];
        if (r.q >= n || r.sn == 0.0) continue;
        {
          const cx<double> ap = A[row + r.p * lda], aq = A[row + r.q * lda];
          // e^{-i phi} aq
          const cx<double> eq = {r.er * aq.x + r.ei * aq.y, r.er * aq.y - r.ei * aq.x};
          A[row + r.p * lda] = {r.cs * ap.x - r.sn * eq.x, r.cs * ap.y - r.sn * eq.y};
          A[row + r.q * lda] = {r.sn * ap.x + r.cs * eq.x, r.sn * ap.y + r.cs * eq.y};
        }
        {
          const cx<double> vp = V[row + (size_t)r.p * ldv], vq = V[row + (size_t)r.q * ldv];
          const cx<double> eq = {r.er * vq.x + r.ei * vq.y, r.er * vq.y - r.ei * vq.x};
          V[row + (size_t)r.p * ldv] = {r.cs * vp.x - r.sn * eq.x, r.cs * vp.y - r.sn * eq.y};
          V[row + (size_t)r.q * ldv] = {r.sn * vp.x + r.cs * eq.x, r.sn * vp.y + r.cs * eq.y};
        }
      }
      __syncthreads();
    }
  }
  // sort: rank of eigenvalue i among all (ascending, ties by index)
  for (int i = t; i < n; i += nt) {
    const double ei = A[i + i * lda].x;
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double ej = A[j + j * lda].x;
      rank += (ej < ei || (ej == ei && j < i)) ? 1 : 0;
    }
    evals[rank] = ei;
    for (int r = 0; r < n; ++r) Vout[r + (size_t)rank * ldv] = V[r + (size_t)i * ldv];
  }
}

}  // namespace

// Y = H X with H = -1/2 Laplacian + V_loc + V_ex (see ace_apply_h).
template <typename T>
ace_status hamiltonian_t(ace_ctx c, const GridInfo& g, const T* vloc, const cx<T>* xi, int nxi,
                         long ldxi, const cx<T>* phi, int nphi, long ldphi, double scale_x,
                         const cx<T>* X, int nx, long ldx, cx<T>* Y, long ldy) {
  ace_status st = ACE_OK;
  bool have = false;  // Y holds a term already
  if (xi) {
    // V_ACE X = -xi (dV xi^H X)
    const size_t mat = align_up((size_t)nxi * nx * sizeof(cx<double>), 256);
    ACE_TRY(ws_begin(c, mat + gemm_cn_partial_bytes(nxi, nx, g.ng, sizeof(cx<T>), kNative, false)));
    cx<double>* C = (cx<double>*)ws_take(c, mat, &st);
    if (!C) return st;
    ACE_TRY(gemm_cn<T>(c, xi, ldxi, nxi, X, ldx, nx, g.ng, -g.dV, C, nxi, kNative));
    ACE_TRY(gemm_nn<T>(c, xi, ldxi, nxi, C, nxi, nx, Y, ldy, g.ng, false));
    have = true;
  } else if (phi) {
    // scale_x V_X[phi] X by pair Poisson solves
    ACE_TRY(build_W_impl<T>(c, g, phi, nphi, ldphi, X, nx, ldx, Y, ldy, scale_x));
    have = true;
  }
  // kinetic term through the pair passes: one orbital of ones, kernel |G|^2/2;
  // the ones sit in a workspace prefix that the build's own pieces skip
  GridInfo gk = g;
  gk.kind = kKindKinetic;
  const size_t ones_bytes = align_up((size_t)g.ng * sizeof(cx<T>), 256);
  const BuildPlan pl = plan_build(c, gk, sizeof(cx<T>), 1, nx, false);
  ACE_TRY(ws_begin(c, ones_bytes + pl.bytes));
  cx<T>* ones = (cx<T>*)ws_take(c, (size_t)g.ng * sizeof(cx<T>), &st);
  if (!ones) return st;
  ACE_TRY(launch(c, "fill_ones", k_fill_ones<T>, dim3((unsigned)((g.ng + 255) / 256)), dim3(256),
                 0, ones, g.ng));
  c->ws_prefix = ones_bytes;
  st = build_W_impl<T>(c, gk, ones, 1, g.ng, X, nx, ldx, Y, ldy, -1.0, nullptr, have);
  c->ws_prefix = 0;
  if (st != ACE_OK) return st;
  if (vloc)
    ACE_TRY(launch(c, "add_local", k_add_local<T>, dim3(stream_blocks((long)g.ng * nx)), dim3(256),
                   0, X, ldx, vloc, Y, ldy, g.ng, nx));
  return ACE_OK;
}

size_t hamiltonian_ws_bytes(ace_ctx c, const GridInfo& g, size_t eb, int nx, int nxi, int nphi) {
  GridInfo gk = g;
  gk.kind = kKindKinetic;
  size_t need = align_up((size_t)g.ng * eb, 256) + plan_build(c, gk, eb, 1, nx, false).bytes;
  if (nxi > 0)
    need = std::max(need, align_up((size_t)nxi * nx * sizeof(cx<double>), 256) +
                              gemm_cn_partial_bytes(nxi, nx, g.ng, eb, kNative, false));
  if (nphi > 0) need = std::max(need, plan_build(c, g, eb, nphi, nx, false).bytes);
  return need;
}

namespace {

template <typename T>
ace_status rayleigh_ritz_t(ace_ctx c, const GridInfo& g, const cx<T>* X, long ldx,
                           const cx<T>* HX, long ldhx, int n, cx<T>* Xout, cx<T>* HXout,
                           long ldo, double* evals) {
  const size_t mat = align_up((size_t)n * n * sizeof(cx<double>), 256);
  ACE_TRY(ws_begin(c, 4 * mat + gemm_cn_scratch_bytes(n, n, g.ng)));
  ace_status st = ACE_OK;
  cx<double>* S = (cx<double>*)ws_take(c, mat, &st);
  cx<double>* A = (cx<double>*)ws_take(c, mat, &st);
  cx<double>* V = (cx<double>*)ws_take(c, mat, &st);
  cx<double>* Q = (cx<double>*)ws_take(c, mat, &st);
  if (!S || !A || !V || !Q) return st;
  // S = dV X^H (H X), Hermitian for Hermitian H: upper tiles, lower mirrored
  ACE_TRY(gemm_cn<T>(c, X, ldx, n, HX, ldhx, n, g.ng, g.dV, S, n,
                     sizeof(T) == 8 ? kNative : kFp64, false, true));
  if (n <= kJacobiLds)
    ACE_TRY(launch(c, "jacobi_eigh", k_jacobi_eigh<true>, dim3(1), dim3(1024), 0,
                   (const cx<double>*)S, n, n, A, V, Q, n, evals, 30, 1e-15));
  else
    ACE_TRY(launch(c, "jacobi_eigh", k_jacobi_eigh<false>, dim3(1), dim3(1024), 0,
                   (const cx<double>*)S, n, n, A, V, Q, n, evals, 30, 1e-15));
  ACE_TRY(gemm_nn<T>(c, X, ldx, n, Q, n, n, Xout, ldo, g.ng, true));
  if (HXout) ACE_TRY(gemm_nn<T>(c, HX, ldhx, n, Q, n, n, HXout, ldo, g.ng, true));
  return ACE_OK;
}

}  // namespace
}  // namespace ace

using namespace ace;

ACE_EXPORT ace_status ace_apply_h(ace_ctx c, const ace_grid* grid, ace_prec prec, const void* vloc,
                                  const void* xi, int n_xi, long ld_xi, const void* phi,
                                  int n_phi, long ld_phi, double scale_x, const void* X, int n_x,
                                  long ld_x, void* Y, long ld_y) {
  if (!c) return ACE_E_ARG;
  GridInfo g;
  ACE_TRY(check_grid(c, grid, prec, &g));
  if (prec == ACE_REAL32 || prec == ACE_REAL64)
    return fail(c, ACE_E_UNSUPPORTED, "ace_apply_h takes complex orbitals");
  if (xi && phi) return fail(c, ACE_E_ARG, "give xi (V_ACE) or phi (V_X), not both");
  ACE_TRY(check_block(c, X, n_x, ld_x, g, "X"));
  ACE_TRY(check_block(c, Y, n_x, ld_y, g, "Y"));
  if (xi) ACE_TRY(check_block(c, xi, n_xi, ld_xi, g, "xi"));
  if (phi) ACE_TRY(check_block(c, phi, n_phi, ld_phi, g, "phi"));
  if (!std::isfinite(scale_x)) return fail(c, ACE_E_ARG, "scale_x must be finite");
  const size_t eb = elem_bytes(prec);
  const Span sy = span_of(Y, n_x, ld_y, g.ng, eb);
  if (overlap(sy, span_of(X, n_x, ld_x, g.ng, eb)) ||
      (xi && overlap(sy, span_of(xi, n_xi, ld_xi, g.ng, eb))) ||
      (phi && overlap(sy, span_of(phi, n_phi, ld_phi, g.ng, eb))))
    return fail(c, ACE_E_ARG, "Y overlaps an input");
  if (prec == ACE_FP64)
    return hamiltonian_t<double>(c, g, (const double*)vloc, (const cx<double>*)xi, n_xi, ld_xi,
                                 (const cx<double>*)phi, n_phi, ld_phi, scale_x,
                                 (const cx<double>*)X, n_x, ld_x, (cx<double>*)Y, ld_y);
  return hamiltonian_t<float>(c, g, (const float*)vloc, (const cx<float>*)xi, n_xi, ld_xi,
                              (const cx<float>*)phi, n_phi, ld_phi, scale_x, (const cx<float>*)X,
                              n_x, ld_x, (cx<float>*)Y, ld_y);
}

ACE_EXPORT ace_status ace_combine(ace_ctx c, const ace_grid* grid, ace_prec prec, int n, double a,
                                  const void* A, long lda, double b, const void* B, long ldb,
                                  double cc, const void* C, long ldc, void* D, long ldd) {
  if (!c) return ACE_E_ARG;
  GridInfo g;
  ACE_TRY(check_grid(c, grid, prec, &g));
  if (prec == ACE_REAL32 || prec == ACE_REAL64)
    return fail(c, ACE_E_UNSUPPORTED, "ace_combine takes complex orbitals");
  if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(cc))
    return fail(c, ACE_E_ARG, "coefficients must be finite");
  ACE_TRY(check_block(c, A, n, lda, g, "A"));
  ACE_TRY(check_block(c, D, n, ldd, g, "D"));
  if (B) ACE_TRY(check_block(c, B, n, ldb, g, "B"));
  if (C) ACE_TRY(check_block(c, C, n, ldc, g, "C"));
  const dim3 grd(stream_blocks((long)g.ng * n));
  if (prec == ACE_FP64)
    return launch(c, "combine", k_combine<double>, grd, dim3(256), 0, a, (const cx<double>*)A, lda,
                  b, (const cx<double>*)B, ldb, cc, (const cx<double>*)C, ldc, (cx<double>*)D, ldd,
                  g.ng, n);
  return launch(c, "combine", k_combine<float>, grd, dim3(256), 0, a, (const cx<float>*)A, lda, b,
                (const cx<float>*)B, ldb, cc, (const cx<float>*)C, ldc, (cx<float>*)D, ldd, g.ng,
                n);
}

ACE_EXPORT ace_status ace_rayleigh_ritz(ace_ctx c, const ace_grid* grid, ace_prec prec,
                                        const void* X, long ld_x, const void* HX, long ld_hx,
                                        int n, void* Xout, void* HXout, long ld_out,
                                        double* evals_dev) {
  if (!c) return ACE_E_ARG;
  GridInfo g;
  ACE_TRY(check_grid(c, grid, prec, &g));
  if (prec == ACE_REAL32 || prec == ACE_REAL64)
    return fail(c, ACE_E_UNSUPPORTED, "ace_rayleigh_ritz takes complex orbitals");
  if (n < 1 || n > kJacobiMax) return fail(c, ACE_E_UNSUPPORTED, "n must be 1..512");
  if (!evals_dev) return fail(c, ACE_E_ARG, "evals_dev is NULL");
  ACE_TRY(check_block(c, X, n, ld_x, g, "X"));
  ACE_TRY(check_block(c, HX, n, ld_hx, g, "HX"));
  ACE_TRY(check_block(c, Xout, n, ld_out, g, "Xout"));
  if (HXout) ACE_TRY(check_block(c, HXout, n, ld_out, g, "HXout"));
  const size_t eb = elem_bytes(prec);
  const Span ins[2] = {span_of(X, n, ld_x, g.ng, eb), span_of(HX, n, ld_hx, g.ng, eb)};
  const Span so = span_of(Xout, n, ld_out, g.ng, eb);
  if (overlap(so, ins[0]) || overlap(so, ins[1]) ||
      (HXout && (overlap(span_of(HXout, n, ld_out, g.ng, eb), ins[0]) ||
                 overlap(span_of(HXout, n, ld_out, g.ng, eb), ins[1]) ||
                 overlap(span_of(HXout, n, ld_out, g.ng, eb), so))))
    return fail(c, ACE_E_ARG, "outputs overlap inputs or each other");
  if (prec == ACE_FP64)
    return rayleigh_ritz_t<double>(c, g, (const cx<double>*)X, ld_x, (const cx<double>*)HX, ld_hx,
                                   n, (cx<double>*)Xout, (cx<double>*)HXout, ld_out, evals_dev);
  return rayleigh_ritz_t<float>(c, g, (const cx<float>*)X, ld_x, (const cx<float>*)HX, ld_hx, n,
                                (cx<float>*)Xout, (cx<float>*)HXout, ld_out, evals_dev);
}
