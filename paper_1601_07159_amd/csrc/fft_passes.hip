// Pair Poisson solves of the exchange operator (Section 2, Eq. applyVX2;
// Section 3, Eq. W): for every pair (i, j)
//     u_ij = ifftn( K * fftn( conj(phi_i) psi_j ) ),   w_j += phi_i * u_ij.
//
// A 3-D FFT of an N^3 field does not fit on one compute unit, so each pair
// crosses HBM three times:
//   slab pass (forward)   one workgroup per (x0 slab, pair): the pair product is
//                         formed while the slab is loaded, then 2-D FFT over
//                         axes 2 and 1 in LDS; spectrum slab written out.
//   plane pass            one workgroup per (k1 plane, pair): along axis 0 the
//                         forward FFT, the multiply by the scaled kernel and
//                         the inverse FFT, then the inverse FFT along axis 2,
//                         all through LDS.
//   pencil pass           one thread per (x0, x2) pencil along axis 1, lanes
//                         on consecutive pencils: loops over the occupied
//                         orbitals i of the block, inverse FFT, multiply by
//                         phi_i, accumulate in thread-private LDS; w_j is
//                         written once per block (no atomics, no barriers).
// The 1/N_g of the inverse transform, the minus sign and the caller's scale are
// folded into the scaled kernel K'(G) = -scale K(G) / N_g, evaluated on the fly
// in the plane pass from the per-axis factors (2 pi / L_a)^2 (no N_g table).
#include <cmath>

#include <vector>

#include "ace_internal.h"
#include "pass_bodies.h"

namespace ace {

namespace {


// Forward slab pass: one group of N threads per (x0, pair).
template <int N, typename T, int P>
__global__ __launch_bounds__(N * P) void k_pair_fwd_slab_t1(const cx<T>* __restrict__ phi, long ldphi,
                                                         const cx<T>* __restrict__ psi, long ldpsi,
                                                         cx<T>* __restrict__ buf, int mode, int i0,
                                                         int A, int j0, long p0, int npairs) {
  __shared__ cx<T> s_all[P * N * (N + 1)];
  const long total = (long)N * npairs;
  const long lid0 = xcd_logical(blockIdx.x, gridDim.x) * P;
  if (lid0 >= total) return;  // the whole workgroup
  slab_t1_body<N, T, P>(s_all, (int)threadIdx.x, false, lid0, total, phi, ldphi, psi, ldpsi, buf,
                        mode, i0, A, j0, p0, npairs);
}

// Plane pass: one group of N threads per (k1 plane, pair).
template <int N, typename T, int P>
__global__ __launch_bounds__(N * P) void k_plane_kernel_t1(cx<T>* __restrict__ buf,
                                                        ace_kspec ks, int npairs) {
  __shared__ cx<T> s_all[P * N * (N + 1)];
  const long total = (long)N * npairs;
  const long lid0 = xcd_logical(blockIdx.x, gridDim.x) * P;
  if (lid0 >= total) return;  // the whole workgroup
  plane_t1_body<N, T, P>(s_all, (int)threadIdx.x, false, lid0, total, buf, ks, npairs);
}

// The slab and plane passes split every line FFT over the 4 lanes of a quad
// (fft_quad_*): a workgroup of 4N threads handles an N x N slab or plane (line
// l = t / 4, quad lane h = t % 4).  LDS rows are kQuadLd(N) elements apart with
// kQuadLd = 4 (mod 16): a 16-lane phase of an 8-byte access then touches 4
// lines x 4 quad lanes in distinct banks, for row reads (l LD + h + 4m) and
// column reads ((h + 4m) LD + l) alike.
template <int N>
constexpr int kQuadLd = N + ((4 - N % 16) + 16) % 16;
// Whether the quad forms stage their strided global accesses through LDS (the
// plane's column loads, the slab's spectrum stores) so that every access
// instruction covers whole rows: measured at N = 64 (plane pass 1.33 -> 1.23
// ms per 640 pairs), but at N = 72, whose 48 KiB plane leaves 4.5 waves per
// workgroup and three workgroups per CU, the two extra barriers cost more
// (plane 2.33 -> 3.33 ms, slab 2.08 -> 2.44 ms per 1,146 pairs).
template <int N>
constexpr bool kQuadStage = N <= 64;

// Forward slab pass: one workgroup per (x0 slab, pair).  The pair product
// conj(phi_i) psi_j is formed while the slab is loaded (coalesced) into LDS;
// 2-D FFT over axis 2 (rows) then axis 1 (columns); the column results go
// straight to global memory, lanes on consecutive columns.
template <int N, typename T>
__global__ __launch_bounds__(4 * N) void k_pair_fwd_slab(const cx<T>* __restrict__ phi, long ldphi,
                                                         const cx<T>* __restrict__ psi, long ldpsi,
                                                         cx<T>* __restrict__ buf, int mode, int i0,
                                                         int A, int j0, long p0, int npairs) {
  constexpr int NN = N * N;
  constexpr int LD = kQuadLd<N>;
  constexpr int M = N / 4;
  __shared__ cx<T> s[N * LD];
  const long lid = xcd_logical(blockIdx.x, gridDim.x);
  if (lid >= (long)N * npairs) return;
  const int x0 = (int)(lid / npairs);
  const int p = (int)(lid - (long)x0 * npairs);
  int i, j;
  pair_of(mode, i0, A, j0, p0, p, &i, &j);
  const cx<T>* a = phi + (size_t)i * ldphi + (size_t)x0 * NN;
  const cx<T>* b = psi + (size_t)j * ldpsi + (size_t)x0 * NN;
  const int t = threadIdx.x;
  const int l = t >> 2, h = t & 3;
  const int rr = t / N, cc = t - rr * N;  // element t + 4N q sits at row 4q + rr, column cc
  cx<T> v[M];
  if constexpr (kQuadStage<N>) {
    cx<T> va[M], vb[M];
#pragma unroll
    for (int q = 0; q < M; ++q) va[q] = a[(4 * q + rr) * N + cc];
#pragma unroll
    for (int q = 0; q < M; ++q) vb[q] = b[(4 * q + rr) * N + cc];
#pragma unroll
    for (int q = 0; q < M; ++q) s[(4 * q + rr) * LD + cc] = cmulc(va[q], vb[q]);
    __syncthreads();
    // axis 2: row l
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = s[l * LD + h + 4 * m];
  } else {
    // row l of the pair product straight from global memory, decimated over
    // the quad (each 16 lanes read 4 rows x 32 contiguous bytes; the rest of
    // those lines are read by the next loads): no LDS pass and no barrier
    // before the row transform
    cx<T> va[M], vb[M];
#pragma unroll
    for (int m = 0; m < M; ++m) va[m] = a[l * N + h + 4 * m];
#pragma unroll
    for (int m = 0; m < M; ++m) vb[m] = b[l * N + h + 4 * m];
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = cmulc(va[m], vb[m]);
  }
  fft_quad_d2b<N, -1, T>(v, h);
#pragma unroll
  for (int k = 0; k < M; ++k) s[l * LD + quad_block_index(k, M, h)] = v[k];
  __syncthreads();
  // axis 1: column l
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = s[(h + 4 * m) * LD + l];
  fft_quad_d2b<N, -1, T>(v, h);
  if constexpr (kQuadStage<N>) {
    // the spectrum slab leaves through LDS, so that every store instruction
    // writes whole rows (a quad's direct stores cover 4 rows x 4 values per
    // 16 lanes)
    __syncthreads();
#pragma unroll
    for (int k = 0; k < M; ++k) s[quad_block_index(k, M, h) * LD + l] = v[k];
    __syncthreads();
    cx<T>* out = buf + (size_t)p * N * NN + (size_t)x0 * NN;
#pragma unroll
    for (int q = 0; q < M; ++q) store_nt(&out[(4 * q + rr) * N + cc], s[(4 * q + rr) * LD + cc]);
  } else {
    // plain stores: a quad writes 4 rows x 4 values per 16 lanes, and
    // streaming stores of such 32-byte pieces bypass the L2's write combining
    // (at N = 72 they wrote 1.23x the spectrum bytes; plain stores 2.08 ->
    // 2.01 ms per 1,146 pairs)
    cx<T>* out = buf + (size_t)p * N * NN + (size_t)x0 * NN + l;
#pragma unroll
    for (int k = 0; k < M; ++k) out[quad_block_index(k, M, h) * N] = v[k];
  }
}

// Plane pass: one workgroup per (k1 plane, pair).  Along axis 0 (column l of
// the plane, read straight from global memory): forward FFT, multiply by K',
// inverse FFT; then through LDS the inverse FFT along axis 2 (row l); coalesced
// store of the plane.
template <int N, typename T>
__global__ __launch_bounds__(4 * N) void k_plane_kernel(cx<T>* __restrict__ buf,
                                                        ace_kspec ks, int npairs) {
  constexpr int NN = N * N;
  constexpr int LD = kQuadLd<N>;
  constexpr int M = N / 4;
  __shared__ cx<T> s[N * LD];
  const long lid = xcd_logical(blockIdx.x, gridDim.x);
  if (lid >= (long)N * npairs) return;
  // planes of one pair on neighbouring workgroups: at every k0 their rows
  // form one contiguous N^2 run of the spectrum (the pairs share no input)
  const int p = (int)(lid / N);
  const int k1 = (int)(lid - (long)p * N);
  const int t = threadIdx.x;
  const int l = t >> 2, h = t & 3;
  cx<T>* plane = buf + (size_t)p * N * NN + (size_t)k1 * N;
  const int rr = t / N, cc = t - rr * N;  // element t + 4N q sits at row 4q + rr, column cc
  cx<T> v[M];
  if constexpr (kQuadStage<N>) {
    // the plane comes in through LDS, so that every load instruction reads
    // whole rows (a quad's direct column loads cover 4 rows x 4 values per
    // 16 lanes)
    {
      cx<T> w[M];
#pragma unroll
      for (int q = 0; q < M; ++q) w[q] = plane[(size_t)(4 * q + rr) * NN + cc];
#pragma unroll
      for (int q = 0; q < M; ++q) s[(4 * q + rr) * LD + cc] = w[q];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = s[(h + 4 * m) * LD + l];
  } else {
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = plane[(size_t)(h + 4 * m) * NN + l];
  }
  fft_quad_d2b<N, -1, T>(v, h);
  {
    const KEval<T> ke(ks);
    const T s12 = ke.part12(k1, l);
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const T kk = ke.at(quad_block_index(k, M, h), s12);
      v[k].x *= kk;
      v[k].y *= kk;
    }
  }
  fft_quad_b2d<N, +1, T>(v, h);
  if constexpr (kQuadStage<N>) __syncthreads();  // every column read before any is rewritten
#pragma unroll
  for (int m = 0; m < M; ++m) s[(h + 4 * m) * LD + l] = v[m];
  __syncthreads();
  if constexpr (kQuadStage<N>) {
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = s[l * LD + h + 4 * m];
    fft_quad_d2b<N, +1, T>(v, h);
    // row l is read and rewritten by its own quad only (one wave, in order)
#pragma unroll
    for (int k = 0; k < M; ++k) s[l * LD + quad_block_index(k, M, h)] = v[k];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < M; ++q) plane[(size_t)(4 * q + rr) * NN + cc] = s[(4 * q + rr) * LD + cc];
  } else {
    // row l read in block layout, transformed to the decimated one, and
    // stored straight from registers (each 16 lanes write 4 rows x 32
    // contiguous bytes; a wave's 18 stores complete its 16 rows): no second
    // LDS pass and no barrier
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = s[l * LD + quad_block_index(k, M, h)];
    fft_quad_b2d<N, +1, T>(v, h);
    cx<T>* row = plane + (size_t)l * NN + h;
#pragma unroll
    for (int m = 0; m < M; ++m) row[4 * m] = v[m];
  }
}

// Split-line forms of the slab and plane passes: every line FFT is split over
// 4 lanes 16 apart (fft_quad_* with lane distance 16: lane p + 16 h of wave w
// holds part h of line l = 16 w + p), so 16 consecutive lanes hold the same
// part of 16 consecutive lines and every global access of 16 lanes is one
// contiguous row segment.  A workgroup of kRowWaves = ceil(N / 16) waves
// handles an N x N slab or plane; lines l >= N (N = 8, 12, 24, 40, 72) are
// idle: they take part in the lane exchanges on clamped data and store
// nothing.  The coalesced flat loads and stores of the plane use the first 4 N
// threads.  LDS rows are kRowLd(N) elements apart, an odd number, so that 16
// lines at one offset fall in distinct banks.
template <int N>
constexpr int kRowWaves = (N + 15) / 16;
template <int N>
constexpr int kRowLd = N + 1 - (N & 1);

// Forward slab pass: one workgroup per (x0 slab, pair).  The pair product
// conj(phi_i) psi_j is formed while the slab is loaded (coalesced) into LDS;
// 2-D FFT over axis 2 (rows) then axis 1 (columns); the column results go
// straight to global memory, 16 lanes on consecutive columns.
template <int N, typename T>
__global__ __launch_bounds__(64 * kRowWaves<N>) void k_pair_fwd_slab_row(
    const cx<T>* __restrict__ phi, long ldphi, const cx<T>* __restrict__ psi, long ldpsi,
    cx<T>* __restrict__ buf, int mode, int i0, int A, int j0, long p0, int npairs) {
  constexpr int NN = N * N;
  constexpr int LD = kRowLd<N>;
  constexpr int M = N / 4;
  __shared__ cx<T> s[N * LD];
  const long lid = xcd_logical(blockIdx.x, gridDim.x);
  if (lid >= (long)N * npairs) return;
  const int x0 = (int)(lid / npairs);
  const int p = (int)(lid - (long)x0 * npairs);
  int i, j;
  pair_of(mode, i0, A, j0, p0, p, &i, &j);
  const cx<T>* a = phi + (size_t)i * ldphi + (size_t)x0 * NN;
  const cx<T>* b = psi + (size_t)j * ldpsi + (size_t)x0 * NN;
  const int t = threadIdx.x;
  const int h = (t >> 4) & 3;
  const int l = ((t >> 6) << 4) + (t & 15);
  const bool live = l < N;
  const int lc = live ? l : N - 1;
  if (t < 4 * N) {
    const int rr = t / N, cc = t - rr * N;  // element t + 4N q sits at row 4q + rr, column cc
    cx<T> va[M], vb[M];
#pragma unroll
    for (int q = 0; q < M; ++q) va[q] = a[(4 * q + rr) * N + cc];
#pragma unroll
    for (int q = 0; q < M; ++q) vb[q] = b[(4 * q + rr) * N + cc];
#pragma unroll
    for (int q = 0; q < M; ++q) s[(4 * q + rr) * LD + cc] = cmulc(va[q], vb[q]);
  }
  __syncthreads();
  cx<T> v[M];
  // axis 2: row l (read and rewritten by its own four lanes only: one wave)
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = s[lc * LD + h + 4 * m];
  fft_quad_d2b<N, -1, T, 16>(v, h);
  if (live) {
#pragma unroll
    for (int k = 0; k < M; ++k) s[l * LD + quad_block_index(k, M, h)] = v[k];
  }
  __syncthreads();
  // axis 1: column l
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = s[(h + 4 * m) * LD + lc];
  fft_quad_d2b<N, -1, T, 16>(v, h);
  if (!live) return;
  cx<T>* out = buf + (size_t)p * N * NN + (size_t)x0 * NN + l;
#pragma unroll
  for (int k = 0; k < M; ++k) store_nt(&out[quad_block_index(k, M, h) * N], v[k]);
}

// Plane pass: one workgroup per (k1 plane, pair).  Along axis 0 (column l of
// the plane, read straight from global memory): forward FFT, multiply by K',
// inverse FFT; then through LDS the inverse FFT along axis 2 (row l); coalesced
// store of the plane.
template <int N, typename T>
__global__ __launch_bounds__(64 * kRowWaves<N>) void k_plane_kernel_row(cx<T>* __restrict__ buf,
                                                                   ace_kspec ks, int npairs) {
  constexpr int NN = N * N;
  constexpr int LD = kRowLd<N>;
  constexpr int M = N / 4;
  __shared__ cx<T> s[N * LD];
  const long lid = xcd_logical(blockIdx.x, gridDim.x);
  if (lid >= (long)N * npairs) return;
  const int p = (int)(lid / N);  // pair-major, as in the quad plane pass
  const int k1 = (int)(lid - (long)p * N);
  const int t = threadIdx.x;
  const int h = (t >> 4) & 3;
  const int l = ((t >> 6) << 4) + (t & 15);
  const bool live = l < N;
  const int lc = live ? l : N - 1;
  cx<T>* plane = buf + (size_t)p * N * NN + (size_t)k1 * N;
  cx<T> v[M];
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = plane[(size_t)(h + 4 * m) * NN + lc];
  fft_quad_d2b<N, -1, T, 16>(v, h);
  {
    const KEval<T> ke(ks);
    const T s12 = ke.part12(k1, lc);
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const T kk = ke.at(quad_block_index(k, M, h), s12);
      v[k].x *= kk;
      v[k].y *= kk;
    }
  }
  fft_quad_b2d<N, +1, T, 16>(v, h);
  if (live) {
#pragma unroll
    for (int m = 0; m < M; ++m) s[(h + 4 * m) * LD + l] = v[m];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = s[lc * LD + h + 4 * m];
  fft_quad_d2b<N, +1, T, 16>(v, h);
  // row l is read and rewritten by its own four lanes only (one wave, in
  // order; idle lanes read a clamped row of their own wave)
  if (live) {
#pragma unroll
    for (int k = 0; k < M; ++k) s[l * LD + quad_block_index(k, M, h)] = v[k];
  }
  __syncthreads();
  if (t < 4 * N) {
    const int rr = t / N, cc = t - rr * N;
#pragma unroll
    for (int q = 0; q < M; ++q) plane[(size_t)(4 * q + rr) * NN + cc] = s[(4 * q + rr) * LD + cc];
  }
}

// Octet forms of the slab and plane passes (N = 8 M lines over the 8 lanes of
// an octet: 8N threads, line l = t / 8, lane h = t % 8).  LDS rows are kOctLd
// apart with kOctLd = 2 (mod 16): a 16-lane phase of an 8-byte column access
// (h + 8m) LD + l then touches 16 distinct banks; row accesses l LD + h + 8m
// of two lines overlap in at most 6 of them.
template <int N>
constexpr int kOctLd = N + ((2 - N % 16) + 16) % 16;

template <int N, typename T>
__global__ __launch_bounds__(8 * N) void k_pair_fwd_slab_oct(const cx<T>* __restrict__ phi,
                                                             long ldphi,
                                                             const cx<T>* __restrict__ psi,
                                                             long ldpsi, cx<T>* __restrict__ buf,
                                                             int mode, int i0, int A, int j0,
                                                             long p0, int npairs) {
  constexpr int NN = N * N;
  constexpr int LD = kOctLd<N>;
  constexpr int M = N / 8;
  __shared__ cx<T> s[N * LD];
  const long lid = xcd_logical(blockIdx.x, gridDim.x);
  if (lid >= (long)N * npairs) return;
  const int x0 = (int)(lid / npairs);
  const int p = (int)(lid - (long)x0 * npairs);
  int i, j;
  pair_of(mode, i0, A, j0, p0, p, &i, &j);
  const cx<T>* a = phi + (size_t)i * ldphi + (size_t)x0 * NN;
  const cx<T>* b = psi + (size_t)j * ldpsi + (size_t)x0 * NN;
  const int t = threadIdx.x;
  const int l = t >> 3, h = t & 7;
  const int rr = t / N, cc = t - rr * N;  // element t + 8N q sits at row 8q + rr, column cc
  const OctTw<N, T> tw = oct_twiddles<N, T>(h);
  {
    cx<T> va[M], vb[M];
#pragma unroll
    for (int q = 0; q < M; ++q) va[q] = a[(8 * q + rr) * N + cc];
#pragma unroll
    for (int q = 0; q < M; ++q) vb[q] = b[(8 * q + rr) * N + cc];
#pragma unroll
    for (int q = 0; q < M; ++q) s[(8 * q + rr) * LD + cc] = cmulc(va[q], vb[q]);
  }
  __syncthreads();
  cx<T> v[M];
  // axis 2: row l (read and rewritten by its own octet only: one wave, in order)
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = s[l * LD + h + 8 * m];
  fft_oct_d2b<N, -1, T>(v, h, tw);
#pragma unroll
  for (int k = 0; k < M; ++k) s[l * LD + oct_block_index(k, M, h)] = v[k];
  __syncthreads();
  // axis 1: column l
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = s[(h + 8 * m) * LD + l];
  fft_oct_d2b<N, -1, T>(v, h, tw);
  cx<T>* out = buf + (size_t)p * N * NN + (size_t)x0 * NN + l;
#pragma unroll
  for (int k = 0; k < M; ++k) store_nt(&out[oct_block_index(k, M, h) * N], v[k]);
}

template <int N, typename T>
__global__ __launch_bounds__(8 * N) void k_plane_kernel_oct(cx<T>* __restrict__ buf,
                                                            ace_kspec ks, int npairs) {
  constexpr int NN = N * N;
  constexpr int LD = kOctLd<N>;
  constexpr int M = N / 8;
  __shared__ cx<T> s[N * LD];
  const long lid = xcd_logical(blockIdx.x, gridDim.x);
  if (lid >= (long)N * npairs) return;
  const int p = (int)(lid / N);  // pair-major, as in the quad plane pass
  const int k1 = (int)(lid - (long)p * N);
  const int t = threadIdx.x;
  const int l = t >> 3, h = t & 7;
  const OctTw<N, T> tw = oct_twiddles<N, T>(h);
  cx<T>* plane = buf + (size_t)p * N * NN + (size_t)k1 * N;
  cx<T> v[M];
  // axis 0 (column l of the plane): forward, kernel, inverse
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = plane[(size_t)(h + 8 * m) * NN + l];
  fft_oct_d2b<N, -1, T>(v, h, tw);
  {
    const KEval<T> ke(ks);
    const T s12 = ke.part12(k1, l);
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const T kk = ke.at(oct_block_index(k, M, h), s12);
      v[k].x *= kk;
      v[k].y *= kk;
    }
  }
  fft_oct_b2d<N, +1, T>(v, h, tw);
#pragma unroll
  for (int m = 0; m < M; ++m) s[(h + 8 * m) * LD + l] = v[m];
  __syncthreads();
  // axis 2 (row l): inverse; the row is read and rewritten by its own octet
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = s[l * LD + h + 8 * m];
  fft_oct_d2b<N, +1, T>(v, h, tw);
#pragma unroll
  for (int k = 0; k < M; ++k) s[l * LD + oct_block_index(k, M, h)] = v[k];
  __syncthreads();
  const int rr = t / N, cc = t - rr * N;
#pragma unroll
  for (int q = 0; q < M; ++q) plane[(size_t)(8 * q + rr) * NN + cc] = s[(8 * q + rr) * LD + cc];
}

// Accumulate pass, one thread per pencil (accum_lds_body), one wave per
// logical workgroup.
template <int N, typename T>
__global__ __launch_bounds__(64) void k_pencil_accum(const cx<T>* __restrict__ phi, long ldphi,
                                                     const cx<T>* __restrict__ buf,
                                                     cx<T>* __restrict__ W, long ldW, int i0,
                                                     int A, int j0, int nbc, int accumulate,
                                                     int mode) {
  constexpr int TILES = (N * N + 63) / 64;
  __shared__ cx<T> acc[N * 64];
  const long lid = xcd_logical(blockIdx.x, gridDim.x);
  if (lid >= (long)TILES * nbc) return;
  accum_lds_body<N, T>(acc, (int)threadIdx.x, lid, phi, ldphi, buf, W, ldW, i0, A, j0, nbc,
                       accumulate, mode);
}

// Accumulate pass on split lines (accum_q_body), one wave per logical
// workgroup.
template <int N, typename T>
__global__ __launch_bounds__(64) void k_pencil_accum_q(const cx<T>* __restrict__ phi, long ldphi,
                                                       const cx<T>* __restrict__ buf,
                                                       cx<T>* __restrict__ W, long ldW, int i0,
                                                       int A, int j0, int nbc, int accumulate,
                                                       int mode) {
  const long lid = xcd_logical(blockIdx.x, gridDim.x);
  if (lid >= (long)(N * N / 16) * nbc) return;
  accum_q_body<N, T>((int)threadIdx.x, lid, phi, ldphi, buf, W, ldW, i0, A, j0, nbc, accumulate,
                     mode);
}

// ---------------------------------------------------------------------------
// Real orbitals (the paper's Gamma-point setting, Section 4): the pair charges
// phi_a psi_j and phi_b psi_j of two occupied orbitals are real, so they are
// transformed together as rho = phi_a psi_j + i phi_b psi_j.  The kernel K is
// real and even, so the solve keeps real fields real:
// u = ifftn(K fftn(rho)) = u_aj + i u_bj, and one complex transform serves
// two pairs (the plane pass is shared with the complex path).
// Unit p of a chunk: orbitals a = i0 + 2m, b = a + 1 (absent when 2m + 1 = A)
// with m = p % Am, band j = j0 + p / Am.
// sym = 1: the packed triangle of the occupied block (psi = phi there), then
// the rectangle of the extra bands j0 = A, ... (units as in plan_build_real).
template <int N, typename T>
__global__ __launch_bounds__(N) void k_pair_fwd_real_t1(const T* __restrict__ phi, long ldphi,
                                                        const T* __restrict__ psi, long ldpsi,
                                                        cx<T>* __restrict__ buf, int i0, int A,
                                                        int Am, int j0, int nunits, int sym) {
  constexpr int NN = N * N;
  constexpr int LD = N + 1;
  __shared__ cx<T> s[N * LD];
  const long lid = xcd_logical(blockIdx.x, gridDim.x);
  if (lid >= (long)N * nunits) return;
  const int x0 = (int)(lid / nunits);
  const int p = (int)(lid - (long)x0 * nunits);
  int ia, jb;
  bool has_b;
  const long tri = sym ? real_tri_units(A) : 0;
  if (p < tri) {
    int cc, mm;
    real_tri_of(p, &cc, &mm);
    ia = 2 * mm;
    has_b = 2 * mm + 1 <= cc;
    jb = cc;
  } else {
    const int q = (int)(p - tri);
    const int m = q % Am;
    ia = i0 + 2 * m;
    has_b = 2 * m + 1 < A;
    jb = j0 + q / Am;
  }
  const T* fa = phi + (size_t)ia * ldphi + (size_t)x0 * NN;
  const T* fb = has_b ? fa + ldphi : fa;
  const T* ps = psi + (size_t)jb * ldpsi + (size_t)x0 * NN;
  const int t = threadIdx.x;
  {
    // issue every load of the slab before the first use
    T va[N], vb[N], vy[N];
#pragma unroll
    for (int r = 0; r < N; ++r) va[r] = fa[r * N + t];
#pragma unroll
    for (int r = 0; r < N; ++r) vb[r] = fb[r * N + t];
#pragma unroll
    for (int r = 0; r < N; ++r) vy[r] = ps[r * N + t];
    const T wb = has_b ? T(1) : T(0);
#pragma unroll
    for (int r = 0; r < N; ++r) s[r * LD + t] = cx<T>{va[r] * vy[r], wb * vb[r] * vy[r]};
  }
  __syncthreads();
  cx<T> v[N];
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = s[t * LD + k];
  fft_line<N, -1, T>(v);
#pragma unroll
  for (int k = 0; k < N; ++k) s[t * LD + k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = s[k * LD + t];
  fft_line<N, -1, T>(v);
  cx<T>* out = buf + (size_t)p * N * NN + (size_t)x0 * NN;
#pragma unroll
  for (int k = 0; k < N; ++k) store_nt(&out[k * N + t], v[k]);
}

// Accumulate pass for real orbitals: one thread per (x0, x2) pencil along
// axis 1, one band per workgroup row; for each unit of the chunk, the inverse
// FFT along axis 1 gives u_aj (real part) and u_bj (imaginary part), and
// w_j += phi_a u_aj + phi_b u_bj in a thread-private LDS column.
template <int N, typename T>
__global__ __launch_bounds__(64) void k_pencil_accum_real(const T* __restrict__ phi, long ldphi,
                                                          const cx<T>* __restrict__ buf,
                                                          T* __restrict__ W, long ldW, int i0,
                                                          int A, int Am, int j0, int nbc,
                                                          int accumulate) {
  constexpr int NN = N * N;
  constexpr int TILES = (NN + 63) / 64;
  __shared__ T acc[N * 64];
  const long lid = xcd_logical(blockIdx.x, gridDim.x);
  if (lid >= (long)TILES * nbc) return;
  const int tile = (int)(lid / nbc);
  const int b = (int)(lid - (long)tile * nbc);
  const int t = threadIdx.x;
  const int q = tile * 64 + t;
  if (q >= NN) return;
  const int x0 = q / N, x2 = q - x0 * N;
  const size_t off = (size_t)x0 * NN + x2;
#pragma unroll
  for (int k = 0; k < N; ++k) acc[k * 64 + t] = T(0);
  for (int m = 0; m < Am; ++m) {
    const int ia = i0 + 2 * m;
    const bool has_b = 2 * m + 1 < A;
    const cx<T>* src = buf + ((size_t)m + (size_t)Am * b) * N * NN + off;
    const T* pa = phi + (size_t)ia * ldphi + off;
    const T* pb = has_b ? pa + ldphi : pa;
    const T wb = has_b ? T(1) : T(0);
    cx<T> v[N];
    T fa[N], fb[N];
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = src[k * N];
#pragma unroll
    for (int k = 0; k < N; ++k) fa[k] = pa[k * N];
#pragma unroll
    for (int k = 0; k < N; ++k) fb[k] = pb[k * N];
    fft_line<N, +1, T>(v);
#pragma unroll
    for (int k = 0; k < N; ++k) acc[k * 64 + t] += fa[k] * v[k].x + wb * fb[k] * v[k].y;
  }
  T* w = W + (size_t)(j0 + b) * ldW + off;
  if (accumulate) {
    T old[N];
#pragma unroll
    for (int k = 0; k < N; ++k) old[k] = w[k * N];
#pragma unroll
    for (int k = 0; k < N; ++k) w[k * N] = old[k] + acc[k * 64 + t];
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) w[k * N] = acc[k * 64 + t];
  }
}

// Accumulate pass of the symmetric real chunk.  Workgroup row g < G = ceil(A/2)
// owns the band pair (j0, j1) = (2g, 2g + 1) of the occupied block (j1
// absent when it reaches A) with two LDS accumulators, so that a unit of a
// column c > j1, which holds u_{j0 c} (real part) and u_{j1 c} (imaginary
// part), is read once for both bands:
//   column j0, units m <= g:    w_j0 += phi_2m u_{2m j0} + phi_2m+1 u_{2m+1 j0}
//   column j1, units m < g:     w_j1 += phi_2m u_{2m j1} + phi_2m+1 u_{2m+1 j1}
//   column j1, unit g:          w_j0 += phi_j1 u_{j0 j1},
//                               w_j1 += phi_j0 u_{j0 j1} + phi_j1 u_{j1 j1}
//   columns c > j1, unit g:     w_j0 += phi_c u_{j0 c},  w_j1 += phi_c u_{j1 c}
// (u_ij = u_ji for real fields).  Rows g >= G are the extra bands A + (g - G),
// accumulated from their rectangle units as in k_pencil_accum_real.
// Two waves per SIMD where the registers allow it without spills (FP32 up to
// N = 48); the compiler would otherwise settle for one at N = 48.
template <int N, typename T>
constexpr int kRealSymWaves = (sizeof(T) == 4 && N <= 48) ? 2 : 1;
template <int N, typename T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kRealSymWaves<N, T>))) void
k_pencil_accum_real_sym(const T* __restrict__ phi,
                                                              long ldphi,
                                                              const cx<T>* __restrict__ buf,
                                                              T* __restrict__ W, long ldW, int A,
                                                              int nrows) {
  constexpr int NN = N * N;
  constexpr int TILES = (NN + 63) / 64;
  __shared__ T acc0[N * 64];
  __shared__ T acc1[N * 64];
  const long lid = xcd_logical(blockIdx.x, gridDim.x);
  if (lid >= (long)TILES * nrows) return;
  const int tile = (int)(lid / nrows);
  const int g = (int)(lid - (long)tile * nrows);
  const int t = threadIdx.x;
  const int q = tile * 64 + t;
  if (q >= NN) return;
  const int x0 = q / N, x2 = q - x0 * N;
  const size_t off = (size_t)x0 * NN + x2;
  const int G = (A + 1) / 2;
  const long tri = real_tri_units(A);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    acc0[k * 64 + t] = T(0);
    acc1[k * 64 + t] = T(0);
  }
  // inverse FFT along axis 1 of unit u at this pencil
  auto unit = [&](long u, cx<T> (&v)[N]) {
    const cx<T>* src = buf + (size_t)u * N * NN + off;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = src[k * N];
    fft_line<N, +1, T>(v);
  };
  // acc += fa * Re v + wb * fb * Im v
  auto add2 = [&](T* acc, const T* pa, const T* pb, T wb, const cx<T> (&v)[N]) {
    T fa[N], fb[N];
#pragma unroll
    for (int k = 0; k < N; ++k) fa[k] = pa[k * N];
#pragma unroll
    for (int k = 0; k < N; ++k) fb[k] = pb[k * N];
#pragma unroll
    for (int k = 0; k < N; ++k) acc[k * 64 + t] += fa[k] * v[k].x + wb * fb[k] * v[k].y;
  };
  cx<T> v[N];
  if (g < G) {
    const int j0 = 2 * g, j1 = 2 * g + 1;
    const bool two = j1 < A;
    // column j0
    for (int m = 0; m <= g; ++m) {
      unit(real_tri_units(j0) + m, v);
      const T* pa = phi + (size_t)(2 * m) * ldphi + off;
      const bool hb = 2 * m + 1 <= j0;
      add2(acc0, pa, hb ? pa + ldphi : pa, hb ? T(1) : T(0), v);
    }
    if (two) {
      // column j1, rows below j0
      for (int m = 0; m < g; ++m) {
        unit(real_tri_units(j1) + m, v);
        const T* pa = phi + (size_t)(2 * m) * ldphi + off;
        add2(acc1, pa, pa + ldphi, T(1), v);
      }
      // unit (j0, j1; column j1)
      unit(real_tri_units(j1) + g, v);
      const T* p0 = phi + (size_t)j0 * ldphi + off;
      const T* p1 = p0 + ldphi;
      {
        T f0[N], f1[N];
#pragma unroll
        for (int k = 0; k < N; ++k) f0[k] = p0[k * N];
#pragma unroll
        for (int k = 0; k < N; ++k) f1[k] = p1[k * N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
          acc0[k * 64 + t] += f1[k] * v[k].x;
          acc1[k * 64 + t] += f0[k] * v[k].x + f1[k] * v[k].y;
        }
      }
    }
    // columns beyond the pair
    for (int c = two ? j1 + 1 : j0 + 1; c < A; ++c) {
      unit(real_tri_units(c) + g, v);
      const T* pc = phi + (size_t)c * ldphi + off;
      T fc[N];
#pragma unroll
      for (int k = 0; k < N; ++k) fc[k] = pc[k * N];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        acc0[k * 64 + t] += fc[k] * v[k].x;
        acc1[k * 64 + t] += fc[k] * v[k].y;
      }
    }
    T* w0 = W + (size_t)j0 * ldW + off;
#pragma unroll
    for (int k = 0; k < N; ++k) w0[k * N] = acc0[k * 64 + t];
    if (two) {
      T* w1 = W + (size_t)j1 * ldW + off;
#pragma unroll
      for (int k = 0; k < N; ++k) w1[k * N] = acc1[k * 64 + t];
    }
  } else {
    const int b = g - G;  // extra band A + b
    for (int m = 0; m < G; ++m) {
      unit(tri + m + (long)G * b, v);
      const T* pa = phi + (size_t)(2 * m) * ldphi + off;
      const bool hb = 2 * m + 1 < A;
      add2(acc0, pa, hb ? pa + ldphi : pa, hb ? T(1) : T(0), v);
    }
    T* w = W + (size_t)(A + b) * ldW + off;
#pragma unroll
    for (int k = 0; k < N; ++k) w[k * N] = acc0[k * 64 + t];
  }
}

// Energy pencil pass: forward FFT along axis 0 and sum_G K |rho^(G)|^2 over 64
// pencils per workgroup; one partial per workgroup, weighted 2 for i < j (the
// pair j, i has the same sum because K(G) = K(-G)).
template <int N, typename T>
__global__ __launch_bounds__(256) void k_pencil_energy(const cx<T>* __restrict__ buf,
                                                       ace_kspec ks, long p0,
                                                       double* __restrict__ partial) {
  constexpr int NN = N * N;
  constexpr int TILES = (NN + 63) / 64;
  constexpr int M = N / 4;
  __shared__ double red[4];
  const int p = blockIdx.x / TILES;
  const int tile = blockIdx.x - p * TILES;
  const int t = threadIdx.x;
  // pencil p_ + 16 (t >> 6) of the tile on lanes p_ + 16 h (split lines, 16
  // consecutive pencils per row segment)
  const int h = (t >> 4) & 3;
  const int q = tile * 64 + ((t >> 6) << 4) + (t & 15);
  double sum = 0.0;
  {
    const int qc = q < NN ? q : NN - 1;  // the lanes of a pencil past the end stay in step
    const cx<T>* base = buf + (size_t)p * N * NN + qc;
    cx<T> v[M];
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = base[(size_t)(h + 4 * m) * NN];
    fft_quad_d2b<N, -1, T, 16>(v, h);
    if (q < NN) {
      const KEval<T> ke(ks);
      const T s12 = ke.part12(q / N, q - (q / N) * N);
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const double kk = (double)ke.at(quad_block_index(k, M, h), s12);
        sum += kk * ((double)v[k].x * v[k].x + (double)v[k].y * v[k].y);
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_down(sum, o, 64);
  if ((t & 63) == 0) red[t >> 6] = sum;
  __syncthreads();
  if (t == 0) {
    int i, j;
    pair_of(1, 0, 1, 0, p0, p, &i, &j);
    partial[(size_t)(p0 + p) * TILES + tile] =
        (i == j ? 1.0 : 2.0) * ((red[0] + red[1]) + (red[2] + red[3]));
  }
}

// Deterministic two-stage sum, *out = s * sum(x[0..n)): kSumBlocks
// workgroups each sum a contiguous range into y[b] (fixed order, tree), then
// one workgroup sums y.
constexpr int kSumBlocks = 256;
__global__ __launch_bounds__(1024) void k_sum_blocks(const double* __restrict__ x, long n,
                                                     double* __restrict__ y) {
  __shared__ double red[1024];
  const long per = (n + gridDim.x - 1) / gridDim.x;
  const long beg = (long)blockIdx.x * per, end = beg + per < n ? beg + per : n;
  double acc = 0.0;
  for (long k = beg + threadIdx.x; k < end; k += 1024) acc += x[k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) y[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(1024) void k_sum_scaled(const double* __restrict__ x, long n,
                                                     double s, double* __restrict__ out) {
  __shared__ double red[1024];
  double acc = 0.0;
  for (long k = threadIdx.x; k < n; k += 1024) acc += x[k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s * red[0];
}

size_t default_pair_budget() { return (size_t)4 << 30; }

}  // namespace

size_t default_pair_budget_bytes() { return default_pair_budget(); }

// Pairs per chunk of the direct energy (triangle i <= j in budget-sized chunks).
long energy_chunk(ace_ctx c, const GridInfo& g, size_t eb, int nocc) {
  const long total = (long)nocc * (nocc + 1) / 2;
  const size_t budget = c->pair_budget ? c->pair_budget : default_pair_budget();
  const long chunk = std::max<long>(1, (long)(budget / ((size_t)g.ng * eb)));
  return std::min(chunk, total);
}

size_t energy_direct_ws_bytes(ace_ctx c, const GridInfo& g, size_t eb, int nocc) {
  const long total = (long)nocc * (nocc + 1) / 2;
  const long tiles = ((long)g.n * g.n + 63) / 64;
  return align_up(((size_t)total * tiles + kSumBlocks) * sizeof(double), 256) +
         align_up((size_t)energy_chunk(c, g, eb, nocc) * g.ng * eb, 256);
}

BuildPlan plan_build(ace_ctx c, const GridInfo& g, size_t eb, int nocc, int nband,
                     bool psi_starts_with_phi) {
  BuildPlan pl;
  const size_t pair_bytes = (size_t)g.ng * eb;
  // explicit knobs first, then an autotuned entry for this grid size, then defaults
  size_t budget = c->pair_budget;
  long jblock = c->jblock;
  if (const auto* t = tuned_for(c, g.n, (int)eb)) {
    if (!budget) budget = (size_t)t->budget;
    if (!jblock) jblock = t->jblock;
  }
  if (!budget) budget = default_pair_budget();
  if (c->budget_cap && budget > c->budget_cap) budget = c->budget_cap;
  long maxpairs = (long)(budget / pair_bytes);
  if (maxpairs < 1) maxpairs = 1;
  // Band block B (all bands unless tuned otherwise): the accumulating pass runs
  // (N^2 / 64) * B one-wave workgroups, each looping over the i block, and W is
  // read-modified-written once per i block.
  // Pair symmetry: when psi's first n_occ orbitals are phi, u_ji = conj(u_ij)
  // on the occupied block and only its triangle i <= j needs FFTs.  When the
  // whole triangle fits the budget it is one chunk; otherwise the occupied
  // orbitals are split into blocks of b, and each block pair I <= J is one
  // chunk (the triangle of I for I = J, the rectangle I x J otherwise) whose
  // spectra serve the bands of J and, conjugated, those of I.
  const long tri = (long)nocc * (nocc + 1) / 2;
  pl.sym = c->use_symmetry && psi_starts_with_phi && nocc >= 2;
  pl.symblk = 0;
  long sym_alloc = 0;
  pl.merged = false;
  if (pl.sym) {
    const long all = tri + (long)nocc * (nband - nocc);
    if (all <= maxpairs && (long)g.n * all < (1L << 31)) {
      // triangle and rectangle of the extra bands in flight together: one
      // launch per pass for the whole build
      pl.merged = true;
      sym_alloc = all;
    } else if (tri <= maxpairs && (long)g.n * tri < (1L << 31)) {
      sym_alloc = tri;
    } else {
      long bmax = (long)std::sqrt((double)maxpairs);
      while ((bmax + 1) * (bmax + 1) <= maxpairs) ++bmax;
      while (bmax > 1 && bmax * bmax > maxpairs) --bmax;
      if (bmax < 2) {
        pl.sym = false;  // budget below a 2 x 2 block
      } else {
        const long nblk = (nocc + bmax - 1) / bmax;
        pl.symblk = (int)((nocc + nblk - 1) / nblk);  // even blocks, last may be short
        sym_alloc = (long)pl.symblk * pl.symblk;
      }
    }
  }
  // the rectangular blocks cover the bands after the occupied block (all of
  // them without symmetry)
  const int nrect = std::max(1, pl.sym ? nband - nocc : nband);
  int B = jblock > 0 ? (int)std::min<long>(nrect, jblock) : nrect;
  B = (int)std::max<long>(1, std::min<long>(B, maxpairs));
  pl.B = B;
  pl.A = (int)std::max<long>(1, std::min<long>(nocc, maxpairs / B));
  pl.pairs_alloc = std::max<size_t>((size_t)pl.A * pl.B, (size_t)sym_alloc);
  pl.bytes = align_up(pl.pairs_alloc * pair_bytes, 256);
  return pl;
}

// Real orbitals: units of two pairs; A orbitals (even unless all of them) x B
// bands per chunk, Am = ceil(A / 2) units per band.
// Real orbitals with psi's first n_occ orbitals equal to phi: u_ij = u_ji on
// the occupied block, so only pairs i <= j are transformed.  Column c of the
// triangle packs rows (2m, 2m + 1), 2m <= c, into unit real_tri_units(c) + m
// (row 2m + 1 absent when it exceeds c); the extra bands follow as rectangle
// units (orbital pair m, band n_occ + k) at real_tri_units(n_occ) + m + Am k.
// Used when all units fit the pair budget (one chunk); otherwise the rectangle
// chunks below.
BuildPlan plan_build_real(ace_ctx c, const GridInfo& g, size_t cx_bytes, int nocc, int nband,
                          bool psi_starts_with_phi) {
  BuildPlan pl;
  const size_t unit_bytes = (size_t)g.ng * cx_bytes;
  size_t budget = c->pair_budget;
  long jblock = c->jblock;
  if (!budget) budget = default_pair_budget();
  long maxunits = (long)(budget / unit_bytes);
  if (maxunits < 1) maxunits = 1;
  pl.symblk = 0;
  pl.merged = false;
  const long sym_units = real_tri_units(nocc) + (long)((nocc + 1) / 2) * (nband - nocc);
  if (c->use_symmetry && psi_starts_with_phi && nocc >= 2 && jblock == 0 &&
      sym_units <= maxunits) {
    pl.sym = true;
    pl.merged = true;
    pl.A = nocc;
    pl.B = nband;
    pl.pairs_alloc = (size_t)sym_units;
  } else {
    int B = jblock > 0 ? (int)std::min<long>(nband, jblock) : nband;
    B = (int)std::max<long>(1, std::min<long>(B, maxunits));
    long am = std::max<long>(1, std::min<long>((nocc + 1) / 2, maxunits / B));
    pl.B = B;
    pl.A = (int)std::min<long>(nocc, 2 * am);
    pl.sym = false;
    pl.pairs_alloc = (size_t)((pl.A + 1) / 2) * pl.B;
  }
  pl.bytes = align_up(pl.pairs_alloc * unit_bytes, 256);
  return pl;
}

namespace {

// The scaled kernel K'(G) = coef * K(G) (* *dscale) of a grid, for the plane
// and energy passes, which evaluate it on the fly.
ace_kspec kspec_of(const GridInfo& g, double coef, const double* dscale = nullptr) {
  ace_kspec k{};
  const double twopi = 6.283185307179586477;
  for (int a = 0; a < 3; ++a) k.t2[a] = (twopi / g.L[a]) * (twopi / g.L[a]);
  k.coef = coef;
  k.inv4mu2 = g.kind == ACE_ERFC ? 1.0 / (4.0 * g.mu * g.mu) : 0.0;
  k.g0 = g.g0;
  k.dscale = dscale;
  k.n = g.n;
  k.kind = g.kind;
  return k;
}

// Line shape of the slab and plane passes: one thread per line (1), a lane
// quad per line with DPP exchanges (4), an octet (8), or a line split over
// lanes 16 apart with permlane exchanges (16).  Defaults from timings on the
// MI355X: slab pass quad from N = 72 (FP32) or 64 (FP64), plane pass quad from
// N = 64 (FP32) or 48 (FP64), one thread per line below.  The split form keeps
// 16-lane accesses contiguous but pays two VALU instructions per exchanged
// word where a DPP quad permutation rides on the consuming instruction: at
// N = 72 it measured slower (slab 2.07 -> 2.72 ms, plane 2.3 -> 3.7 ms per
// 1,146 pairs), at N = 48 too, so it is used only when asked for.  The tuning
// knob ACE_TUNE_FFT_SHAPE overrides both passes, else an autotuned shape for
// this grid size and element size.
int line_shape(ace_ctx c, int n, int eb) {
  if (c->fft_shape) return c->fft_shape;
  const auto* t = tuned_for(c, n, eb);
  return t ? t->shape : 0;
}

template <int N, typename T>
constexpr bool kOctOk = N % 8 == 0 && N >= 16;

// Form of the slab (plane_pass false) or plane pass: 1, 4, 8 or 16 as above.
template <int N, typename T>
int pass_form(ace_ctx c, bool plane_pass) {
  const int sh = line_shape(c, N, (int)sizeof(cx<T>));
  if (sh == 8) return kOctOk<N, T> ? 8 : 4;
  if (sh == 1 || sh == 4 || sh == 16) return sh;
  if (sizeof(T) == 8) return (plane_pass ? N >= 48 : N >= 64) ? 4 : 1;
  return (plane_pass ? N >= 64 : N >= 72) ? 4 : 1;
}

// Octet lines (N a multiple of 8 from 16) only on request (knob value 8):
// measured slower than the defaults at every size (at N = 72 FP32 the slab
// pass 8.1 vs 5.6 ms and the plane pass 7.5 vs 6.2 ms for 64 x 80 pairs),
// as the third exchange, the per-lane twiddles and the 64-byte row segments
// of the plane's column loads cost more than the full waves gain.
template <int N, typename T>
ace_status fwd_slab(ace_ctx c, const cx<T>* phi, long ldphi, const cx<T>* psi, long ldpsi,
                    cx<T>* buf, int mode, int i0, int A, int j0, long p0, int np) {
  if (c->record) {
    // the persistent kernel runs the one-thread-per-line form
    ace_plaunch l{};
    l.kind = kPassSlab;
    l.units = (long)N * np;
    l.phi = phi;
    l.ldphi = ldphi;
    l.psi = psi;
    l.ldpsi = ldpsi;
    l.buf = buf;
    l.mode = mode;
    l.i0 = i0;
    l.A = A;
    l.j0 = j0;
    l.p0 = p0;
    l.npairs = np;
    c->record->push_back(l);
    return ACE_OK;
  }
  const dim3 grid(xcd_pad((long)N * np));
  const int form = pass_form<N, T>(c, false);
  if constexpr (kOctOk<N, T>)
    if (form == 8)
      return launch(c, "pair_fwd_slab", k_pair_fwd_slab_oct<N, T>, grid, dim3(8 * N), 0, phi,
                    ldphi, psi, ldpsi, buf, mode, i0, A, j0, p0, np);
  if (form == 16)
    return launch(c, "pair_fwd_slab", k_pair_fwd_slab_row<N, T>, grid, dim3(64 * kRowWaves<N>), 0,
                  phi, ldphi, psi, ldpsi, buf, mode, i0, A, j0, p0, np);
  if (form == 4)
    return launch(c, "pair_fwd_slab", k_pair_fwd_slab<N, T>, grid, dim3(4 * N), 0, phi, ldphi, psi,
                  ldpsi, buf, mode, i0, A, j0, p0, np);
  constexpr int P = t1_group<N, T>(40 * 1024);
  return launch(c, "pair_fwd_slab", k_pair_fwd_slab_t1<N, T, P>,
                dim3(xcd_pad(((long)N * np + P - 1) / P)), dim3(N * P), 0, phi, ldphi, psi, ldpsi,
                buf, mode, i0, A, j0, p0, np);
}

template <int N, typename T>
ace_status plane(ace_ctx c, cx<T>* buf, const ace_kspec& ks, int np) {
  if (c->record) {
    ace_plaunch l{};
    l.kind = kPassPlane;
    l.units = (long)N * np;
    l.buf = buf;
    l.ks = ks;
    l.npairs = np;
    c->record->push_back(l);
    return ACE_OK;
  }
  const dim3 grid(xcd_pad((long)N * np));
  const int form = pass_form<N, T>(c, true);
  if constexpr (kOctOk<N, T>)
    if (form == 8)
      return launch(c, "plane_kernel", k_plane_kernel_oct<N, T>, grid, dim3(8 * N), 0, buf, ks,
                    np);
  if (form == 16)
    return launch(c, "plane_kernel", k_plane_kernel_row<N, T>, grid, dim3(64 * kRowWaves<N>), 0,
                  buf, ks, np);
  if (form == 4)
    return launch(c, "plane_kernel", k_plane_kernel<N, T>, grid, dim3(4 * N), 0, buf, ks, np);
  constexpr int P = t1_group<N, T>(80 * 1024);
  return launch(c, "plane_kernel", k_plane_kernel_t1<N, T, P>,
                dim3(xcd_pad(((long)N * np + P - 1) / P)), dim3(N * P), 0, buf, ks, np);
}

// Form of the accumulate pass: one thread per pencil with the accumulator in
// LDS (1), or pencils split over lanes 16 apart with register accumulators
// (16).  Measured per build (FP32): 48^3 split 0.92 ms vs LDS 1.03 ms
// (5,120 pairs), 64^3 0.90 vs 0.90, 72^3 1.11 vs 0.95 ms per launch (the
// split form needs 226 registers there, two waves per SIMD, and the permlane
// exchanges add VALU work): split up to N = 64, LDS above.  The knob
// ACE_TUNE_ACCUM_SHAPE overrides it, else an autotuned form.
template <int N, typename T>
int accum_form(ace_ctx c) {
  if (c->accum_shape) return c->accum_shape;
  const auto* t = tuned_for(c, N, (int)sizeof(cx<T>));
  if (t && t->accum) return t->accum;
  return N <= 64 ? 16 : 1;
}

template <int N, typename T>
ace_status accum(ace_ctx c, const cx<T>* phi, long ldphi, const cx<T>* buf, cx<T>* W, long ldW,
                 int i0, int A, int j0, int nbc, int accumulate, int mode) {
  if (c->record) {
    const bool q = accum_form<N, T>(c) != 1;
    ace_plaunch l{};
    l.kind = q ? kPassAccumQ : kPassAccum;
    l.units = (q ? (long)(N * N / 16) : (long)((N * N + 63) / 64)) * nbc;
    l.phi = phi;
    l.ldphi = ldphi;
    l.buf = (void*)buf;
    l.W = W;
    l.ldW = ldW;
    l.i0 = i0;
    l.A = A;
    l.j0 = j0;
    l.nbc = nbc;
    l.accumulate = accumulate;
    l.mode = mode;
    c->record->push_back(l);
    return ACE_OK;
  }
  if (accum_form<N, T>(c) == 1) {
    constexpr int TILES = (N * N + 63) / 64;
    return launch(c, "pencil_accum", k_pencil_accum<N, T>, dim3(xcd_pad((long)TILES * nbc)),
                  dim3(64), 0, phi, ldphi, buf, W, ldW, i0, A, j0, nbc, accumulate, mode);
  }
  constexpr int TQ = N * N / 16;
  return launch(c, "pencil_accum", k_pencil_accum_q<N, T>, dim3(xcd_pad((long)TQ * nbc)),
                dim3(64), 0, phi, ldphi, buf, W, ldW, i0, A, j0, nbc, accumulate, mode);
}

template <int N, typename T>
ace_status build_W_n(ace_ctx c, const GridInfo& g, const cx<T>* phi, int nocc, long ldphi,
                     const cx<T>* psi, int nband, long ldpsi, cx<T>* W, long ldW, double scale,
                     const double* dscale, bool accumulate) {
  const int acc0 = accumulate ? 1 : 0;  // the first contribution to a band adds to W
  constexpr int NN = N * N;
  constexpr int TILES = (NN + 63) / 64;
  const size_t pair_bytes = (size_t)g.ng * sizeof(cx<T>);
  const BuildPlan pl = plan_build(c, g, sizeof(cx<T>), nocc, nband, psi == phi && ldpsi == ldphi);
  const int A = pl.A, B = pl.B;
  const bool sym = pl.sym;
  const size_t pairs_alloc = pl.pairs_alloc;
  ace_status st;
  if ((st = ws_begin(c, pl.bytes)) != ACE_OK) return st;
  cx<T>* buf = (cx<T>*)ws_take(c, pairs_alloc * pair_bytes, &st);
  if (!buf) return st;
  if (c->record && dscale) return fail(c, ACE_E_UNSUPPORTED, "recorded build with a device scale");
  const ace_kspec ks = kspec_of(g, -scale / (double)g.ng, dscale);
  int jstart = 0;
  if (pl.merged) {
    const long all = (long)nocc * (nocc + 1) / 2 + (long)nocc * (nband - nocc);
    if ((st = fwd_slab<N, T>(c, phi, ldphi, psi, ldpsi, buf, 3, 0, nocc, nocc, 0L,
                             (int)all)) != ACE_OK)
      return st;
    if ((st = plane<N, T>(c, buf, ks, (int)all)) != ACE_OK) return st;
    return accum<N, T>(c, phi, ldphi, buf, W, ldW, 0, nocc, 0, nband, acc0, 3);
  }
  if (sym && pl.symblk == 0) {
    // occupied block: the triangle i <= j of pair spectra, every column j < n_occ
    // accumulates all i from it (u_ij = conj(u_ji))
    const long tri = (long)nocc * (nocc + 1) / 2;
    if ((st = fwd_slab<N, T>(c, phi, ldphi, phi, ldphi, buf, 1, 0, 1, 0, 0L, (int)tri)) !=
        ACE_OK)
      return st;
    if ((st = plane<N, T>(c, buf, ks, (int)tri)) != ACE_OK) return st;
    if ((st = accum<N, T>(c, phi, ldphi, buf, W, ldW, 0, nocc, 0, nocc, acc0, 1)) != ACE_OK)
      return st;
    jstart = nocc;
  } else if (sym) {
    // occupied block in blocks of b: chunk (I, J), I <= J, in a fixed order;
    // a band is written by its first contribution and accumulated afterwards
    const int b = pl.symblk, nblk = (nocc + b - 1) / b;
    std::vector<char> started(nblk, (char)acc0);
    for (int J = 0; J < nblk; ++J)
      for (int I = 0; I <= J; ++I) {
        const int i0 = I * b, ni = std::min(b, nocc - i0);
        const int j0 = J * b, nj = std::min(b, nocc - j0);
        if (I == J) {
          const int np = ni * (ni + 1) / 2;
          if ((st = fwd_slab<N, T>(c, phi, ldphi, phi, ldphi, buf, 1, i0, 1, i0, 0L, np)) !=
              ACE_OK)
            return st;
          if ((st = plane<N, T>(c, buf, ks, np)) != ACE_OK) return st;
          if ((st = accum<N, T>(c, phi, ldphi, buf, W, ldW, i0, ni, i0, ni, (int)started[I], 1)) !=
              ACE_OK)
            return st;
          started[I] = 1;
        } else {
          const int np = ni * nj;
          if ((st = fwd_slab<N, T>(c, phi, ldphi, phi, ldphi, buf, 0, i0, ni, j0, 0L, np)) !=
              ACE_OK)
            return st;
          if ((st = plane<N, T>(c, buf, ks, np)) != ACE_OK) return st;
          // bands of J from the orbitals of I, then bands of I from those of J
          if ((st = accum<N, T>(c, phi, ldphi, buf, W, ldW, i0, ni, j0, nj, (int)started[J], 0)) !=
              ACE_OK)
            return st;
          started[J] = 1;
          if ((st = accum<N, T>(c, phi, ldphi, buf, W, ldW, j0, nj, i0, ni, (int)started[I], 2)) !=
              ACE_OK)
            return st;
          started[I] = 1;
        }
      }
    jstart = nocc;
  }
  for (int j0 = jstart; j0 < nband; j0 += B) {
    const int Bc = std::min(B, nband - j0);
    for (int i0 = 0; i0 < nocc; i0 += A) {
      const int Ac = std::min(A, nocc - i0);
      const int np = Ac * Bc;
      if ((st = fwd_slab<N, T>(c, phi, ldphi, psi, ldpsi, buf, 0, i0, Ac, j0, 0L, np)) !=
          ACE_OK)
        return st;
      if ((st = plane<N, T>(c, buf, ks, np)) != ACE_OK) return st;
      if ((st = accum<N, T>(c, phi, ldphi, buf, W, ldW, i0, Ac, j0, Bc, (i0 > 0 || accumulate) ? 1 : 0, 0)) !=
          ACE_OK)
        return st;
    }
  }
  return ACE_OK;
}

template <int N, typename T>
ace_status build_W_real_n(ace_ctx c, const GridInfo& g, const T* phi, int nocc, long ldphi,
                          const T* psi, int nband, long ldpsi, T* W, long ldW, double scale,
                          const double* dscale) {
  constexpr int NN = N * N;
  constexpr int TILES = (NN + 63) / 64;
  const size_t unit_bytes = (size_t)g.ng * sizeof(cx<T>);
  // the symmetric accumulate kernel spills heavily in FP64 above N = 48
  const bool sym_ok = sizeof(T) == 4 || N <= 48;
  const BuildPlan pl =
      plan_build_real(c, g, sizeof(cx<T>), nocc, nband, sym_ok && psi == phi && ldpsi == ldphi);
  ace_status st;
  if ((st = ws_begin(c, pl.bytes)) != ACE_OK) return st;
  cx<T>* buf = (cx<T>*)ws_take(c, pl.pairs_alloc * unit_bytes, &st);
  if (!buf) return st;
  const ace_kspec ks = kspec_of(g, -scale / (double)g.ng, dscale);
  if (pl.sym) {
    const int G = (nocc + 1) / 2, nu = (int)pl.pairs_alloc;
    if ((st = launch(c, "pair_fwd_real", k_pair_fwd_real_t1<N, T>, dim3(xcd_pad((long)N * nu)),
                     dim3(N), 0, phi, ldphi, psi, ldpsi, buf, 0, nocc, G, nocc, nu, 1)) != ACE_OK)
      return st;
    if ((st = plane<N, T>(c, buf, ks, nu)) != ACE_OK) return st;
    const int nrows = G + (nband - nocc);
    return launch(c, "pencil_accum_real", k_pencil_accum_real_sym<N, T>,
                  dim3(xcd_pad((long)TILES * nrows)), dim3(64), 0, phi, ldphi, (const cx<T>*)buf,
                  W, ldW, nocc, nrows);
  }
  for (int j0 = 0; j0 < nband; j0 += pl.B) {
    const int Bc = std::min(pl.B, nband - j0);
    for (int i0 = 0; i0 < nocc; i0 += pl.A) {
      const int Ac = std::min(pl.A, nocc - i0);
      const int Am = (Ac + 1) / 2;
      const int nu = Am * Bc;
      if ((st = launch(c, "pair_fwd_real", k_pair_fwd_real_t1<N, T>,
                       dim3(xcd_pad((long)N * nu)), dim3(N), 0, phi, ldphi, psi, ldpsi, buf, i0,
                       Ac, Am, j0, nu, 0)) != ACE_OK)
        return st;
      if ((st = plane<N, T>(c, buf, ks, nu)) != ACE_OK) return st;
      if ((st = launch(c, "pencil_accum_real", k_pencil_accum_real<N, T>,
                       dim3(xcd_pad((long)TILES * Bc)), dim3(64), 0, phi, ldphi,
                       (const cx<T>*)buf, W, ldW, i0, Ac, Am, j0, Bc, i0 > 0 ? 1 : 0)) != ACE_OK)
        return st;
    }
  }
  return ACE_OK;
}

template <int N, typename T>
ace_status energy_direct_n(ace_ctx c, const GridInfo& g, const cx<T>* phi, int nocc, long ldphi,
                           double* ex_dev) {
  constexpr int NN = N * N;
  constexpr int TILES = (NN + 63) / 64;
  const long total = (long)nocc * (nocc + 1) / 2;
  const size_t pair_bytes = (size_t)g.ng * sizeof(cx<T>);
  const long chunk = energy_chunk(c, g, sizeof(cx<T>), nocc);
  const size_t part_bytes = align_up(((size_t)total * TILES + kSumBlocks) * sizeof(double), 256);
  ace_status st;
  if ((st = ws_begin(c, energy_direct_ws_bytes(c, g, sizeof(cx<T>), nocc))) != ACE_OK) return st;
  double* partial = (double*)ws_take(c, part_bytes, &st);
  cx<T>* buf = (cx<T>*)ws_take(c, (size_t)chunk * pair_bytes, &st);
  if (!partial || !buf) return st;
  const ace_kspec ks = kspec_of(g, 1.0);
  for (long p0 = 0; p0 < total; p0 += chunk) {
    const int np = (int)std::min(chunk, total - p0);
    if ((st = fwd_slab<N, T>(c, phi, ldphi, phi, ldphi, buf, 1, 0, 1, 0, p0,
                             np)) != ACE_OK)
      return st;
    if ((st = launch(c, "pencil_energy", k_pencil_energy<N, T>, dim3(np * TILES), dim3(256), 0,
                     (const cx<T>*)buf, ks, p0, partial)) != ACE_OK)
      return st;
  }
  double* blocks = partial + (size_t)total * TILES;
  if ((st = launch(c, "sum_blocks", k_sum_blocks, dim3(kSumBlocks), dim3(1024), 0,
                   (const double*)partial, total * TILES, blocks)) != ACE_OK)
    return st;
  return launch(c, "sum_scaled", k_sum_scaled, dim3(1), dim3(1024), 0, (const double*)blocks,
                (long)kSumBlocks, -0.5 * g.dV / (double)g.ng, ex_dev);
}

}  // namespace

template <typename T>
ace_status build_W_impl(ace_ctx c, const GridInfo& g, const cx<T>* phi, int nocc, long ldphi,
                        const cx<T>* psi, int nband, long ldpsi, cx<T>* W, long ldW,
                        double scale, const double* dscale, bool accumulate) {
  switch (g.n) {
#define ACE_CASE(NV)                                                                    \
  case NV:                                                                              \
    return build_W_n<NV, T>(c, g, phi, nocc, ldphi, psi, nband, ldpsi, W, ldW, scale, dscale, \
                            accumulate);
    ACE_FOR_EACH_N(ACE_CASE)
#undef ACE_CASE
    default:
      return fail(c, ACE_E_UNSUPPORTED, "grid size not compiled into the library");
  }
}

template <typename T>
ace_status energy_direct_impl(ace_ctx c, const GridInfo& g, const cx<T>* phi, int nocc,
                              long ldphi, double* ex_dev) {
  switch (g.n) {
#define ACE_CASE(NV) \
  case NV:           \
    return energy_direct_n<NV, T>(c, g, phi, nocc, ldphi, ex_dev);
    ACE_FOR_EACH_N(ACE_CASE)
#undef ACE_CASE
    default:
      return fail(c, ACE_E_UNSUPPORTED, "grid size not compiled into the library");
  }
}

template <typename T>
ace_status build_W_real_impl(ace_ctx c, const GridInfo& g, const T* phi, int nocc, long ldphi,
                             const T* psi, int nband, long ldpsi, T* W, long ldW, double scale,
                             const double* dscale) {
  switch (g.n) {
#define ACE_CASE(NV) \
  case NV:           \
    return build_W_real_n<NV, T>(c, g, phi, nocc, ldphi, psi, nband, ldpsi, W, ldW, scale, dscale);
    ACE_FOR_EACH_N(ACE_CASE)
#undef ACE_CASE
    default:
      return fail(c, ACE_E_UNSUPPORTED, "grid size not compiled into the library");
  }
}

template ace_status build_W_real_impl<float>(ace_ctx, const GridInfo&, const float*, int, long,
                                             const float*, int, long, float*, long, double,
                                             const double*);
template ace_status build_W_real_impl<double>(ace_ctx, const GridInfo&, const double*, int, long,
                                              const double*, int, long, double*, long, double,
                                              const double*);
template ace_status build_W_impl<float>(ace_ctx, const GridInfo&, const cx<float>*, int, long,
                                        const cx<float>*, int, long, cx<float>*, long, double,
                                        const double*, bool);
template ace_status build_W_impl<double>(ace_ctx, const GridInfo&, const cx<double>*, int, long,
                                         const cx<double>*, int, long, cx<double>*, long, double,
                                         const double*, bool);
template ace_status energy_direct_impl<float>(ace_ctx, const GridInfo&, const cx<float>*, int,
                                              long, double*);
template ace_status energy_direct_impl<double>(ace_ctx, const GridInfo&, const cx<double>*, int,
                                               long, double*);

}  // namespace ace
