// Host-side internals of libace shared by the translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/ace.h"
#include "fft_core.h"

// The scaled kernel of one build, K'(G) = coef * K(G) (times *dscale when
// dscale is set), evaluated on the fly from the per-axis factors
// (2 pi / L_a)^2: K = 4 pi / |G|^2 for G != 0, times -expm1(-|G|^2 / (4 mu^2))
// for the screened kernel; K(0) = g0; |G|^2 / 2 for the kinetic kind.
struct ace_kspec {
  double t2[3];          // (2 pi / L_a)^2
  double coef;
  double inv4mu2;        // 1 / (4 mu^2), screened kernel
  double g0;
  const double* dscale;  // nullable device factor (read by every thread)
  int n;
  int kind;
};

// One pass launch of a build, recorded for the persistent batched kernel
// (plain data, copied to device memory).
struct ace_plaunch {
  int kind;  // ace::PassKind
  int mode, i0, A, j0, nbc, accumulate, npairs;
  long p0;
  long units;  // logical units of the launch (slabs, planes, pencil tiles)
  const void* phi;
  const void* psi;
  void* buf;
  void* W;
  long ldphi, ldpsi, ldW;
  ace_kspec ks;  // plane pass
};

// One task of the persistent kernel: units [u0, u1) of launch `launch`, run
// once every task of launch `wait` (-1: none) has finished (wait_count tasks).
struct ace_ptask {
  int launch;
  int wait;
  int wait_count;
  int pad;
  long u0, u1;
};

struct ace_ctx_s {
  hipStream_t stream = nullptr;
  int device = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  size_t ws_used = 0;
  // Bytes at the start of the workspace that ws_begin / ws_take skip (a piece
  // one entry point keeps alive across an inner call that carves its own).
  size_t ws_prefix = 0;
  // Sub-arena (batched builds): while sub_base is set, ws_begin/ws_take carve
  // from [sub_base, sub_base + sub_bytes) and never reallocate.
  char* sub_base = nullptr;
  size_t sub_bytes = 0;
  // batched build: branch streams, fork/join events, cached graph
  // autotuned build settings per (grid size, element bytes): {pair budget, band
  // block, line shape of the slab and plane passes (0 = defaults)}; tune_gen
  // counts changes (it keys the batched build's cached graph)
  struct Tuned {
    int n;
    int eb;
    long budget;
    long jblock;
    int shape;
    int accum;  // form of the accumulate pass (0 = default)
  };
  std::vector<Tuned> tuned;
  unsigned tune_gen = 0;
  hipStream_t capture_stream = nullptr;
  std::vector<hipStream_t> branch_streams;
  std::vector<hipEvent_t> branch_events;
  hipEvent_t fork_event = nullptr;
  std::vector<unsigned char> graph_key;
  hipGraphExec_t graph_exec = nullptr;
  size_t pair_budget = 0;  // 0 = default
  long jblock = 0;         // band block of the build; 0 = automatic
  bool use_symmetry = true;  // i <-> j pair symmetry on the occupied block
  int fft_shape = 0;         // slab/plane line shape: 0 auto, 1 thread, 4 quad, 8 octet, 16 split
  int accum_shape = 0;       // accumulate pass: 0 auto, 1 thread per pencil, 16 split lines
  int branches = 4;          // branch streams of the batched build
  int batch_form = 0;        // batched build: 0 default, 1 per-instance launches, 2 persistent
  // Batched build, persistent form: while `record` is set, the pass launchers
  // of build_W_impl append descriptors there instead of launching, and
  // plan_build caps the pair budget at budget_cap (0 = no cap).
  std::vector<struct ace_plaunch>* record = nullptr;
  size_t budget_cap = 0;
  std::vector<void*> graph_bufs;  // device buffers the cached graph reads
  int num_cus = 256;
  std::string last_error;
  std::string tune_cache;              // default cache file of ace_autotune ("" = none)
  // ACE_TUNE at creation: -1 unset (tuned settings used, none made implicitly),
  // 0 library defaults only (the tuned table is not consulted), 1 a complex
  // build of a grid size with no tuned setting first runs the autotuner
  int tune_mode = -1;
  FILE* log = nullptr;                 // ACE_LOG target (stderr or an appended file)
  bool log_owned = false;              // log was opened here (closed on destroy)
  hipEvent_t stream_event = nullptr;   // orders a new stream after the old one
  // profiling
  bool profiling = false;
  struct ProfEntry {
    std::string name;
    long launches = 0;
    double ms = 0.0;
  };
  std::vector<ProfEntry> prof;
  struct Pending {
    int entry;
    hipEvent_t e0, e1;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> free_events;
};

namespace ace {

// Supported grid sizes per axis (cubic grids).  Each needs a radix plan in
// fft_core.h and instantiations in fft_passes.hip.
#define ACE_FOR_EACH_N(X) X(8) X(12) X(16) X(24) X(32) X(40) X(48) X(64) X(72)

ace_status fail(ace_ctx c, ace_status s, const std::string& msg);
ace_status hip_fail(ace_ctx c, hipError_t e, const char* where);
// True when the context stream is being captured into a graph (also when the
// legacy default stream may not be used because another stream captures).
bool stream_capturing(ace_ctx c);
// Reads a tuning cache ("n eb budget jblock [shape]" per line) into the
// context; a missing file returns false.
bool tune_cache_read(ace_ctx c, const char* path);
// The tuned setting for (grid size, element bytes), or null when there is none
// or ACE_TUNE=0 switched tuned settings off.
const ace_ctx_s::Tuned* tuned_for(ace_ctx c, int n, int eb);
// Writes one line to the ACE_LOG target, if any (printf-style).
void log_line(ace_ctx c, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
// Looks up, once per device and with that device current, the device address
// of the allocation-free apply's static scratch array (noalloc.hip).
void noalloc_setup(int device);

#define ACE_TRY(x)               \
  do {                           \
    ace_status _s = (x);         \
    if (_s != ACE_OK) return _s; \
  } while (0)

struct GridInfo {
  int n;          // points per axis
  long ng;        // n^3
  double L[3];
  int kind;
  double mu, g0;
  double omega, dV;
};

// Context workspace, a bump allocator over one device buffer.  Each entry
// point first calls ws_begin with the total it will carve (the buffer grows if
// needed, which synchronises the device; nothing is carved yet at that point),
// then ws_take hands out 256-byte aligned pieces.  ws_take returns nullptr and
// sets *st if a piece exceeds what ws_begin reserved.
ace_status ws_begin(ace_ctx c, size_t total_bytes);
void* ws_take(ace_ctx c, size_t bytes, ace_status* st);
// Scratch bytes gemm_cn takes from the workspace for these sizes (the most
// over every arithmetic and the Hermitian shapes).
size_t gemm_cn_scratch_bytes(int na, int nb, long K);

// Blocking of the build: A occupied orbitals x B bands per pair block, or the
// symmetric occupied triangle; `bytes` is the workspace the build takes.
struct BuildPlan {
  int A, B;       // rectangle chunks: A orbitals x B bands
  bool sym;       // i <-> j symmetry on the occupied block
  int symblk;     // 0: the whole occupied triangle is one chunk; else block size
  bool merged;    // triangle and the extra bands' rectangle form one chunk
  size_t pairs_alloc;
  size_t bytes;
};
BuildPlan plan_build(ace_ctx c, const GridInfo& g, size_t elem_bytes, int nocc, int nband,
                     bool psi_starts_with_phi);
// Workspace of ace_apply_h for n_x vectors (exchange from n_xi projection
// vectors or n_phi orbitals; 0 for none).
size_t hamiltonian_ws_bytes(ace_ctx c, const GridInfo& g, size_t eb, int nx, int nxi, int nphi);
// Workspace the compression takes for n_band vectors; alias_eb > 0 adds the
// copy of xi (n_band x N_g elements of alias_eb bytes) that xi == W needs.
size_t compress_ws_bytes(int nb, long ng, size_t alias_eb = 0);
// Workspace of the orthonormalisation of n vectors (element size eb).
size_t orth_ws_bytes(int n, long ng, size_t eb);
// Direct exchange energy: pairs per chunk and workspace.
long energy_chunk(ace_ctx c, const GridInfo& g, size_t eb, int nocc);
size_t energy_direct_ws_bytes(ace_ctx c, const GridInfo& g, size_t eb, int nocc);
size_t default_pair_budget_bytes();

// Profiling hooks around one launch.
void prof_begin(ace_ctx c, const char* name, int* entry, hipEvent_t* e0);
void prof_end(ace_ctx c, int entry, hipEvent_t e0);

template <typename... KArgs, typename... Args>
ace_status launch(ace_ctx c, const char* name, void (*kern)(KArgs...), dim3 grid, dim3 block,
                  size_t shmem, Args... args) {
  if (grid.x == 0 || grid.y == 0 || grid.z == 0) return ACE_OK;
  int entry = -1;
  hipEvent_t e0 = nullptr;
  if (c->profiling) prof_begin(c, name, &entry, &e0);
  hipLaunchKernelGGL(kern, grid, block, shmem, c->stream, static_cast<KArgs>(args)...);
  hipError_t e = hipGetLastError();
  if (c->profiling) prof_end(c, entry, e0);
  if (e != hipSuccess) return hip_fail(c, e, name);
  return ACE_OK;
}

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }


// Pass kinds of a recorded launch.
enum PassKind { kPassSlab = 1, kPassPlane = 2, kPassAccum = 3, kPassAccumQ = 4 };

// Persistent batched kernel (persist.hip) for grid size n and element bytes eb
// (8: complex64, 16: complex128): units per step of a pass kind, and the
// co-resident workgroups per CU.
int persist_step(int n, size_t eb, int kind);
ace_status persist_blocks_per_cu(ace_ctx c, int n, size_t eb, bool accq, int* out);
// Enqueues (on c->stream) the reset of ctl/done, the persistent kernel over
// ntasks tasks on `grid` workgroups, and the poisoning of every accumulated W
// (NaN in its first element) if a wait timed out.
ace_status persist_run(ace_ctx c, int n, size_t eb, bool accq, const ace_plaunch* L, int nlaunch,
                       const ace_ptask* tasks, int ntasks, int* ctl, int* done, int grid,
                       long long spin_ticks);

// Kernel kind used internally for the kinetic operator -1/2 Laplacian: the
// pair machinery with one "orbital" of ones and the kernel |G|^2 / 2 gives
// ifftn(|G|^2/2 fftn(x)) (scale -1).
constexpr int kKindKinetic = 2;

// Pair FFT stages (fft_passes.hip).
// W = scale * (*dscale if dscale else 1) * V_X[phi] psi   (accumulate: W += ...)
template <typename T>
ace_status build_W_impl(ace_ctx c, const GridInfo& g, const cx<T>* phi, int nocc, long ldphi,
                        const cx<T>* psi, int nband, long ldpsi, cx<T>* W, long ldW, double scale,
                        const double* dscale = nullptr, bool accumulate = false);
template <typename T>
ace_status energy_direct_impl(ace_ctx c, const GridInfo& g, const cx<T>* phi, int nocc,
                              long ldphi, double* ex_dev);
// Real orbitals (arrays of N_g reals): two pairs per complex transform.
template <typename T>
ace_status build_W_real_impl(ace_ctx c, const GridInfo& g, const T* phi, int nocc, long ldphi,
                             const T* psi, int nband, long ldpsi, T* W, long ldW, double scale,
                             const double* dscale = nullptr);
BuildPlan plan_build_real(ace_ctx c, const GridInfo& g, size_t cx_bytes, int nocc, int nband,
                          bool psi_starts_with_phi);

// Argument checks shared by the entry points (api.hip).
ace_status check_grid(ace_ctx c, const ace_grid* g, ace_prec prec, GridInfo* out);
ace_status check_block(ace_ctx c, const void* p, int count, long ld, const GridInfo& g,
                       const char* what);
size_t elem_bytes(ace_prec p);
struct Span {
  const char* lo;
  const char* hi;
};
Span span_of(const void* p, int count, long ld, long ng, size_t eb);
bool overlap(Span a, Span b);

// Compression of one instance (api.hip): M, Cholesky, xi = W L^{-H}.
// real: the orbital blocks hold real values viewed as N_g / 2 complex numbers
// (g.ng halved, ld halved); the small matrices then keep only their real part.
// Arithmetic of a reduction product C = alpha A^H B (gemm_cn): kNative in the
// data type (FP32 MFMA for complex64, FP64 for complex128), kBf16Split the
// BF16 hi/lo products with FP32 accumulation (complex64 only), kFp64 FP64 MFMA
// products of complex64 data with FP64 accumulation.
enum CnMode { kNative = 0, kBf16Split = 1, kFp64 = 2 };
// Exact scratch bytes of one gemm_cn call (complex data of data_bytes per
// element, arithmetic mode, Hermitian shape or not).
size_t gemm_cn_partial_bytes(int na, int nb, long K, size_t data_bytes, CnMode mode, bool herm);
// Mode of M for a precision.
inline CnMode compress_mode(ace_prec p) {
  return (p == ACE_MIXED || p == ACE_REAL32) ? kBf16Split : p == ACE_FP32 ? kFp64 : kNative;
}
// Mode of the Gram matrices of the orthonormalisation: FP64 products for
// ACE_FP32, the data type's own MFMA otherwise.  (Not BF16-split: a Gram
// diagonal sums |x|^2, so the dropped lo*lo term of every product is positive
// and biases the sum instead of averaging out.)
inline CnMode gram_mode(ace_prec p) { return p == ACE_FP32 ? kFp64 : kNative; }
template <typename T>
ace_status compress_impl(ace_ctx c, const GridInfo& g, const cx<T>* psi, long ldpsi,
                         const cx<T>* W, long ldW, int nb, cx<T>* xi, long ldxi,
                         cx<double>* L_out, int* info_dev, CnMode mode, bool real = false);

// Dense stages (dense.hip).  Small matrices are complex128, column-major.
// C[a + b*ldc] = alpha * sum_r conj(A_a[r]) B_b[r]   (real_part: imaginary part
// written as 0; for real data viewed as complex pairs the real part is the
// real dot product).  herm (na == nb, C Hermitian): only the 32 x 32 tiles on
// or above the diagonal are computed, the others are their conjugates.
template <typename T>
ace_status gemm_cn(ace_ctx c, const cx<T>* A, long lda, int na, const cx<T>* B, long ldb, int nb,
                   long K, double alpha, cx<double>* C, int ldc, CnMode mode,
                   bool real_part = false, bool herm = false);
// Y_b[r] = sum_a A_a[r] C[a + b*ldc]      (r < K); c_upper: C is upper
// triangular and its zero blocks are skipped
template <typename T>
ace_status gemm_nn(ace_ctx c, const cx<T>* A, long lda, int na, const cx<double>* C, int ldc,
                   int nb, cx<T>* Y, long ldy, long K, bool fp64_accumulate,
                   bool c_upper = false);
// Fused: A = s (M + M^H)/2, A = L L^H, Lout = L (nullable), C = L^{-H}.
// scratch: chol_scratch_elems(n) complex128 (used when n > 88).  info_dev gets
// 0 or the first failing pivot; a nonzero *prior (nullable) is propagated.
// real_only: A = s Re(M + M^T)/2 (the imaginary part of M is ignored).
ace_status chol_inv(ace_ctx c, const cx<double>* M, int n, double s, cx<double>* Lout,
                    cx<double>* C, cx<double>* scratch, int* info_dev,
                    const int* prior = nullptr, bool real_only = false);
inline size_t chol_scratch_elems(int n) { return (size_t)n * n + (size_t)16 * n; }
// *out = s * sum |A_ij|^2 over an m x n column-major block
ace_status sumsq(ace_ctx c, const cx<double>* A, long count, double s, double* out);

}  // namespace ace
