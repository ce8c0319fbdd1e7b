/*
 * libace: the adaptively compressed exchange (ACE) build on one AMD Instinct
 * MI355X (gfx950).  C ABI: plain pointers and sizes, no C++ or framework types.
 *
 * Method: L. Lin, "Adaptively Compressed Exchange Operator",
 * J. Chem. Theory Comput. 12, 2242 (2016).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid.   A periodic orthorhombic cell with edges L[0..2] (bohr) sampled on
 *         n[0] x n[1] x n[2] points (this release: n[0] = n[1] = n[2], a value
 *         listed by ace_supported_n).  N_g = n0 n1 n2, Omega = L0 L1 L2,
 *         dV = Omega / N_g.
 * Orbitals.  Device arrays of complex numbers with interleaved (re, im)
 *         parts: complex128 (two doubles) when prec == ACE_FP64, complex64
 *         (two floats) for ACE_FP32 and ACE_MIXED.  A block of N orbitals is
 *         orbital-major: orbital b starts at element b * ld (ld >= N_g, in
 *         complex elements) and holds its N_g grid values in C order
 *         (index (x0 * n1 + x1) * n2 + x2).  This is an N_g x N column-major
 *         matrix with leading dimension ld.
 * Real orbitals.  With ACE_REAL64 / ACE_REAL32 every orbital block (inputs
 *         and outputs) holds N_g reals per orbital, ld counted in reals; ld
 *         must be even and each orbital start aligned to two values.  The
 *         build transforms two pair charges per complex FFT (phi_a psi_j +
 *         i phi_b psi_j: both real, and the real even kernel keeps the two
 *         potentials apart as real and imaginary parts).  Small matrices
 *         (L_out) stay complex128 with zero imaginary parts.  Not available
 *         for real orbitals: the direct energy form (xi == NULL), the batched
 *         build, the tuner and the eigensolver pieces (ACE_E_UNSUPPORTED).
 * Inner product.  <f, g> = dV * sum_r conj(f(r)) g(r); orbitals are expected
 *         to satisfy <phi_i, phi_j> = delta_ij where the paper says so.
 * Ownership.  The caller owns every pointer passed in; the library never frees
 *         or retains them beyond the call.  The context owns its workspace.
 * Execution.  Every call is asynchronous and ordered on the context's HIP
 *         stream; outputs are valid once that stream reaches the call.  The
 *         only calls that may synchronise are those documented to do so.
 * Errors.  Argument errors are detected before any work is enqueued and return
 *         ACE_E_ARG or ACE_E_UNSUPPORTED with nothing written.  HIP runtime
 *         failures return ACE_E_HIP; ace_last_error() gives the text.
 *         Calls on one context must not overlap from several host threads.
 * Graph capture.  The compute entry points (build, compress, apply, energy,
 *         gradient, orthonormalise, batched build) may be called while the
 *         context stream is being captured into a HIP graph once the workspace
 *         is large enough for them (ace_reserve with at least their sizes, or
 *         an earlier uncaptured call of the same sizes).  A call that would
 *         have to grow the workspace, or synchronise (info_dev == NULL), on a
 *         capturing stream returns ACE_E_CAPTURE before it enqueues anything
 *         and leaves the capture and the workspace intact.
 */
#ifndef ACE_H
#define ACE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ace_ctx_s* ace_ctx;

typedef enum {
  ACE_OK = 0,
  ACE_E_ARG = 1,          /* invalid argument (null pointer, ld < N_g, sizes) */
  ACE_E_NOT_PD = 2,       /* -M (or the Gram matrix) is not positive definite */
  ACE_E_NOMEM = 3,        /* device workspace allocation failed */
  ACE_E_HIP = 4,          /* a HIP runtime call failed */
  ACE_E_UNSUPPORTED = 5,  /* grid shape or precision not built into the library */
  ACE_E_CAPTURE = 6       /* the call would allocate or synchronise while its stream
                             is being captured (see "Graph capture" above) */
} ace_status;

typedef enum {
  ACE_FP64 = 0,   /* complex128 data; FFTs, products and factorisations in FP64 */
  ACE_FP32 = 1,   /* complex64 data; FFTs and apply in FP32 (FP32 MFMA products); the
                     compression in FP64: M = dV psi^H W and the Gram matrices of
                     ace_orthonormalize as FP64 MFMA products of the FP32 data with FP64
                     accumulation, Cholesky, L^{-H} and xi = W L^{-H} in FP64 */
  ACE_MIXED = 2,  /* complex64 data; FFTs and apply in FP32; M by BF16-split MFMA
                     products (hi/lo halves, three products) with FP32 accumulation
                     inside each K chunk and FP64 across chunks; the Gram matrices of
                     ace_orthonormalize by FP32 MFMA products (same accumulation);
                     Cholesky, L^{-H} and xi = W L^{-H} in FP64 */
  ACE_REAL64 = 3, /* real orbitals (the Gamma-point setting of Section 4): arrays of
                     doubles; everything in FP64 */
  ACE_REAL32 = 4  /* real orbitals, arrays of floats; arithmetic as ACE_MIXED */
} ace_prec;

typedef enum {
  ACE_COULOMB = 0, /* v(r) = 1/r, Fourier kernel 4 pi / |G|^2 (Section 2, Eq. VXkernel) */
  ACE_ERFC = 1     /* v(r) = erfc(mu r)/r, kernel 4 pi/|G|^2 (1 - exp(-|G|^2/(4 mu^2)))
                      (Section 2, Eq. EXSR: the short-range screened exchange) */
} ace_kernel;

typedef struct {
  int n[3];      /* grid points per axis, n[0] slowest */
  double L[3];   /* cell edges in bohr */
  int kind;      /* ace_kernel */
  double mu;     /* screening parameter (bohr^-1) for ACE_ERFC, ignored otherwise */
  double g0;     /* kernel value used at G = 0, where 4 pi/|G|^2 is undefined; 0 removes
                    the G = 0 component */
} ace_grid;

/* Create a context bound to a HIP stream (hipStream_t passed as void*; NULL
 * means the default stream).  The context allocates device workspace lazily on
 * the device current at creation.
 * tune_cache (nullable): path of a tuning cache written by ace_autotune; the
 * settings it holds are loaded now (a file that does not exist yet is not an
 * error), and later ace_autotune calls with cache_path == NULL append their
 * results to it.
 * Environment, read here once per context:
 *   ACE_TUNE_CACHE  path used as tune_cache when the argument is NULL;
 *   ACE_TUNE        "0": library defaults only, tuned settings (loaded or made
 *                   by ace_autotune) are kept but not used; "1": the first
 *                   ace_build_W of a complex precision on a grid size and
 *                   element size with no tuned setting runs ace_autotune on
 *                   scratch orbitals of that call's sizes first (that call then
 *                   allocates and synchronises; skipped under stream capture)
 *                   and appends the result to the tuning cache; unset: tuned
 *                   settings are used, none is made implicitly;
 *   ACE_LOG         "1" or "stderr": one line per failed call (status and
 *                   message), workspace growth, tuning results and context
 *                   creation go to stderr; another value other than "0" names
 *                   a file they are appended to.
 * Fails with ACE_E_HIP when no HIP device is current. */
ace_status ace_create(ace_ctx* out, void* hip_stream, const char* tune_cache);
ace_status ace_destroy(ace_ctx ctx);
/* Rebind the stream used by later calls.  All calls share the context's one
 * workspace, so when the stream changes the new stream is first made to wait
 * for the work already enqueued on the old one (an event recorded on the old
 * stream); the calls of one context are therefore never concurrent.  When
 * either stream is being captured no such wait is added and the caller must
 * order the two streams itself. */
ace_status ace_set_stream(ace_ctx ctx, void* hip_stream);

/* Grow the context workspace now so that later calls with at most these sizes
 * allocate nothing.  Optional. */
ace_status ace_reserve(ace_ctx ctx, const ace_grid* grid, ace_prec prec,
                       int max_nocc, int max_nband, int max_nx);

/*
 * W = scale * V_X[phi] psi                      (Section 2, Eq. applyVX2; Section 3, Eq. W)
 *
 * For every band j < n_band:
 *   W_j(r) = -scale * sum_{i < n_occ} phi_i(r) u_ij(r),
 *   u_ij   = ifftn( K(G) * fftn( conj(phi_i) * psi_j ) ),
 * i.e. n_occ * n_band pair Poisson solves, each a 3-D FFT of the pair charge,
 * a multiply by the kernel K(G) of the grid, an inverse 3-D FFT (1/N_g
 * included) and an accumulation into w_j.  phi are the n_occ orbitals that
 * define the exchange operator; psi the n_band >= 1 vectors it is applied to
 * (psi = phi gives Eq. W; n_band > n_occ is the oversampled build at the end of
 * Section 3).  scale = 1 is the Fock exchange; 1/4 the PBE0/HSE fraction.
 * W must not overlap phi or psi.  ld_* >= N_g.
 */
ace_status ace_build_W(ace_ctx ctx, const ace_grid* grid, ace_prec prec,
                       const void* phi, int n_occ, long ld_phi,
                       const void* psi, int n_band, long ld_psi,
                       void* W, long ld_W, double scale);

/*
 * Compression (Section 3, Eqs. ACEconstruct2, Wtilde, ACE):
 *   M = dV * psi^H W  (n_band x n_band), symmetrised M <- (M + M^H)/2,
 *   -M = L L^H with L lower triangular, positive real diagonal,
 *   xi = W L^{-H}     (n_band projection vectors, same layout as W).
 * Afterwards V_ACE = -xi xi^H reproduces W on span(psi).
 * L_out (nullable): n_band x n_band complex128, column-major, device memory;
 *   receives L.
 * info_dev (nullable): device int; receives 0 on success or k >= 1, the first
 *   non-positive pivot (LAPACK potrf convention); xi and L_out are then
 *   unspecified.
 *   When info_dev is NULL the call synchronises the stream and returns
 *   ACE_E_NOT_PD on failure.
 * xi may be W itself (same pointer and ld: xi then overwrites W, through a
 * workspace copy of n_band orbitals); otherwise xi must not overlap psi or W.
 */
ace_status ace_compress(ace_ctx ctx, const ace_grid* grid, ace_prec prec,
                        const void* psi, long ld_psi, const void* W, long ld_W,
                        int n_band, void* xi, long ld_xi,
                        void* L_out, int* info_dev);

/*
 * Y = V_ACE X = -xi (dV xi^H X)                  (Section 3, Eq. ACE)
 * xi: n_band projection vectors; X, Y: n_x orbitals.  Y must not overlap xi or X.
 */
ace_status ace_apply(ace_ctx ctx, const ace_grid* grid, ace_prec prec,
                     const void* xi, int n_band, long ld_xi,
                     const void* X, int n_x, long ld_x, void* Y, long ld_y);

/*
 * Allocation-free variant of ace_apply, for callers that cannot allocate
 * device memory (code under HIP graph capture on a context whose workspace
 * was never sized, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, result and kernels as ace_apply; the scratch the kernels
 * need (the n_band x n_x matrix dV xi^H X and the reduction's split-K partial
 * sums) lives in a static device array of 48 MiB inside the library instead of
 * the context workspace, so the call allocates nothing, never synchronises and
 * never grows the workspace.  Each GPU that loads the library holds its own
 * copy of the array until the process ends.  Limit: the scratch must fit the
 * 48 MiB (n_band x n_x up to 256 x 256 at any supported grid and precision);
 * larger sizes return ACE_E_UNSUPPORTED before anything is enqueued.  All
 * calls on one GPU share that GPU's array: two calls that may overlap on one
 * GPU (other contexts, or other streams not ordered after this one) race and
 * must be serialised by the caller.
 */
ace_status ace_apply_noalloc(ace_ctx ctx, const ace_grid* grid, ace_prec prec,
                             const void* xi, int n_band, long ld_xi,
                             const void* X, int n_x, long ld_x, void* Y, long ld_y);

/*
 * Fock exchange energy of the n_occ orbitals phi, written to *ex_dev (one
 * device double).
 *  xi != NULL: E_X = -1/2 sum_{i,k} |<xi_k, phi_i>|^2   (Eq. EX_ACE, no Poisson solve)
 *  xi == NULL: E_X = -1/2 sum_{i,j} <rho_ji, v * rho_ji>, rho_ji = conj(phi_j) phi_i
 *              (Eq. EX), by forward FFTs of the pairs i <= j and Parseval.
 */
ace_status ace_exchange_energy(ace_ctx ctx, const ace_grid* grid, ace_prec prec,
                               const void* phi, int n_occ, long ld_phi,
                               const void* xi, int n_band, long ld_xi,
                               double* ex_dev);

/*
 * Orbital gradient of E_X(phi) = 1/2 sum_i <phi_i, V_X[phi] phi_i>  (Eq. EX),
 * written in the convention PyTorch uses for complex leaves (twice the
 * conjugate Wirtinger derivative), scaled by an upstream gradient:
 *   G_i = 2 gbar dE_X/dphi_i^* = 2 gbar dV (V_X[phi] phi)_i,
 * because each of the two conj(phi) factors of the quartic E_X contributes one
 * half.  gbar_dev: one device double (nullable: 1).  The pair FFTs are
 * recomputed, none is stored between forward and backward.  G: n_occ orbitals,
 * must not overlap phi.
 */
ace_status ace_exchange_energy_grad(ace_ctx ctx, const ace_grid* grid, ace_prec prec,
                                    const void* phi, int n_occ, long ld_phi,
                                    const double* gbar_dev, void* G, long ld_G);

/*
 * Orthonormalise n vectors: Q = X R^{-1} with <Q_a, Q_b> = delta_ab and R upper
 * triangular with positive real diagonal (the constraint of Eq. HF).  Computed
 * as two rounds of Cholesky QR (Gram matrix, Cholesky, triangular solve); the
 * Gram matrices as FP64 MFMA products for ACE_FP64, ACE_FP32 and ACE_REAL64,
 * FP32 MFMA products (FP32 accumulation inside each K chunk, FP64 across
 * chunks) for ACE_MIXED and ACE_REAL32; the Cholesky and the inverse in FP64.
 * Q must not overlap X.  info_dev as in ace_compress.
 */
ace_status ace_orthonormalize(ace_ctx ctx, const ace_grid* grid, ace_prec prec,
                              const void* X, int n, long ld_x, void* Q, long ld_q,
                              int* info_dev);

/*
 * Hamiltonian application for the linear eigenvalue problem of the inner
 * iterations (Section 2, Eq. HFlineig, with a fixed local potential standing
 * for V_ion + V_H; Alg. 1 applies V_X[phi] directly, Alg. 2 applies V_ACE):
 *   Y = -1/2 Laplacian X + V_loc X + V_ex X,
 *   V_ex = V_ACE = -xi (dV xi^H .)   when xi != NULL (n_xi vectors),
 *          scale_x V_X[phi]            when phi != NULL (n_phi orbitals; the
 *                                      pair solves of ace_build_W),
 *          0                           when both are NULL (not both non-NULL).
 * The Laplacian is spectral on the periodic grid: -1/2 Laplacian x =
 * ifftn(|G|^2/2 fftn(x)) with G = 2 pi m / L per axis (the same G as the
 * exchange kernel).  vloc (nullable): N_g reals in C order, double for ACE_FP64,
 * float for ACE_FP32 / ACE_MIXED.  Complex precisions only.  Y must not overlap
 * X, xi or phi.
 */
ace_status ace_apply_h(ace_ctx ctx, const ace_grid* grid, ace_prec prec, const void* vloc,
                       const void* xi, int n_xi, long ld_xi,
                       const void* phi, int n_phi, long ld_phi, double scale_x,
                       const void* X, int n_x, long ld_x, void* Y, long ld_y);

/*
 * D = a A + b B + c C on blocks of n orbitals (real coefficients; B and C
 * nullable, their terms then absent): the vector updates of polynomial
 * filters in the eigensolver.  D may be A, B or C itself (same ld).
 */
ace_status ace_combine(ace_ctx ctx, const ace_grid* grid, ace_prec prec, int n,
                       double a, const void* A, long ld_a, double b, const void* B, long ld_b,
                       double c, const void* C, long ld_c, void* D, long ld_d);

/*
 * Rayleigh-Ritz step on span(X) for the linear eigenvalue problem (Eq.
 * HFlineig): S = dV X^H (HX) (n x n, FP64 products, made Hermitian),
 * S = Q diag(e) Q^H with e ascending (parallel cyclic Jacobi in FP64,
 * n <= 512), Xout = X Q, HXout = (HX) Q (nullable), evals_dev = e (n device
 * doubles).  X should be orthonormal (<x_a, x_b> = delta_ab) and HX = H X.
 * The outputs must not overlap the inputs or each other.
 */
ace_status ace_rayleigh_ritz(ace_ctx ctx, const ace_grid* grid, ace_prec prec,
                             const void* X, long ld_x, const void* HX, long ld_hx, int n,
                             void* Xout, void* HXout, long ld_out, double* evals_dev);

/*
 * Batched build (Section 3 for many independent systems): for every instance,
 * W = scale * V_X[phi] psi as ace_build_W, then (when xi != NULL) the
 * compression of ace_compress with L not returned and the pivot status in
 * *info_dev (required then).  Instances may differ in grid, cell, kernel,
 * sizes and complex precision (ACE_FP64, ACE_FP32 or ACE_MIXED each).  Two
 * forms of the W stage (tuning knob ACE_TUNE_BATCH_FORM):
 *   1 (launches): each instance's pass kernels run on one of several
 *     concurrent branch streams (ACE_TUNE_BRANCHES, 1..16, default 4), each
 *     with its own workspace slice;
 *   2 (persistent): one persistent kernel per (grid size, precision) runs the
 *     passes of all instances of that size as tasks from a device queue with
 *     dependency counters, on the co-resident workgroups; it uses the
 *     one-thread-per-line slab and plane passes (ACE_TUNE_FFT_SHAPE 1 gives
 *     single calls with the same arithmetic) and caps each instance's pair
 *     budget so that one size's buffers stay within min(24 GiB, a quarter of
 *     the free device memory).  A wait that exceeds 10 s (a defect) ends the
 *     kernel and leaves NaN in W, which the compression reports as a failed
 *     factorisation.
 * The compressions run on the branch streams.  The whole batch is captured
 * into one HIP graph that is launched on the context stream.  A later call
 * with an identical instance array (same pointers, sizes and settings)
 * replays that graph without re-enqueueing and never synchronises; the data
 * behind the pointers may change between calls.  A call that captures anew
 * may wait for the context stream (when the workspace grows, and before the
 * task lists of the previous persistent graph are freed).  Instances run
 * concurrently, so an instance's W or xi overlapping another instance's W,
 * xi, phi or psi is an argument error (ACE_E_ARG, checked before anything is
 * enqueued); inputs may be shared.  xi may not alias W here.
 */
typedef struct {
  ace_grid grid;
  int prec;               /* ace_prec of this instance (complex precisions) */
  const void* phi; int n_occ; long ld_phi;
  const void* psi; int n_band; long ld_psi;
  void* W; long ld_W;
  void* xi; long ld_xi;   /* nullable: build only */
  int* info_dev;          /* device int, required when xi != NULL */
  double scale;
} ace_instance;
ace_status ace_build_W_batched(ace_ctx ctx, int n_inst, const ace_instance* inst);

/*
 * Autotuner of the build for one grid size and precision: times ace_build_W on
 * scratch orbitals (n_occ of n_band, allocated and freed here, so this call
 * allocates and synchronises) over candidate pair budgets (the number of pair
 * spectra in flight) and band blocks, then, at the fastest of those, over the
 * line shapes of the FFT passes (ACE_TUNE_FFT_SHAPE values 1, 4, 8 and 16) and
 * then the forms of the accumulate pass (ACE_TUNE_ACCUM_SHAPE 1 and 16), and
 * keeps the fastest in the context; later builds of that grid size and
 * element size use it where the explicit knobs are not set.  cache_path
 * (nullable; NULL means the context's tune_cache, if any): the result is
 * appended as a text line "n element_bytes budget jblock shape accum".
 * Outputs (nullable): the choice (shape or accum 0 = the defaults) and its time
 * per build in ms.  Complex precisions only (ACE_E_UNSUPPORTED for the real
 * ones).
 */
ace_status ace_autotune(ace_ctx ctx, const ace_grid* grid, ace_prec prec, int n_occ, int n_band,
                        const char* cache_path, long* best_budget, long* best_jblock,
                        int* best_shape, int* best_accum, double* best_ms);
/* Load tuning results written by ace_autotune (later lines win; a line
 * without the shape or accum field reads as 0 there). */
ace_status ace_tune_load(ace_ctx ctx, const char* cache_path);

/* Grid sizes n (per axis) compiled into this library; returns how many were
 * written (at most cap). */
int ace_supported_n(int* out, int cap);

/* Per-kernel timing: when enabled every kernel launch is bracketed by HIP
 * events on the context stream.  ace_profile_get synchronises the stream and
 * reports, for entry idx, the kernel name, launch count and total time. */
ace_status ace_profile_enable(ace_ctx ctx, int on);
ace_status ace_profile_reset(ace_ctx ctx);
int ace_profile_count(ace_ctx ctx);
ace_status ace_profile_get(ace_ctx ctx, int idx, const char** name, long* launches,
                           double* total_ms);

/* Tuning knob: device bytes the build may use for in-flight pair spectra
 * (the FFT intermediates of a block of pairs).  0 restores the default. */
ace_status ace_set_pair_budget(ace_ctx ctx, long bytes);

/* Tuning knobs of the build (values >= 0):
 *  ACE_TUNE_PAIR_BUDGET  same as ace_set_pair_budget (bytes; 0 = default)
 *  ACE_TUNE_JBLOCK       bands j per pair block of the build (0 = all)
 *  ACE_TUNE_SYMMETRY     1 (default): when psi's first n_occ orbitals are phi
 *                        (same pointer and ld), FFT only the pairs i <= j of the
 *                        occupied block and use u_ji = conj(u_ij); 0: all pairs
 *  ACE_TUNE_FFT_SHAPE    line FFTs of the slab and plane passes: 1 one thread
 *                        per line, 4 a lane quad per line, 8 an octet of lanes
 *                        per line (grids whose n is a multiple of 8 from 16;
 *                        quads otherwise), 16 a line split over four lanes 16
 *                        apart, 0 (default) automatic
 *  ACE_TUNE_ACCUM_SHAPE  accumulate pass: 1 one thread per pencil (accumulator
 *                        in LDS), 16 a pencil split over four lanes 16 apart
 *                        (accumulator in registers), 0 (default) automatic
 *  ACE_TUNE_BRANCHES     concurrent branch streams of ace_build_W_batched
 *                        (1..16; 0 restores the default 4)
 *  ACE_TUNE_BATCH_FORM   W stage of ace_build_W_batched: 1 launches on branch
 *                        streams, 2 persistent kernels, 0 (default) form 1
 * They change speed only; results agree to rounding. */
enum { ACE_TUNE_PAIR_BUDGET = 0, ACE_TUNE_JBLOCK = 1, ACE_TUNE_SYMMETRY = 2,
       ACE_TUNE_FFT_SHAPE = 3, ACE_TUNE_ACCUM_SHAPE = 4, ACE_TUNE_BRANCHES = 5,
       ACE_TUNE_BATCH_FORM = 6 };
ace_status ace_set_tuning(ace_ctx ctx, int key, long value);
ace_status ace_get_tuning(ace_ctx ctx, int key, long* value);

const char* ace_status_string(ace_status s);
const char* ace_last_error(ace_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* ACE_H */
