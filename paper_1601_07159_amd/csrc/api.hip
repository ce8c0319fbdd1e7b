// C ABI of libace: argument validation, workspace, dispatch to the kernels.
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <new>

#include "ace_internal.h"

#define ACE_EXPORT extern "C" __attribute__((visibility("default")))

namespace ace {

void log_line(ace_ctx c, const char* fmt, ...) {
  if (!c || !c->log) return;
  va_list ap;
  va_start(ap, fmt);
  std::fputs("[ace] ", c->log);
  std::vfprintf(c->log, fmt, ap);
  std::fputc('\n', c->log);
  va_end(ap);
  std::fflush(c->log);
}

ace_status fail(ace_ctx c, ace_status s, const std::string& msg) {
  if (c) {
    c->last_error = msg;
    log_line(c, "%s: %s", ace_status_string(s), msg.c_str());
  }
  return s;
}

const ace_ctx_s::Tuned* tuned_for(ace_ctx c, int n, int eb) {
  if (c->tune_mode == 0) return nullptr;
  for (const auto& t : c->tuned)
    if (t.n == n && t.eb == eb) return &t;
  return nullptr;
}

ace_status hip_fail(ace_ctx c, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(c, ACE_E_HIP, m);
}

bool stream_capturing(ace_ctx c) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const hipError_t e = hipStreamIsCapturing(c->stream, &cs);
  if (e == hipErrorStreamCaptureImplicit || e == hipErrorStreamCaptureUnsupported) {
    (void)hipGetLastError();
    return true;  // the legacy stream while another stream captures globally
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return cs != hipStreamCaptureStatusNone;
}

ace_status ws_begin(ace_ctx c, size_t total) {
  total = align_up(total ? total : 256, 256);
  if (c->sub_base) {
    c->ws_used = 0;
    if (total > c->sub_bytes) return fail(c, ACE_E_NOMEM, "internal: batched workspace plan");
    return ACE_OK;
  }
  c->ws_used = c->ws_prefix;
  if (c->ws_prefix + total <= c->ws_bytes) return ACE_OK;
  if (c->ws_prefix) return fail(c, ACE_E_NOMEM, "internal: workspace plan with a kept prefix");
  // Growing synchronises and allocates, neither of which a stream capture
  // allows: refuse before touching the capture or the current buffer.
  if (stream_capturing(c))
    return fail(c, ACE_E_CAPTURE,
                "the workspace must grow, which is not possible while the stream is captured "
                "(call ace_reserve, or the same call once, before capturing)");
  if (c->ws) {
    // queued kernels of earlier calls may still use the old buffer; every call
    // of the context is ordered on its stream (ace_set_stream chains a new
    // stream after the old one), so waiting for that stream suffices
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize(workspace)");
    e = hipFree(c->ws);
    if (e != hipSuccess) return hip_fail(c, e, "hipFree(workspace)");
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, total);
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    char buf[128];
    snprintf(buf, sizeof buf, "workspace allocation of %zu bytes failed", total);
    return fail(c, ACE_E_NOMEM, buf);
  }
  c->ws = p;
  c->ws_bytes = total;
  log_line(c, "workspace grown to %.1f MiB", total / 1048576.0);
  return ACE_OK;
}

void* ws_take(ace_ctx c, size_t bytes, ace_status* st) {
  bytes = align_up(bytes ? bytes : 256, 256);
  char* base = c->sub_base ? c->sub_base : (char*)c->ws;
  const size_t limit = c->sub_base ? c->sub_bytes : c->ws_bytes;
  if (c->ws_used + bytes > limit) {
    *st = fail(c, ACE_E_NOMEM, "internal: workspace carve exceeds reservation");
    return nullptr;
  }
  void* p = base + c->ws_used;
  c->ws_used += bytes;
  return p;
}

size_t orth_ws_bytes(int n, long ng, size_t eb) {
  const size_t mat = align_up((size_t)n * n * sizeof(cx<double>), 256);
  const size_t tmp = align_up((size_t)n * ng * eb, 256);
  const size_t scr = align_up(chol_scratch_elems(n) * sizeof(cx<double>), 256);
  return 2 * mat + scr + 2 * 256 + tmp + 2 * gemm_cn_scratch_bytes(n, n, ng);
}

size_t compress_ws_bytes(int nb, long ng, size_t alias_eb) {
  const size_t mat = align_up((size_t)nb * nb * sizeof(cx<double>), 256);
  const size_t scr = align_up(chol_scratch_elems(nb) * sizeof(cx<double>), 256);
  const size_t copy = alias_eb ? align_up((size_t)nb * ng * alias_eb, 256) : 0;
  return 2 * mat + scr + 256 + gemm_cn_scratch_bytes(nb, nb, ng) + copy;
}

void prof_begin(ace_ctx c, const char* name, int* entry, hipEvent_t* e0) {
  int idx = -1;
  for (size_t k = 0; k < c->prof.size(); ++k)
    if (c->prof[k].name == name) idx = (int)k;
  if (idx < 0) {
    c->prof.push_back({name, 0, 0.0});
    idx = (int)c->prof.size() - 1;
  }
  hipEvent_t e = nullptr;
  if (!c->free_events.empty()) {
    e = c->free_events.back();
    c->free_events.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  if (e) hipEventRecord(e, c->stream);
  *entry = idx;
  *e0 = e;
}

void prof_end(ace_ctx c, int entry, hipEvent_t e0) {
  if (!e0) return;
  hipEvent_t e1 = nullptr;
  if (!c->free_events.empty()) {
    e1 = c->free_events.back();
    c->free_events.pop_back();
  } else if (hipEventCreate(&e1) != hipSuccess) {
    c->free_events.push_back(e0);
    return;
  }
  hipEventRecord(e1, c->stream);
  c->pending.push_back({entry, e0, e1});
}

static void prof_collect(ace_ctx c) {
  for (auto& p : c->pending) {
    hipEventSynchronize(p.e1);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
      c->prof[p.entry].ms += ms;
      c->prof[p.entry].launches += 1;
    }
    c->free_events.push_back(p.e0);
    c->free_events.push_back(p.e1);
  }
  c->pending.clear();
}

static bool grid_supported(int n) {
  switch (n) {
#define ACE_CASE(NV) \
  case NV:           \
    return true;
    ACE_FOR_EACH_N(ACE_CASE)
#undef ACE_CASE
    default:
      return false;
  }
}

ace_status check_grid(ace_ctx c, const ace_grid* g, ace_prec prec, GridInfo* out) {
  if (!g) return fail(c, ACE_E_ARG, "grid is NULL");
  if (prec != ACE_FP64 && prec != ACE_FP32 && prec != ACE_MIXED && prec != ACE_REAL32 &&
      prec != ACE_REAL64)
    return fail(c, ACE_E_ARG, "unknown precision");
  for (int a = 0; a < 3; ++a) {
    if (g->n[a] <= 0) return fail(c, ACE_E_ARG, "grid size must be positive");
    if (!(g->L[a] > 0.0) || !std::isfinite(g->L[a]))
      return fail(c, ACE_E_ARG, "cell edges must be positive and finite");
  }
  if (g->kind != ACE_COULOMB && g->kind != ACE_ERFC) return fail(c, ACE_E_ARG, "unknown kernel");
  if (g->kind == ACE_ERFC && !(g->mu > 0.0 && std::isfinite(g->mu)))
    return fail(c, ACE_E_ARG, "screened kernel needs mu > 0");
  if (!std::isfinite(g->g0)) return fail(c, ACE_E_ARG, "g0 must be finite");
  if (g->n[0] != g->n[1] || g->n[1] != g->n[2] || !grid_supported(g->n[0]))
    return fail(c, ACE_E_UNSUPPORTED, "grid must be cubic with n listed by ace_supported_n");
  out->n = g->n[0];
  out->ng = (long)g->n[0] * g->n[1] * g->n[2];
  for (int a = 0; a < 3; ++a) out->L[a] = g->L[a];
  out->kind = g->kind;
  out->mu = g->mu;
  out->g0 = g->g0;
  out->omega = g->L[0] * g->L[1] * g->L[2];
  out->dV = out->omega / (double)out->ng;
  return ACE_OK;
}

size_t elem_bytes(ace_prec p) {
  switch (p) {
    case ACE_FP64: return 16;
    case ACE_REAL32: return 4;
    case ACE_REAL64: return 8;
    default: return 8;
  }
}

static bool is_real(ace_prec p) { return p == ACE_REAL32 || p == ACE_REAL64; }

// Real orbitals reuse the complex reduction/expansion kernels on N_g / 2
// complex pairs (x0 + i x1, x2 + i x3, ...): the real part of a complex dot
// product of two such views is the real dot product, and a real small matrix
// maps pairs to pairs.  Needs an even ld and pair-aligned orbital starts.
static ace_status check_real_view(ace_ctx c, const void* p, long ld, size_t eb,
                                  const char* what) {
  if (ld % 2 != 0 || ((uintptr_t)p % (2 * eb)) != 0)
    return fail(c, ACE_E_ARG, std::string(what) +
                                  ": real orbitals need an even ld and a start aligned to two values");
  return ACE_OK;
}

static GridInfo half_view(const GridInfo& g) {
  GridInfo h = g;
  h.ng = g.ng / 2;  // every supported n is even
  return h;
}

Span span_of(const void* p, int count, long ld, long ng, size_t eb) {
  const char* b = (const char*)p;
  return {b, b + ((size_t)(count - 1) * ld + ng) * eb};
}
bool overlap(Span a, Span b) { return a.lo < b.hi && b.lo < a.hi; }

ace_status check_block(ace_ctx c, const void* p, int count, long ld, const GridInfo& g,
                              const char* what) {
  if (!p) return fail(c, ACE_E_ARG, std::string(what) + " is NULL");
  if (count < 1) return fail(c, ACE_E_ARG, std::string(what) + ": count must be >= 1");
  if (ld < g.ng) return fail(c, ACE_E_ARG, std::string(what) + ": ld < N_g");
  return ACE_OK;
}


// Cholesky failure reporting shared by compress and orthonormalize.
static ace_status finish_info(ace_ctx c, int* info_ws, int* info_dev) {
  if (info_dev) {
    hipError_t e = hipMemcpyAsync(info_dev, info_ws, sizeof(int), hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync(info)");
    return ACE_OK;
  }
  int h = 0;
  hipError_t e = hipMemcpyAsync(&h, info_ws, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "info readback");
  if (h != 0) {
    char buf[96];
    snprintf(buf, sizeof buf, "matrix not positive definite: pivot %d", h);
    return fail(c, ACE_E_NOT_PD, buf);
  }
  return ACE_OK;
}

template <typename T>
ace_status compress_impl(ace_ctx c, const GridInfo& g, const cx<T>* psi, long ldpsi,
                         const cx<T>* W, long ldW, int nb, cx<T>* xi, long ldxi,
                         cx<double>* L_out, int* info_dev, CnMode mode, bool real) {
  const size_t mat = align_up((size_t)nb * nb * sizeof(cx<double>), 256);
  // xi == W: the expansion's column blocks read every column of W for their
  // rows, so xi is formed in a workspace copy and copied over W at the end
  const bool alias = (const void*)xi == (const void*)W;
  ACE_TRY(ws_begin(c, compress_ws_bytes(nb, g.ng, alias ? sizeof(cx<T>) : 0)));
  ace_status st = ACE_OK;
  cx<double>* M = (cx<double>*)ws_take(c, mat, &st);
  cx<double>* X = (cx<double>*)ws_take(c, chol_scratch_elems(nb) * sizeof(cx<double>), &st);
  cx<double>* C = (cx<double>*)ws_take(c, mat, &st);
  int* info = (int*)ws_take(c, 256, &st);
  cx<T>* tmp = alias ? (cx<T>*)ws_take(c, (size_t)nb * g.ng * sizeof(cx<T>), &st) : nullptr;
  if (!M || !X || !C || !info || (alias && !tmp)) return st;
  // M = dV psi^H W; M is Hermitian (V_X is): its upper triangle of tiles
  // defines it
  ACE_TRY(gemm_cn<T>(c, psi, ldpsi, nb, W, ldW, nb, g.ng, g.dV, M, nb, mode, real, true));
  // -M made exactly Hermitian, -M = L L^H, C = L^{-H}
  ACE_TRY(chol_inv(c, M, nb, -1.0, L_out, C, X, info, nullptr, real));
  ACE_TRY(gemm_nn<T>(c, W, ldW, nb, C, nb, nb, alias ? tmp : xi, alias ? g.ng : ldxi, g.ng, true,
                     true));
  if (alias) {
    const hipError_t e = hipMemcpy2DAsync(xi, (size_t)ldxi * sizeof(cx<T>), tmp,
                                          (size_t)g.ng * sizeof(cx<T>), (size_t)g.ng * sizeof(cx<T>),
                                          (size_t)nb, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy2DAsync(xi)");
  }
  return finish_info(c, info, info_dev);
}

template ace_status compress_impl<float>(ace_ctx, const GridInfo&, const cx<float>*, long,
                                         const cx<float>*, long, int, cx<float>*, long,
                                         cx<double>*, int*, CnMode, bool);
template ace_status compress_impl<double>(ace_ctx, const GridInfo&, const cx<double>*, long,
                                          const cx<double>*, long, int, cx<double>*, long,
                                          cx<double>*, int*, CnMode, bool);

template <typename T>
static ace_status apply_t(ace_ctx c, const GridInfo& g, const cx<T>* xi, int nb, long ldxi,
                          const cx<T>* X, int nx, long ldx, cx<T>* Y, long ldy,
                          bool real = false) {
  const size_t mat = align_up((size_t)nb * nx * sizeof(cx<double>), 256);
  ACE_TRY(ws_begin(c, mat + gemm_cn_partial_bytes(nb, nx, g.ng, sizeof(cx<T>), kNative, false)));
  ace_status st = ACE_OK;
  cx<double>* C = (cx<double>*)ws_take(c, mat, &st);
  if (!C) return st;
  ACE_TRY(gemm_cn<T>(c, xi, ldxi, nb, X, ldx, nx, g.ng, -g.dV, C, nb, kNative, real));
  return gemm_nn<T>(c, xi, ldxi, nb, C, nb, nx, Y, ldy, g.ng, false);
}

template <typename T>
static ace_status energy_ace_t(ace_ctx c, const GridInfo& g, const cx<T>* phi, int nocc,
                               long ldphi, const cx<T>* xi, int nb, long ldxi, double* ex,
                               bool real = false) {
  const size_t mat = align_up((size_t)nb * nocc * sizeof(cx<double>), 256);
  ACE_TRY(ws_begin(c, mat + gemm_cn_scratch_bytes(nb, nocc, g.ng)));
  ace_status st = ACE_OK;
  cx<double>* C = (cx<double>*)ws_take(c, mat, &st);
  if (!C) return st;
  ACE_TRY(gemm_cn<T>(c, xi, ldxi, nb, phi, ldphi, nocc, g.ng, g.dV, C, nb, kNative, real));
  return sumsq(c, C, (long)nb * nocc, -0.5, ex);
}

template <typename T>
static ace_status orth_t(ace_ctx c, const GridInfo& g, const cx<T>* X, int n, long ldx, cx<T>* Q,
                         long ldq, int* info_dev, CnMode mode, bool real = false) {
  const size_t mat = align_up((size_t)n * n * sizeof(cx<double>), 256);
  const size_t tmp = align_up((size_t)n * g.ng * sizeof(cx<T>), 256);
  const size_t scr = align_up(chol_scratch_elems(n) * sizeof(cx<double>), 256);
  ACE_TRY(ws_begin(c, orth_ws_bytes(n, g.ng, sizeof(cx<T>))));
  ace_status st = ACE_OK;
  cx<double>* S = (cx<double>*)ws_take(c, mat, &st);
  cx<double>* Xs = (cx<double>*)ws_take(c, scr, &st);
  cx<double>* C = (cx<double>*)ws_take(c, mat, &st);
  int* info1 = (int*)ws_take(c, 256, &st);
  int* info2 = (int*)ws_take(c, 256, &st);
  cx<T>* Y = (cx<T>*)ws_take(c, tmp, &st);
  if (!S || !Xs || !C || !info1 || !info2 || !Y) return st;
  // first pass: Y = X R1^{-1}, S = dV X^H X = R1^H R1 with R1 = L^H
  ACE_TRY(gemm_cn<T>(c, X, ldx, n, X, ldx, n, g.ng, g.dV, S, n, mode, real, true));
  ACE_TRY(chol_inv(c, S, n, 1.0, nullptr, C, Xs, info1, nullptr, real));
  ACE_TRY(gemm_nn<T>(c, X, ldx, n, C, n, n, Y, g.ng, g.ng, true, true));
  // the second pass on Y restores orthogonality lost to rounding in the first
  ACE_TRY(gemm_cn<T>(c, Y, g.ng, n, Y, g.ng, n, g.ng, g.dV, S, n, mode, real, true));
  ACE_TRY(chol_inv(c, S, n, 1.0, nullptr, C, Xs, info2, info1, real));
  ACE_TRY(gemm_nn<T>(c, Y, g.ng, n, C, n, n, Q, ldq, g.ng, true, true));
  return finish_info(c, info2, info_dev);
}

}  // namespace ace

using namespace ace;

ACE_EXPORT const char* ace_status_string(ace_status s) {
  switch (s) {
    case ACE_OK: return "ok";
    case ACE_E_ARG: return "invalid argument";
    case ACE_E_NOT_PD: return "matrix not positive definite";
    case ACE_E_NOMEM: return "out of device memory";
    case ACE_E_HIP: return "HIP runtime error";
    case ACE_E_UNSUPPORTED: return "unsupported configuration";
    case ACE_E_CAPTURE: return "not allowed while the stream is being captured";
  }
  return "unknown status";
}

ACE_EXPORT const char* ace_last_error(ace_ctx c) { return c ? c->last_error.c_str() : ""; }

ACE_EXPORT int ace_supported_n(int* out, int cap) {
  static const int list[] = {
#define ACE_ITEM(NV) NV,
      ACE_FOR_EACH_N(ACE_ITEM)
#undef ACE_ITEM
  };
  const int count = (int)(sizeof(list) / sizeof(list[0]));
  int k = 0;
  for (; k < count && k < cap; ++k)
    if (out) out[k] = list[k];
  return out ? k : count;
}

ACE_EXPORT ace_status ace_create(ace_ctx* out, void* stream, const char* tune_cache) {
  if (!out) return ACE_E_ARG;
  *out = nullptr;
  ace_ctx c = new (std::nothrow) ace_ctx_s();
  if (!c) return ACE_E_NOMEM;
  c->stream = (hipStream_t)stream;
  // ACE_LOG: "1" or "stderr" logs to stderr, another non-empty value other
  // than "0" names a file the log is appended to
  if (const char* lg = std::getenv("ACE_LOG")) {
    if (!std::strcmp(lg, "1") || !std::strcmp(lg, "stderr")) {
      c->log = stderr;
    } else if (*lg && std::strcmp(lg, "0")) {
      c->log = std::fopen(lg, "a");
      c->log_owned = c->log != nullptr;
    }
  }
  if (const char* tm = std::getenv("ACE_TUNE")) {
    if (!std::strcmp(tm, "0")) c->tune_mode = 0;
    else if (!std::strcmp(tm, "1")) c->tune_mode = 1;
  }
  // ACE_TUNE_CACHE names the tuning cache when the caller passes none
  if (!tune_cache) {
    const char* env = std::getenv("ACE_TUNE_CACHE");
    if (env && *env) tune_cache = env;
  }
  if (tune_cache) {
    c->tune_cache = tune_cache;
    // a cache not written yet is not an error
    const bool found = tune_cache_read(c, tune_cache);
    log_line(c, "tuning cache %s: %s, %zu settings", tune_cache, found ? "read" : "not found",
             c->tuned.size());
  }
  if (hipGetDevice(&c->device) != hipSuccess) {
    if (c->log_owned) std::fclose(c->log);
    delete c;
    return ACE_E_HIP;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) ==
          hipSuccess &&
      cus > 0)
    c->num_cus = cus;
  noalloc_setup(c->device);  // device address of the allocation-free apply's scratch
  log_line(c, "context on device %d (%d CUs), stream %p, ACE_TUNE mode %d", c->device,
           c->num_cus, stream, c->tune_mode);
  *out = c;
  return ACE_OK;
}

ACE_EXPORT ace_status ace_destroy(ace_ctx c) {
  if (!c) return ACE_E_ARG;
  if (c->graph_exec) hipGraphExecDestroy(c->graph_exec);
  for (auto s : c->branch_streams) {
    hipStreamSynchronize(s);
    hipStreamDestroy(s);
  }
  for (auto e : c->branch_events) hipEventDestroy(e);
  if (c->capture_stream) {
    hipStreamSynchronize(c->capture_stream);
    hipStreamDestroy(c->capture_stream);
  }
  if (c->fork_event) hipEventDestroy(c->fork_event);
  if (c->stream_event) hipEventDestroy(c->stream_event);
  if (c->ws || !c->graph_bufs.empty()) hipStreamSynchronize(c->stream);
  if (c->ws) hipFree(c->ws);
  for (void* p : c->graph_bufs) hipFree(p);
  for (auto& p : c->pending) {
    hipEventDestroy(p.e0);
    hipEventDestroy(p.e1);
  }
  for (auto e : c->free_events) hipEventDestroy(e);
  if (c->log_owned) std::fclose(c->log);
  delete c;
  return ACE_OK;
}

ACE_EXPORT ace_status ace_set_stream(ace_ctx c, void* stream) {
  if (!c) return ACE_E_ARG;
  const hipStream_t next = (hipStream_t)stream;
  if (next == c->stream) return ACE_OK;
  // The calls share one workspace: the new stream waits for what the old one
  // has queued (skipped when either is capturing; the caller orders them then).
  const hipStream_t prev = c->stream;
  const bool prev_cap = stream_capturing(c);
  c->stream = next;
  const bool next_cap = stream_capturing(c);
  if (prev_cap || next_cap) return ACE_OK;
  if (!c->stream_event) {
    const hipError_t e = hipEventCreateWithFlags(&c->stream_event, hipEventDisableTiming);
    if (e != hipSuccess) {
      c->stream_event = nullptr;
      c->stream = prev;
      return hip_fail(c, e, "hipEventCreateWithFlags");
    }
  }
  hipError_t e = hipEventRecord(c->stream_event, prev);
  if (e == hipSuccess) e = hipStreamWaitEvent(next, c->stream_event, 0);
  if (e != hipSuccess) return hip_fail(c, e, "ordering the new stream");
  return ACE_OK;
}

ACE_EXPORT ace_status ace_set_pair_budget(ace_ctx c, long bytes) {
  if (!c || bytes < 0) return ACE_E_ARG;
  c->pair_budget = (size_t)bytes;
  return ACE_OK;
}

ACE_EXPORT ace_status ace_set_tuning(ace_ctx c, int key, long value) {
  if (!c || value < 0) return ACE_E_ARG;
  switch (key) {
    case ACE_TUNE_PAIR_BUDGET: c->pair_budget = (size_t)value; return ACE_OK;
    case ACE_TUNE_JBLOCK: c->jblock = value; return ACE_OK;
    case ACE_TUNE_SYMMETRY: c->use_symmetry = value != 0; return ACE_OK;
    case ACE_TUNE_FFT_SHAPE:
      if (value != 0 && value != 1 && value != 4 && value != 8 && value != 16)
        return fail(c, ACE_E_ARG, "fft shape 0, 1, 4, 8 or 16");
      c->fft_shape = (int)value;
      return ACE_OK;
    case ACE_TUNE_ACCUM_SHAPE:
      if (value != 0 && value != 1 && value != 16)
        return fail(c, ACE_E_ARG, "accumulate shape 0, 1 or 16");
      c->accum_shape = (int)value;
      return ACE_OK;
    case ACE_TUNE_BRANCHES:
      if (value > 16) return fail(c, ACE_E_ARG, "branches 1..16 (0 = default)");
      c->branches = value ? (int)value : 4;
      return ACE_OK;
    case ACE_TUNE_BATCH_FORM:
      if (value > 2) return fail(c, ACE_E_ARG, "batch form 0, 1 or 2");
      c->batch_form = (int)value;
      return ACE_OK;
    default: return fail(c, ACE_E_ARG, "unknown tuning key");
  }
}

ACE_EXPORT ace_status ace_get_tuning(ace_ctx c, int key, long* value) {
  if (!c || !value) return ACE_E_ARG;
  switch (key) {
    case ACE_TUNE_PAIR_BUDGET: *value = (long)c->pair_budget; return ACE_OK;
    case ACE_TUNE_JBLOCK: *value = c->jblock; return ACE_OK;
    case ACE_TUNE_SYMMETRY: *value = c->use_symmetry ? 1 : 0; return ACE_OK;
    case ACE_TUNE_FFT_SHAPE: *value = c->fft_shape; return ACE_OK;
    case ACE_TUNE_ACCUM_SHAPE: *value = c->accum_shape; return ACE_OK;
    case ACE_TUNE_BRANCHES: *value = c->branches; return ACE_OK;
    case ACE_TUNE_BATCH_FORM: *value = c->batch_form; return ACE_OK;
    default: return fail(c, ACE_E_ARG, "unknown tuning key");
  }
}

ACE_EXPORT ace_status ace_reserve(ace_ctx c, const ace_grid* grid, ace_prec prec, int max_nocc,
                                  int max_nband, int max_nx) {
  if (!c) return ACE_E_ARG;
  GridInfo g;
  ACE_TRY(check_grid(c, grid, prec, &g));
  if (max_nocc < 1 || max_nband < 1 || max_nx < 0) return fail(c, ACE_E_ARG, "sizes");
  const size_t eb = elem_bytes(prec);
  // the largest workspace any call with these sizes takes (so that later
  // calls, also under graph capture, need no allocation)
  const int nmax = std::max(max_nband, std::max(max_nx, max_nocc));
  const size_t mat = align_up((size_t)nmax * nmax * sizeof(cx<double>), 256);
  if (is_real(prec)) {
    const GridInfo gh = half_view(g);
    size_t need = 0;
    for (int symm = 0; symm < 2; ++symm) {
      need = std::max(need, plan_build_real(c, g, 2 * eb, max_nocc, max_nband, symm).bytes);
      need = std::max(need, plan_build_real(c, g, 2 * eb, max_nocc, max_nocc, symm).bytes);
    }
    need = std::max(need, compress_ws_bytes(max_nband, gh.ng, 2 * eb));
    need = std::max(need, orth_ws_bytes(nmax, gh.ng, 2 * eb));
    need = std::max(need, mat + gemm_cn_scratch_bytes(max_nband, std::max(max_nx, 1), gh.ng));
    need = std::max(need, mat + gemm_cn_scratch_bytes(max_nband, max_nocc, gh.ng));
    return ws_begin(c, need);
  }
  size_t need = std::max(plan_build(c, g, eb, max_nocc, max_nband, true).bytes,
                         plan_build(c, g, eb, max_nocc, max_nband, false).bytes);
  need = std::max(need, plan_build(c, g, eb, max_nocc, max_nocc, true).bytes);
  need = std::max(need, compress_ws_bytes(max_nband, g.ng, eb));
  need = std::max(need, orth_ws_bytes(nmax, g.ng, eb));
  need = std::max(need, mat + gemm_cn_scratch_bytes(max_nband, std::max(max_nx, 1), g.ng));
  need = std::max(need, mat + gemm_cn_scratch_bytes(max_nband, max_nocc, g.ng));
  need = std::max(need, energy_direct_ws_bytes(c, g, eb, max_nocc));
  // ace_apply_h (exchange from xi or from the occupied orbitals) and the
  // Rayleigh-Ritz step of the eigensolver on up to max(n_band, n_x) vectors
  need = std::max(need, hamiltonian_ws_bytes(c, g, eb, std::max(max_nx, 1), max_nband, max_nocc));
  need = std::max(need, 4 * mat + gemm_cn_scratch_bytes(nmax, nmax, g.ng));
  return ws_begin(c, need);
}

ACE_EXPORT ace_status ace_build_W(ace_ctx c, const ace_grid* grid, ace_prec prec, const void* phi,
                                  int n_occ, long ld_phi, const void* psi, int n_band, long ld_psi,
                                  void* W, long ld_W, double scale) {
  if (!c) return ACE_E_ARG;
  GridInfo g;
  ACE_TRY(check_grid(c, grid, prec, &g));
  ACE_TRY(check_block(c, phi, n_occ, ld_phi, g, "phi"));
  ACE_TRY(check_block(c, psi, n_band, ld_psi, g, "psi"));
  ACE_TRY(check_block(c, W, n_band, ld_W, g, "W"));
  if (!std::isfinite(scale)) return fail(c, ACE_E_ARG, "scale must be finite");
  const size_t eb = elem_bytes(prec);
  const Span sw = span_of(W, n_band, ld_W, g.ng, eb);
  if (overlap(sw, span_of(phi, n_occ, ld_phi, g.ng, eb)) ||
      overlap(sw, span_of(psi, n_band, ld_psi, g.ng, eb)))
    return fail(c, ACE_E_ARG, "W overlaps an input");
  if (c->tune_mode == 1 && (prec == ACE_FP64 || prec == ACE_FP32 || prec == ACE_MIXED) &&
      !tuned_for(c, g.n, (int)eb) && !stream_capturing(c)) {
    // ACE_TUNE=1: tune this grid size and element size once, on scratch
    // orbitals of this call's sizes (allocates and synchronises); a failed
    // tuning run is logged and the defaults are kept for this size
    long bb = 0, bj = 0;
    int bs = 0, ba = 0;
    double ms = 0.0;
    const ace_status ts = ace_autotune(c, grid, prec, n_occ, n_band, nullptr, &bb, &bj, &bs,
                                       &ba, &ms);
    if (ts == ACE_OK) {
      log_line(c, "tuned n=%d elem_bytes=%zu: budget %ld, band block %ld, shape %d, accum %d "
               "(%.3f ms per build)", g.n, eb, bb, bj, bs, ba, ms);
    } else {
      log_line(c, "tuning n=%d elem_bytes=%zu failed (%s); defaults kept", g.n, eb,
               ace_status_string(ts));
      c->tuned.push_back({g.n, (int)eb, 0, 0, 0, 0});
      ++c->tune_gen;
      c->last_error.clear();
    }
  }
  if (prec == ACE_REAL64)
    return build_W_real_impl<double>(c, g, (const double*)phi, n_occ, ld_phi, (const double*)psi,
                                     n_band, ld_psi, (double*)W, ld_W, scale);
  if (prec == ACE_REAL32)
    return build_W_real_impl<float>(c, g, (const float*)phi, n_occ, ld_phi, (const float*)psi,
                                    n_band, ld_psi, (float*)W, ld_W, scale);
  if (prec == ACE_FP64)
    return build_W_impl<double>(c, g, (const cx<double>*)phi, n_occ, ld_phi,
                                (const cx<double>*)psi, n_band, ld_psi, (cx<double>*)W, ld_W,
                                scale);
  return build_W_impl<float>(c, g, (const cx<float>*)phi, n_occ, ld_phi, (const cx<float>*)psi,
                             n_band, ld_psi, (cx<float>*)W, ld_W, scale);
}

ACE_EXPORT ace_status ace_compress(ace_ctx c, const ace_grid* grid, ace_prec prec, const void* psi,
                                   long ld_psi, const void* W, long ld_W, int n_band, void* xi,
                                   long ld_xi, void* L_out, int* info_dev) {
  if (!c) return ACE_E_ARG;
  GridInfo g;
  ACE_TRY(check_grid(c, grid, prec, &g));
  ACE_TRY(check_block(c, psi, n_band, ld_psi, g, "psi"));
  ACE_TRY(check_block(c, W, n_band, ld_W, g, "W"));
  ACE_TRY(check_block(c, xi, n_band, ld_xi, g, "xi"));
  if (n_band > 4096) return fail(c, ACE_E_UNSUPPORTED, "n_band above 4096");
  const size_t eb = elem_bytes(prec);
  const Span sx = span_of(xi, n_band, ld_xi, g.ng, eb);
  const bool alias = xi == W && ld_xi == ld_W;
  if (overlap(sx, span_of(psi, n_band, ld_psi, g.ng, eb)) ||
      (!alias && overlap(sx, span_of(W, n_band, ld_W, g.ng, eb))))
    return fail(c, ACE_E_ARG, "xi overlaps an input (it may only be W itself, same ld)");
  if (!info_dev && stream_capturing(c))
    return fail(c, ACE_E_CAPTURE, "info_dev == NULL synchronises, which a capture does not allow");
  if (is_real(prec)) {
    ACE_TRY(check_real_view(c, psi, ld_psi, eb, "psi"));
    ACE_TRY(check_real_view(c, W, ld_W, eb, "W"));
    ACE_TRY(check_real_view(c, xi, ld_xi, eb, "xi"));
    const GridInfo gh = half_view(g);
    if (prec == ACE_REAL64)
      return compress_impl<double>(c, gh, (const cx<double>*)psi, ld_psi / 2,
                                   (const cx<double>*)W, ld_W / 2, n_band, (cx<double>*)xi,
                                   ld_xi / 2, (cx<double>*)L_out, info_dev, kNative, true);
    return compress_impl<float>(c, gh, (const cx<float>*)psi, ld_psi / 2, (const cx<float>*)W,
                                ld_W / 2, n_band, (cx<float>*)xi, ld_xi / 2, (cx<double>*)L_out,
                                info_dev, compress_mode(prec), true);
  }
  if (prec == ACE_FP64)
    return compress_impl<double>(c, g, (const cx<double>*)psi, ld_psi, (const cx<double>*)W, ld_W,
                                 n_band, (cx<double>*)xi, ld_xi, (cx<double>*)L_out, info_dev,
                                 kNative);
  return compress_impl<float>(c, g, (const cx<float>*)psi, ld_psi, (const cx<float>*)W, ld_W, n_band,
                              (cx<float>*)xi, ld_xi, (cx<double>*)L_out, info_dev,
                              compress_mode(prec));
}

namespace ace {
// The apply on the context workspace (sub == nullptr) or on a caller-provided
// device arena [sub, sub + sub_bytes) that it never grows (sizes that need
// more are refused before anything is enqueued).
ace_status apply_entry(ace_ctx c, const ace_grid* grid, ace_prec prec, const void* xi, int n_band,
                       long ld_xi, const void* X, int n_x, long ld_x, void* Y, long ld_y,
                       char* sub, size_t sub_bytes);
}  // namespace ace

ACE_EXPORT ace_status ace_apply(ace_ctx c, const ace_grid* grid, ace_prec prec, const void* xi,
                                int n_band, long ld_xi, const void* X, int n_x, long ld_x, void* Y,
                                long ld_y) {
  if (!c) return ACE_E_ARG;
  return apply_entry(c, grid, prec, xi, n_band, ld_xi, X, n_x, ld_x, Y, ld_y, nullptr, 0);
}

ace_status ace::apply_entry(ace_ctx c, const ace_grid* grid, ace_prec prec, const void* xi,
                            int n_band, long ld_xi, const void* X, int n_x, long ld_x, void* Y,
                            long ld_y, char* sub, size_t sub_bytes) {
  GridInfo g;
  ACE_TRY(check_grid(c, grid, prec, &g));
  ACE_TRY(check_block(c, xi, n_band, ld_xi, g, "xi"));
  ACE_TRY(check_block(c, X, n_x, ld_x, g, "X"));
  ACE_TRY(check_block(c, Y, n_x, ld_y, g, "Y"));
  const size_t eb = elem_bytes(prec);
  const Span sy = span_of(Y, n_x, ld_y, g.ng, eb);
  if (overlap(sy, span_of(xi, n_band, ld_xi, g.ng, eb)) ||
      overlap(sy, span_of(X, n_x, ld_x, g.ng, eb)))
    return fail(c, ACE_E_ARG, "Y overlaps an input");
  if (is_real(prec)) {
    ACE_TRY(check_real_view(c, xi, ld_xi, eb, "xi"));
    ACE_TRY(check_real_view(c, X, ld_x, eb, "X"));
    ACE_TRY(check_real_view(c, Y, ld_y, eb, "Y"));
  }
  const GridInfo gv = is_real(prec) ? half_view(g) : g;
  if (sub) {
    // workspace of apply_t: the n_band x n_x matrix and the split-K partials
    const size_t need = align_up((size_t)n_band * n_x * sizeof(cx<double>), 256) +
                        gemm_cn_partial_bytes(n_band, n_x, gv.ng, is_real(prec) ? 2 * eb : eb,
                                              kNative, false);
    if (need > sub_bytes) {
      char buf[160];
      snprintf(buf, sizeof buf,
               "n_band x n_x too large for the allocation-free apply: needs %zu bytes of "
               "scratch, the library holds %zu", need, sub_bytes);
      return fail(c, ACE_E_UNSUPPORTED, buf);
    }
    c->sub_base = sub;
    c->sub_bytes = sub_bytes;
  }
  ace_status st;
  if (prec == ACE_REAL64)
    st = apply_t<double>(c, gv, (const cx<double>*)xi, n_band, ld_xi / 2, (const cx<double>*)X,
                         n_x, ld_x / 2, (cx<double>*)Y, ld_y / 2, true);
  else if (prec == ACE_REAL32)
    st = apply_t<float>(c, gv, (const cx<float>*)xi, n_band, ld_xi / 2, (const cx<float>*)X, n_x,
                        ld_x / 2, (cx<float>*)Y, ld_y / 2, true);
  else if (prec == ACE_FP64)
    st = apply_t<double>(c, gv, (const cx<double>*)xi, n_band, ld_xi, (const cx<double>*)X, n_x,
                         ld_x, (cx<double>*)Y, ld_y);
  else
    st = apply_t<float>(c, gv, (const cx<float>*)xi, n_band, ld_xi, (const cx<float>*)X, n_x,
                        ld_x, (cx<float>*)Y, ld_y);
  if (sub) {
    c->sub_base = nullptr;
    c->sub_bytes = 0;
  }
  return st;
}

ACE_EXPORT ace_status ace_exchange_energy(ace_ctx c, const ace_grid* grid, ace_prec prec,
                                          const void* phi, int n_occ, long ld_phi, const void* xi,
                                          int n_band, long ld_xi, double* ex_dev) {
  if (!c) return ACE_E_ARG;
  GridInfo g;
  ACE_TRY(check_grid(c, grid, prec, &g));
  ACE_TRY(check_block(c, phi, n_occ, ld_phi, g, "phi"));
  if (!ex_dev) return fail(c, ACE_E_ARG, "ex_dev is NULL");
  if (xi && is_real(prec)) {
    ACE_TRY(check_block(c, xi, n_band, ld_xi, g, "xi"));
    const size_t eb = elem_bytes(prec);
    ACE_TRY(check_real_view(c, phi, ld_phi, eb, "phi"));
    ACE_TRY(check_real_view(c, xi, ld_xi, eb, "xi"));
    const GridInfo gh = half_view(g);
    if (prec == ACE_REAL64)
      return energy_ace_t<double>(c, gh, (const cx<double>*)phi, n_occ, ld_phi / 2,
                                  (const cx<double>*)xi, n_band, ld_xi / 2, ex_dev, true);
    return energy_ace_t<float>(c, gh, (const cx<float>*)phi, n_occ, ld_phi / 2,
                               (const cx<float>*)xi, n_band, ld_xi / 2, ex_dev, true);
  }
  if (is_real(prec))
    return fail(c, ACE_E_UNSUPPORTED, "direct energy form for real orbitals (pass xi)");
  if (xi) {
    ACE_TRY(check_block(c, xi, n_band, ld_xi, g, "xi"));
    if (prec == ACE_FP64)
      return energy_ace_t<double>(c, g, (const cx<double>*)phi, n_occ, ld_phi,
                                  (const cx<double>*)xi, n_band, ld_xi, ex_dev);
    return energy_ace_t<float>(c, g, (const cx<float>*)phi, n_occ, ld_phi, (const cx<float>*)xi,
                               n_band, ld_xi, ex_dev);
  }
  if (prec == ACE_FP64)
    return energy_direct_impl<double>(c, g, (const cx<double>*)phi, n_occ, ld_phi, ex_dev);
  return energy_direct_impl<float>(c, g, (const cx<float>*)phi, n_occ, ld_phi, ex_dev);
}

ACE_EXPORT ace_status ace_exchange_energy_grad(ace_ctx c, const ace_grid* grid, ace_prec prec,
                                               const void* phi, int n_occ, long ld_phi,
                                               const double* gbar_dev, void* G, long ld_G) {
  if (!c) return ACE_E_ARG;
  GridInfo g;
  ACE_TRY(check_grid(c, grid, prec, &g));
  ACE_TRY(check_block(c, phi, n_occ, ld_phi, g, "phi"));
  ACE_TRY(check_block(c, G, n_occ, ld_G, g, "G"));
  const size_t eb = elem_bytes(prec);
  if (overlap(span_of(G, n_occ, ld_G, g.ng, eb), span_of(phi, n_occ, ld_phi, g.ng, eb)))
    return fail(c, ACE_E_ARG, "G overlaps phi");
  // G = 2 gbar dV V_X[phi] phi: the pair FFTs are recomputed (pairs i <= j)
  const double scale = 2.0 * g.dV;
  if (prec == ACE_REAL64)
    return build_W_real_impl<double>(c, g, (const double*)phi, n_occ, ld_phi, (const double*)phi,
                                     n_occ, ld_phi, (double*)G, ld_G, scale, gbar_dev);
  if (prec == ACE_REAL32)
    return build_W_real_impl<float>(c, g, (const float*)phi, n_occ, ld_phi, (const float*)phi,
                                    n_occ, ld_phi, (float*)G, ld_G, scale, gbar_dev);
  if (prec == ACE_FP64)
    return build_W_impl<double>(c, g, (const cx<double>*)phi, n_occ, ld_phi,
                                (const cx<double>*)phi, n_occ, ld_phi, (cx<double>*)G, ld_G, scale,
                                gbar_dev);
  return build_W_impl<float>(c, g, (const cx<float>*)phi, n_occ, ld_phi, (const cx<float>*)phi,
                             n_occ, ld_phi, (cx<float>*)G, ld_G, scale, gbar_dev);
}

ACE_EXPORT ace_status ace_orthonormalize(ace_ctx c, const ace_grid* grid, ace_prec prec,
                                         const void* X, int n, long ld_x, void* Q, long ld_q,
                                         int* info_dev) {
  if (!c) return ACE_E_ARG;
  GridInfo g;
  ACE_TRY(check_grid(c, grid, prec, &g));
  ACE_TRY(check_block(c, X, n, ld_x, g, "X"));
  ACE_TRY(check_block(c, Q, n, ld_q, g, "Q"));
  if (n > 4096) return fail(c, ACE_E_UNSUPPORTED, "n above 4096");
  const size_t eb = elem_bytes(prec);
  if (overlap(span_of(Q, n, ld_q, g.ng, eb), span_of(X, n, ld_x, g.ng, eb)))
    return fail(c, ACE_E_ARG, "Q overlaps X");
  if (!info_dev && stream_capturing(c))
    return fail(c, ACE_E_CAPTURE, "info_dev == NULL synchronises, which a capture does not allow");
  const CnMode mode = gram_mode(prec);
  if (is_real(prec)) {
    ACE_TRY(check_real_view(c, X, ld_x, eb, "X"));
    ACE_TRY(check_real_view(c, Q, ld_q, eb, "Q"));
    const GridInfo gh = half_view(g);
    if (prec == ACE_REAL64)
      return orth_t<double>(c, gh, (const cx<double>*)X, n, ld_x / 2, (cx<double>*)Q, ld_q / 2,
                            info_dev, mode, true);
    return orth_t<float>(c, gh, (const cx<float>*)X, n, ld_x / 2, (cx<float>*)Q, ld_q / 2,
                         info_dev, mode, true);
  }
  if (prec == ACE_FP64)
    return orth_t<double>(c, g, (const cx<double>*)X, n, ld_x, (cx<double>*)Q, ld_q, info_dev,
                          mode);
  return orth_t<float>(c, g, (const cx<float>*)X, n, ld_x, (cx<float>*)Q, ld_q, info_dev, mode);
}

ACE_EXPORT ace_status ace_profile_enable(ace_ctx c, int on) {
  if (!c) return ACE_E_ARG;
  c->profiling = on != 0;
  return ACE_OK;
}

ACE_EXPORT ace_status ace_profile_reset(ace_ctx c) {
  if (!c) return ACE_E_ARG;
  prof_collect(c);
  c->prof.clear();
  return ACE_OK;
}

ACE_EXPORT int ace_profile_count(ace_ctx c) {
  if (!c) return 0;
  prof_collect(c);
  return (int)c->prof.size();
}

ACE_EXPORT ace_status ace_profile_get(ace_ctx c, int idx, const char** name, long* launches,
                                      double* total_ms) {
  if (!c) return ACE_E_ARG;
  prof_collect(c);
  if (idx < 0 || idx >= (int)c->prof.size()) return ACE_E_ARG;
  if (name) *name = c->prof[idx].name.c_str();
  if (launches) *launches = c->prof[idx].launches;
  if (total_ms) *total_ms = c->prof[idx].ms;
  return ACE_OK;
}
