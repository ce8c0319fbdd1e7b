// Autotuner of the build: for one grid size and precision it times the build
// on scratch orbitals over candidate pair budgets (how many pair spectra are in
// flight, i.e. the pair-batch width) and band blocks, then, at the fastest of
// those, over the line shapes of the slab and plane FFT passes (one thread,
// a quad or an octet of lanes per line; the tile of a line FFT); keeps the
// fastest in the context, and optionally appends it to a text cache file
// ("n elem_bytes budget jblock shape" per line) that ace_tune_load reads back.
#include <cerrno>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "ace_internal.h"

#define ACE_EXPORT extern "C" __attribute__((visibility("default")))

namespace ace {
namespace {

// Smooth, finite scratch orbitals: a few plane waves per orbital.
template <typename T>
__global__ __launch_bounds__(256) void k_fill_scratch(cx<T>* x, int n, int count) {
  const long ng = (long)n * n * n;
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= ng * count) return;
  const int b = (int)(idx / ng);
  const long r = idx - (long)b * ng;
  const int x2 = (int)(r % n), x1 = (int)((r / n) % n), x0 = (int)(r / ((long)n * n));
  const double ph = 6.283185307179586 * ((b % 5 + 1) * x0 + (b % 3) * x1 + (b % 7) * x2) / n;
  x[idx] = {T(cos(ph) * (1.0 + 0.1 * b)), T(sin(ph))};
}

void upsert(ace_ctx c, int n, int eb, long budget, long jblock, int shape, int accum) {
  ++c->tune_gen;
  for (auto& t : c->tuned)
    if (t.n == n && t.eb == eb) {
      t.budget = budget;
      t.jblock = jblock;
      t.shape = shape;
      t.accum = accum;
      return;
    }
  c->tuned.push_back({n, eb, budget, jblock, shape, accum});
}

}  // namespace
}  // namespace ace

using namespace ace;

ACE_EXPORT ace_status ace_autotune(ace_ctx c, const ace_grid* grid, ace_prec prec, int n_occ,
                                   int n_band, const char* cache_path, long* best_budget,
                                   long* best_jblock, int* best_shape, int* best_accum,
                                   double* best_ms) {
  if (!c) return ACE_E_ARG;
  GridInfo g;
  ACE_TRY(check_grid(c, grid, prec, &g));
  if (n_occ < 1 || n_band < n_occ) return fail(c, ACE_E_ARG, "need 1 <= n_occ <= n_band");
  if (prec == ACE_REAL32 || prec == ACE_REAL64)
    return fail(c, ACE_E_UNSUPPORTED, "the tuner times the complex build");
  if (stream_capturing(c))
    return fail(c, ACE_E_CAPTURE, "the tuner allocates and synchronises");
  if (!cache_path && !c->tune_cache.empty()) cache_path = c->tune_cache.c_str();
  const size_t eb = elem_bytes(prec);
  void* psi = nullptr;
  void* W = nullptr;
  hipError_t e = hipMalloc(&psi, (size_t)n_band * g.ng * eb);
  if (e == hipSuccess) e = hipMalloc(&W, (size_t)n_band * g.ng * eb);
  if (e != hipSuccess) {
    if (psi) hipFree(psi);
    (void)hipGetLastError();
    return fail(c, ACE_E_NOMEM, "autotune scratch allocation");
  }
  const long total = (long)n_band * g.ng;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  ace_status st = prec == ACE_FP64
                      ? launch(c, "fill_scratch", k_fill_scratch<double>, dim3(blocks), dim3(256), 0,
                               (cx<double>*)psi, g.n, n_band)
                      : launch(c, "fill_scratch", k_fill_scratch<float>, dim3(blocks), dim3(256), 0,
                               (cx<float>*)psi, g.n, n_band);
  const size_t save_budget = c->pair_budget;
  const long save_jblock = c->jblock;
  const int save_shape = c->fft_shape;
  const int save_accum = c->accum_shape;
  const bool save_prof = c->profiling;
  c->profiling = false;
  const long budgets[] = {256L << 20, 512L << 20, 1L << 30, 2L << 30, 4L << 30, 8L << 30};
  std::vector<long> jblocks = {0};
  if (n_band >= 32) jblocks.push_back((n_band + 1) / 2);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  double best = 1e300;
  long bb = 0, bj = 0;
  int bs = 0;
  const size_t pair_bytes = (size_t)g.ng * eb;
  auto run = [&]() {
    return prec == ACE_FP64
               ? build_W_impl<double>(c, g, (const cx<double>*)psi, n_occ, g.ng,
                                      (const cx<double>*)psi, n_band, g.ng, (cx<double>*)W, g.ng,
                                      1.0)
               : build_W_impl<float>(c, g, (const cx<float>*)psi, n_occ, g.ng,
                                     (const cx<float>*)psi, n_band, g.ng, (cx<float>*)W, g.ng,
                                     1.0);
  };
  // time of one build (mean of three after a warm-up that also grows the
  // workspace), or a negative value on failure
  auto time_build = [&]() -> double {
    if ((st = run()) != ACE_OK) return -1.0;
    float ms = 0.f;
    hipEventRecord(e0, c->stream);
    for (int r = 0; r < 3 && st == ACE_OK; ++r) st = run();
    hipEventRecord(e1, c->stream);
    hipEventSynchronize(e1);
    hipEventElapsedTime(&ms, e0, e1);
    return st == ACE_OK ? ms / 3.0 : -1.0;
  };
  c->fft_shape = 0;
  for (long bud : budgets) {
    if (st != ACE_OK) break;
    // skip budgets that change nothing: larger than every pair at once
    if ((size_t)bud / 2 >= pair_bytes * (size_t)n_occ * n_band && bud != budgets[0]) continue;
    for (long jb : jblocks) {
      c->pair_budget = (size_t)bud;
      c->jblock = jb;
      const double ms = time_build();
      if (ms < 0) break;
      if (ms < best) {
        best = ms;
        bb = bud;
        bj = jb;
      }
    }
  }
  // line shapes at the chosen blocking (0, the defaults, was timed above)
  const int shapes[] = {1, 4, 8, 16};
  c->pair_budget = (size_t)bb;
  c->jblock = bj;
  for (int sh : shapes) {
    if (st != ACE_OK) break;
    if (sh == 8 && (g.n % 8 != 0 || g.n < 16)) continue;
    c->fft_shape = sh;
    const double ms = time_build();
    if (ms < 0) break;
    if (ms < best) {
      best = ms;
      bs = sh;
    }
  }
  // accumulate-pass forms at the chosen blocking and line shape (0, the
  // default, was timed above)
  const int accums[] = {1, 16};
  int ba = 0;
  c->fft_shape = bs;
  for (int af : accums) {
    if (st != ACE_OK) break;
    c->accum_shape = af;
    const double ms = time_build();
    if (ms < 0) break;
    if (ms < best) {
      best = ms;
      ba = af;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  c->pair_budget = save_budget;
  c->jblock = save_jblock;
  c->fft_shape = save_shape;
  c->accum_shape = save_accum;
  c->profiling = save_prof;
  hipStreamSynchronize(c->stream);
  hipFree(psi);
  hipFree(W);
  if (st != ACE_OK) return st;
  upsert(c, g.n, (int)eb, bb, bj, bs, ba);
  if (cache_path) {
    FILE* f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "%d %d %ld %ld %d %d\n", g.n, (int)eb, bb, bj, bs, ba);
      fclose(f);
    }
  }
  if (best_budget) *best_budget = bb;
  if (best_jblock) *best_jblock = bj;
  if (best_shape) *best_shape = bs;
  if (best_accum) *best_accum = ba;
  if (best_ms) *best_ms = best;
  return ACE_OK;
}

namespace ace {
// One whole line of f into out (without the newline); false at end of file.
static bool read_line(FILE* f, std::string& out) {
  out.clear();
  int ch;
  while ((ch = std::fgetc(f)) != EOF && ch != '\n') out.push_back((char)ch);
  return ch != EOF || !out.empty();
}

// Parses up to 6 integers separated by blanks; returns how many, or -1 when the
// line holds anything else (a value out of range of long included).
static int parse_fields(const std::string& line, long* v) {
  const char* p = line.c_str();
  int got = 0;
  while (true) {
    while (*p == ' ' || *p == '\t' || *p == '\r') ++p;
    if (!*p) return got;
    if (got == 6) return -1;
    char* end = nullptr;
    errno = 0;
    const long x = std::strtol(p, &end, 10);
    if (end == p || errno == ERANGE) return -1;
    if (*end && *end != ' ' && *end != '\t' && *end != '\r') return -1;
    v[got++] = x;
    p = end;
  }
}

bool tune_cache_read(ace_ctx c, const char* cache_path) {
  FILE* f = std::fopen(cache_path, "r");
  if (!f) return false;
  // one setting per line: "n eb budget jblock [shape [accum]]" (0 when absent);
  // lines that do not parse or hold values out of range are skipped
  std::string line;
  while (read_line(f, line)) {
    long v[6] = {0, 0, 0, 0, 0, 0};
    const int got = parse_fields(line, v);
    if (got < 4) continue;
    const long n = v[0], eb = v[1], bud = v[2], jb = v[3], shape = v[4], accum = v[5];
    if (n > 0 && n <= 4096 && (eb == 8 || eb == 16) && bud >= 0 && jb >= 0 && jb <= INT32_MAX &&
        (shape == 0 || shape == 1 || shape == 4 || shape == 8 || shape == 16) &&
        (accum == 0 || accum == 1 || accum == 16))
      upsert(c, (int)n, (int)eb, bud, jb, (int)shape, (int)accum);
  }
  std::fclose(f);
  return true;
}
}  // namespace ace

ACE_EXPORT ace_status ace_tune_load(ace_ctx c, const char* cache_path) {
  if (!c || !cache_path) return ACE_E_ARG;
  if (!tune_cache_read(c, cache_path)) return fail(c, ACE_E_ARG, "cannot open tuning cache");
  return ACE_OK;
}
