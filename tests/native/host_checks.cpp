// Host-side checks of libace through its C ABI, built together with the
// library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
// (the device code is built as usual).  They run every entry point on small
// inputs and through its argument errors, workspace growth, stream changes,
// the tuning cache reader (including malformed files), the environment read
// at context creation, profiling and graph-capture refusals, so that a
// host-side out-of-bounds access, use after free, leak or undefined operation
// in the argument and workspace logic stops the program.
//
// Without a HIP device, or with the argument --no-device, only the checks that
// need no context run.
// Exit status: 0 when every check held, 1 otherwise; a sanitizer report
// aborts with its own status.
#include <hip/hip_runtime_api.h>
#include <sanitizer/lsan_interface.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <unistd.h>
#include <vector>

#include "../../include/ace.h"

namespace {

int g_checks = 0, g_failures = 0;

void expect(bool ok, const char* what, int line) {
  ++g_checks;
  if (!ok) {
    ++g_failures;
    std::printf("FAIL line %d: %s\n", line, what);
  }
}
#define EXPECT(cond) expect((cond), #cond, __LINE__)
#define EXPECT_ST(call, st) expect((call) == (st), #call " == " #st, __LINE__)

struct c128 {
  double re, im;
};
struct c64 {
  float re, im;
};

// Smooth orbitals: a few plane waves each, distinct per band, not normalised.
std::vector<c128> orbitals(int n, int count) {
  const long ng = (long)n * n * n;
  std::vector<c128> x(ng * count);
  for (int b = 0; b < count; ++b)
    for (long r = 0; r < ng; ++r) {
      const int x2 = (int)(r % n), x1 = (int)((r / n) % n), x0 = (int)(r / ((long)n * n));
      const double ph = 6.283185307179586 * ((b % 5 + 1) * x0 + (b % 3) * x1 + (b % 7) * x2) / n;
      x[b * ng + r] = {std::cos(ph) * (1.0 + 0.1 * b), std::sin(ph) + 0.05 * std::cos(2 * ph)};
    }
  return x;
}

template <typename T>
T* dev_alloc(size_t count) {
  void* p = nullptr;
  if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
    std::printf("hipMalloc of %zu bytes failed\n", count * sizeof(T));
    std::exit(1);
  }
  hipMemset(p, 0, count * sizeof(T));
  return (T*)p;
}

template <typename T>
void upload(T* d, const std::vector<T>& h) {
  hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
}

template <typename T>
std::vector<T> download(const T* d, size_t count) {
  std::vector<T> h(count);
  hipMemcpy(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost);
  return h;
}

double rel_diff(const std::vector<c128>& a, const std::vector<c128>& b) {
  double num = 0, den = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    num += (a[i].re - b[i].re) * (a[i].re - b[i].re) + (a[i].im - b[i].im) * (a[i].im - b[i].im);
    den += b[i].re * b[i].re + b[i].im * b[i].im;
  }
  return std::sqrt(num / den);
}

ace_grid cubic(int n, double L, int kind = ACE_COULOMB, double mu = 0.0) {
  ace_grid g;
  g.n[0] = g.n[1] = g.n[2] = n;
  g.L[0] = g.L[1] = g.L[2] = L;
  g.kind = kind;
  g.mu = mu;
  g.g0 = 0.0;
  return g;
}

std::string temp_path(const char* stem) {
  const char* dir = std::getenv("TMPDIR");
  std::string p = std::string(dir && *dir ? dir : "/tmp") + "/" + stem + "_" +
                  std::to_string((long)getpid());
  return p;
}

void checks_without_context() {
  ace_grid g = cubic(16, 7.0);
  EXPECT_ST(ace_create(nullptr, nullptr, nullptr), ACE_E_ARG);
  EXPECT_ST(ace_destroy(nullptr), ACE_E_ARG);
  EXPECT_ST(ace_set_stream(nullptr, nullptr), ACE_E_ARG);
  EXPECT_ST(ace_reserve(nullptr, &g, ACE_FP64, 1, 1, 1), ACE_E_ARG);
  EXPECT_ST(ace_build_W(nullptr, &g, ACE_FP64, nullptr, 1, 1, nullptr, 1, 1, nullptr, 1, 1.0),
            ACE_E_ARG);
  EXPECT_ST(ace_compress(nullptr, &g, ACE_FP64, nullptr, 1, nullptr, 1, 1, nullptr, 1, nullptr,
                         nullptr),
            ACE_E_ARG);
  EXPECT_ST(ace_apply(nullptr, &g, ACE_FP64, nullptr, 1, 1, nullptr, 1, 1, nullptr, 1),
            ACE_E_ARG);
  EXPECT_ST(ace_apply_noalloc(nullptr, &g, ACE_FP64, nullptr, 1, 1, nullptr, 1, 1, nullptr, 1),
            ACE_E_ARG);
  EXPECT_ST(ace_exchange_energy(nullptr, &g, ACE_FP64, nullptr, 1, 1, nullptr, 1, 1, nullptr),
            ACE_E_ARG);
  EXPECT_ST(ace_exchange_energy_grad(nullptr, &g, ACE_FP64, nullptr, 1, 1, nullptr, nullptr, 1),
            ACE_E_ARG);
  EXPECT_ST(ace_orthonormalize(nullptr, &g, ACE_FP64, nullptr, 1, 1, nullptr, 1, nullptr),
            ACE_E_ARG);
  EXPECT_ST(ace_build_W_batched(nullptr, 0, nullptr), ACE_E_ARG);
  EXPECT_ST(ace_tune_load(nullptr, "x"), ACE_E_ARG);
  EXPECT_ST(ace_profile_enable(nullptr, 1), ACE_E_ARG);
  EXPECT(ace_profile_count(nullptr) <= 0);
  EXPECT_ST(ace_set_tuning(nullptr, ACE_TUNE_JBLOCK, 0), ACE_E_ARG);
  EXPECT(std::strlen(ace_last_error(nullptr)) == 0);
  for (int s = 0; s <= 7; ++s) EXPECT(ace_status_string((ace_status)s) != nullptr);
  int sizes[64];
  const int k = ace_supported_n(sizes, 64);
  EXPECT(k >= 6 && k <= 64);
  EXPECT(ace_supported_n(sizes, 0) == k || ace_supported_n(sizes, 0) == 0);
  EXPECT(ace_supported_n(sizes, 2) >= 0);
}

void checks_with_context() {
  const int n = 16, nocc = 3, nb = 5;
  const long ng = (long)n * n * n;
  const ace_grid g = cubic(n, 7.0);
  const ace_grid gs = cubic(n, 7.0, ACE_ERFC, 0.4);
  const std::vector<c128> h_psi = orbitals(n, nb);

  ace_ctx c = nullptr;
  EXPECT_ST(ace_create(&c, nullptr, nullptr), ACE_OK);
  if (!c) return;

  c128* psi = dev_alloc<c128>(ng * nb);
  c128* W = dev_alloc<c128>(ng * nb);
  c128* xi = dev_alloc<c128>(ng * nb);
  c128* Y = dev_alloc<c128>(ng * nb);
  c128* Q = dev_alloc<c128>(ng * nb);
  c128* L = dev_alloc<c128>((size_t)nb * nb);
  int* info = dev_alloc<int>(4);
  double* dd = dev_alloc<double>(64);
  upload(psi, h_psi);

  // argument errors with a live context
  ace_grid bad = g;
  bad.n[1] = 20;
  EXPECT_ST(ace_build_W(c, &bad, ACE_FP64, psi, nocc, ng, psi, nb, ng, W, ng, 1.0),
            ACE_E_UNSUPPORTED);
  bad = g;
  bad.L[2] = -1.0;
  EXPECT(ace_build_W(c, &bad, ACE_FP64, psi, nocc, ng, psi, nb, ng, W, ng, 1.0) != ACE_OK);
  EXPECT(std::strlen(ace_last_error(c)) > 0);
  EXPECT(ace_build_W(c, &g, (ace_prec)7, psi, nocc, ng, psi, nb, ng, W, ng, 1.0) != ACE_OK);
  EXPECT_ST(ace_build_W(c, &g, ACE_FP64, psi, nocc, ng - 1, psi, nb, ng, W, ng, 1.0), ACE_E_ARG);
  EXPECT_ST(ace_build_W(c, &g, ACE_FP64, psi, nocc, ng, psi, nb, ng, psi, ng, 1.0), ACE_E_ARG);
  EXPECT_ST(ace_build_W(c, &g, ACE_FP64, psi, nocc, ng, psi, nb, ng, W, ng, NAN), ACE_E_ARG);
  EXPECT_ST(ace_build_W(c, &g, ACE_FP64, psi, 0, ng, psi, nb, ng, W, ng, 1.0), ACE_E_ARG);
  EXPECT_ST(ace_build_W(c, &g, ACE_FP64, nullptr, nocc, ng, psi, nb, ng, W, ng, 1.0), ACE_E_ARG);
  EXPECT_ST(ace_compress(c, &g, ACE_FP64, psi, ng, W, ng, 5000, xi, ng, nullptr, nullptr),
            ACE_E_UNSUPPORTED);
  EXPECT_ST(ace_set_tuning(c, 99, 1), ACE_E_ARG);
  EXPECT_ST(ace_get_tuning(c, ACE_TUNE_JBLOCK, nullptr), ACE_E_ARG);

  // the path: W, xi, V_ACE psi = W, energy, gradient
  EXPECT_ST(ace_build_W(c, &g, ACE_FP64, psi, nocc, ng, psi, nb, ng, W, ng, 1.0), ACE_OK);
  EXPECT_ST(ace_compress(c, &g, ACE_FP64, psi, ng, W, ng, nb, xi, ng, L, info), ACE_OK);
  EXPECT_ST(ace_apply(c, &g, ACE_FP64, xi, nb, ng, psi, nb, ng, Y, ng), ACE_OK);
  hipDeviceSynchronize();
  const std::vector<c128> hW = download(W, ng * nb), hY = download(Y, ng * nb);
  EXPECT(rel_diff(hY, hW) < 1e-9);
  EXPECT(download(info, 1)[0] == 0);
  EXPECT_ST(ace_apply_noalloc(c, &g, ACE_FP64, xi, nb, ng, psi, 2, ng, Y, ng), ACE_OK);
  EXPECT(ace_apply_noalloc(c, &g, ACE_FP64, xi, 300, ng, psi, 300, ng, Y, ng) != ACE_OK);
  EXPECT_ST(ace_exchange_energy(c, &g, ACE_FP64, psi, nocc, ng, xi, nb, ng, dd), ACE_OK);
  EXPECT_ST(ace_exchange_energy(c, &g, ACE_FP64, psi, nocc, ng, nullptr, 0, 0, dd + 1), ACE_OK);
  EXPECT_ST(ace_exchange_energy_grad(c, &g, ACE_FP64, psi, nocc, ng, nullptr, Y, ng), ACE_OK);
  hipDeviceSynchronize();
  const std::vector<double> e = download(dd, 2);
  EXPECT(std::isfinite(e[0]) && std::fabs(e[0] - e[1]) <= 1e-9 * std::fabs(e[1]));

  // orthonormalisation and the eigensolver pieces
  EXPECT_ST(ace_orthonormalize(c, &g, ACE_FP64, psi, nb, ng, Q, ng, info), ACE_OK);
  double* vloc = dev_alloc<double>(ng);
  EXPECT_ST(ace_apply_h(c, &g, ACE_FP64, vloc, xi, nb, ng, nullptr, 0, 0, 1.0, Q, nb, ng, Y, ng),
            ACE_OK);
  EXPECT_ST(ace_apply_h(c, &g, ACE_FP64, nullptr, nullptr, 0, 0, psi, nocc, ng, 1.0, Q, nb, ng,
                        W, ng),
            ACE_OK);
  EXPECT(ace_apply_h(c, &g, ACE_FP64, nullptr, xi, nb, ng, psi, nocc, ng, 1.0, Q, nb, ng, W,
                     ng) != ACE_OK);
  c128* Xo = dev_alloc<c128>(ng * nb);
  c128* HXo = dev_alloc<c128>(ng * nb);
  EXPECT_ST(ace_rayleigh_ritz(c, &g, ACE_FP64, Q, ng, Y, ng, nb, Xo, HXo, ng, dd + 8), ACE_OK);
  EXPECT_ST(ace_combine(c, &g, ACE_FP64, nb, 0.5, Xo, ng, -1.0, HXo, ng, 0.0, nullptr, 0, Xo, ng),
            ACE_OK);

  // single precision and the real forms, with a screened kernel
  c64* s_psi = dev_alloc<c64>(ng * nb);
  c64* s_W = dev_alloc<c64>(ng * nb);
  c64* s_xi = dev_alloc<c64>(ng * nb);
  {
    std::vector<c64> h(ng * nb);
    for (size_t i = 0; i < h.size(); ++i) h[i] = {(float)h_psi[i].re, (float)h_psi[i].im};
    upload(s_psi, h);
  }
  for (ace_prec p : {ACE_FP32, ACE_MIXED}) {
    EXPECT_ST(ace_build_W(c, &gs, p, s_psi, nocc, ng, s_psi, nb, ng, s_W, ng, 1.0), ACE_OK);
    EXPECT_ST(ace_compress(c, &gs, p, s_psi, ng, s_W, ng, nb, s_xi, ng, nullptr, info), ACE_OK);
  }
  double* r_psi = (double*)psi;  // the complex buffer read as 2 nb real orbitals
  double* r_W = (double*)W;
  EXPECT_ST(ace_build_W(c, &gs, ACE_REAL64, r_psi, nocc, ng, r_psi, nb, ng, r_W, ng, 1.0),
            ACE_OK);
  float* f_psi = (float*)s_psi;
  float* f_W = (float*)s_W;
  EXPECT_ST(ace_build_W(c, &gs, ACE_REAL32, f_psi, nocc, ng, f_psi, nb, ng, f_W, ng, 1.0), ACE_OK);

  // workspace growth after a reservation, a larger build, a smaller one
  EXPECT_ST(ace_reserve(c, &g, ACE_FP64, 1, 2, 2), ACE_OK);
  c128* big = dev_alloc<c128>(ng * 24);
  c128* bigW = dev_alloc<c128>(ng * 24);
  {
    std::vector<c128> h = orbitals(n, 24);
    upload(big, h);
  }
  EXPECT_ST(ace_build_W(c, &g, ACE_FP64, big, 20, ng, big, 24, ng, bigW, ng, 1.0), ACE_OK);
  EXPECT_ST(ace_build_W(c, &g, ACE_FP64, big, 2, ng, big, 3, ng, bigW, ng, 1.0), ACE_OK);

  // tuning knobs, profiling
  long v = -1;
  EXPECT_ST(ace_set_tuning(c, ACE_TUNE_FFT_SHAPE, 4), ACE_OK);
  EXPECT_ST(ace_get_tuning(c, ACE_TUNE_FFT_SHAPE, &v), ACE_OK);
  EXPECT(v == 4);
  EXPECT_ST(ace_profile_enable(c, 1), ACE_OK);
  EXPECT_ST(ace_build_W(c, &g, ACE_FP64, psi, nocc, ng, psi, nb, ng, W, ng, 1.0), ACE_OK);
  const int np = ace_profile_count(c);
  EXPECT(np > 0);
  for (int i = 0; i < np; ++i) {
    const char* name = nullptr;
    long launches = 0;
    double ms = 0;
    EXPECT_ST(ace_profile_get(c, i, &name, &launches, &ms), ACE_OK);
    EXPECT(name && std::strlen(name) > 0 && launches > 0);
  }
  EXPECT(ace_profile_get(c, np, nullptr, nullptr, nullptr) != ACE_OK);
  EXPECT_ST(ace_profile_reset(c), ACE_OK);
  EXPECT_ST(ace_profile_enable(c, 0), ACE_OK);
  EXPECT_ST(ace_set_tuning(c, ACE_TUNE_FFT_SHAPE, 0), ACE_OK);

  // batched build, both forms, mixed sizes and precisions
  ace_instance inst[3];
  std::memset(inst, 0, sizeof inst);
  for (int i = 0; i < 3; ++i) {
    inst[i].grid = i == 1 ? gs : g;
    inst[i].prec = ACE_FP64;
    inst[i].phi = i == 2 ? big : psi;
    inst[i].n_occ = i == 2 ? 6 : nocc;
    inst[i].ld_phi = ng;
    inst[i].psi = i == 2 ? big : psi;
    inst[i].n_band = i == 2 ? 8 : nb;
    inst[i].ld_psi = ng;
    inst[i].scale = 1.0;
  }
  inst[0].W = W;
  inst[1].W = Y;
  inst[2].W = bigW;
  inst[2].ld_W = inst[1].ld_W = inst[0].ld_W = ng;
  inst[0].xi = xi;
  inst[0].ld_xi = ng;
  inst[0].info_dev = info;
  for (long form : {1L, 2L}) {
    EXPECT_ST(ace_set_tuning(c, ACE_TUNE_BATCH_FORM, form), ACE_OK);
    EXPECT_ST(ace_build_W_batched(c, 3, inst), ACE_OK);
    EXPECT_ST(ace_build_W_batched(c, 2, inst), ACE_OK);
  }
  inst[1].W = W;  // two instances writing one W
  EXPECT(ace_build_W_batched(c, 2, inst) != ACE_OK);
  EXPECT_ST(ace_build_W_batched(c, -1, inst), ACE_E_ARG);

  // a stream of its own, then back
  hipStream_t s = nullptr;
  hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  EXPECT_ST(ace_set_stream(c, s), ACE_OK);
  EXPECT_ST(ace_build_W(c, &g, ACE_FP64, psi, nocc, ng, psi, nb, ng, W, ng, 1.0), ACE_OK);
  EXPECT_ST(ace_set_stream(c, nullptr), ACE_OK);
  hipStreamSynchronize(s);

  // capture: a fresh context must refuse to grow its workspace
  ace_ctx c2 = nullptr;
  EXPECT_ST(ace_create(&c2, s, nullptr), ACE_OK);
  if (c2) {
    hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    EXPECT_ST(ace_build_W(c2, &g, ACE_FP64, psi, nocc, ng, psi, nb, ng, W, ng, 1.0),
              ACE_E_CAPTURE);
    EXPECT_ST(ace_autotune(c2, &g, ACE_FP64, nocc, nb, nullptr, nullptr, nullptr, nullptr,
                           nullptr, nullptr),
              ACE_E_CAPTURE);
    hipGraph_t graph = nullptr;
    hipStreamEndCapture(s, &graph);
    if (graph) hipGraphDestroy(graph);
    EXPECT_ST(ace_destroy(c2), ACE_OK);
  }

  // tuning cache: the tuner's output, then malformed files
  const std::string cache = temp_path("ace_tune_cache");
  std::remove(cache.c_str());
  long bb = 0, bj = 0;
  int bs = 0, ba = 0;
  double ms = 0;
  EXPECT_ST(ace_autotune(c, &g, ACE_FP32, nocc, nb, cache.c_str(), &bb, &bj, &bs, &ba, &ms),
            ACE_OK);
  EXPECT(bb > 0 && ms > 0);
  EXPECT_ST(ace_tune_load(c, cache.c_str()), ACE_OK);
  {
    FILE* f = std::fopen(cache.c_str(), "w");
    std::string longline(1000, '7');
    std::fprintf(f, "%s\n16 8\n-5 8 1 1 1 1\n16 8 1 2 3 4\n\n16 16 99999999999999999999 0\n",
                 longline.c_str());
    const unsigned char junk[] = {0xff, 0x00, 0x31, 0x36, 0x20, 0x0a, 0x80, 0x7f};
    std::fwrite(junk, 1, sizeof junk, f);
    std::fclose(f);
  }
  EXPECT_ST(ace_tune_load(c, cache.c_str()), ACE_OK);
  EXPECT_ST(ace_build_W(c, &g, ACE_FP32, s_psi, nocc, ng, s_psi, nb, ng, s_W, ng, 1.0), ACE_OK);
  EXPECT(ace_tune_load(c, (cache + ".absent").c_str()) != ACE_OK);

  // the environment read at creation: log file, tuning cache, tune on first build
  const std::string log = temp_path("ace_log");
  std::remove(log.c_str());
  std::remove(cache.c_str());
  setenv("ACE_LOG", log.c_str(), 1);
  setenv("ACE_TUNE_CACHE", cache.c_str(), 1);
  setenv("ACE_TUNE", "1", 1);
  ace_ctx c3 = nullptr;
  EXPECT_ST(ace_create(&c3, nullptr, nullptr), ACE_OK);
  if (c3) {
    EXPECT_ST(ace_build_W(c3, &g, ACE_FP32, s_psi, nocc, ng, s_psi, nb, ng, s_W, ng, 1.0),
              ACE_OK);
    EXPECT_ST(ace_build_W(c3, &g, ACE_FP32, s_psi, nocc, ng, s_psi, nb, ng, s_W, ng, NAN),
              ACE_E_ARG);
    EXPECT_ST(ace_destroy(c3), ACE_OK);
  }
  unsetenv("ACE_LOG");
  unsetenv("ACE_TUNE_CACHE");
  unsetenv("ACE_TUNE");
  {
    FILE* f = std::fopen(log.c_str(), "r");
    EXPECT(f != nullptr);
    std::string text;
    char buf[512];
    while (f && std::fgets(buf, sizeof buf, f)) text += buf;
    if (f) std::fclose(f);
    EXPECT(text.find("tuned n=16") != std::string::npos);
    EXPECT(text.find("scale must be finite") != std::string::npos);
  }
  std::remove(log.c_str());
  std::remove(cache.c_str());

  hipDeviceSynchronize();
  EXPECT_ST(ace_destroy(c), ACE_OK);
  hipStreamDestroy(s);
  for (void* p : {(void*)psi, (void*)W, (void*)xi, (void*)Y, (void*)Q, (void*)L, (void*)info,
                  (void*)dd, (void*)vloc, (void*)Xo, (void*)HXo, (void*)s_psi, (void*)s_W,
                  (void*)s_xi, (void*)big, (void*)bigW})
    hipFree(p);
}

}  // namespace

// Ends the program after the leak check, without the static destructors of the
// ROCm runtime libraries: under AddressSanitizer those free memory after the
// sanitizer's hook of the HIP device allocator is gone, which its allocator
// treats as a fatal internal error unrelated to the code checked here.
[[noreturn]] void finish(int code) {
  std::fflush(stdout);
  __lsan_do_leak_check();
  _exit(code);
}

int main(int argc, char** argv) {
  setvbuf(stdout, nullptr, _IOLBF, 0);
  checks_without_context();
  const bool no_device = argc > 1 && !std::strcmp(argv[1], "--no-device");
  int dev = 0;
  if (no_device || hipGetDeviceCount(&dev) != hipSuccess || dev < 1) {
    std::printf("host checks: %d checks, %d failures (no HIP device: context checks skipped)\n",
                g_checks, g_failures);
    finish(g_failures ? 1 : 0);
  }
  checks_with_context();
  std::printf("host checks: %d checks, %d failures\n", g_checks, g_failures);
  finish(g_failures ? 1 : 0);
}
