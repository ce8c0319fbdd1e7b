// Batched ACE build: many independent instances (each with its own grid,
// orbitals and sizes) of the build and compression of Section 3, enqueued on
// several branch streams with a private workspace slice per branch, captured
// once into a HIP graph and replayed while the instance descriptors stay the
// same.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "ace_internal.h"

#define ACE_EXPORT extern "C" __attribute__((visibility("default")))

namespace ace {
namespace {

struct Planned {
  GridInfo g;
  size_t bytes;
  double cost;
  int branch;
};

ace_status ensure_branches(ace_ctx c, int nb) {
  if (!c->capture_stream) {
    hipError_t e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamCreateWithFlags");
  }
  while ((int)c->branch_streams.size() < nb) {
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamCreateWithFlags");
    c->branch_streams.push_back(s);
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventCreateWithFlags");
    c->branch_events.push_back(ev);
  }
  if (!c->fork_event) {
    hipError_t e = hipEventCreateWithFlags(&c->fork_event, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventCreateWithFlags");
  }
  return ACE_OK;
}

template <typename T>
ace_status enqueue_instance(ace_ctx c, const ace_instance& in, const GridInfo& g, CnMode mode) {
  ACE_TRY(build_W_impl<T>(c, g, (const cx<T>*)in.phi, in.n_occ, in.ld_phi, (const cx<T>*)in.psi,
                          in.n_band, in.ld_psi, (cx<T>*)in.W, in.ld_W, in.scale));
  if (in.xi)
    ACE_TRY(compress_impl<T>(c, g, (const cx<T>*)in.psi, in.ld_psi, (const cx<T>*)in.W, in.ld_W,
                             in.n_band, (cx<T>*)in.xi, in.ld_xi, nullptr, in.info_dev, mode));
  return ACE_OK;
}

std::vector<unsigned char> make_key(ace_ctx c, int n, const ace_instance* inst, int nbr) {
  std::vector<unsigned char> k(sizeof(ace_instance) * n + 72);
  std::memcpy(k.data(), inst, sizeof(ace_instance) * n);
  unsigned char* t = k.data() + sizeof(ace_instance) * n;
  const void* ws = c->ws;
  std::memcpy(t + 8, &nbr, sizeof nbr);
  std::memcpy(t + 16, &ws, sizeof ws);
  std::memcpy(t + 24, &c->ws_bytes, sizeof c->ws_bytes);
  std::memcpy(t + 32, &c->pair_budget, sizeof c->pair_budget);
  std::memcpy(t + 40, &c->jblock, sizeof c->jblock);
  const int symm = c->use_symmetry ? 1 : 0;
  std::memcpy(t + 48, &symm, sizeof symm);
  std::memcpy(t + 52, &c->fft_shape, sizeof c->fft_shape);
  std::memcpy(t + 56, &c->tune_gen, sizeof c->tune_gen);
  std::memcpy(t + 64, &c->accum_shape, sizeof c->accum_shape);
  return k;
}

}  // namespace
}  // namespace ace

using namespace ace;

ACE_EXPORT ace_status ace_build_W_batched(ace_ctx c, int n_inst, const ace_instance* inst) {
  if (!c) return ACE_E_ARG;
  if (n_inst < 1 || !inst) return fail(c, ACE_E_ARG, "no instances");
  const int n_branches = c->branches;
  std::vector<Planned> plan(n_inst);
  for (int k = 0; k < n_inst; ++k) {
    const ace_instance& in = inst[k];
    const ace_prec prec = (ace_prec)in.prec;
    if (prec != ACE_FP64 && prec != ACE_FP32 && prec != ACE_MIXED)
      return fail(c, prec == ACE_REAL32 || prec == ACE_REAL64 ? ACE_E_UNSUPPORTED : ACE_E_ARG,
                  "batched builds take complex precisions (ACE_FP64, ACE_FP32, ACE_MIXED)");
    const size_t eb = elem_bytes(prec);
    ACE_TRY(check_grid(c, &in.grid, prec, &plan[k].g));
    const GridInfo& g = plan[k].g;
    ACE_TRY(check_block(c, in.phi, in.n_occ, in.ld_phi, g, "instance phi"));
    ACE_TRY(check_block(c, in.psi, in.n_band, in.ld_psi, g, "instance psi"));
    ACE_TRY(check_block(c, in.W, in.n_band, in.ld_W, g, "instance W"));
    if (!std::isfinite(in.scale)) return fail(c, ACE_E_ARG, "instance scale");
    const Span sw = span_of(in.W, in.n_band, in.ld_W, g.ng, eb);
    if (overlap(sw, span_of(in.phi, in.n_occ, in.ld_phi, g.ng, eb)) ||
        overlap(sw, span_of(in.psi, in.n_band, in.ld_psi, g.ng, eb)))
      return fail(c, ACE_E_ARG, "instance W overlaps an input");
    if (in.xi) {
      ACE_TRY(check_block(c, in.xi, in.n_band, in.ld_xi, g, "instance xi"));
      if (!in.info_dev) return fail(c, ACE_E_ARG, "instance with xi needs info_dev");
      if (in.n_band > 4096) return fail(c, ACE_E_UNSUPPORTED, "n_band above 4096");
      const Span sx = span_of(in.xi, in.n_band, in.ld_xi, g.ng, eb);
      if (overlap(sx, sw) || overlap(sx, span_of(in.psi, in.n_band, in.ld_psi, g.ng, eb)))
        return fail(c, ACE_E_ARG, "instance xi overlaps an input");
    }
    const BuildPlan bp = plan_build(c, g, eb, in.n_occ, in.n_band,
                                    in.psi == in.phi && in.ld_psi == in.ld_phi);
    plan[k].bytes = std::max(bp.bytes, in.xi ? compress_ws_bytes(in.n_band, g.ng) : (size_t)0);
    plan[k].cost = (double)in.n_occ * in.n_band * (double)g.ng;
  }
  // longest-processing-time assignment of instances to branches
  const int nbr = std::min(n_branches, n_inst);
  std::vector<int> order(n_inst);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return plan[a].cost > plan[b].cost; });
  std::vector<double> load(nbr, 0.0);
  std::vector<size_t> bbytes(nbr, 0);
  for (int k : order) {
    const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    plan[k].branch = b;
    load[b] += plan[k].cost;
    bbytes[b] = std::max(bbytes[b], align_up(plan[k].bytes, 256));
  }
  std::vector<size_t> boff(nbr, 0);
  size_t total = 0;
  for (int b = 0; b < nbr; ++b) {
    boff[b] = total;
    total += bbytes[b];
  }
  ACE_TRY(ws_begin(c, total));  // grows the workspace before any capture
  ACE_TRY(ensure_branches(c, nbr));

  std::vector<unsigned char> key = make_key(c, n_inst, inst, nbr);
  if (c->graph_exec && key == c->graph_key) {
    hipError_t e = hipGraphLaunch(c->graph_exec, c->stream);  // replay
    return e == hipSuccess ? ACE_OK : hip_fail(c, e, "hipGraphLaunch");
  }
  if (c->graph_exec) {
    hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
    c->graph_key.clear();
  }

  // Capture on a stream of the context (the caller's stream may be the legacy
  // default stream, which cannot be captured); the graph is then launched on
  // the caller's stream, which orders it after the caller's earlier work.
  hipStream_t caller = c->stream;
  hipStream_t main = c->capture_stream;
  const bool prof = c->profiling;
  c->profiling = false;  // no timing events inside a capture
  hipError_t e = hipStreamBeginCapture(main, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    c->profiling = prof;
    return hip_fail(c, e, "hipStreamBeginCapture");
  }
  ace_status st = ACE_OK;
  e = hipEventRecord(c->fork_event, main);
  for (int b = 0; b < nbr && e == hipSuccess; ++b)
    e = hipStreamWaitEvent(c->branch_streams[b], c->fork_event, 0);
  if (e != hipSuccess) st = hip_fail(c, e, "fork");
  for (int b = 0; b < nbr && st == ACE_OK; ++b) {
    c->stream = c->branch_streams[b];
    c->sub_base = (char*)c->ws + boff[b];
    c->sub_bytes = bbytes[b];
    for (int k = 0; k < n_inst && st == ACE_OK; ++k) {
      if (plan[k].branch != b) continue;
      const ace_prec prec = (ace_prec)inst[k].prec;
      st = prec == ACE_FP64 ? enqueue_instance<double>(c, inst[k], plan[k].g, kNative)
                            : enqueue_instance<float>(c, inst[k], plan[k].g, compress_mode(prec));
    }
    if (st == ACE_OK) {
      e = hipEventRecord(c->branch_events[b], c->stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(main, c->branch_events[b], 0);
      if (e != hipSuccess) st = hip_fail(c, e, "join");
    }
  }
  c->stream = caller;
  c->sub_base = nullptr;
  c->sub_bytes = 0;
  c->profiling = prof;
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(main, &graph);
  if (st != ACE_OK) {
    if (graph) hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
  c->graph_exec = exec;
  c->graph_key = std::move(key);
  e = hipGraphLaunch(exec, caller);
  return e == hipSuccess ? ACE_OK : hip_fail(c, e, "hipGraphLaunch");
}
