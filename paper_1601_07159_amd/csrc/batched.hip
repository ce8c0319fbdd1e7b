// Batched ACE build: many independent instances (each with its own grid,
// orbitals and sizes) of the build and compression of Section 3, captured once
// into a HIP graph and replayed while the instance descriptors stay the same.
// Two forms of the W stage:
//  - launches: every instance's pass kernels on one of several branch
//    streams, with a private workspace slice per branch;
//  - persistent: one persistent kernel per grid size runs the pass launches of
//    all instances of that size from a task queue with dependency counters
//    (persist.hip); the compressions follow on the branch streams.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "ace_internal.h"

#define ACE_EXPORT extern "C" __attribute__((visibility("default")))

namespace ace {
namespace {

// Form of the W stage when ACE_TUNE_BATCH_FORM is 0.
constexpr int kDefaultBatchForm = 1;

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


std::vector<unsigned char> make_key(ace_ctx c, int n, const ace_instance* inst, int nbr,
                                    int form) {
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
  std::memcpy(t + 68, &form, sizeof form);
  return k;
}

// Drops the cached graph and the device buffers it reads (after the work
// already queued on the context stream, which may still replay it).
void drop_graph(ace_ctx c) {
  if (c->graph_exec) {
    hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
    c->graph_key.clear();
  }
  if (!c->graph_bufs.empty()) {
    (void)hipStreamSynchronize(c->stream);
    for (void* p : c->graph_bufs) (void)hipFree(p);
    c->graph_bufs.clear();
  }
}

// Longest-processing-time assignment of the instances flagged in `use` to nbr
// branches; returns each branch's largest slice (`bytes` per instance).
std::vector<size_t> assign_branches(std::vector<Planned>& plan, const std::vector<char>& use,
                                    const std::vector<size_t>& bytes, int nbr) {
  const int n = (int)plan.size();
  std::vector<int> order;
  for (int k = 0; k < n; ++k)
    if (use[k]) order.push_back(k);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return plan[a].cost > plan[b].cost; });
  std::vector<double> load(nbr, 0.0);
  std::vector<size_t> bbytes(nbr, 0);
  for (int k : order) {
    const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    plan[k].branch = b;
    load[b] += plan[k].cost;
    bbytes[b] = std::max(bbytes[b], align_up(bytes[k], 256));
  }
  return bbytes;
}

// Captures `body` (which enqueues on c->stream = the capture stream and may
// fork to branch streams) into a graph, caches it under `key` and launches it
// on the caller's stream.
template <typename F>
ace_status capture_and_launch(ace_ctx c, std::vector<unsigned char>&& key, F&& body) {
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
  c->stream = main;
  ace_status st = body(main);
  c->stream = caller;
  c->sub_base = nullptr;
  c->sub_bytes = 0;
  c->record = nullptr;
  c->budget_cap = 0;
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

template <typename T>
ace_status compress_instance(ace_ctx c, const ace_instance& in, const GridInfo& g) {
  if (!in.xi) return ACE_OK;
  const CnMode mode = sizeof(T) == 8 ? kNative : compress_mode((ace_prec)in.prec);
  return compress_impl<T>(c, g, (const cx<T>*)in.psi, in.ld_psi, (const cx<T>*)in.W, in.ld_W,
                          in.n_band, (cx<T>*)in.xi, in.ld_xi, nullptr, in.info_dev, mode);
}

template <typename T>
ace_status record_instance(ace_ctx c, const ace_instance& in, const GridInfo& g) {
  return build_W_impl<T>(c, g, (const cx<T>*)in.phi, in.n_occ, in.ld_phi, (const cx<T>*)in.psi,
                         in.n_band, in.ld_psi, (cx<T>*)in.W, in.ld_W, in.scale);
}

// ---------------------------------------------------------------------------
// Launches form.
ace_status batched_launches(ace_ctx c, int n_inst, const ace_instance* inst,
                            std::vector<Planned>& plan) {
  const int nbr = std::min(c->branches, n_inst);
  std::vector<char> all(n_inst, 1);
  std::vector<size_t> bytes(n_inst);
  for (int k = 0; k < n_inst; ++k) bytes[k] = plan[k].bytes;
  const std::vector<size_t> bbytes = assign_branches(plan, all, bytes, nbr);
  std::vector<size_t> boff(nbr, 0);
  size_t total = 0;
  for (int b = 0; b < nbr; ++b) {
    boff[b] = total;
    total += bbytes[b];
  }
  ACE_TRY(ws_begin(c, total));  // grows the workspace before any capture
  ACE_TRY(ensure_branches(c, nbr));
  std::vector<unsigned char> key = make_key(c, n_inst, inst, nbr, 1);
  if (c->graph_exec && key == c->graph_key) {
    hipError_t e = hipGraphLaunch(c->graph_exec, c->stream);  // replay
    return e == hipSuccess ? ACE_OK : hip_fail(c, e, "hipGraphLaunch");
  }
  drop_graph(c);
  return capture_and_launch(c, std::move(key), [&](hipStream_t main) -> ace_status {
    ace_status st = ACE_OK;
    hipError_t e = hipEventRecord(c->fork_event, main);
    for (int b = 0; b < nbr && e == hipSuccess; ++b)
      e = hipStreamWaitEvent(c->branch_streams[b], c->fork_event, 0);
    if (e != hipSuccess) return hip_fail(c, e, "fork");
    for (int b = 0; b < nbr && st == ACE_OK; ++b) {
      c->stream = c->branch_streams[b];
      c->sub_base = (char*)c->ws + boff[b];
      c->sub_bytes = bbytes[b];
      for (int k = 0; k < n_inst && st == ACE_OK; ++k) {
        if (plan[k].branch != b) continue;
        const ace_prec prec = (ace_prec)inst[k].prec;
        if (prec == ACE_FP64) {
          st = record_instance<double>(c, inst[k], plan[k].g);
          if (st == ACE_OK) st = compress_instance<double>(c, inst[k], plan[k].g);
        } else {
          st = record_instance<float>(c, inst[k], plan[k].g);
          if (st == ACE_OK) st = compress_instance<float>(c, inst[k], plan[k].g);
        }
      }
      if (st == ACE_OK) {
        e = hipEventRecord(c->branch_events[b], c->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(main, c->branch_events[b], 0);
        if (e != hipSuccess) st = hip_fail(c, e, "join");
      }
    }
    return st;
  });
}

// ---------------------------------------------------------------------------
// Persistent form.
struct Bucket {
  int n;
  size_t eb;
  std::vector<int> members;   // by decreasing cost
  std::vector<size_t> off;    // pair-region offset of each member
  std::vector<size_t> bytes;  // build workspace of each member
  size_t cap;                 // pair budget cap of each member
  size_t total;
  // recorded run
  bool accq = false;
  int nlaunch = 0, ntasks = 0, grid = 0;
  ace_plaunch* dL = nullptr;
  ace_ptask* dT = nullptr;
  int* ctl = nullptr;
  int* done = nullptr;
};

// Tasks of the recorded launches: the launches of the members interleave (the
// s-th launch of every member, then the (s+1)-th ...), so every task comes
// after the tasks it waits for (the previous launch of its instance).  A
// launch is cut into tasks of up to kMaxTaskSteps steps, about one task per
// workgroup when it is large (every task ends with a release, which writes
// back the XCD's L2).
constexpr long kMaxTaskSteps = 64;

std::vector<ace_ptask> make_tasks(const Bucket& bk, const std::vector<ace_plaunch>& L,
                                  const std::vector<int>& first) {
  std::vector<ace_ptask> tasks;
  std::vector<int> ntask(L.size(), 0);
  const int m = (int)bk.members.size();
  std::vector<int> pos(m, 0);
  for (bool any = true; any;) {
    any = false;
    for (int q = 0; q < m; ++q) {
      const int li = first[q] + pos[q];
      if (li >= first[q + 1]) continue;
      any = true;
      const ace_plaunch& l = L[li];
      const long step = persist_step(bk.n, bk.eb, l.kind);
      const long iters = (l.units + step - 1) / step;
      const long per = std::max<long>(
          1, std::min<long>(kMaxTaskSteps, (iters + bk.grid - 1) / bk.grid));
      for (long it = 0; it < iters; it += per) {
        ace_ptask t{};
        t.launch = li;
        t.wait = pos[q] > 0 ? li - 1 : -1;
        t.wait_count = pos[q] > 0 ? ntask[li - 1] : 0;
        t.u0 = it * step;
        t.u1 = std::min(l.units, (it + per) * step);
        tasks.push_back(t);
        ++ntask[li];
      }
      ++pos[q];
    }
  }
  return tasks;
}

ace_status batched_persistent(ace_ctx c, int n_inst, const ace_instance* inst,
                              std::vector<Planned>& plan) {
  std::vector<Bucket> bks;
  std::vector<size_t> ebs(n_inst);
  for (int k = 0; k < n_inst; ++k) {
    ebs[k] = (ace_prec)inst[k].prec == ACE_FP64 ? 16 : 8;
    int b = 0;
    while (b < (int)bks.size() && !(bks[b].n == plan[k].g.n && bks[b].eb == ebs[k])) ++b;
    if (b == (int)bks.size()) {
      bks.emplace_back();
      bks[b].n = plan[k].g.n;
      bks[b].eb = ebs[k];
    }
    bks[b].members.push_back(k);
  }
  // The members of a size run concurrently, each with its own pair buffers:
  // their pair budgets are capped so that one size's buffers take at most
  // min(24 GiB, a quarter of the free device memory).
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    fr = (size_t)64 << 30;
  }
  const size_t region_cap = std::min<size_t>((size_t)24 << 30, fr / 4);
  size_t region = 0;
  for (auto& bk : bks) {
    std::sort(bk.members.begin(), bk.members.end(),
              [&](int a, int b) { return plan[a].cost > plan[b].cost; });
    bk.cap = std::max<size_t>(region_cap / bk.members.size(), (size_t)64 << 20);
    c->budget_cap = bk.cap;
    bk.total = 0;
    for (int k : bk.members) {
      const ace_instance& in = inst[k];
      const BuildPlan bp = plan_build(c, plan[k].g, ebs[k], in.n_occ, in.n_band,
                                      in.psi == in.phi && in.ld_psi == in.ld_phi);
      bk.off.push_back(bk.total);
      bk.bytes.push_back(align_up(bp.bytes, 256));
      bk.total += bk.bytes.back();
    }
    c->budget_cap = 0;
    region = std::max(region, bk.total);
  }
  std::vector<char> has_xi(n_inst);
  std::vector<size_t> cbytes(n_inst, 0);
  int n_xi = 0;
  for (int k = 0; k < n_inst; ++k) {
    has_xi[k] = inst[k].xi != nullptr;
    n_xi += has_xi[k];
    if (has_xi[k]) cbytes[k] = compress_ws_bytes(inst[k].n_band, plan[k].g.ng);
  }
  const int nbr = std::max(1, std::min(c->branches, n_xi));
  const std::vector<size_t> bbytes = assign_branches(plan, has_xi, cbytes, nbr);
  std::vector<size_t> boff(nbr, 0);
  size_t total = align_up(region, 256);
  for (int b = 0; b < nbr; ++b) {
    boff[b] = total;
    total += bbytes[b];
  }
  ACE_TRY(ws_begin(c, total));
  ACE_TRY(ensure_branches(c, nbr));
  std::vector<unsigned char> key = make_key(c, n_inst, inst, nbr, 2);
  if (c->graph_exec && key == c->graph_key) {
    hipError_t e = hipGraphLaunch(c->graph_exec, c->stream);  // replay
    return e == hipSuccess ? ACE_OK : hip_fail(c, e, "hipGraphLaunch");
  }
  drop_graph(c);

  // record each size's launches (nothing runs), build its task list and copy
  // both to device memory
  ace_status st = ACE_OK;
  for (auto& bk : bks) {
    std::vector<ace_plaunch> L;
    std::vector<int> first(1, 0);
    for (size_t q = 0; q < bk.members.size() && st == ACE_OK; ++q) {
      const int k = bk.members[q];
      c->record = &L;
      c->budget_cap = bk.cap;
      c->sub_base = (char*)c->ws + bk.off[q];
      c->sub_bytes = bk.bytes[q];
      st = bk.eb == 16 ? record_instance<double>(c, inst[k], plan[k].g)
                       : record_instance<float>(c, inst[k], plan[k].g);
      c->record = nullptr;
      c->budget_cap = 0;
      c->sub_base = nullptr;
      c->sub_bytes = 0;
      first.push_back((int)L.size());
    }
    if (st != ACE_OK) return st;
    int nq = 0, nl = 0;
    for (const auto& l : L) {
      nq += l.kind == kPassAccumQ;
      nl += l.kind == kPassAccum;
    }
    if (nq && nl) return fail(c, ACE_E_ARG, "internal: mixed accumulate forms in one size");
    bk.accq = nq > 0;
    int bpc = 0;
    ACE_TRY(persist_blocks_per_cu(c, bk.n, bk.eb, bk.accq, &bpc));
    if (bpc < 1) return fail(c, ACE_E_UNSUPPORTED, "persistent kernel does not fit a CU");
    bk.grid = bpc * c->num_cus;
    const std::vector<ace_ptask> tasks = make_tasks(bk, L, first);
    // the kernel trusts these: every task in its launch's range, every wait on
    // an earlier launch with all its tasks before the waiting one
    {
      std::vector<int> seen(L.size(), 0);
      for (const ace_ptask& t : tasks) {
        const bool ok = t.launch >= 0 && t.launch < (int)L.size() && t.u0 >= 0 && t.u0 < t.u1 &&
                        t.u1 <= L[t.launch].units &&
                        (t.wait < 0 || (t.wait < t.launch && seen[t.wait] == t.wait_count));
        if (!ok) return fail(c, ACE_E_ARG, "internal: persistent task list");
        ++seen[t.launch];
      }
    }
    bk.nlaunch = (int)L.size();
    bk.ntasks = (int)tasks.size();
    const size_t lb = align_up(L.size() * sizeof(ace_plaunch), 256);
    const size_t tb = align_up(tasks.size() * sizeof(ace_ptask), 256);
    const size_t cb = align_up((2 + L.size()) * sizeof(int), 256);
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, lb + tb + cb);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, ACE_E_NOMEM, "task list allocation");
    }
    c->graph_bufs.push_back(d);
    bk.dL = (ace_plaunch*)d;
    bk.dT = (ace_ptask*)((char*)d + lb);
    bk.ctl = (int*)((char*)d + lb + tb);
    bk.done = bk.ctl + 2;
    e = hipMemcpy(bk.dL, L.data(), L.size() * sizeof(ace_plaunch), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(bk.dT, tasks.data(), tasks.size() * sizeof(ace_ptask), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "task list upload");
  }
  // a wait that lasts 10 s means a defect: give up rather than hang
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) != hipSuccess ||
      khz <= 0) {
    (void)hipGetLastError();
    khz = 100000;
  }
  const long long spin_ticks = (long long)khz * 1000 * 10;

  return capture_and_launch(c, std::move(key), [&](hipStream_t main) -> ace_status {
    std::vector<char> forked(nbr, 0);
    for (auto& bk : bks) {
      c->stream = main;
      ACE_TRY(persist_run(c, bk.n, bk.eb, bk.accq, bk.dL, bk.nlaunch, bk.dT, bk.ntasks, bk.ctl,
                          bk.done, bk.grid, spin_ticks));
      // the compressions of this size's instances follow on the branches
      hipError_t e = hipEventRecord(c->fork_event, main);
      if (e != hipSuccess) return hip_fail(c, e, "fork");
      std::fill(forked.begin(), forked.end(), 0);
      for (int k : bk.members) {
        if (!has_xi[k]) continue;
        const int b = plan[k].branch;
        if (!forked[b]) {
          e = hipStreamWaitEvent(c->branch_streams[b], c->fork_event, 0);
          if (e != hipSuccess) return hip_fail(c, e, "fork");
          forked[b] = 1;
        }
        c->stream = c->branch_streams[b];
        c->sub_base = (char*)c->ws + boff[b];
        c->sub_bytes = bbytes[b];
        ACE_TRY(bk.eb == 16 ? compress_instance<double>(c, inst[k], plan[k].g)
                            : compress_instance<float>(c, inst[k], plan[k].g));
      }
      c->sub_base = nullptr;
      c->sub_bytes = 0;
    }
    for (int b = 0; b < nbr; ++b) {
      hipError_t e = hipEventRecord(c->branch_events[b], c->branch_streams[b]);
      if (e == hipSuccess) e = hipStreamWaitEvent(main, c->branch_events[b], 0);
      if (e != hipSuccess) return hip_fail(c, e, "join");
    }
    return ACE_OK;
  });
}

}  // namespace
}  // namespace ace

using namespace ace;

ACE_EXPORT ace_status ace_build_W_batched(ace_ctx c, int n_inst, const ace_instance* inst) {
  if (!c) return ACE_E_ARG;
  if (n_inst < 1 || !inst) return fail(c, ACE_E_ARG, "no instances");
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
  // Instances run concurrently: no instance's output may overlap another
  // instance's inputs or outputs.
  auto outs = [&](int k, Span* o) {
    const ace_instance& in = inst[k];
    const size_t eb = elem_bytes((ace_prec)in.prec);
    o[0] = span_of(in.W, in.n_band, in.ld_W, plan[k].g.ng, eb);
    o[1] = in.xi ? span_of(in.xi, in.n_band, in.ld_xi, plan[k].g.ng, eb) : Span{};
  };
  for (int k = 0; k < n_inst; ++k) {
    Span ok[2];
    outs(k, ok);
    for (int m = 0; m < n_inst; ++m) {
      if (m == k) continue;
      const ace_instance& im = inst[m];
      const size_t eb = elem_bytes((ace_prec)im.prec);
      Span om[4];
      outs(m, om);
      om[2] = span_of(im.phi, im.n_occ, im.ld_phi, plan[m].g.ng, eb);
      om[3] = span_of(im.psi, im.n_band, im.ld_psi, plan[m].g.ng, eb);
      for (const Span& a : ok)
        for (const Span& b : om)
          if (overlap(a, b)) {
            char buf[96];
            snprintf(buf, sizeof buf, "an output of instance %d overlaps instance %d", k, m);
            return fail(c, ACE_E_ARG, buf);
          }
    }
  }
  const int form = c->batch_form ? c->batch_form : kDefaultBatchForm;
  return form == 2 ? batched_persistent(c, n_inst, inst, plan)
                   : batched_launches(c, n_inst, inst, plan);
}
