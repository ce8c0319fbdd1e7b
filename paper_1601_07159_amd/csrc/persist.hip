// Persistent form of the batched build (the W stage of Section 3, Eq. W, for
// many independent instances): one launch per grid size runs the pass
// launches of every instance of that size, recorded from the single-instance
// build (slab, plane and accumulate passes, chunk by chunk), as tasks pulled
// from a queue in device memory.
//
// Each workgroup loops: count its previous task as finished (after a release
// fence), take the next task index from an atomic counter; if the task's
// launch depends on an earlier launch of the same instance, wait until that
// launch's finished-task counter reaches its task count; run the task's units
// with the same device bodies as the per-pass kernels.  The task list is ordered so that
// every task comes after all tasks it waits for, so the oldest unfinished
// dequeued task never waits on anything unfinished: the queue drains whatever
// the number of co-resident workgroups.  Every wait is bounded in time as well;
// a wait that runs out sets an error flag, every workgroup then stops, and a
// follow-up kernel writes NaN into each instance's W so that the failure shows
// (the compression then reports a failed factorisation).
#include "ace_internal.h"
#include "pass_bodies.h"

namespace ace {
namespace {

// LDS per workgroup of the slab and plane groups: with more, LDS rather than
// registers sets the occupancy (and the compiler then spends registers freely).
constexpr long kPersistLdsLimit = 40 * 1024;

// Lane use of the slab and plane groups (P groups of N threads in 64 wv
// threads) for a workgroup of wv waves.
template <int N, typename T>
constexpr int persist_groups(int wv) {
  const long plane = (long)N * (N + 1) * (long)sizeof(cx<T>);
  int p = 64 * wv / N;
  while (p > 1 && p * plane > kPersistLdsLimit) --p;
  return p < 1 ? 1 : p;
}

// Waves per workgroup: the best lane use of the slab and plane groups, fewer
// waves on a tie.
template <int N, typename T>
constexpr int persist_waves() {
  int best = 1;
  double best_use = 0.0;
  for (int wv = 1; wv <= 4; ++wv) {
    const int p = persist_groups<N, T>(wv);
    if (p * N > 64 * wv) continue;
    const double use = (double)(p * N) / (64.0 * wv);
    if (use > best_use + 1e-9) {
      best_use = use;
      best = wv;
    }
  }
  return best;
}

template <int N, typename T, bool AccQ>
struct PShape {
  static constexpr int WV = persist_waves<N, T>();
  static constexpr int P = persist_groups<N, T>(WV);
  static constexpr int kThreads = 64 * WV;
  static constexpr long kPlaneLds = (long)P * N * (N + 1);
  static constexpr long kAccLds = AccQ ? 0 : (long)WV * N * 64;
  static constexpr long kLds = kPlaneLds > kAccLds ? kPlaneLds : kAccLds;  // elements
  // slab rows loaded per batch (keeps the slab pass's registers near the
  // other passes' so that the kernel is not limited by its heaviest body)
  static constexpr int kLoadBatch = N % 8 == 0 ? 8 : 4;
};

// Value of lane 0 in every lane (a scalar register): the queue logic below
// keeps all its branches wave-uniform.  With a divergent "lane 0 takes the
// task" branch, a workgroup of one wave (whose barriers the compiler drops)
// was compiled into an inner loop in which the other lanes re-read the task
// slot without lane 0 ever taking the next task.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <int N, typename T, bool AccQ>
__global__ __launch_bounds__((PShape<N, T, AccQ>::kThreads)) void k_build_persistent(
    const ace_plaunch* __restrict__ L, const ace_ptask* __restrict__ tasks, int ntasks,
    int* __restrict__ ctl, int* __restrict__ done, long long spin_ticks) {
  using S = PShape<N, T, AccQ>;
  __shared__ cx<T> lds[S::kLds];
  __shared__ int cur;
  const int tid = threadIdx.x;
  const int wave = uni(tid >> 6), lane = tid & 63;
  int prev = -1;  // launch of this workgroup's last task, counted at the next take
  for (;;) {
    if (wave == 0) {
      // every lane of wave 0 runs this; only lane 0 adds 1
      if (prev >= 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(&done[prev], lane == 0 ? 1 : 0, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      }
      int t = uni(__hip_atomic_fetch_add(&ctl[0], lane == 0 ? 1 : 0, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT));
      if (t < ntasks && uni(__hip_atomic_load(&ctl[1], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT)) != 0)
        t = ntasks;  // another workgroup gave up
      if (t < ntasks) {
        const int w = uni(tasks[t].wait), need = uni(tasks[t].wait_count);
        if (w >= 0) {
          const long long t0 = wall_clock64();
          while (uni(__hip_atomic_load(&done[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) <
                 need) {
            if (uni(__hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0 ||
                wall_clock64() - t0 > spin_ticks) {
              __hip_atomic_store(&ctl[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              t = ntasks;
              break;
            }
            __builtin_amdgcn_s_sleep(2);
          }
          // the finished launch's results become visible to this workgroup
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
      }
      cur = t;
    }
    __syncthreads();
    const int t = uni(cur);
    if (t >= ntasks) break;
    const ace_ptask tk = tasks[t];
    const ace_plaunch& l = L[tk.launch];
    switch (l.kind) {
      case kPassSlab:
        for (long u = tk.u0; u < tk.u1; u += S::P) {
          slab_t1_body<N, T, S::P, S::kLoadBatch>(lds, tid, tid >= S::P * N, u, tk.u1,
                                                  (const cx<T>*)l.phi, l.ldphi,
                                                  (const cx<T>*)l.psi, l.ldpsi, (cx<T>*)l.buf,
                                                  l.mode, l.i0, l.A, l.j0, l.p0, l.npairs);
          __syncthreads();  // the LDS planes are rewritten by the next step
        }
        break;
      case kPassPlane:
        for (long u = tk.u0; u < tk.u1; u += S::P) {
          plane_t1_body<N, T, S::P>(lds, tid, tid >= S::P * N, u, tk.u1, (cx<T>*)l.buf, l.ks,
                                    l.npairs);
          __syncthreads();
        }
        break;
      default:
        if constexpr (AccQ) {
          for (long u = tk.u0 + wave; u < tk.u1; u += S::WV)
            accum_q_body<N, T>(lane, u, (const cx<T>*)l.phi, l.ldphi, (const cx<T>*)l.buf,
                               (cx<T>*)l.W, l.ldW, l.i0, l.A, l.j0, l.nbc, l.accumulate, l.mode);
        } else {
          for (long u = tk.u0 + wave; u < tk.u1; u += S::WV)
            accum_lds_body<N, T>(lds + wave * N * 64, lane, u, (const cx<T>*)l.phi, l.ldphi,
                                 (const cx<T>*)l.buf, (cx<T>*)l.W, l.ldW, l.i0, l.A, l.j0, l.nbc,
                                 l.accumulate, l.mode);
        }
        break;
    }
    // the workgroup's results are published by wave 0's release at the next
    // take (after this barrier), as in a grid barrier; a release fence in
    // every wave cost a write-back of the XCD's L2 per wave and task (cfg 4:
    // 115 ms of 427)
    __syncthreads();
    prev = tk.launch;
  }
}

__global__ __launch_bounds__(256) void k_zero_ints(int* __restrict__ p, int n) {
  for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) p[k] = 0;
}

template <typename T>
__global__ __launch_bounds__(64) void k_poison_on_error(const ace_plaunch* __restrict__ L,
                                                        int nlaunch, const int* __restrict__ ctl) {
  if (ctl[1] == 0) return;
  for (int k = threadIdx.x; k < nlaunch; k += 64)
    if (L[k].kind == kPassAccum || L[k].kind == kPassAccumQ) {
      cx<T>* w = (cx<T>*)L[k].W + (size_t)L[k].j0 * L[k].ldW;
      w[0] = cx<T>{T(NAN), T(NAN)};
    }
}

template <int N, typename T, bool AccQ>
ace_status run_n(ace_ctx c, const ace_plaunch* L, int nlaunch, const ace_ptask* tasks,
                 int ntasks, int* ctl, int* done, int grid, long long spin_ticks) {
  ACE_TRY(launch(c, "persist_reset", k_zero_ints, dim3(1), dim3(256), 0, ctl, 2));
  ACE_TRY(launch(c, "persist_reset", k_zero_ints, dim3((nlaunch + 255) / 256), dim3(256), 0, done,
                 nlaunch));
  ACE_TRY(launch(c, "build_persistent", k_build_persistent<N, T, AccQ>, dim3(grid),
                 dim3(PShape<N, T, AccQ>::kThreads), 0, L, tasks, ntasks, ctl, done, spin_ticks));
  return launch(c, "persist_check", k_poison_on_error<T>, dim3(1), dim3(64), 0, L, nlaunch,
                (const int*)ctl);
}

template <int N, typename T, bool AccQ>
ace_status occupancy_n(ace_ctx c, int* out) {
  int b = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &b, k_build_persistent<N, T, AccQ>, PShape<N, T, AccQ>::kThreads, 0);
  if (e != hipSuccess) return hip_fail(c, e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
  *out = b;
  return ACE_OK;
}

}  // namespace

int persist_step(int n, size_t eb, int kind) {
#define ACE_CASE(NV)                                                                 \
  if (n == NV) {                                                                     \
    const int wv = eb == 16 ? PShape<NV, double, false>::WV : PShape<NV, float, false>::WV; \
    const int p = eb == 16 ? PShape<NV, double, false>::P : PShape<NV, float, false>::P;    \
    return (kind == kPassSlab || kind == kPassPlane) ? p : wv;                             \
  }
  ACE_FOR_EACH_N(ACE_CASE)
#undef ACE_CASE
  return 0;
}

ace_status persist_blocks_per_cu(ace_ctx c, int n, size_t eb, bool accq, int* out) {
#define ACE_CASE(NV)                                                         \
  if (n == NV) {                                                             \
    if (eb == 16)                                                            \
      return accq ? occupancy_n<NV, double, true>(c, out)                    \
                  : occupancy_n<NV, double, false>(c, out);                  \
    return accq ? occupancy_n<NV, float, true>(c, out) : occupancy_n<NV, float, false>(c, out); \
  }
  ACE_FOR_EACH_N(ACE_CASE)
#undef ACE_CASE
  return fail(c, ACE_E_UNSUPPORTED, "grid size");
}

ace_status persist_run(ace_ctx c, int n, size_t eb, bool accq, const ace_plaunch* L, int nlaunch,
                       const ace_ptask* tasks, int ntasks, int* ctl, int* done, int grid,
                       long long spin_ticks) {
#define ACE_CASE(NV)                                                                        \
  if (n == NV) {                                                                            \
    if (eb == 16)                                                                           \
      return accq ? run_n<NV, double, true>(c, L, nlaunch, tasks, ntasks, ctl, done, grid, \
                                            spin_ticks)                                     \
                  : run_n<NV, double, false>(c, L, nlaunch, tasks, ntasks, ctl, done, grid, \
                                             spin_ticks);                                   \
    return accq ? run_n<NV, float, true>(c, L, nlaunch, tasks, ntasks, ctl, done, grid,    \
                                         spin_ticks)                                        \
                : run_n<NV, float, false>(c, L, nlaunch, tasks, ntasks, ctl, done, grid,   \
                                          spin_ticks);                                      \
  }
  ACE_FOR_EACH_N(ACE_CASE)
#undef ACE_CASE
  return fail(c, ACE_E_UNSUPPORTED, "grid size");
}

}  // namespace ace
