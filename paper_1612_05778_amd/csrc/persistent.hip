// All stages of all products of a batch in one persistent launch.
//
// The tiles of the batch's grouped launches, in the same order (level by level), form one
// task list.  Each workgroup repeatedly takes the next task number from a ticket counter,
// waits until the tiles of the previous stage of that task's product are done, runs the
// stage body, and counts its tile as done.  A task's dependencies (the previous stage of
// its own product) always have smaller task numbers, so the unfinished task with the
// smallest number never waits on anything unfinished: its workgroup (which is running,
// since it took the ticket) proceeds.  The launch therefore completes whatever the number
// of workgroups resident at once and whatever order the hardware dispatches them in.
//
// Visibility across the XCDs' separate L2 caches: a finished tile's stores are made
// visible with an agent-scope release fence in every lane (write-back of this XCD's L2)
// before one lane's agent-scope increment of the stage counter; a waiting workgroup polls
// that counter with agent-scope atomic loads (coherent reads that do not invalidate any
// cache) and, once it is complete, every lane takes an agent-scope acquire fence (L1 and
// L2 invalidation) before reading the previous stage's output.
//
// Every wait is bounded: past `spin_limit` polls the workgroup raises the abort flag,
// every workgroup stops at its next poll or ticket, and the host reports the batch as
// failed.  The kernel therefore always exits.
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "stages.hpp"

namespace zpm {

__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int find_seg_p(const GroupSeg *__restrict__ segs, int32_t nseg, int64_t b) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].start <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int NP>
__device__ __forceinline__ void run_convert(uint32_t *s, const JobDev &jb, int64_t tile,
                                            const PrimeDev *__restrict__ primes) {
  const bool ob = tile >= jb.tiles_a;
  const int32_t N = ob ? jb.Nb : jb.Na;
  body_convert_in<NP>(s, ob ? tile - jb.tiles_a : tile, ob ? jb.b : jb.a, ob ? jb.db : jb.da, N,
                      (N + 63) / 64, jb.K, jb.M, NP, jb.X, jb.L, ob ? jb.K : 0, jb.log_ti_in,
                      primes, jb.plan);
}

template <int NP>
__device__ __forceinline__ void run_recover(uint32_t *s, const JobDev &jb, int64_t tile,
                                            const PrimeDev *__restrict__ primes) {
  body_recover<NP>(reinterpret_cast<uint64_t *>(s), tile, jb.X, jb.L, jb.K, jb.M, jb.nout, jb.nw32,
                   jb.wc, jb.log_ti_out, primes, jb.plan, jb.c);
}

__device__ void run_task(uint32_t *s, const Group &gr, const GroupSeg &sg, const JobDev &jb,
                         int64_t tile, const PrimeDev *__restrict__ primes) {
  const int64_t L = jb.L;
  switch (gr.kind) {
    case SK_CONVERT:
      switch (gr.variant) {
#define ZPM_P(NP_) \
  case NP_: run_convert<NP_>(s, jb, tile, primes); break;
        ZPM_P(1) ZPM_P(2) ZPM_P(3) ZPM_P(4) ZPM_P(5) ZPM_P(6) ZPM_P(7) ZPM_P(8)
        ZPM_P(9) ZPM_P(10) ZPM_P(11) ZPM_P(12) ZPM_P(13) ZPM_P(14) ZPM_P(15) ZPM_P(16)
#undef ZPM_P
        default: break;
      }
      break;
    case SK_RECOVER:
      switch (gr.variant) {
#define ZPM_P(NP_) \
  case NP_: run_recover<NP_>(s, jb, tile, primes); break;
        ZPM_P(1) ZPM_P(2) ZPM_P(3) ZPM_P(4) ZPM_P(5) ZPM_P(6) ZPM_P(7) ZPM_P(8)
        ZPM_P(9) ZPM_P(10) ZPM_P(11) ZPM_P(12) ZPM_P(13) ZPM_P(14) ZPM_P(15) ZPM_P(16)
#undef ZPM_P
        default: break;
      }
      break;
    case SK_COL_FWD:
    case SK_COL_INV: {
      // every pass shape through the runtime-shape body
      const int inverse = gr.kind == SK_COL_INV ? 1 : 0;
      const int c = sg.pass;
      const bool outer = c == 0;
      body_col_pass<-1, -1>(s, tile, jb.X, L, 2 * jb.K, jb.col_logn[c], jb.col_S[c], jb.col_logT[c],
                            (outer && !inverse) ? jb.da : L, (outer && !inverse) ? jb.db : L, jb.K,
                            (outer && inverse) ? jb.nout : L, inverse, primes,
                            (jb.square && !inverse) ? jb.K : 2 * jb.K, 0);
      break;
    }
    case SK_CONVOLVE: {
      const bool direct = jb.ncol == 0;
      const int64_t nza = direct ? jb.da : L, nzb = direct ? jb.db : L, nl = direct ? jb.nout : L;
      if (gr.variant >= 64 || gr.variant == 0) {
        int logK = 0;
        while ((1 << logK) < jb.K) ++logK;
        body_convolve<-1, -1>(s, tile, jb.X, L, jb.K, logK, jb.logL1, nza, nzb, nl, primes, jb.plan,
                              jb.square ? CM_SQUARE : CM_PRODUCT, nullptr);
        break;
      }
      const bool sq = (gr.variant & 16) != 0;
      switch (gr.variant & 15) {
#define ZPM_P(LK_)                                                                                  \
  case LK_:                                                                                         \
    if (sq) body_convolve_reg<LK_, CM_SQUARE, -1>(s, tile, jb.X, L, jb.logL1, nza, nzb, nl, primes, \
                                                  jb.plan, nullptr);                               \
    else body_convolve_reg<LK_, CM_PRODUCT, -1>(s, tile, jb.X, L, jb.logL1, nza, nzb, nl, primes,   \
                                                jb.plan, nullptr);                                 \
    break;
        ZPM_P(1) ZPM_P(2) ZPM_P(3) ZPM_P(4)
#undef ZPM_P
        default: break;
      }
      break;
    }
    default:
      break;
  }
}

// Called by every thread of the workgroup (all the lane-0 work of the task loop lives
// here, so that the loop in the kernel has no divergent branch next to its head or its
// back edge; otherwise the structurizer nests a lane-divergent inner loop around the
// barrier and the task, in which lanes 1..63 of wave 0 re-run the last task while lane 0,
// which writes the next one, waits outside it).  Lane 0 counts the previous task (prev >= 0:
// its done-counter slot; the caller made every lane's stores visible before this call),
// takes the next ticket and waits for its dependencies.  Returns the task number, or -1
// when there is none left or the launch was aborted; *gi / *si get its group and segment.
__device__ __noinline__ int64_t next_task(const GroupSeg *__restrict__ segs,
                                          const Group *__restrict__ groups,
                                          const int64_t *__restrict__ gstart, int32_t ngroups,
                                          int64_t ntasks, const uint32_t *__restrict__ need,
                                          uint32_t *done, PersistCtl *ctl, uint32_t spin_limit,
                                          int64_t prev, int32_t *gi, int32_t *si) {
  __shared__ int64_t sh_task;
  __shared__ int32_t sh_group, sh_seg;
  if (threadIdx.x == 0) {
    if (prev >= 0)
      __hip_atomic_fetch_add(done + prev, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int64_t t = -1;
    int32_t g = 0, sgi = 0;
    if (!ld_agent(&ctl->abort)) {
      t = (int64_t)__hip_atomic_fetch_add(&ctl->ticket, 1ull, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
      if (t >= ntasks) {
        t = -1;
      } else {
        int lo = 0, hi = ngroups - 1;   // last group with gstart <= t
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (gstart[mid] <= t) lo = mid;
          else hi = mid - 1;
        }
        g = lo;
        const Group &gr = groups[g];
        sgi = (int32_t)gr.seg0 + find_seg_p(segs + gr.seg0, gr.nseg, t - gstart[g]);
        if (gr.level > 0) {
          // the tiles of the previous stage of this product
          const int64_t slot = (int64_t)segs[sgi].job * PERSIST_LEVELS + gr.level - 1;
          const uint32_t want = need[slot];
          uint32_t spins = 0;
          while (ld_agent(done + slot) < want) {
            if (ld_agent(&ctl->abort)) {
              t = -1;
              break;
            }
            if (++spins > spin_limit) {
              __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              t = -1;
              break;
            }
            __builtin_amdgcn_s_sleep(2);
          }
        }
      }
    }
    sh_task = t;
    sh_group = g;
    sh_seg = sgi;
  }
  __syncthreads();
  *gi = sh_group;
  *si = sh_seg;
  const int64_t t = sh_task;
  __syncthreads();   // sh_* are rewritten by the next call
  return t;
}

__device__ __forceinline__ int64_t uniform64(int64_t v) {
  return (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(v >> 32)) << 32) |
                   (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)v));
}

__global__ __launch_bounds__(BLOCK) void k_batch_persistent(
    const JobDev *__restrict__ jobs, const GroupSeg *__restrict__ segs,
    const Group *__restrict__ groups, const int64_t *__restrict__ gstart, int32_t ngroups,
    int64_t ntasks, const uint32_t *__restrict__ need, uint32_t *done, PersistCtl *ctl,
    const PrimeDev *__restrict__ primes, uint32_t spin_limit) {
  extern __shared__ uint64_t S64[];
  uint32_t *s = reinterpret_cast<uint32_t *>(S64);
  int64_t prev = -1;
  for (;;) {
    int32_t gv, sv;
    const int64_t t = uniform64(next_task(segs, groups, gstart, ngroups, ntasks, need, done, ctl,
                                          spin_limit, prev, &gv, &sv));
    if (t < 0) break;
    const int32_t gi = __builtin_amdgcn_readfirstlane(gv);
    const int32_t si = __builtin_amdgcn_readfirstlane(sv);
    // the previous stage's output, written on any XCD, is read fresh
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const Group gr = groups[gi];
    const GroupSeg sg = segs[si];
    const JobDev &jb = jobs[sg.job];
    run_task(s, gr, sg, jb, t - gstart[gi] - sg.start, primes);
    // every lane's stores written back before the tile is counted (by the next call)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    prev = (int64_t)sg.job * PERSIST_LEVELS + gr.level;
  }
}

__global__ __launch_bounds__(BLOCK) void k_persist_zero(uint32_t *done, int64_t n, PersistCtl *ctl) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) done[i] = 0;
  if (i == 0) {
    ctl->ticket = 0;
    ctl->abort = 0;
  }
}

hipError_t launch_persistent(const JobDev *jobs, const GroupSeg *segs, const Group *groups,
                             const int64_t *gstart, int32_t ngroups, int64_t ntasks,
                             const uint32_t *need, uint32_t *done, int64_t nslots, PersistCtl *ctl,
                             const PrimeDev *primes, size_t lds, uint32_t spin_limit, int ncu,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_persist_zero, dim3((unsigned)((nslots + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0,
                     st, done, nslots, ctl);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persistent, BLOCK, lds) !=
      hipSuccess)
    return hipErrorInvalidValue;
  per_cu = per_cu < 1 ? 1 : per_cu;
  int64_t grid = (int64_t)per_cu * ncu;
  if (grid > ntasks) grid = ntasks;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_batch_persistent, dim3((unsigned)grid), dim3(BLOCK), lds, st, jobs, segs,
                     groups, gstart, ngroups, ntasks, need, done, ctl, primes, spin_limit);
  return hipGetLastError();
}

}  // namespace zpm
