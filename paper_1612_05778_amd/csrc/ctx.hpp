// Library context: resident twiddle tables, per-plan constants, workspace.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/zpm.h"
#include "batch.hpp"
#include "kernels.hpp"
#include "zpm_internal.hpp"

namespace zpm {

// Host-side schedule of a batch (see Ctx::schedule_batch).
struct BatchHost {
  std::vector<Plan> plans;       // per job of the call (only live jobs are planned)
  std::vector<JobDev> jobs;      // live jobs; X = workspace offset in words
  std::vector<int32_t> job_plan; // live job -> index into plans
  std::vector<GroupSeg> segs;    // segments of all launches, launch after launch
  std::vector<Group> groups;     // launches in order
  int64_t ws_words = 0, H = 2, TP = 64;
  int npmax = 1;
};

// Device and pinned host buffers of one batch, plus its captured graph.
struct BatchState {
  BatchHost host;
  uint32_t *ws = nullptr;
  int64_t ws_cap = 0;
  JobDev *jobs_h = nullptr, *jobs_d = nullptr;
  int64_t jobs_hcap = 0, jobs_dcap = 0;
  GroupSeg *segs_h = nullptr, *segs_d = nullptr;
  int64_t segs_hcap = 0, segs_dcap = 0;
  int32_t nseg = 0;
  int64_t nlive = 0;
  hipEvent_t upload_done = nullptr;
  hipGraphExec_t exec = nullptr;
  // persistent launch: groups, their first task numbers, tiles per product stage, the
  // done counters and the ticket/abort words
  Group *groups_h = nullptr, *groups_d = nullptr;
  int64_t *gstart_h = nullptr, *gstart_d = nullptr;
  uint32_t *need_h = nullptr, *need_d = nullptr, *done_d = nullptr;
  int64_t groups_hcap = 0, groups_dcap = 0, gstart_hcap = 0, gstart_dcap = 0;
  int64_t need_hcap = 0, need_dcap = 0, done_dcap = 0;
  PersistCtl *ctl_h = nullptr, *ctl_d = nullptr;
  uint64_t key = 0;
  static uint64_t hash(const zpm_job *jobs, int64_t n, int32_t K_force, int32_t T_force,
                       const uint32_t *const *specs = nullptr, const Plan *given = nullptr);
  void release();
};

// Autotuned choice for a size class: limb count K and column-tile width T.
struct TuneChoice {
  int32_t K = 0, T = 0;
};
using TuneTable = std::map<int32_t, TuneChoice>;

// Plan of a product for the batch kernels: the tuned K and column tile of its size
// class when `tuned` has them (and they are feasible), else the planner's choice,
// limited to what the batch kernels support.  K_force / T_force != 0 force K / T.
int plan_for_batch(const TuneTable &tuned, int64_t da, int32_t Na, int64_t db, int32_t Nb,
                   int32_t K_force, int32_t T_force, Plan *out);

// Kronecker reshaping of a product with wide coefficients: chunks of w bits, y -> z^S.
struct KronPlan {
  int32_t w = 0, wq = 0, sa = 0, sb = 0, S = 0, N2 = 0, wc2 = 0;
  int64_t da2 = 0, db2 = 0, nout2 = 0;
  Plan inner;          // plan of the reshaped product (da2, N2) x (db2, N2)
  double cost = 0;
};
// Chooses the chunk width (chunk_bits, a multiple of 64, or 0 for the cheapest of
// 256 ... 16384 by the planner's cost model); false when no reshaping has a plan.
bool kron_plan(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t chunk_bits, KronPlan *out);

struct P64State;   // tables and workspace of the 64-bit prime variant
struct GfpState;   // tables and workspace of the generalized Fermat prime variant

struct Ctx {
  int device = 0;
  P64State *p64 = nullptr;
  GfpState *gfp = nullptr;
  PrimeDev *primes = nullptr;   // MAXNP entries
  uint2 *heaps = nullptr;       // np_built primes x (forward H, inverse H)
  int np_built = 0;
  int64_t H_built = 0;
  int64_t TP_built = 0;         // entries of each prime's 2^(32 t) table
  std::map<std::tuple<int, int, int, int>, PlanDev *> consts;
  std::vector<PlanDev *> consts_owned;          // allocated one by one (before zpm_reserve)
  // zpm_reserve: tables, workspace and plan-constant slots are fixed; products that
  // need more get ZPM_ENOMEM instead of a reallocation
  bool reserved = false;
  PlanDev *pool_d = nullptr, *pool_h = nullptr; // plan-constant slots and their pinned copies
  int pool_cap = 0, pool_used = 0;
  std::vector<std::pair<PlanDev *, PlanDev *>> pool_old;   // earlier, smaller pools
  // checked-input mode (ZPM_OPT_CHECK_INPUTS)
  int check_inputs = 0;
  uint32_t *flag_d = nullptr, *flag_h = nullptr;
  std::map<std::tuple<int64_t, int32_t, int64_t, int32_t, int32_t, int32_t, int32_t>, Plan> plans;
  uint32_t *ws = nullptr;
  int64_t ws_words = 0;
  uint64_t *kbuf = nullptr;     // reshaped operands and product of mul_kronecker
  int64_t kbuf_words = 0;
  std::mutex mu;
  Profiler prof;
  TuneTable tuned;                             // size class -> choice of zpm_tune
  BatchState batch_eager, batch_graph;
  hipStream_t capture_stream = nullptr;        // graph capture only (default priority)

  int ensure_tables(int np, int64_t H, int64_t TP);
  // st: stream of the call that needs the constants (a reserved slot is uploaded there)
  int plan_consts(const Plan &pl, PlanDev **out, hipStream_t st = nullptr);
  int reserve(size_t ws_bytes, int64_t max_len, int32_t max_bits, int32_t max_plans);
  // checked-input mode: ZPM_ERANGE if a coefficient of src has bits >= N that are not
  // copies of bit N-1 (waits for the check on st); ZPM_OK when the mode is off
  int check_range(const uint64_t *src, int64_t d, int32_t N, hipStream_t st);
  int ensure_ws(int64_t words);
  int ensure_kbuf(int64_t words);
  int mul_kronecker(const uint64_t *a, int64_t da, int32_t Na, const uint64_t *b, int64_t db,
                    int32_t Nb, uint64_t *c, int32_t wc, int32_t chunk_bits, hipStream_t st);
  // alone: the plan of a product that runs by itself (the row-group floor applies);
  // false for a resident operand, whose plan also serves batches
  int get_plan(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K, int32_t np, Plan *out,
               bool alone = true);
  int prepare(const Plan &pl, DevState *ds, hipStream_t st = nullptr);
  int get_plan_batch(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K_force,
                     int32_t T_force, Plan *out);
  // given: plans per job (from plan_for_batch) instead of the context's choice; specs:
  // per job, b's resident spectra (an operand's, whose plan given[] then holds) or null
  int schedule_batch(const zpm_job *jobs, int64_t n, int32_t K_force, BatchHost &bh,
                     const Plan *given = nullptr, int32_t T_force = 0,
                     const uint32_t *const *specs = nullptr);
  // ws_ext: workspace of ws_ext_words words to use instead of the state's own buffer
  int build_batch(const zpm_job *jobs, int64_t n, int32_t K_force, BatchState &bs,
                  const Plan *given = nullptr, uint32_t *ws_ext = nullptr, int64_t ws_ext_words = 0,
                  int32_t T_force = 0, const uint32_t *const *specs = nullptr);
  // sizes the descriptor buffers of bs for batches of up to `jobs` products and `segs`
  // segments, so that later batches within those bounds allocate nothing
  int reserve_batch(BatchState &bs, int64_t jobs, int64_t segs);
  int enqueue_batch(BatchState &bs, hipStream_t st);
  // the whole batch as one persistent launch; waits for it (ZPM_EDEVICE if a wait of the
  // kernel exceeded its bound)
  int enqueue_persistent(BatchState &bs, hipStream_t st);
  int ncu = 0;                                 // compute units of the device (persistent grid)
  int mul_batch(const zpm_job *jobs, int64_t n, int32_t flags, int32_t K_force, hipStream_t st,
                int32_t T_force = 0, const Plan *given = nullptr,
                const uint32_t *const *specs = nullptr);
  int tune(const zpm_job *sample, int64_t n, hipStream_t st);
  ~Ctx();
};

}  // namespace zpm

// A resident operand: b's spectra under a plan sized for products with any a of at
// most da_max coefficients and Na_max bits.
struct zpm_operand {
  zpm::Ctx *cx;
  zpm::Plan pl;        // plan for (da_max, Na_max, db, Nb)
  uint32_t *spec;      // np * 2K * L words: b's forward transforms
  const uint64_t *b;   // the operand's words, for the overlap check only
  int64_t db, da_max;
  int32_t Nb, Na_max;
};

namespace zpm {

// The operand's plan for a product with an a of da coefficients and Na bits: K, M, np
// and L are the operand's.
Plan operand_plan(const zpm_operand &op, int64_t da, int32_t Na);
// c = a * (the operand's b) under pl (from operand_plan) with workspace ws of pl.ws_words
// words, on st; the caller holds cx.mu.
int operand_product(Ctx &cx, const zpm_operand &op, const Plan &pl, const uint64_t *a, uint64_t *c,
                    int32_t wc, uint32_t *ws, hipStream_t st);

}  // namespace zpm
