// Host side of batched multiplication: per-product plans, job descriptors, grouped
// launches level by level, and the optional capture of the whole sequence in a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>

#include "../../include/zpm.h"
#include "batch.hpp"
#include "ctx.hpp"
#include "plan.hpp"

namespace zpm {

static int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

int plan_for_batch(const TuneTable &tuned, int64_t da, int32_t Na, int64_t db, int32_t Nb,
                   int32_t K_force, int32_t T_force, Plan *out) {
  PlanLimits lim;
  lim.np_max = 16;
  lim.reg_k_max = 16;
  int32_t K = K_force, T = T_force;
  if (!K && !T) {
    auto it = tuned.find(size_class(da, Na, db, Nb));
    if (it != tuned.end()) {
      K = it->second.K;
      T = it->second.T;
    }
  }
  lim.col_tile = T;
  Plan pl;
  const char *why = nullptr;
  bool ok = make_plan(da, Na, db, Nb, K, 0, pl, &why, &lim);
  if (!ok && K && !K_force) {      // tuned choice infeasible for this member of the class
    lim.col_tile = T_force;
    ok = make_plan(da, Na, db, Nb, 0, 0, pl, &why, &lim);
  }
  if (!ok || !batch_supports(pl)) return ZPM_EUNSUPPORTED;
  *out = pl;
  return ZPM_OK;
}

int Ctx::get_plan_batch(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K_force,
                        int32_t T_force, Plan *out) {
  int32_t K = K_force, T = T_force;
  if (!K && !T) {
    auto it = tuned.find(size_class(da, Na, db, Nb));
    if (it != tuned.end()) {
      K = it->second.K;
      T = it->second.T;
    }
  }
  auto key = std::make_tuple(da, Na, db, Nb, K, T, (int32_t)-1);
  auto it = plans.find(key);
  if (it != plans.end()) { *out = it->second; return ZPM_OK; }
  Plan pl;
  const int rc = plan_for_batch(tuned, da, Na, db, Nb, K_force, T_force, &pl);
  if (rc != ZPM_OK) return rc;
  if (plans.size() > 65536) plans.clear();
  plans[key] = pl;
  *out = pl;
  return ZPM_OK;
}

template <typename T>
static int grow_dev(T **p, int64_t *cap, int64_t n) {
  if (n <= *cap) return ZPM_OK;
  if (*p) {
    // earlier batches on any stream may still read the old buffer
    if (hipDeviceSynchronize() != hipSuccess) return ZPM_EDEVICE;
    (void)hipFree(*p);
  }
  *p = nullptr;
  *cap = 0;
  const int64_t c = n + n / 4;
  if (hipMalloc(p, sizeof(T) * (size_t)c) != hipSuccess) return ZPM_ENOMEM;
  *cap = c;
  return ZPM_OK;
}

template <typename T>
static int grow_host(T **p, int64_t *cap, int64_t n) {
  if (n <= *cap) return ZPM_OK;
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  *cap = 0;
  if (hipHostMalloc(p, sizeof(T) * (size_t)n, hipHostMallocDefault) != hipSuccess) return ZPM_ENOMEM;
  *cap = n;
  return ZPM_OK;
}

uint64_t BatchState::hash(const zpm_job *jobs, int64_t n, int32_t K_force, int32_t T_force,
                          const uint32_t *const *specs, const Plan *given) {
  uint64_t h = 1469598103934665603ull ^ (uint64_t)n ^ ((uint64_t)K_force << 40) ^
               ((uint64_t)T_force << 52);
  const unsigned char *p = reinterpret_cast<const unsigned char *>(jobs);
  for (size_t i = 0; i < sizeof(zpm_job) * (size_t)n; ++i) h = (h ^ p[i]) * 1099511628211ull;
  if (specs) {
    p = reinterpret_cast<const unsigned char *>(specs);
    h = (h ^ 0x5bu) * 1099511628211ull;
    for (size_t i = 0; i < sizeof(*specs) * (size_t)n; ++i) h = (h ^ p[i]) * 1099511628211ull;
  }
  if (given) {
    p = reinterpret_cast<const unsigned char *>(given);
    h = (h ^ 0xa7u) * 1099511628211ull;
    for (size_t i = 0; i < sizeof(*given) * (size_t)n; ++i) h = (h ^ p[i]) * 1099511628211ull;
  }
  return h;
}

// Stage at position `lev` of a product's pipeline: convert-in, forward column passes
// (outermost first), row convolutions, inverse column passes (innermost first),
// recovery.
static void stage_of(const Plan &pl, int lev, int *kind, int *pass) {
  const int nlev = 3 + 2 * pl.ncol;
  *pass = 0;
  if (lev == 0) {
    *kind = SK_CONVERT;
  } else if (lev <= pl.ncol) {
    *kind = SK_COL_FWD;
    *pass = lev - 1;
  } else if (lev == pl.ncol + 1) {
    *kind = SK_CONVOLVE;
  } else if (lev < nlev - 1) {
    *kind = SK_COL_INV;
    *pass = pl.ncol - 1 - (lev - pl.ncol - 2);
  } else {
    *kind = SK_RECOVER;
  }
}

// Tiles of a stage: the grid of the corresponding per-stage kernel.
static int64_t stage_tiles(const Plan &pl, int kind, int pass) {
  const int64_t L = (int64_t)1 << pl.logL;
  switch (kind) {
    case SK_CONVERT: {
      const int64_t ti = (int64_t)1 << pl.log_ti_in;
      return (pl.da + ti - 1) / ti + ((pl.square || pl.spec) ? 0 : (pl.db + ti - 1) / ti);
    }
    case SK_COL_FWD:
    case SK_COL_INV: {
      const int64_t S = pl.col[pass].S;
      const int64_t nn = (int64_t)1 << pl.col[pass].logn;
      const int64_t cols = ((pl.square || pl.spec) && kind == SK_COL_FWD) ? pl.K : 2 * pl.K;
      return (S / pl.col_tile[pass]) * (L / (nn * S)) * pl.np * cols;
    }
    case SK_CONVOLVE:
      return (int64_t)pl.np * (L >> pl.logL1);
    default: {
      const int64_t ti = (int64_t)1 << pl.log_ti_out;
      return (pl.nout + ti - 1) / ti;
    }
  }
}

// Compiled kernel a stage's tiles run in (tiles of one level with the same kind and
// variant share a launch).
static int stage_variant(const Plan &pl, int kind, int pass) {
  if (kind == SK_CONVERT || kind == SK_RECOVER) return pl.np;
  int lk = 0;
  while ((1 << lk) < pl.K) ++lk;
  if (kind == SK_CONVOLVE && pl.conv_reg) {
    // squares and products with resident spectra have register kernels of their own;
    // so has the full inner factor
    return lk + (pl.spec ? 128 : pl.square ? 16 : 0) + (fixed_reg_l1(lk, pl.logL1) ? 32 : 0);
  }
  if (kind == SK_CONVOLVE) return fixed_lds_kl1(lk, pl.logL1) ? 64 + lk : 0;
  if (kind == SK_COL_FWD || kind == SK_COL_INV) {
    int lt = 0;
    while ((1 << lt) < pl.col_tile[pass]) ++lt;
    return fixed_col_index(pl.col[pass].logn, lt);
  }
  return 0;
}

// Host part of a batch: plans, job descriptors (X holds the workspace offset in words
// until the buffer exists), grouped launches in level order.  No device work.
int Ctx::schedule_batch(const zpm_job *jobs, int64_t n, int32_t K_force, BatchHost &bh,
                        const Plan *given, int32_t T_force, const uint32_t *const *specs) {
  int rc;
  bh = BatchHost();
  std::vector<Plan> &pls = bh.plans;
  pls.assign((size_t)n, Plan());
  std::vector<char> live((size_t)n, 0);
  int maxlev = 0;
  for (int64_t i = 0; i < n; ++i) {
    const zpm_job &j = jobs[i];
    if (j.da < 0 || j.db < 0 || j.Na < 1 || j.Nb < 1) return ZPM_EINVAL;
    if (j.da == 0 || j.db == 0) continue;
    if (j.wc < (out_bits(j.da, j.Na, j.db, j.Nb) + 63) / 64) return ZPM_EINVAL;
    const bool sp = specs && specs[i];
    if (sp && !given) return ZPM_EINVAL;   // resident spectra come with their operand's plan
    if (given) {
      if (!batch_supports(given[i])) return ZPM_EUNSUPPORTED;
      pls[i] = given[i];
    } else if ((rc = get_plan_batch(j.da, j.Na, j.db, j.Nb, K_force, T_force, &pls[i])) != ZPM_OK) {
      return rc;
    }
    // one operand passed twice is transformed once; resident spectra are not transformed
    pls[i].spec = sp ? 1 : 0;
    pls[i].square = (!sp && j.a && j.a == j.b && j.da == j.db && j.Na == j.Nb) ? 1 : 0;
    live[i] = 1;
    const Plan &pl = pls[i];
    bh.npmax = std::max(bh.npmax, pl.np);
    bh.H = std::max<int64_t>(bh.H, std::max<int64_t>((int64_t)1 << pl.logL, 2 * (int64_t)pl.K));
    bh.TP = std::max<int64_t>(bh.TP, (pl.M + 31) / 32 + 1);
    maxlev = std::max(maxlev, 3 + 2 * pl.ncol);
  }
  std::vector<int32_t> slot((size_t)n, -1);
  int64_t off = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!live[i]) continue;
    const Plan &pl = pls[i];
    JobDev jd;
    std::memset(&jd, 0, sizeof(jd));
    jd.a = jobs[i].a; jd.b = jobs[i].b; jd.c = jobs[i].c;
    jd.spec = pl.spec ? specs[i] : nullptr;
    jd.X = reinterpret_cast<uint32_t *>((uintptr_t)off);
    off += align_up(pl.ws_words, 64);
    jd.da = pl.da; jd.db = pl.db; jd.nout = pl.nout; jd.L = (int64_t)1 << pl.logL;
    jd.tiles_a = (pl.da + (1 << pl.log_ti_in) - 1) >> pl.log_ti_in;   // b's tiles follow
    for (int c = 0; c < pl.ncol; ++c) {
      jd.col_S[c] = pl.col[c].S;
      jd.col_logn[c] = pl.col[c].logn;
      int lt = 0;
      while ((1 << lt) < pl.col_tile[c]) ++lt;
      jd.col_logT[c] = lt;
    }
    jd.Na = pl.Na; jd.Nb = pl.Nb; jd.wc = jobs[i].wc; jd.K = pl.K; jd.M = pl.M; jd.np = pl.np;
    jd.logL = pl.logL; jd.logL1 = pl.logL1; jd.ncol = pl.ncol; jd.conv_reg = pl.conv_reg;
    jd.log_ti_in = pl.log_ti_in; jd.log_ti_out = pl.log_ti_out;
    jd.nw32 = 2 * ((pl.nout_bits + 63) / 64);
    jd.square = pl.square;
    slot[i] = (int32_t)bh.jobs.size();
    bh.jobs.push_back(jd);
    bh.job_plan.push_back((int32_t)i);
  }
  bh.ws_words = off;
  // groups: per level, one launch per (stage kind, compiled variant)
  for (int lev = 0; lev < maxlev; ++lev) {
    std::map<std::pair<int, int>, std::vector<GroupSeg>> by;
    std::map<std::pair<int, int>, size_t> lds;
    for (int64_t i = 0; i < n; ++i) {
      if (!live[i]) continue;
      const Plan &pl = pls[i];
      if (lev >= 3 + 2 * pl.ncol) continue;
      int kind, pass;
      stage_of(pl, lev, &kind, &pass);
      const auto key = std::make_pair(kind, stage_variant(pl, kind, pass));
      GroupSeg g;
      std::memset(&g, 0, sizeof(g));
      g.ntiles = stage_tiles(pl, kind, pass);
      g.job = slot[i];
      g.pass = pass;
      by[key].push_back(g);
      lds[key] = std::max(lds[key], stage_lds(pl, kind, pass));
    }
    for (auto &kv : by) {
      Group gr;
      std::memset(&gr, 0, sizeof(gr));
      gr.level = lev;
      gr.kind = kv.first.first;
      gr.variant = kv.first.second;
      gr.seg0 = (int64_t)bh.segs.size();
      gr.nseg = (int32_t)kv.second.size();
      int64_t start = 0;
      for (GroupSeg g : kv.second) {
        g.start = start;
        start += g.ntiles;
        bh.segs.push_back(g);
      }
      gr.blocks = start;
      gr.lds = lds[kv.first];
      bh.groups.push_back(gr);
    }
  }
  return ZPM_OK;
}

int Ctx::build_batch(const zpm_job *jobs, int64_t n, int32_t K_force, BatchState &bs,
                     const Plan *given, uint32_t *ws_ext, int64_t ws_ext_words, int32_t T_force,
                     const uint32_t *const *specs) {
  int rc;
  // the previous upload from the pinned buffers must be done before they are rewritten
  if (bs.upload_done) (void)hipEventSynchronize(bs.upload_done);
  for (int64_t i = 0; i < n; ++i)
    if (jobs[i].da > 0 && jobs[i].db > 0 && (!jobs[i].a || !jobs[i].b || !jobs[i].c))
      return ZPM_EINVAL;
  BatchHost &bh = bs.host;
  if ((rc = schedule_batch(jobs, n, K_force, bh, given, T_force, specs)) != ZPM_OK) return rc;
  const int64_t nlive = (int64_t)bh.jobs.size();
  if ((rc = ensure_tables(bh.npmax, bh.H, bh.TP)) != ZPM_OK) return rc;
  uint32_t *base = ws_ext;
  if (ws_ext) {
    if (bh.ws_words > ws_ext_words) return ZPM_EINVAL;
  } else {
    if ((rc = grow_dev(&bs.ws, &bs.ws_cap, std::max<int64_t>(bh.ws_words, 1))) != ZPM_OK) return rc;
    base = bs.ws;
  }
  if ((rc = grow_host(&bs.jobs_h, &bs.jobs_hcap, std::max<int64_t>(nlive, 1))) != ZPM_OK) return rc;
  for (int64_t s = 0; s < nlive; ++s) {
    JobDev jd = bh.jobs[s];
    PlanDev *pd = nullptr;
    if ((rc = plan_consts(bh.plans[bh.job_plan[s]], &pd)) != ZPM_OK) return rc;
    jd.plan = pd;
    jd.X = base + (int64_t)reinterpret_cast<uintptr_t>(jd.X);
    bs.jobs_h[s] = jd;
  }
  const int64_t nseg = (int64_t)bh.segs.size();
  if ((rc = grow_host(&bs.segs_h, &bs.segs_hcap, std::max<int64_t>(nseg, 1))) != ZPM_OK) return rc;
  if (nseg) std::memcpy(bs.segs_h, bh.segs.data(), sizeof(GroupSeg) * (size_t)nseg);
  if ((rc = grow_dev(&bs.jobs_d, &bs.jobs_dcap, std::max<int64_t>(nlive, 1))) != ZPM_OK) return rc;
  if ((rc = grow_dev(&bs.segs_d, &bs.segs_dcap, std::max<int64_t>(nseg, 1))) != ZPM_OK) return rc;
  bs.nseg = (int32_t)nseg;
  bs.nlive = nlive;
  return ZPM_OK;
}

int Ctx::enqueue_batch(BatchState &bs, hipStream_t st) {
  if (bs.host.groups.empty()) return ZPM_OK;
  if (hipMemcpyAsync(bs.jobs_d, bs.jobs_h, sizeof(JobDev) * (size_t)bs.nlive, hipMemcpyHostToDevice,
                     st) != hipSuccess)
    return ZPM_EDEVICE;
  if (hipMemcpyAsync(bs.segs_d, bs.segs_h, sizeof(GroupSeg) * (size_t)bs.nseg, hipMemcpyHostToDevice,
                     st) != hipSuccess)
    return ZPM_EDEVICE;
  prof.begin(KK_BATCH, st);
  for (const Group &gr : bs.host.groups) {
    if (launch_group(gr, bs.jobs_d, bs.segs_d, primes, st) != hipSuccess) {
      prof.end(st);
      return ZPM_EDEVICE;
    }
  }
  prof.end(st);
  return ZPM_OK;
}

int Ctx::enqueue_persistent(BatchState &bs, hipStream_t st) {
  int rc;
  const BatchHost &bh = bs.host;
  if (bh.groups.empty()) return ZPM_OK;
  const int64_t ng = (int64_t)bh.groups.size();
  const int64_t nslots = bs.nlive * PERSIST_LEVELS;
  if (!ncu && hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return ZPM_EDEVICE;
  if ((rc = grow_host(&bs.groups_h, &bs.groups_hcap, ng)) != ZPM_OK) return rc;
  if ((rc = grow_host(&bs.gstart_h, &bs.gstart_hcap, ng + 1)) != ZPM_OK) return rc;
  if ((rc = grow_host(&bs.need_h, &bs.need_hcap, nslots)) != ZPM_OK) return rc;
  if ((rc = grow_dev(&bs.groups_d, &bs.groups_dcap, ng)) != ZPM_OK) return rc;
  if ((rc = grow_dev(&bs.gstart_d, &bs.gstart_dcap, ng + 1)) != ZPM_OK) return rc;
  if ((rc = grow_dev(&bs.need_d, &bs.need_dcap, nslots)) != ZPM_OK) return rc;
  if ((rc = grow_dev(&bs.done_d, &bs.done_dcap, nslots)) != ZPM_OK) return rc;
  if (!bs.ctl_d && hipMalloc(&bs.ctl_d, sizeof(PersistCtl)) != hipSuccess) return ZPM_ENOMEM;
  if (!bs.ctl_h && hipHostMalloc(&bs.ctl_h, sizeof(PersistCtl), hipHostMallocDefault) != hipSuccess)
    return ZPM_ENOMEM;
  // tasks in the order of the grouped launches (level by level); a stage's tiles are one
  // segment of one group
  int64_t t = 0;
  size_t lds = 0;
  std::memset(bs.need_h, 0, sizeof(uint32_t) * (size_t)nslots);
  for (int64_t g = 0; g < ng; ++g) {
    const Group &gr = bh.groups[g];
    bs.groups_h[g] = gr;
    bs.gstart_h[g] = t;
    t += gr.blocks;
    lds = std::max(lds, gr.lds);
    if (gr.level >= PERSIST_LEVELS) return ZPM_EINVAL;
    if ((gr.kind == SK_CONVERT || gr.kind == SK_RECOVER) && gr.variant > PERSIST_NP_MAX)
      return ZPM_EUNSUPPORTED;
    for (int32_t k = 0; k < gr.nseg; ++k) {
      const GroupSeg &sg = bh.segs[gr.seg0 + k];
      bs.need_h[(int64_t)sg.job * PERSIST_LEVELS + gr.level] = (uint32_t)sg.ntiles;
    }
  }
  bs.gstart_h[ng] = t;
  const int64_t ntasks = t;
  if (hipMemcpyAsync(bs.jobs_d, bs.jobs_h, sizeof(JobDev) * (size_t)bs.nlive, hipMemcpyHostToDevice,
                     st) != hipSuccess ||
      hipMemcpyAsync(bs.segs_d, bs.segs_h, sizeof(GroupSeg) * (size_t)bs.nseg, hipMemcpyHostToDevice,
                     st) != hipSuccess ||
      hipMemcpyAsync(bs.groups_d, bs.groups_h, sizeof(Group) * (size_t)ng, hipMemcpyHostToDevice,
                     st) != hipSuccess ||
      hipMemcpyAsync(bs.gstart_d, bs.gstart_h, sizeof(int64_t) * (size_t)(ng + 1),
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(bs.need_d, bs.need_h, sizeof(uint32_t) * (size_t)nslots, hipMemcpyHostToDevice,
                     st) != hipSuccess)
    return ZPM_EDEVICE;
  prof.begin(KK_BATCH, st);
  const hipError_t e = launch_persistent(bs.jobs_d, bs.segs_d, bs.groups_d, bs.gstart_d, (int32_t)ng,
                                         ntasks, bs.need_d, bs.done_d, nslots, bs.ctl_d, primes, lds,
                                         1u << 20, ncu, st);
  prof.end(st);
  if (e != hipSuccess) return ZPM_EDEVICE;
  bs.ctl_h->abort = 0;
  if (hipMemcpyAsync(bs.ctl_h, bs.ctl_d, sizeof(PersistCtl), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return ZPM_EDEVICE;
  return bs.ctl_h->abort ? ZPM_EDEVICE : ZPM_OK;
}

int Ctx::mul_batch(const zpm_job *jobs, int64_t n, int32_t flags, int32_t K_force, hipStream_t st,
                   int32_t T_force, const Plan *given, const uint32_t *const *specs) {
  int rc;
  if (flags & ZPM_BATCH_PERSISTENT) {
    for (int64_t i = 0; specs && i < n; ++i)
      if (specs[i]) return ZPM_ENOTIMPL;   // the persistent kernel has no resident-spectra mode
    BatchState &bs = batch_eager;
    if (!bs.upload_done &&
        hipEventCreateWithFlags(&bs.upload_done, hipEventDisableTiming) != hipSuccess)
      return ZPM_EDEVICE;
    if ((rc = build_batch(jobs, n, K_force, bs, given, nullptr, 0, T_force)) != ZPM_OK) return rc;
    rc = enqueue_persistent(bs, st);
    if (hipEventRecord(bs.upload_done, st) != hipSuccess && rc == ZPM_OK) rc = ZPM_EDEVICE;
    return rc;
  }
  const bool graph = (flags & ZPM_BATCH_GRAPH) != 0;
  BatchState &bs = graph ? batch_graph : batch_eager;
  if (!bs.upload_done && hipEventCreateWithFlags(&bs.upload_done, hipEventDisableTiming) != hipSuccess)
    return ZPM_EDEVICE;
  if (graph) {
    // every launch of the graph is followed by upload_done on the caller's stream: the
    // graph reads the pinned descriptors (its copy nodes), the device descriptors and
    // the workspace until then, so none of them is rewritten, freed or destroyed before
    const uint64_t h = BatchState::hash(jobs, n, K_force, T_force, specs, given);
    if (bs.exec && bs.key == h) {
      prof.begin(KK_BATCH, st);
      const hipError_t e = hipGraphLaunch(bs.exec, st);
      prof.end(st);
      if (e != hipSuccess || hipEventRecord(bs.upload_done, st) != hipSuccess) return ZPM_EDEVICE;
      return ZPM_OK;
    }
    if (bs.exec) {
      if (hipEventSynchronize(bs.upload_done) != hipSuccess) return ZPM_EDEVICE;
      (void)hipGraphExecDestroy(bs.exec);
      bs.exec = nullptr;
    }
    if ((rc = build_batch(jobs, n, K_force, bs, given, nullptr, 0, T_force, specs)) != ZPM_OK)
      return rc;
    if (bs.host.groups.empty()) return ZPM_OK;
    // capture on a stream of our own (the caller's may be the legacy default stream,
    // which cannot be captured); the graph is then launched on the caller's stream
    if (!capture_stream &&
        hipStreamCreateWithFlags(&capture_stream, hipStreamNonBlocking) != hipSuccess)
      return ZPM_EDEVICE;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return ZPM_EDEVICE;
    const bool was_on = prof.on;
    prof.on = false;   // no event records inside the graph
    rc = enqueue_batch(bs, capture_stream);
    prof.on = was_on;
    if (hipStreamEndCapture(capture_stream, &g) != hipSuccess || rc != ZPM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc != ZPM_OK ? rc : ZPM_EDEVICE;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      return ZPM_EDEVICE;
    }
    (void)hipGraphDestroy(g);
    bs.exec = ex;
    bs.key = h;
    prof.begin(KK_BATCH, st);
    const hipError_t e = hipGraphLaunch(bs.exec, st);
    prof.end(st);
    if (e != hipSuccess || hipEventRecord(bs.upload_done, st) != hipSuccess) return ZPM_EDEVICE;
    return ZPM_OK;
  }
  if ((rc = build_batch(jobs, n, K_force, bs, given, nullptr, 0, T_force, specs)) != ZPM_OK) return rc;
  rc = enqueue_batch(bs, st);
  // recorded even after a failed enqueue: what was enqueued may still read the buffers
  if (hipEventRecord(bs.upload_done, st) != hipSuccess && rc == ZPM_OK) rc = ZPM_EDEVICE;
  return rc;
}

int Ctx::reserve_batch(BatchState &bs, int64_t jobs, int64_t segs) {
  int rc;
  if ((rc = grow_host(&bs.jobs_h, &bs.jobs_hcap, jobs)) != ZPM_OK) return rc;
  if ((rc = grow_host(&bs.segs_h, &bs.segs_hcap, segs)) != ZPM_OK) return rc;
  if ((rc = grow_dev(&bs.jobs_d, &bs.jobs_dcap, jobs)) != ZPM_OK) return rc;
  return grow_dev(&bs.segs_d, &bs.segs_dcap, segs);
}

void BatchState::release() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (upload_done) (void)hipEventDestroy(upload_done);
  if (ws) (void)hipFree(ws);
  if (jobs_d) (void)hipFree(jobs_d);
  if (segs_d) (void)hipFree(segs_d);
  if (jobs_h) (void)hipHostFree(jobs_h);
  if (segs_h) (void)hipHostFree(segs_h);
  if (groups_d) (void)hipFree(groups_d);
  if (gstart_d) (void)hipFree(gstart_d);
  if (need_d) (void)hipFree(need_d);
  if (done_d) (void)hipFree(done_d);
  if (ctl_d) (void)hipFree(ctl_d);
  if (groups_h) (void)hipHostFree(groups_h);
  if (gstart_h) (void)hipHostFree(gstart_h);
  if (need_h) (void)hipHostFree(need_h);
  if (ctl_h) (void)hipHostFree(ctl_h);
  *this = BatchState();
}

}  // namespace zpm

// Host-only view of a batch schedule, for tests and tools.
extern "C" int zpm_batch_schedule(const zpm_job *jobs, int64_t n, int32_t K, int64_t *nlaunch,
                                  int64_t *out, int64_t cap) {
  if (n < 0 || (n > 0 && !jobs) || !nlaunch || K < 0 || (cap > 0 && !out)) return ZPM_EINVAL;
  static zpm::Ctx host_ctx;   // plans only; never touches a device
  std::lock_guard<std::mutex> lock(host_ctx.mu);
  zpm::BatchHost bh;
  const int rc = host_ctx.schedule_batch(jobs, n, K, bh);
  if (rc != ZPM_OK) return rc;
  *nlaunch = (int64_t)bh.groups.size();
  for (int64_t g = 0; g < (int64_t)bh.groups.size() && g < cap; ++g) {
    const zpm::Group &gr = bh.groups[g];
    int64_t *o = out + 6 * g;
    o[0] = gr.level; o[1] = gr.kind; o[2] = gr.variant; o[3] = gr.nseg; o[4] = gr.blocks;
    o[5] = (int64_t)gr.lds;
  }
  return ZPM_OK;
}

extern "C" int zpm_mul_batch(zpm_ctx *ctx, const zpm_job *jobs, int64_t n, int32_t flags,
                             void *stream) {
  return zpm_mul_batch_ex(ctx, jobs, n, flags, 0, stream);
}

extern "C" int zpm_mul_batch_ex(zpm_ctx *ctx, const zpm_job *jobs, int64_t n, int32_t flags,
                                int32_t K, void *stream) {
  if (!ctx || n < 0 || (n > 0 && !jobs) || K < 0) return ZPM_EINVAL;
  if (flags != 0 && flags != ZPM_BATCH_GRAPH && flags != ZPM_BATCH_PERSISTENT) return ZPM_EINVAL;
  zpm::Ctx *cx = reinterpret_cast<zpm::Ctx *>(ctx);
  std::lock_guard<std::mutex> lock(cx->mu);
  if (hipSetDevice(cx->device) != hipSuccess) return ZPM_EDEVICE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (int64_t i = 0; cx->check_inputs && i < n; ++i) {
    const zpm_job &j = jobs[i];
    if (j.da <= 0 || j.db <= 0) continue;
    if (!j.a || !j.b || j.Na < 1 || j.Nb < 1) return ZPM_EINVAL;
    int rc = cx->check_range(j.a, j.da, j.Na, st);
    if (rc == ZPM_OK) rc = cx->check_range(j.b, j.db, j.Nb, st);
    if (rc != ZPM_OK) return rc;
  }
  return cx->mul_batch(jobs, n, flags, K, st);
}
