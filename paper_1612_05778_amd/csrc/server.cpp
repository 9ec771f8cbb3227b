// Continuous-batching server.
//
// A worker thread owns n_streams device streams and a workspace pool of a fixed number
// of bytes, allocated once.  Submitted products wait in one of two FIFO lanes (small
// and large, by output bits).  Whenever a stream is free the worker takes work from
// the head of a lane, admitting requests in order while their workspace fits in the
// largest free range of the pool.  Small requests form batches that run with the
// grouped batch kernels; a large request fills the device by itself and runs alone
// through the single-product path, so that its latency is its own; so do products
// the batch kernels do not cover and every request in single-product mode (the
// unbatched baseline).  Work on different streams overlaps on the device, and
// requests that arrive meanwhile wait for the next free stream.  Large requests may
// occupy at most large_streams streams (half of them by default): while large
// kernels fill the device, small kernels wait for free compute units, so the fewer
// large requests run at once, the shorter small requests' tail latency, at some cost
// in throughput.  While the device is busy, a small batch of fewer than min_batch
// requests is held until its oldest request has waited linger_s, so that arrivals
// coalesce into fewer, larger batches.  Twiddle tables and plan constants stay resident
// in the context, and requests against a resident operand (zpm_operand) take its
// spectra as they are: only their a is converted and transformed, in a batch beside
// ordinary requests or alone.
//
// The executor is an interface so that the admission and batching policy can also run
// against a simulated device (no computation, a modelled duration per batch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/zpm.h"
#include "batch.hpp"
#include "ctx.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace zpm {
namespace {

using Clock = std::chrono::steady_clock;

constexpr int32_t kMaxStreams = 16;
constexpr int32_t kMaxBatch = 4096;
constexpr int32_t kPending = 1;
constexpr size_t kMaxLatencySamples = size_t(1) << 22;

static int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

static double seconds(Clock::duration d) { return std::chrono::duration<double>(d).count(); }

struct SReq {
  uint64_t ticket = 0;
  zpm_job job;
  const zpm_operand *op = nullptr;   // resident b (job.b is then the operand's words)
  Plan plan;
  bool batch = true;       // planned for the batch kernels
  bool large = false;
  int64_t bytes = 0;       // workspace footprint in the pool
  double bits = 0;         // output bits, (da + db - 1) * out_bits
  Clock::time_point t0;    // submission
};

struct Flight {
  std::vector<SReq> reqs;
  int64_t off = 0, bytes = 0;
  bool large = false, batch = true;
  Clock::time_point t_launch;
  double sim_s = 0;
  bool sim_fail = false;
};

// First-fit allocator over byte offsets [0, size), with coalescing on release.
class FreeList {
 public:
  void init(int64_t size) {
    free_.clear();
    if (size > 0) free_[0] = size;
  }
  int64_t largest() const {
    int64_t m = 0;
    for (auto &kv : free_) m = std::max(m, kv.second);
    return m;
  }
  bool alloc(int64_t n, int64_t *off) {
    if (n == 0) { *off = 0; return true; }
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const int64_t rest = it->second - n, at = it->first + n;
      free_.erase(it);
      if (rest) free_[at] = rest;
      return true;
    }
    return false;
  }
  void release(int64_t off, int64_t n) {
    if (n == 0) return;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<int64_t, int64_t> free_;
};

class Exec {
 public:
  virtual ~Exec() = default;
  virtual int start(int nslots) = 0;                 // on the worker thread, before any launch
  virtual int launch(int slot, Flight &f) = 0;
  virtual int query(int slot, Flight &f) = 0;        // 1 running, 0 done, < 0 error
  virtual void finish() = 0;                         // on the worker thread, after the last query
};

class GpuExec final : public Exec {
 public:
  GpuExec(Ctx *cx, uint8_t *pool, int32_t max_batch) : cx_(cx), pool_(pool), max_batch_(max_batch) {}

  int start(int nslots) override {
    if (hipSetDevice(cx_->device) != hipSuccess) return ZPM_EDEVICE;
    st_.assign(nslots, nullptr);
    ev_.assign(nslots, nullptr);
    bs_.resize(nslots);
    for (int s = 0; s < nslots; ++s) {
      if (hipStreamCreateWithFlags(&st_[s], hipStreamNonBlocking) != hipSuccess) return ZPM_EDEVICE;
      if (hipEventCreateWithFlags(&ev_[s], hipEventDisableTiming) != hipSuccess) return ZPM_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(cx_->mu);
    for (int s = 0; s < nslots; ++s) {
      const int rc = cx_->reserve_batch(bs_[s], max_batch_, (int64_t)max_batch_ * (3 + 2 * MAX_COL_PASSES));
      if (rc != ZPM_OK) return rc;
    }
    // tables for every plan the batch kernels take up to y-length 2^17; larger
    // products grow them (with a device-wide wait) on first use
    return cx_->ensure_tables(16, (int64_t)1 << 17, 160);
  }

  int launch(int slot, Flight &f) override {
    std::lock_guard<std::mutex> lock(cx_->mu);
    int rc;
    hipStream_t st = st_[slot];
    uint32_t *ws = reinterpret_cast<uint32_t *>(pool_ + f.off);
    if (f.batch) {
      jobs_.clear();
      plans_.clear();
      specs_.clear();
      for (const SReq &r : f.reqs) {
        jobs_.push_back(r.job);
        plans_.push_back(r.plan);
        specs_.push_back(r.op ? r.op->spec : nullptr);
      }
      const bool was_on = cx_->prof.on;
      cx_->prof.on = false;
      rc = cx_->build_batch(jobs_.data(), (int64_t)jobs_.size(), 0, bs_[slot], plans_.data(), ws,
                            f.bytes / 4, 0, specs_.data());
      if (rc == ZPM_OK) rc = cx_->enqueue_batch(bs_[slot], st);
      cx_->prof.on = was_on;
      if (rc != ZPM_OK) return rc;
    } else {
      const SReq &r = f.reqs[0];
      const Plan &pl = r.plan;
      if (r.op) {   // the operand's tables were built when it was created
        rc = operand_product(*cx_, *r.op, pl, r.job.a, r.job.c, r.job.wc, ws, st);
        if (rc != ZPM_OK) return rc;
        return hipEventRecord(ev_[slot], st) == hipSuccess ? ZPM_OK : ZPM_EDEVICE;
      }
      const int64_t H = std::max<int64_t>((int64_t)1 << pl.logL, 2 * (int64_t)pl.K);
      if ((rc = cx_->ensure_tables(pl.np, H, (pl.M + 31) / 32 + 1)) != ZPM_OK) return rc;
      PlanDev *pd = nullptr;
      if ((rc = cx_->plan_consts(pl, &pd)) != ZPM_OK) return rc;
      DevState ds;
      ds.X = ws;
      ds.primes = cx_->primes;
      ds.plan = pd;
      if (launch_mul(pl, ds, r.job.a, r.job.b, r.job.c, r.job.wc, 0, st, nullptr) != hipSuccess)
        return ZPM_EDEVICE;
    }
    return hipEventRecord(ev_[slot], st) == hipSuccess ? ZPM_OK : ZPM_EDEVICE;
  }

  int query(int slot, Flight &) override {
    const hipError_t e = hipEventQuery(ev_[slot]);
    if (e == hipSuccess) return 0;
    if (e == hipErrorNotReady) return 1;
    return ZPM_EDEVICE;
  }

  void finish() override {
    for (hipStream_t s : st_)
      if (s) (void)hipStreamSynchronize(s);
    for (hipEvent_t e : ev_)
      if (e) (void)hipEventDestroy(e);
    for (hipStream_t s : st_)
      if (s) (void)hipStreamDestroy(s);
    for (BatchState &b : bs_) b.release();
    st_.clear();
    ev_.clear();
    bs_.clear();
  }

 private:
  Ctx *cx_;
  uint8_t *pool_;
  int32_t max_batch_;
  std::vector<hipStream_t> st_;
  std::vector<hipEvent_t> ev_;
  std::vector<BatchState> bs_;
  std::vector<zpm_job> jobs_;
  std::vector<Plan> plans_;
  std::vector<const uint32_t *> specs_;
};

// Simulated device: a batch takes overhead_s + (its output bits) / bits_per_s seconds
// of wall-clock time from its launch; nothing is computed or written.
class SimExec final : public Exec {
 public:
  SimExec(double bits_per_s, double overhead_s, int32_t fail_after)
      : rate_(bits_per_s), overhead_(overhead_s), fail_after_(fail_after) {}
  int start(int) override { return ZPM_OK; }
  int launch(int, Flight &f) override {
    double bits = 0;
    for (const SReq &r : f.reqs) bits += r.bits;
    f.t_launch = Clock::now();
    f.sim_s = overhead_ + bits / rate_;
    f.sim_fail = fail_after_ >= 0 && launches_ >= fail_after_;
    ++launches_;
    return ZPM_OK;
  }
  int query(int, Flight &f) override {
    if (seconds(Clock::now() - f.t_launch) < f.sim_s) return 1;
    return f.sim_fail ? ZPM_EDEVICE : 0;
  }
  void finish() override {}

 private:
  double rate_, overhead_;
  int32_t fail_after_;
  int64_t launches_ = 0;
};

}  // namespace

struct Server {
  struct Rec {
    int32_t state = kPending;
    double lat = 0;
  };

  Ctx *cx = nullptr;                  // null for a simulated server
  std::unique_ptr<Exec> ex;
  TuneTable tuned;                    // the context's tuned choices at creation
  zpm_server_config cfg;
  uint8_t *pool = nullptr;
  int64_t pool_bytes = 0;
  FreeList fl;                        // worker thread only

  std::mutex pm;                      // plan cache
  std::map<std::tuple<int64_t, int32_t, int64_t, int32_t>, std::pair<Plan, bool>> plan_cache;

  std::mutex m;                       // everything below
  std::condition_variable cv_work, cv_done;
  std::deque<SReq> lane[2];           // 0 small, 1 large
  uint64_t waited[2] = {0, 0};        // head ticket already counted as an admission wait
  std::unordered_map<uint64_t, Rec> recs;
  std::deque<uint64_t> done_order;
  uint64_t next_ticket = 1;
  bool stopping = false;
  int dead = ZPM_OK;

  // statistics since creation or the last reset
  uint64_t submitted = 0, completed = 0, failed = 0, rejected = 0, batches = 0, adm_waits = 0;
  uint64_t batch_reqs = 0;
  std::vector<double> lat;
  double bits_done = 0, lat_sum = 0, lat_max = 0;
  bool have_first = false, have_last = false;
  Clock::time_point t_first, t_last;
  int64_t hbm_in_use = 0, hbm_peak = 0, inflight = 0, inflight_peak = 0;

  std::thread worker;

  int plan_req(SReq &r);
  bool take(int ln, Flight &f);
  bool form(Flight &f, int busy_large, int busy_any);
  void retire(Flight &f, int status);
  void fail_queued(int status);
  void run();
};

int Server::plan_req(SReq &r) {
  const zpm_job &j = r.job;
  r.bits = (double)(j.da + j.db - 1) * (double)out_bits(j.da, j.Na, j.db, j.Nb);
  r.large = r.bits >= cfg.large_bits;
  if (r.op) {
    // the operand fixes K, M, np and L; small requests join batches when the batch
    // kernels cover that plan
    r.plan = operand_plan(*r.op, j.da, j.Na);
    r.batch = !cfg.single_product && !r.large && batch_supports(r.plan);
    r.bytes = align_up(r.plan.ws_words, 64) * 4;
    return ZPM_OK;
  }
  const auto key = std::make_tuple(j.da, j.Na, j.db, j.Nb);
  {
    std::lock_guard<std::mutex> lock(pm);
    auto it = plan_cache.find(key);
    if (it != plan_cache.end()) {
      r.plan = it->second.first;
      r.batch = it->second.second;
    } else {
      // small requests are batched; large ones (which fill the device by themselves)
      // and products beyond the batch kernels run alone with the single-product plan
      Plan pl;
      bool batch = !cfg.single_product && !r.large &&
                   plan_for_batch(tuned, j.da, j.Na, j.db, j.Nb, 0, 0, &pl) == ZPM_OK;
      if (!batch) {
        const char *why = nullptr;
        PlanLimits lim;
        lim.row_groups_min = ROW_GROUPS_MIN;
        if (!make_plan(j.da, j.Na, j.db, j.Nb, 0, 0, pl, &why, &lim)) return ZPM_EUNSUPPORTED;
      }
      if (plan_cache.size() > 65536) plan_cache.clear();
      plan_cache[key] = std::make_pair(pl, batch);
      r.plan = pl;
      r.batch = batch;
    }
  }
  r.plan.square = (j.a == j.b && j.da == j.db && j.Na == j.Nb) ? 1 : 0;
  r.bytes = align_up(r.plan.ws_words, 64) * 4;
  return ZPM_OK;
}

// Forms a batch from the head of lane ln (under m).  False when the lane is empty or
// its head does not fit in the largest free range of the pool.
bool Server::take(int ln, Flight &f) {
  std::deque<SReq> &q = lane[ln];
  if (q.empty()) return false;
  const int64_t avail = fl.largest();
  if (q.front().bytes > avail) {
    if (waited[ln] != q.front().ticket) {
      waited[ln] = q.front().ticket;
      ++adm_waits;
    }
    return false;
  }
  f.large = ln == 1;
  f.batch = q.front().batch;
  int64_t tot = 0;
  if (!f.batch) {
    tot = q.front().bytes;
    f.reqs.push_back(std::move(q.front()));
    q.pop_front();
  } else {
    while (!q.empty() && q.front().batch && (int32_t)f.reqs.size() < cfg.max_batch &&
           tot + q.front().bytes <= avail) {
      tot += q.front().bytes;
      f.reqs.push_back(std::move(q.front()));
      q.pop_front();
    }
  }
  if (!fl.alloc(tot, &f.off)) {   // cannot happen: tot <= largest free range
    for (auto it = f.reqs.rbegin(); it != f.reqs.rend(); ++it) q.push_front(std::move(*it));
    f.reqs.clear();
    return false;
  }
  f.bytes = tot;
  hbm_in_use += tot;
  hbm_peak = std::max(hbm_peak, hbm_in_use);
  inflight += (int64_t)f.reqs.size();
  inflight_peak = std::max(inflight_peak, inflight);
  ++batches;
  batch_reqs += f.reqs.size();
  return true;
}

// Picks the lane whose head arrived first among those allowed a stream (under m).  While
// other work occupies the device, a small batch of fewer than min_batch requests waits
// until its oldest request has waited linger_s, so that requests arriving meanwhile
// join it (an idle device takes whatever is queued at once).
bool Server::form(Flight &f, int busy_large, int busy_any) {
  const bool large_ok = !lane[1].empty() && busy_large < cfg.large_streams;
  bool small_ok = !lane[0].empty();
  if (small_ok && busy_any && (int32_t)lane[0].size() < cfg.min_batch &&
      seconds(Clock::now() - lane[0].front().t0) < cfg.linger_s)
    small_ok = false;
  int order[2] = {0, 1};
  if (large_ok && small_ok && lane[1].front().t0 < lane[0].front().t0) std::swap(order[0], order[1]);
  for (int ln : order) {
    if (ln == 1 && !large_ok) continue;
    if (ln == 0 && !small_ok) continue;
    if (take(ln, f)) return true;
  }
  return false;
}

void Server::retire(Flight &f, int status) {
  const Clock::time_point now = Clock::now();
  std::lock_guard<std::mutex> lock(m);
  for (const SReq &r : f.reqs) {
    Rec &rec = recs[r.ticket];
    rec.state = status;
    rec.lat = seconds(now - r.t0);
    done_order.push_back(r.ticket);
    if (status == ZPM_OK) {
      ++completed;
      bits_done += r.bits;
      lat_sum += rec.lat;
      lat_max = std::max(lat_max, rec.lat);
      if (lat.size() < kMaxLatencySamples) lat.push_back(rec.lat);
      t_last = now;
      have_last = true;
    } else {
      ++failed;
    }
  }
  fl.release(f.off, f.bytes);
  hbm_in_use -= f.bytes;
  inflight -= (int64_t)f.reqs.size();
  f.reqs.clear();
  cv_done.notify_all();
}

void Server::fail_queued(int status) {   // under m
  for (auto &q : lane) {
    for (const SReq &r : q) {
      Rec &rec = recs[r.ticket];
      rec.state = status;
      rec.lat = seconds(Clock::now() - r.t0);
      done_order.push_back(r.ticket);
      ++failed;
    }
    q.clear();
  }
  cv_done.notify_all();
}

void Server::run() {
  const int S = cfg.n_streams;
  int rc = ex->start(S);
  if (rc != ZPM_OK) {
    std::lock_guard<std::mutex> lock(m);
    dead = rc;
    fail_queued(rc);
  }
  std::vector<Flight> fls(S);
  std::vector<char> busy(S, 0);
  for (;;) {
    bool active = false;
    for (int s = 0; s < S; ++s) {
      if (!busy[s]) continue;
      const int q = ex->query(s, fls[s]);
      if (q == 1) {
        active = true;
        continue;
      }
      retire(fls[s], q);
      busy[s] = 0;
      if (q < 0) {
        std::lock_guard<std::mutex> lock(m);
        dead = q;
        fail_queued(q);
      }
    }
    for (;;) {
      int s = 0;
      while (s < S && busy[s]) ++s;
      if (s == S) break;
      int busy_large = 0, busy_any = 0;
      for (int t = 0; t < S; ++t) {
        busy_large += busy[t] && fls[t].large;
        busy_any += busy[t];
      }
      Flight f;
      {
        std::lock_guard<std::mutex> lock(m);
        if (dead != ZPM_OK || !form(f, busy_large, busy_any)) break;
      }
      const int lr = ex->launch(s, f);
      if (lr != ZPM_OK) {
        retire(f, lr);
        if (lr == ZPM_EDEVICE) {
          std::lock_guard<std::mutex> lock(m);
          dead = lr;
          fail_queued(lr);
        }
        continue;
      }
      fls[s] = std::move(f);
      busy[s] = 1;
      active = true;
    }
    std::unique_lock<std::mutex> lk(m);
    const bool queued = !lane[0].empty() || !lane[1].empty();
    if (!active) {
      if (stopping && !queued) break;
      // nothing on the device: a queued head always fits the empty pool (larger
      // requests are rejected at submission), so only an empty queue waits here
      if (!queued) cv_work.wait(lk, [&] { return stopping || !lane[0].empty() || !lane[1].empty(); });
      continue;
    }
    lk.unlock();
    std::this_thread::yield();
  }
  ex->finish();
}

static int check_job(const zpm_job &j) {
  if (j.da < 0 || j.db < 0 || j.Na < 1 || j.Nb < 1) return ZPM_EINVAL;
  if (j.da == 0 || j.db == 0) return ZPM_OK;
  if (!j.a || !j.b || !j.c) return ZPM_EINVAL;
  if (j.wc < (out_bits(j.da, j.Na, j.db, j.Nb) + 63) / 64) return ZPM_EINVAL;
  return ZPM_OK;
}

static int fill_config(const zpm_server_config *in, zpm_server_config *out) {
  zpm_server_config c;
  std::memset(&c, 0, sizeof(c));
  if (in) c = *in;
  if (c.n_streams == 0) c.n_streams = 4;
  if (c.min_batch == 0) c.min_batch = 4;
  if (c.linger_s == 0) c.linger_s = 150e-6;
  if (c.linger_s < 0) c.linger_s = 0;
  if (c.max_batch == 0) c.max_batch = kMaxBatch;
  if (c.large_bits == 0) c.large_bits = 67108864.0;
  if (c.large_streams == 0 && c.n_streams >= 1) c.large_streams = std::max(1, c.n_streams / 2);
  if (c.n_streams < 1 || c.n_streams > kMaxStreams || c.max_batch < 1 || c.max_batch > kMaxBatch ||
      !(c.large_bits > 0) || (c.single_product != 0 && c.single_product != 1) ||
      c.large_streams < 1 || c.large_streams > c.n_streams || c.min_batch < 1 ||
      !(c.linger_s <= 1.0))
    return ZPM_EINVAL;
  *out = c;
  return ZPM_OK;
}

}  // namespace zpm

using zpm::Server;

extern "C" int zpm_server_create_ex(zpm_ctx *ctx, const zpm_server_config *cfg, zpm_server **out) {
  if (!ctx || !out) return ZPM_EINVAL;
  *out = nullptr;
  std::unique_ptr<Server> sv(new Server());
  int rc = zpm::fill_config(cfg, &sv->cfg);
  if (rc != ZPM_OK) return rc;
  zpm::Ctx *cx = reinterpret_cast<zpm::Ctx *>(ctx);
  sv->cx = cx;
  {
    std::lock_guard<std::mutex> lock(cx->mu);
    sv->tuned = cx->tuned;
  }
  if (hipSetDevice(cx->device) != hipSuccess) return ZPM_EDEVICE;
  size_t budget = sv->cfg.hbm_budget;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return ZPM_EDEVICE;
    budget = fr / 2;
  }
  budget = budget / 256 * 256;
  if (budget < 256) return ZPM_EINVAL;
  if (hipMalloc(&sv->pool, budget) != hipSuccess) return ZPM_ENOMEM;
  sv->pool_bytes = (int64_t)budget;
  sv->cfg.hbm_budget = budget;
  sv->fl.init(sv->pool_bytes);
  sv->ex.reset(new zpm::GpuExec(cx, sv->pool, sv->cfg.max_batch));
  Server *raw = sv.get();
  sv->worker = std::thread([raw] { raw->run(); });
  *out = reinterpret_cast<zpm_server *>(sv.release());
  return ZPM_OK;
}

extern "C" int zpm_server_create(zpm_ctx *ctx, size_t hbm_budget, int32_t n_streams,
                                 zpm_server **out) {
  zpm_server_config c;
  std::memset(&c, 0, sizeof(c));
  c.hbm_budget = hbm_budget;
  c.n_streams = n_streams;
  return zpm_server_create_ex(ctx, &c, out);
}

extern "C" int zpm_server_create_simulated(const zpm_server_config *cfg, double bits_per_s,
                                           double overhead_s, int32_t fail_after, zpm_server **out) {
  if (!out || !cfg || cfg->hbm_budget < 256 || !(bits_per_s > 0) || !(overhead_s >= 0))
    return ZPM_EINVAL;
  *out = nullptr;
  std::unique_ptr<Server> sv(new Server());
  int rc = zpm::fill_config(cfg, &sv->cfg);
  if (rc != ZPM_OK) return rc;
  sv->pool_bytes = (int64_t)(cfg->hbm_budget / 256 * 256);
  sv->cfg.hbm_budget = (size_t)sv->pool_bytes;
  sv->fl.init(sv->pool_bytes);
  sv->ex.reset(new zpm::SimExec(bits_per_s, overhead_s, fail_after));
  Server *raw = sv.get();
  sv->worker = std::thread([raw] { raw->run(); });
  *out = reinterpret_cast<zpm_server *>(sv.release());
  return ZPM_OK;
}

namespace zpm {

// Plans and queues r (its job checked); the ticket goes to *ticket.
static int submit(Server *sv, SReq &r, uint64_t *ticket) {
  int rc;
  const zpm_job *job = &r.job;
  r.t0 = Clock::now();
  const bool empty = job->da == 0 || job->db == 0;
  if (!empty) {
    if ((rc = sv->plan_req(r)) != ZPM_OK) return rc;
  }
  std::lock_guard<std::mutex> lock(sv->m);
  if (sv->dead != ZPM_OK) return sv->dead;
  if (sv->stopping) return ZPM_EBUSY;
  if (!empty && r.bytes > sv->pool_bytes) {
    ++sv->rejected;
    return ZPM_ENOMEM;
  }
  r.ticket = sv->next_ticket++;
  *ticket = r.ticket;
  ++sv->submitted;
  if (!sv->have_first) {
    sv->t_first = r.t0;
    sv->have_first = true;
  }
  Server::Rec &rec = sv->recs[r.ticket];
  if (empty) {   // nothing to compute: finished at once
    rec.state = ZPM_OK;
    rec.lat = 0;
    sv->done_order.push_back(r.ticket);
    ++sv->completed;
    if (sv->lat.size() < zpm::kMaxLatencySamples) sv->lat.push_back(0.0);
    sv->cv_done.notify_all();
    return ZPM_OK;
  }
  sv->lane[r.large ? 1 : 0].push_back(std::move(r));
  sv->cv_work.notify_one();
  return ZPM_OK;
}

}  // namespace zpm

extern "C" int zpm_server_submit(zpm_server *srv, const zpm_job *job, uint64_t *ticket) {
  if (!srv || !job || !ticket) return ZPM_EINVAL;
  Server *sv = reinterpret_cast<Server *>(srv);
  int rc = zpm::check_job(*job);
  if (rc != ZPM_OK) return rc;
  zpm::SReq r;
  r.job = *job;
  return zpm::submit(sv, r, ticket);
}

extern "C" int zpm_server_submit_operand(zpm_server *srv, const zpm_operand_job *job,
                                         uint64_t *ticket) {
  if (!srv || !job || !ticket || !job->op) return ZPM_EINVAL;
  Server *sv = reinterpret_cast<Server *>(srv);
  const zpm_operand *op = job->op;
  if (!sv->cx || op->cx != sv->cx || job->da > op->da_max || job->Na > op->Na_max)
    return ZPM_EINVAL;
  zpm::SReq r;
  r.job.a = job->a;
  r.job.da = job->da;
  r.job.Na = job->Na;
  r.job.b = op->b;
  r.job.db = op->db;
  r.job.Nb = op->Nb;
  r.job.c = job->c;
  r.job.wc = job->wc;
  r.op = op;
  int rc = zpm::check_job(r.job);
  if (rc != ZPM_OK) return rc;
  if (job->da > 0) {   // c may overlap neither a nor the operand's words
    const uint64_t *c_end = job->c + (size_t)(job->da + op->db - 1) * job->wc;
    const uint64_t *a_end = job->a + (size_t)job->da * ((job->Na + 63) / 64);
    const uint64_t *b_end = op->b + (size_t)op->db * ((op->Nb + 63) / 64);
    if ((job->c < a_end && job->a < c_end) || (job->c < b_end && op->b < c_end)) return ZPM_EINVAL;
  }
  return zpm::submit(sv, r, ticket);
}

extern "C" int zpm_server_poll(zpm_server *srv, uint64_t ticket, int32_t *status, double *latency_s) {
  if (!srv || !status) return ZPM_EINVAL;
  Server *sv = reinterpret_cast<Server *>(srv);
  std::lock_guard<std::mutex> lock(sv->m);
  auto it = sv->recs.find(ticket);
  if (it == sv->recs.end()) return ZPM_ENOTFOUND;
  *status = it->second.state;
  if (latency_s) *latency_s = it->second.lat;
  if (it->second.state != zpm::kPending) sv->recs.erase(it);
  return ZPM_OK;
}

extern "C" int zpm_server_wait(zpm_server *srv, uint64_t ticket, double timeout_s, int32_t *status,
                               double *latency_s) {
  if (!srv || !status) return ZPM_EINVAL;
  Server *sv = reinterpret_cast<Server *>(srv);
  std::unique_lock<std::mutex> lk(sv->m);
  auto done = [&] {
    auto it = sv->recs.find(ticket);
    return it == sv->recs.end() || it->second.state != zpm::kPending;
  };
  if (timeout_s < 0) {
    sv->cv_done.wait(lk, done);
  } else {
    sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done);
  }
  auto it = sv->recs.find(ticket);
  if (it == sv->recs.end()) return ZPM_ENOTFOUND;
  *status = it->second.state;
  if (latency_s) *latency_s = it->second.lat;
  if (it->second.state == zpm::kPending) return ZPM_EBUSY;
  sv->recs.erase(it);
  return ZPM_OK;
}

extern "C" int zpm_server_completions(zpm_server *srv, uint64_t *tickets, int32_t *status,
                                      double *latency_s, int64_t cap, int64_t *n) {
  if (!srv || !n || cap < 0 || (cap > 0 && (!tickets || !status))) return ZPM_EINVAL;
  Server *sv = reinterpret_cast<Server *>(srv);
  std::lock_guard<std::mutex> lock(sv->m);
  int64_t k = 0;
  while (k < cap && !sv->done_order.empty()) {
    const uint64_t t = sv->done_order.front();
    sv->done_order.pop_front();
    auto it = sv->recs.find(t);
    if (it == sv->recs.end()) continue;   // already reported by poll or wait
    tickets[k] = t;
    status[k] = it->second.state;
    if (latency_s) latency_s[k] = it->second.lat;
    sv->recs.erase(it);
    ++k;
  }
  *n = k;
  return ZPM_OK;
}

extern "C" int zpm_server_stats(zpm_server *srv, zpm_server_report *out) {
  if (!srv || !out) return ZPM_EINVAL;
  Server *sv = reinterpret_cast<Server *>(srv);
  std::vector<double> l;
  std::memset(out, 0, sizeof(*out));
  {
    std::lock_guard<std::mutex> lock(sv->m);
    out->submitted = sv->submitted;
    out->completed = sv->completed;
    out->failed = sv->failed;
    out->rejected = sv->rejected;
    out->batches = sv->batches;
    out->admission_waits = sv->adm_waits;
    out->out_bits = sv->bits_done;
    out->max_s = sv->lat_max;
    out->mean_s = sv->completed ? sv->lat_sum / (double)sv->completed : 0;
    if (sv->have_first && sv->have_last) {
      const double span = zpm::seconds(sv->t_last - sv->t_first);
      out->bits_per_s = span > 0 ? sv->bits_done / span : 0;
    }
    out->hbm_budget = sv->pool_bytes;
    out->hbm_peak = sv->hbm_peak;
    out->hbm_in_use = sv->hbm_in_use;
    out->inflight = sv->inflight;
    out->inflight_peak = sv->inflight_peak;
    out->queued = (int64_t)(sv->lane[0].size() + sv->lane[1].size());
    out->mean_batch = sv->batches ? (double)sv->batch_reqs / (double)sv->batches : 0;
    l = sv->lat;
  }
  if (!l.empty()) {
    auto pct = [&](double q) {
      size_t k = (size_t)(q * (double)(l.size() - 1) + 0.5);
      std::nth_element(l.begin(), l.begin() + (std::ptrdiff_t)k, l.end());
      return l[k];
    };
    out->p50_s = pct(0.50);
    out->p99_s = pct(0.99);
  }
  return ZPM_OK;
}

extern "C" int zpm_server_reset_stats(zpm_server *srv) {
  if (!srv) return ZPM_EINVAL;
  Server *sv = reinterpret_cast<Server *>(srv);
  std::lock_guard<std::mutex> lock(sv->m);
  sv->submitted = sv->completed = sv->failed = sv->rejected = 0;
  sv->batches = sv->adm_waits = sv->batch_reqs = 0;
  sv->lat.clear();
  sv->bits_done = sv->lat_sum = sv->lat_max = 0;
  sv->have_first = sv->have_last = false;
  sv->hbm_peak = sv->hbm_in_use;
  sv->inflight_peak = sv->inflight;
  return ZPM_OK;
}

extern "C" void zpm_server_destroy(zpm_server *srv) {
  if (!srv) return;
  Server *sv = reinterpret_cast<Server *>(srv);
  {
    std::lock_guard<std::mutex> lock(sv->m);
    sv->stopping = true;
    sv->cv_work.notify_all();
  }
  if (sv->worker.joinable()) sv->worker.join();
  if (sv->pool) {
    (void)hipSetDevice(sv->cx->device);
    (void)hipFree(sv->pool);
  }
  delete sv;
}
