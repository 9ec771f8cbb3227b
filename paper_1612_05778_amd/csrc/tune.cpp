// Autotuner: choose the limb count K (and with it M and the prime count) and the
// column-tile width of the y passes per size class, by measuring batched throughput.
//
// The size class of a product is (ceil log2 of its length da + db - 1, ceil log2 of
// ceil(N / 32)).  For each class present in a sample the tuner takes the median
// product (by output bits), builds a batch of replicas of it, and times the batched
// path once per feasible (K, T): K <= 64 that the batch kernels support (at most 16
// primes) and column tiles T of 8, 16 and 32 inner indices, keeping the fastest.  The
// choice is stored in the context and, on request, in a JSON file that zpm_tune_load
// reads back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/zpm.h"
#include "ctx.hpp"
#include "plan.hpp"

namespace zpm {

static double product_bits(const zpm_job &j) {
  return (double)(j.da + j.db - 1) * out_bits(j.da, j.Na, j.db, j.Nb);
}

int Ctx::tune(const zpm_job *sample, int64_t n, hipStream_t st) {
  std::map<int32_t, std::vector<int64_t>> classes;
  for (int64_t i = 0; i < n; ++i) {
    const zpm_job &j = sample[i];
    if (j.da < 1 || j.db < 1 || j.Na < 1 || j.Nb < 1 || !j.a || !j.b) return ZPM_EINVAL;
    classes[size_class(j.da, j.Na, j.db, j.Nb)].push_back(i);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return ZPM_EDEVICE;
  uint64_t *scratch = nullptr;
  int64_t scratch_words = 0;
  int rc = ZPM_OK;
  for (auto &kv : classes) {
    std::vector<int64_t> &ids = kv.second;
    std::sort(ids.begin(), ids.end(), [&](int64_t x, int64_t y) {
      return product_bits(sample[x]) < product_bits(sample[y]);
    });
    zpm_job rep = sample[ids[ids.size() / 2]];
    const int32_t wc = (out_bits(rep.da, rep.Na, rep.db, rep.Nb) + 63) / 64;
    rep.wc = wc;
    const int64_t nout = rep.da + rep.db - 1;
    // replicas: enough work for a stable time, bounded memory
    const double bits = product_bits(rep);
    int64_t R = (int64_t)std::min(256.0, std::max(4.0, 5e8 / std::max(bits, 1.0)));
    R = std::min<int64_t>(R, std::max<int64_t>(8, (int64_t)(1 << 27) / std::max<int64_t>(nout * wc, 1)));
    const int64_t need = R * nout * wc;
    if (need > scratch_words) {
      if (scratch) {
        (void)hipDeviceSynchronize();
        (void)hipFree(scratch);
      }
      scratch = nullptr;
      if (hipMalloc(&scratch, sizeof(uint64_t) * (size_t)need) != hipSuccess) { rc = ZPM_ENOMEM; break; }
      scratch_words = need;
    }
    std::vector<zpm_job> reps((size_t)R, rep);
    for (int64_t r = 0; r < R; ++r) reps[r].c = scratch + r * nout * wc;
    float best_ms = 1e30f;
    TuneChoice best;
    for (int32_t K = 2; K <= 64 && rc == ZPM_OK; K *= 2) {
      int32_t last_tiles[MAX_COL_PASSES] = {-1, -1, -1, -1};
      for (int32_t T : {8, 16, 32}) {
        Plan pl;
        if (get_plan_batch(rep.da, rep.Na, rep.db, rep.Nb, K, T, &pl) != ZPM_OK) continue;
        // a tile wider than a pass allows gives the plan of a narrower one: skip repeats
        if (std::equal(pl.col_tile, pl.col_tile + MAX_COL_PASSES, last_tiles)) continue;
        std::copy(pl.col_tile, pl.col_tile + MAX_COL_PASSES, last_tiles);
        // first call captures the graph (and sizes tables and buffers); replays are timed
        if (mul_batch(reps.data(), R, ZPM_BATCH_GRAPH, K, st, T) != ZPM_OK) continue;
        float ms = 1e30f;
        for (int t = 0; t < 2; ++t) {
          (void)hipEventRecord(e0, st);
          if ((rc = mul_batch(reps.data(), R, ZPM_BATCH_GRAPH, K, st, T)) != ZPM_OK) break;
          (void)hipEventRecord(e1, st);
          if (hipEventSynchronize(e1) != hipSuccess) { rc = ZPM_EDEVICE; break; }
          float x = 0;
          (void)hipEventElapsedTime(&x, e0, e1);
          ms = std::min(ms, x);
        }
        if (rc != ZPM_OK) break;
        if (ms < best_ms) {
          best_ms = ms;
          best.K = K;
          best.T = T;
        }
      }
    }
    if (rc != ZPM_OK) break;
    if (best.K) tuned[kv.first] = best;
  }
  (void)hipStreamSynchronize(st);
  if (scratch) (void)hipFree(scratch);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // plans cached before tuning may carry the old K
  plans.clear();
  return rc;
}

static std::string device_name(int device) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
  return std::string(p.gcnArchName);
}

}  // namespace zpm

extern "C" int zpm_tune(zpm_ctx *ctx, const zpm_job *sample, int64_t n, const char *cache_path,
                        void *stream) {
  if (!ctx || n < 0 || (n > 0 && !sample)) return ZPM_EINVAL;
  zpm::Ctx *cx = reinterpret_cast<zpm::Ctx *>(ctx);
  std::lock_guard<std::mutex> lock(cx->mu);
  if (hipSetDevice(cx->device) != hipSuccess) return ZPM_EDEVICE;
  int rc = cx->tune(sample, n, reinterpret_cast<hipStream_t>(stream));
  if (rc != ZPM_OK || !cache_path) return rc;
  FILE *f = std::fopen(cache_path, "w");
  if (!f) return ZPM_EINVAL;
  std::fprintf(f, "{\n  \"device\": \"%s\",\n  \"version\": %d,\n  \"classes\": {",
               zpm::device_name(cx->device).c_str(), zpm_version());
  bool first = true;
  for (auto &kv : cx->tuned) {
    std::fprintf(f, "%s\n    \"%d\": [%d, %d]", first ? "" : ",", kv.first, kv.second.K,
                 kv.second.T);
    first = false;
  }
  std::fprintf(f, "\n  }\n}\n");
  std::fclose(f);
  return ZPM_OK;
}

extern "C" int zpm_tune_load(zpm_ctx *ctx, const char *cache_path) {
  if (!ctx || !cache_path) return ZPM_EINVAL;
  zpm::Ctx *cx = reinterpret_cast<zpm::Ctx *>(ctx);
  FILE *f = std::fopen(cache_path, "r");
  if (!f) return ZPM_EINVAL;
  std::string s;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, k);
  std::fclose(f);
  // minimal reader for the format written by zpm_tune:
  // "version": v, "classes": {"c": [K, T], ...}
  const size_t vpos = s.find("\"version\":");
  if (vpos == std::string::npos || std::atoi(s.c_str() + vpos + 10) != zpm_version()) return ZPM_EINVAL;
  const size_t cpos = s.find("\"classes\"");
  if (cpos == std::string::npos) return ZPM_EINVAL;
  std::lock_guard<std::mutex> lock(cx->mu);
  size_t p = s.find('{', cpos);
  zpm::TuneTable got;
  while (p != std::string::npos) {
    const size_t q1 = s.find('"', p + 1);
    if (q1 == std::string::npos) break;
    const size_t q2 = s.find('"', q1 + 1);
    if (q2 == std::string::npos) break;
    const size_t lb = s.find('[', q2), rb = s.find(']', q2);
    if (lb == std::string::npos || rb == std::string::npos || rb < lb) return ZPM_EINVAL;
    const int32_t cls = std::atoi(s.c_str() + q1 + 1);
    zpm::TuneChoice c;
    char *end = nullptr;
    c.K = (int32_t)std::strtol(s.c_str() + lb + 1, &end, 10);
    const size_t comma = s.find(',', lb);
    if (comma == std::string::npos || comma > rb) return ZPM_EINVAL;
    c.T = (int32_t)std::strtol(s.c_str() + comma + 1, &end, 10);
    const bool pow2 = c.K >= 2 && (c.K & (c.K - 1)) == 0 && c.T >= 1 && c.T <= 64 &&
                      (c.T & (c.T - 1)) == 0;
    if (!pow2) return ZPM_EINVAL;
    got[cls] = c;
    p = rb;
  }
  for (auto &kv : got) cx->tuned[kv.first] = kv.second;
  cx->plans.clear();
  return ZPM_OK;
}

extern "C" int zpm_tune_get(zpm_ctx *ctx, int32_t *classes, int32_t *ks, int32_t *tiles, int32_t cap,
                            int32_t *n) {
  if (!ctx || !n || (cap > 0 && (!classes || !ks))) return ZPM_EINVAL;
  zpm::Ctx *cx = reinterpret_cast<zpm::Ctx *>(ctx);
  std::lock_guard<std::mutex> lock(cx->mu);
  int32_t i = 0;
  for (auto &kv : cx->tuned) {
    if (i < cap) {
      classes[i] = kv.first;
      ks[i] = kv.second.K;
      if (tiles) tiles[i] = kv.second.T;
    }
    ++i;
  }
  *n = i;
  return ZPM_OK;
}
