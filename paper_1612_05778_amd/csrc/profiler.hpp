// Optional per-kernel timing with HIP events recorded on the launch stream.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

namespace zpm {

enum KernelKind {
  KK_CONVERT_IN = 0,
  KK_COL_FWD = 1,
  KK_CONVOLVE = 2,
  KK_COL_INV = 3,
  KK_RECOVER = 4,
  KK_BATCH = 5,
  KK_P64_CONVERT = 6,   // 64-bit prime variant
  KK_P64_YFWD = 7,
  KK_P64_X = 8,
  KK_P64_YINV = 9,
  KK_P64_RECOVER = 10,
  KK_GFP_CONVERT = 11,  // single generalized Fermat prime variant
  KK_GFP_YFWD = 12,
  KK_GFP_X = 13,
  KK_GFP_YINV = 14,
  KK_GFP_RECOVER = 15,
  KK_COUNT = 16
};

struct Profiler {
  bool on = false;
  uint32_t mask = ~0u;   // kinds recorded while on (bit k = KernelKind k)
  bool open = false;     // begin() recorded a start event that end() has not closed
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;

  hipEvent_t take() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  void begin(int kind, hipStream_t st) {
    open = false;
    if (!on || !((mask >> kind) & 1u)) return;
    Rec r{kind, take(), take()};
    if (r.a && r.b) {
      (void)hipEventRecord(r.a, st);
      recs.push_back(r);
      open = true;
    }
  }
  // A start/stop pair for a kind that is being recorded (false otherwise), for a launch
  // that records the events itself.
  bool take_pair(int kind, hipEvent_t *a, hipEvent_t *b) {
    if (!on || !((mask >> kind) & 1u)) return false;
    Rec r{kind, take(), take()};
    if (!r.a || !r.b) return false;
    recs.push_back(r);
    *a = r.a;
    *b = r.b;
    return true;
  }
  void end(hipStream_t st) {
    if (!on || !open) return;
    (void)hipEventRecord(recs.back().b, st);
    open = false;
  }
  void reset() {
    recs.clear();
    used = 0;
    open = false;
  }
  ~Profiler() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace zpm
