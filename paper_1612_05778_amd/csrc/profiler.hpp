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
  KK_COUNT = 11
};

struct Profiler {
  bool on = false;
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
    if (!on) return;
    Rec r{kind, take(), take()};
    if (r.a && r.b) {
      (void)hipEventRecord(r.a, st);
      recs.push_back(r);
    }
  }
  void end(hipStream_t st) {
    if (!on || recs.empty()) return;
    (void)hipEventRecord(recs.back().b, st);
  }
  void reset() {
    recs.clear();
    used = 0;
  }
  ~Profiler() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace zpm
