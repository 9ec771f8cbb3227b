// Library context: resident twiddle tables, per-plan constants, workspace.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>

#include "kernels.hpp"
#include "zpm_internal.hpp"

namespace zpm {

struct Ctx {
  int device = 0;
  PrimeDev *primes = nullptr;   // MAXNP entries
  uint2 *heaps = nullptr;       // np_built primes x (forward H, inverse H)
  int np_built = 0;
  int64_t H_built = 0;
  int64_t TP_built = 0;         // entries of each prime's 2^(32 t) table
  std::map<std::tuple<int, int, int, int>, PlanDev *> consts;
  std::map<std::tuple<int64_t, int32_t, int64_t, int32_t, int32_t, int32_t>, Plan> plans;
  uint32_t *ws = nullptr;
  int64_t ws_words = 0;
  std::mutex mu;
  Profiler prof;

  int ensure_tables(int np, int64_t H, int64_t TP);
  int plan_consts(const Plan &pl, PlanDev **out);
  int ensure_ws(int64_t words);
  int get_plan(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K, int32_t np, Plan *out);
  int prepare(const Plan &pl, DevState *ds);
  ~Ctx();
};

}  // namespace zpm
