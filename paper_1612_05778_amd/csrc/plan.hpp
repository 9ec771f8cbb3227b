#pragma once
#include <stdint.h>

#include "zpm_internal.hpp"

namespace zpm {

int32_t out_bits(int64_t da, int32_t Na, int64_t db, int32_t Nb);
struct PlanLimits {
  int32_t np_max = MAXNP;    // largest prime count
  int32_t k_max = 1 << 20;   // largest K
  int32_t reg_k_max = 32;    // largest K for the register x-transform kernels
  int32_t col_tile = 0;      // widest column tile (power of two); 0 = the default
  // products that run alone, K and np not forced: with the x-transforms in registers, at
  // most one column pass and an inner factor of 2^10 or more, shrink the inner factor
  // (adding or lengthening the column pass) until the fused row kernel has this many
  // workgroups; 0 = off
  int32_t row_groups_min = 0;
};

// The row-group floor of products that run alone (single products, the server's lone
// requests).  Batches and resident operands keep the cost model's plan: their row
// kernels share launches, and an extra column pass costs them more than it saves.
constexpr int32_t ROW_GROUPS_MIN = 128;

// K_force / np_force: 0 = choose; otherwise the plan must use that value.
bool make_plan(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K_force, int32_t np_force,
               Plan &out, const char **why, const PlanLimits *lim = nullptr);
// Class of a product for tuning: (ceil log2 of da + db - 1, ceil log2 of ceil(max N / 32)).
int32_t size_class(int64_t da, int32_t Na, int64_t db, int32_t Nb);

}  // namespace zpm
