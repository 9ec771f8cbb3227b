#pragma once
#include <stdint.h>

#include "zpm_internal.hpp"

namespace zpm {

int32_t out_bits(int64_t da, int32_t Na, int64_t db, int32_t Nb);
// K_force / np_force: 0 = choose; otherwise the plan must use that value.
bool make_plan(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K_force, int32_t np_force,
               Plan &out, const char **why);

}  // namespace zpm
