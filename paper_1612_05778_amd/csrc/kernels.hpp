#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "profiler.hpp"
#include "zpm_internal.hpp"

namespace zpm {

// Device pointers a launch needs.
struct DevState {
  uint32_t *X;               // workspace, np * 2K * L words
  const PrimeDev *primes;    // MAXNP entries
  const PlanDev *plan;       // constants of this plan
};

hipError_t launch_convert_in(const Plan &pl, const DevState &ds, const uint64_t *src, int64_t d,
                             int32_t N, int32_t col_off, hipStream_t st);
// fwd_cols / col0: forward passes over fwd_cols columns per prime from col0 on
// (0: both operands', or a's alone for a square); inverse passes cover all 2K.
hipError_t launch_col(const Plan &pl, const DevState &ds, int c, bool inverse, hipStream_t st,
                      int32_t fwd_cols = 0, int32_t col0 = 0);
// mode: a ConvMode (-1: the product, or the square when pl.square); spec: b's spectra
// for CM_WITH_SPECTRUM.
hipError_t launch_convolve(const Plan &pl, const DevState &ds, hipStream_t st, int32_t mode = -1,
                           const uint32_t *spec = nullptr);
hipError_t launch_recover(const Plan &pl, const DevState &ds, uint64_t *out, int32_t wc,
                          hipStream_t st);
// stop_after: 0 = everything; 1..4 = stop after convert-in / forward column passes /
// row convolutions / inverse column passes (the workspace then holds that stage).
hipError_t launch_mul(const Plan &pl, const DevState &ds, const uint64_t *a, const uint64_t *b,
                      uint64_t *c, int32_t wc, int stop_after, hipStream_t st,
                      Profiler *prof = nullptr);

}  // namespace zpm
