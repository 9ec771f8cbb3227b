#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "profiler.hpp"
#include "zpm_internal.hpp"

namespace zpm {

// Column-pass shapes with a compile-time kernel: the planner's default tile for each pass
// length from 2^1 to 2^10 (log2 length, log2 tile), and 8-column tiles for the longer
// ones.  Index + 1, or 0 for any other shape.
constexpr int FIXED_COL[][2] = {{5, 6}, {6, 5}, {7, 4}, {8, 3}, {9, 3}, {10, 3},
                                 {8, 4}, {9, 4}, {10, 4}, {1, 8}, {2, 8}, {3, 8}, {4, 7}};
inline int fixed_col_index(int logn, int logT) {
  for (int i = 0; i < (int)(sizeof(FIXED_COL) / sizeof(FIXED_COL[0])); ++i)
    if (FIXED_COL[i][0] == logn && FIXED_COL[i][1] == logT) return i + 1;
  return 0;
}
// Register row kernels have a compile-time kernel for their full inner factor
// 2^(12 - log2 K); the LDS row kernel for K = 64, 128, 256 with 4 K L1 = 8192 words.
inline bool fixed_reg_l1(int logK, int logL1) { return logL1 == 12 - logK; }
inline bool fixed_lds_kl1(int logK, int logL1) { return logK >= 6 && logK <= 8 && logL1 == 11 - logK; }

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
// Sets *flag to 1 if some coefficient of src (d coefficients of N bits, ceil(N/64) words
// each) has a bit at or above N that differs from bit N-1.
hipError_t launch_check_range(const uint64_t *src, int64_t d, int32_t N, uint32_t *flag,
                              hipStream_t st);
// stop_after: 0 = everything; 1..4 = stop after convert-in / forward column passes /
// row convolutions / inverse column passes (the workspace then holds that stage).
hipError_t launch_mul(const Plan &pl, const DevState &ds, const uint64_t *a, const uint64_t *b,
                      uint64_t *c, int32_t wc, int stop_after, hipStream_t st,
                      Profiler *prof = nullptr);

// Looks up the device address of the no-allocation scratch array on `device` (the
// current device), once per device.
hipError_t noalloc_init(int device);

}  // namespace zpm
