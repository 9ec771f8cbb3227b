// Many independent products per launch: every stage of every product of a batch is a
// segment of one grouped launch per pipeline level, stage kind and compiled variant.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zpm_internal.hpp"

namespace zpm {

enum StageKind : int32_t {
  SK_CONVERT = 0,
  SK_COL_FWD = 1,
  SK_CONVOLVE = 2,
  SK_COL_INV = 3,
  SK_RECOVER = 4
};

// One product of a batch, with its plan, on the device.
struct JobDev {
  const uint64_t *a, *b;
  uint64_t *c;
  uint32_t *X;              // this product's workspace slice (np * 2K * L words)
  const PlanDev *plan;
  const uint32_t *spec;     // b's resident spectra (an operand's), or null
  int64_t da, db, nout, L;
  int64_t tiles_a;          // convert-in tiles of a; the following tiles convert b
  int64_t col_S[MAX_COL_PASSES];
  int32_t col_logn[MAX_COL_PASSES];
  int32_t col_logT[MAX_COL_PASSES];
  int32_t Na, Nb, wc, K, M, np, logL, logL1, ncol, conv_reg, log_ti_in, log_ti_out, nw32, square;
};

// A run of consecutive blocks of one grouped launch: all tiles of one stage of one
// product.  Block b of the launch belongs to the last segment with start <= b.
struct GroupSeg {
  int64_t start;
  int64_t ntiles;
  int32_t job, pass;
};

// One launch of a batch: a stage kind, its compiled variant (prime count for convert-in
// and recovery, log2 K for the register convolution, 0 otherwise) and its segments.
struct Group {
  int32_t level, kind, variant;
  int64_t seg0;      // first segment in the batch's segment array
  int32_t nseg;
  int64_t blocks;
  size_t lds;
};

hipError_t launch_group(const Group &gr, const JobDev *jobs, const GroupSeg *segs,
                        const PrimeDev *primes, hipStream_t st);

// Persistent launch: every tile of every group as one task list (see persistent.hip).
// done[job * PERSIST_LEVELS + level] counts the finished tiles of a product's stage, need[]
// holds how many there are.
constexpr int PERSIST_LEVELS = 3 + 2 * MAX_COL_PASSES;
struct PersistCtl {
  unsigned long long ticket;   // next task number
  uint32_t abort;              // set when a wait exceeded its bound
  uint32_t pad;
};
hipError_t launch_persistent(const JobDev *jobs, const GroupSeg *segs, const Group *groups,
                             const int64_t *gstart, int32_t ngroups, int64_t ntasks,
                             const uint32_t *need, uint32_t *done, int64_t nslots, PersistCtl *ctl,
                             const PrimeDev *primes, size_t lds, uint32_t spin_limit, int ncu,
                             hipStream_t st);
// LDS bytes a stage of a plan needs (same formulas as the per-stage launchers).
size_t stage_lds(const Plan &pl, int kind, int pass);
// Whether the batch kernels have code for this plan.  They take up to BATCH_NP_MAX
// primes (the batch planner itself stays within 16; larger counts come with resident
// operands planned for single products), the persistent kernel up to 16.
constexpr int BATCH_NP_MAX = 20;
constexpr int PERSIST_NP_MAX = 16;
bool batch_supports(const Plan &pl);

}  // namespace zpm
