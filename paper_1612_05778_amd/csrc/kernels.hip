// gfx950 kernels for exact Z[y] multiplication by two convolutions
// (cyclic mod x^K - 1 and negacyclic mod x^K + 1) over word-size Fourier primes.
//
// Workspace X, one buffer of np * 2K * L 32-bit residues, column-major:
//   column (k, j) of prime k is X[(k*2K + j) * L + i], i in [0, L)
//   columns j <  K : limb j of a   (A(x, y) of Section 2, y-index i)
//   columns j >= K : limb j-K of b (B(x, y))
// and, after the pointwise product, column j in [0, 2K) holds c_{i,j} mod p_k.
//
// Stages (each a kernel):
//   bivariate_representation : a, b -> limb residues        (Section 2, BivariateRepresentation)
//   col_fwd                  : outer factors of the y-NTT   (Section 3.3, K FFTs along y)
//   convolve_rows            : inner y factor, 2K-point x-transform whose first stage is the
//                              twist by theta^j (Section 2.1, NegacyclicConvolution) and whose
//                              even half is the cyclic transform (CyclicConvolution),
//                              pointwise product, inverses, untwist and (c- +- c+)/2
//   col_inv                  : outer factors of the inverse y-NTT
//   recovering_product       : CRT over the primes, evaluation at x = 2^M with carries
//                              (Section 2.2, RecoveringProduct)
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "kernels.hpp"

#include "stages.hpp"

namespace zpm {

// Smallest log2 K whose x-transforms run one K-point half at a time (below it the whole
// 2K-point transform fits in registers).  K = 32 is the largest register plan: for
// K = 64 the halves still need about 256 VGPRs and the LDS kernel is faster.
#ifndef ZPM_SPLIT_LOGK
#define ZPM_SPLIT_LOGK 5
#endif

static inline int64_t xcd_grid(int64_t ntiles) { return 8 * ((ntiles + 7) >> 3); }
// Products whose two conversions together take at most this many workgroups convert
// both operands in one launch.
constexpr int64_t CONVERT_PAIR_BLOCKS = 2048;

// Timing events for the next stage kernel this thread launches (set by launch_mul while
// the profiler records that kind): hipExtLaunchKernelGGL records them in the kernel's own
// dispatch, so timing a kernel adds no packets, and no gaps, between the kernels.
static thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;
#define ZPM_LAUNCH(KERN_, GRID_, BLK_, LDS_, ST_, ...)                                        \
  do {                                                                                     \
    if (t_ev_start) {                                                                      \
      hipExtLaunchKernelGGL(KERN_, GRID_, BLK_, (std::uint32_t)(LDS_), ST_, t_ev_start, t_ev_stop, \
                            0u, __VA_ARGS__);                                              \
      t_ev_start = t_ev_stop = nullptr;                                                    \
    } else {                                                                               \
      hipLaunchKernelGGL(KERN_, GRID_, BLK_, LDS_, ST_, __VA_ARGS__);                   \
    }                                                                                      \
  } while (0)
// the same with its arguments expanded first (for argument lists held in a macro)
#define ZPM_LAUNCH_X(...) ZPM_LAUNCH(__VA_ARGS__)

template <int NP>
__global__ __launch_bounds__(BLOCK) void k_bivariate_representation(
    const uint64_t *__restrict__ src, int64_t d, int32_t N, int32_t w, int32_t K, int32_t M,
    int32_t np, uint32_t *__restrict__ X, int64_t L, int32_t col_off, int32_t logTI,
    const PrimeDev *__restrict__ primes, const PlanDev *__restrict__ pd) {
  extern __shared__ uint32_t s[];
  body_convert_in<NP>(s, xcd_tile((d + (1 << logTI) - 1) >> logTI), src, d, N, w, K, M, np, X, L,
                      col_off, logTI, primes, pd);
}

// Both operands in one launch (small products, where a launch takes longer than the
// conversion): blocks below ga convert a into columns 0..K-1, the others b into columns
// K..2K-1.  ga is a multiple of 8, so b's blocks keep the XCD order of a launch of their own.
template <int NP>
__global__ __launch_bounds__(BLOCK) void k_bivariate_representation_pair(
    const uint64_t *__restrict__ a, int64_t da, int32_t Na, int32_t wa,
    const uint64_t *__restrict__ b, int64_t db, int32_t Nb, int32_t wb, int64_t ga, int32_t K,
    int32_t M, int32_t np, uint32_t *__restrict__ X, int64_t L, int32_t logTI,
    const PrimeDev *__restrict__ primes, const PlanDev *__restrict__ pd) {
  extern __shared__ uint32_t s[];
  const bool second = (int64_t)blockIdx.x >= ga;
  const int64_t bid = second ? (int64_t)blockIdx.x - ga : (int64_t)blockIdx.x;
  const int64_t d = second ? db : da;
  body_convert_in<NP>(s, xcd_tile_of(bid, (d + (1 << logTI) - 1) >> logTI), second ? b : a, d,
                      second ? Nb : Na, second ? wb : wa, K, M, np, X, L, second ? K : 0, logTI,
                      primes, pd);
}

// Neighbouring tiles of a column read the two halves of the same 128-byte lines when
// a tile is 16 columns wide: they are placed on one XCD, next to each other in its
// dispatch order, so that the second read hits that XCD's L2.
// CLOGN / CLOGT >= 0: a pass of 2^CLOGN points on tiles of 2^CLOGT columns, fixed at
// compile time; -1, -1: any pass.
template <int CLOGN, int CLOGT>
__global__ __launch_bounds__(BLOCK) void k_col_pass(
    uint32_t *__restrict__ X, int64_t L, int32_t twoK, int32_t logn, int64_t S, int32_t logT,
    int64_t nz_a, int64_t nz_b, int32_t K, int64_t nlimit, int32_t inverse,
    const PrimeDev *__restrict__ primes, int64_t nblocks, int32_t cols, int32_t col0) {
  extern __shared__ uint32_t s[];
  const int64_t bid = xcd_tile(nblocks);
  if (bid >= nblocks) return;
  body_col_pass<CLOGN, CLOGT>(s, bid, X, L, twoK, logn, S, logT, nz_a, nz_b, K, nlimit, inverse,
                              primes, cols, col0);
}

template <int CLOGK, int CLOGL1>
__global__ __launch_bounds__(BLOCK) void k_convolve_rows(
    uint32_t *__restrict__ X, int64_t L, int32_t K, int32_t logK, int32_t logL1, int64_t nz_a,
    int64_t nz_b, int64_t nlimit, const PrimeDev *__restrict__ primes,
    const PlanDev *__restrict__ pd, int32_t mode, const uint32_t *__restrict__ spec) {
  extern __shared__ uint32_t s[];
  body_convolve<CLOGK, CLOGL1>(s, blockIdx.x, X, L, K, logK, logL1, nz_a, nz_b, nlimit, primes, pd,
                               mode, spec);
}

// CLOGL1 >= 0: inner factor fixed at compile time (the largest that fits, 2^(12 - LOGK));
// -1: any.
template <int LOGK, int MODE, int CLOGL1>
__global__ __launch_bounds__(BLOCK) void k_convolve_rows_reg(
    uint32_t *__restrict__ X, int64_t L, int32_t logL1, int64_t nz_a, int64_t nz_b, int64_t nlimit,
    const PrimeDev *__restrict__ primes, const PlanDev *__restrict__ pd,
    const uint32_t *__restrict__ spec) {
  extern __shared__ uint32_t s[];
  body_convolve_reg<LOGK, MODE, CLOGL1>(s, blockIdx.x, X, L, logL1, nz_a, nz_b, nlimit, primes, pd,
                                        spec);
}

template <int LOGK, int MODE, int CLOGL1>
__global__ __launch_bounds__(BLOCK) void k_convolve_rows_split(
    uint32_t *__restrict__ X, int64_t L, int32_t logL1, int64_t nz_a, int64_t nz_b, int64_t nlimit,
    const PrimeDev *__restrict__ primes, const PlanDev *__restrict__ pd,
    const uint32_t *__restrict__ spec) {
  extern __shared__ uint32_t s[];
  body_convolve_split<LOGK, MODE, CLOGL1>(s, blockIdx.x, X, L, logL1, nz_a, nz_b, nlimit, primes,
                                          pd, spec);
}

template <int NP, int FORM>
__global__ __launch_bounds__(BLOCK) void k_recovering_product(
    const uint32_t *__restrict__ X, int64_t L, int32_t K, int32_t M, int64_t nout, int32_t nw32,
    int32_t wc, int32_t logTI, const PrimeDev *__restrict__ primes, const PlanDev *__restrict__ pd,
    uint64_t *__restrict__ out) {
  extern __shared__ uint64_t S[];
  body_recover<NP, FORM>(S, xcd_tile((nout + (1 << logTI) - 1) >> logTI), X, L, K, M, nout, nw32,
                         wc, logTI, primes, pd, out);
}

// Range check of the inputs (checked-input mode): in the top word of each coefficient the
// bits above bit N-1 must repeat it, i.e. -2^(N-1) <= a_i < 2^(N-1) (Relation
// (definingN)).  One thread per coefficient; any violation sets *flag.
__global__ __launch_bounds__(BLOCK) void k_check_range(const uint64_t *__restrict__ src, int64_t d,
                                                       int32_t w, int32_t tb, uint32_t *flag) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= d) return;
  const uint64_t top = src[i * w + (w - 1)];
  const int sh = 63 - tb;          // bits above bit tb of the top word
  const uint64_t ext = (uint64_t)((int64_t)(top << sh) >> sh);
  if (ext != top) atomicOr(flag, 1u);
}

// ------------------------------------------------------------------------------------
// host launchers
// ------------------------------------------------------------------------------------
static inline int ilog2(int64_t x) {
  int r = 0;
  while (((int64_t)1 << (r + 1)) <= x) ++r;
  return r;
}

#define ZPM_NP_CASES(X_) \
  X_(1) X_(2) X_(3) X_(4) X_(5) X_(6) X_(7) X_(8) X_(9) X_(10) X_(11) X_(12) X_(13) X_(14) \
  X_(15) X_(16) X_(17) X_(18) X_(19) X_(20) X_(21) X_(22) X_(23) X_(24) X_(26) X_(28) X_(30) \
  X_(32) X_(36) X_(40) X_(44) X_(48)

hipError_t launch_convert_in(const Plan &pl, const DevState &ds, const uint64_t *src, int64_t d,
                             int32_t N, int32_t col_off, hipStream_t st) {
  const int w = (N + 63) / 64;
  const int logTI = pl.log_ti_in;
  const int64_t blocks = xcd_grid((d + (1 << logTI) - 1) >> logTI);
  const int nchunks = (pl.M + 31) >> 5;
  const size_t lds = sizeof(uint32_t) * ((((size_t)1 << logTI) * (2 * w + 1) + 1) & ~(size_t)1) +
                     sizeof(uint2) * (size_t)nchunks * pl.np;
#define ZPM_CIN(NP_)                                                                          \
  case NP_:                                                                                   \
    ZPM_LAUNCH(k_bivariate_representation<NP_>, dim3((unsigned)blocks), dim3(BLOCK),  \
                       lds, st, src, d, N, w, pl.K, pl.M, pl.np, ds.X, (int64_t)1 << pl.logL,  \
                       col_off, logTI, ds.primes, ds.plan);                                   \
    break;
  switch (pl.np) {
    ZPM_NP_CASES(ZPM_CIN)
    default: return hipErrorInvalidValue;
  }
#undef ZPM_CIN
  return hipGetLastError();
}

hipError_t launch_convert_in_pair(const Plan &pl, const DevState &ds, const uint64_t *a,
                                  const uint64_t *b, hipStream_t st) {
  const int wa = (pl.Na + 63) / 64, wb = (pl.Nb + 63) / 64;
  const int logTI = pl.log_ti_in;
  const int64_t ga = xcd_grid((pl.da + (1 << logTI) - 1) >> logTI);
  const int64_t blocks = ga + xcd_grid((pl.db + (1 << logTI) - 1) >> logTI);
  const int nchunks = (pl.M + 31) >> 5;
  const size_t lds = sizeof(uint32_t) * ((((size_t)1 << logTI) * (2 * (wa > wb ? wa : wb) + 1) + 1) & ~(size_t)1) +
                     sizeof(uint2) * (size_t)nchunks * pl.np;
#define ZPM_CIN2(NP_)                                                                        \
  case NP_:                                                                                  \
    ZPM_LAUNCH(k_bivariate_representation_pair<NP_>, dim3((unsigned)blocks), dim3(BLOCK), lds, \
               st, a, pl.da, pl.Na, wa, b, pl.db, pl.Nb, wb, ga, pl.K, pl.M, pl.np, ds.X,        \
               (int64_t)1 << pl.logL, logTI, ds.primes, ds.plan);                              \
    break;
  switch (pl.np) {
    ZPM_NP_CASES(ZPM_CIN2)
    default: return hipErrorInvalidValue;
  }
#undef ZPM_CIN2
  return hipGetLastError();
}

hipError_t launch_col(const Plan &pl, const DevState &ds, int c, bool inverse, hipStream_t st,
                      int32_t fwd_cols, int32_t col0) {
  const int64_t L = (int64_t)1 << pl.logL;
  const int logn = pl.col[c].logn;
  const int64_t S = pl.col[c].S;
  const int T = pl.col_tile[c];
  if (T < 1 || T > BLOCK) return hipErrorInvalidValue;   // the kernel steps by BLOCK / T
  const int logT = ilog2(T);
  const int64_t tiles = (S >> logT) * (L / (((int64_t)1 << logn) * S));
  // forward passes of a square cover a's limbs only; fwd_cols / col0 select other sets
  const int32_t cols = inverse ? 2 * pl.K : (fwd_cols ? fwd_cols : (pl.square ? pl.K : 2 * pl.K));
  if (inverse) col0 = 0;
  const int64_t blocks = tiles * pl.np * cols;
  const size_t lds = sizeof(uint32_t) * ((size_t)T << logn);
  const int64_t nz_a = (c == 0 && !inverse) ? pl.da : L;
  const int64_t nz_b = (c == 0 && !inverse) ? pl.db : L;
  const int64_t nlimit = (c == 0 && inverse) ? pl.nout : L;
  const int64_t grid = 8 * ((blocks + 7) / 8);   // xcd_tile's shape
#define ZPM_COL_ARGS                                                                         \
  dim3((unsigned)grid), dim3(BLOCK), lds, st, ds.X, L, 2 * pl.K, logn, S, logT, nz_a, nz_b,   \
      pl.K, nlimit, inverse ? 1 : 0, ds.primes, blocks, cols, col0
  switch (fixed_col_index(logn, logT)) {
#define ZPM_COL_FIXED(I, LN, LT)                                                             \
  case I: ZPM_LAUNCH_X((k_col_pass<LN, LT>), ZPM_COL_ARGS); break;
    ZPM_COL_FIXED(1, 5, 6) ZPM_COL_FIXED(2, 6, 5) ZPM_COL_FIXED(3, 7, 4)
    ZPM_COL_FIXED(4, 8, 3) ZPM_COL_FIXED(5, 9, 3) ZPM_COL_FIXED(6, 10, 3)
    ZPM_COL_FIXED(7, 8, 4) ZPM_COL_FIXED(8, 9, 4) ZPM_COL_FIXED(9, 10, 4)
    ZPM_COL_FIXED(10, 1, 8) ZPM_COL_FIXED(11, 2, 8) ZPM_COL_FIXED(12, 3, 8)
    ZPM_COL_FIXED(13, 4, 7)
#undef ZPM_COL_FIXED
    default: ZPM_LAUNCH_X((k_col_pass<-1, -1>), ZPM_COL_ARGS); break;
  }
#undef ZPM_COL_ARGS
  return hipGetLastError();
}

hipError_t launch_convolve(const Plan &pl, const DevState &ds, hipStream_t st, int32_t mode,
                           const uint32_t *spec) {
  if (mode < 0) mode = pl.square ? CM_SQUARE : CM_PRODUCT;
  const int64_t L = (int64_t)1 << pl.logL;
  const int64_t blocks = (int64_t)pl.np * (L >> pl.logL1);
  const bool direct = pl.ncol == 0;
  const int64_t nz_a = direct ? pl.da : L, nz_b = direct ? pl.db : L, nl = direct ? pl.nout : L;
  if (pl.conv_reg) {
    const size_t lds = sizeof(uint32_t) * (size_t)(2 * pl.K) * (((size_t)1 << pl.logL1) + 1);
    // the planner's inner factor for long products is the largest whose 2K rows fit:
    // 2K (L1 + 1) <= LDS_WORDS, i.e. L1 = 2^(12 - log2 K)
    const bool full_l1 = fixed_reg_l1(ilog2(pl.K), pl.logL1);
#define ZPM_CONV_LAUNCH(KERN, LK_, M_, C_)                                                     \
  ZPM_LAUNCH((KERN<LK_, M_, C_>), dim3((unsigned)blocks), dim3(BLOCK), lds, st, ds.X, L, \
                     pl.logL1, nz_a, nz_b, nl, ds.primes, ds.plan, spec)
#define ZPM_CONV_M(LK_, M_)                                                                    \
  if constexpr (LK_ >= ZPM_SPLIT_LOGK) {                                                       \
    /* a fixed L1 raises this kernel to 192 VGPRs (two waves per SIMD instead of three) */     \
    ZPM_CONV_LAUNCH(k_convolve_rows_split, LK_, M_, -1);                                        \
  } else {                                                                                     \
    if (full_l1) ZPM_CONV_LAUNCH(k_convolve_rows_reg, LK_, M_, 12 - LK_);                       \
    else ZPM_CONV_LAUNCH(k_convolve_rows_reg, LK_, M_, -1);                                     \
  }
#define ZPM_CONV(LK_)                                        \
  switch (mode) {                                            \
    case CM_PRODUCT: ZPM_CONV_M(LK_, CM_PRODUCT); break;     \
    case CM_SQUARE: ZPM_CONV_M(LK_, CM_SQUARE); break;       \
    case CM_SPECTRUM: ZPM_CONV_M(LK_, CM_SPECTRUM); break;   \
    default: ZPM_CONV_M(LK_, CM_WITH_SPECTRUM); break;       \
  }
    switch (ilog2(pl.K)) {
      case 1: ZPM_CONV(1); break;
      case 2: ZPM_CONV(2); break;
      case 3: ZPM_CONV(3); break;
      case 4: ZPM_CONV(4); break;
      default: ZPM_CONV(5); break;
    }
#undef ZPM_CONV
#undef ZPM_CONV_M
#undef ZPM_CONV_LAUNCH
    return hipGetLastError();
  }
  const size_t lds = sizeof(uint32_t) * (size_t)4 * pl.K << pl.logL1;
  // K = 64, 128, 256 with the planner's inner factor (4 K L1 = LDS_WORDS / 2) fixed at
  // compile time
  const int lk = ilog2(pl.K);
#define ZPM_CONV_LDS(LK_, LL1_)                                                                \
  ZPM_LAUNCH((k_convolve_rows<LK_, LL1_>), dim3((unsigned)blocks), dim3(BLOCK), lds, st, \
                     ds.X, L, pl.K, lk, pl.logL1, nz_a, nz_b, nl, ds.primes, ds.plan, mode, spec)
  if (!fixed_lds_kl1(lk, pl.logL1)) ZPM_CONV_LDS(-1, -1);
  else if (lk == 6) ZPM_CONV_LDS(6, 5);
  else if (lk == 7) ZPM_CONV_LDS(7, 4);
  else ZPM_CONV_LDS(8, 3);
#undef ZPM_CONV_LDS
  return hipGetLastError();
}

hipError_t launch_recover(const Plan &pl, const DevState &ds, uint64_t *out, int32_t wc,
                          hipStream_t st) {
  const int64_t L = (int64_t)1 << pl.logL;
  const int nw32 = 2 * ((pl.nout_bits + 63) / 64);
  const int logTI = pl.log_ti_out;
  const int64_t blocks = xcd_grid((pl.nout + (1 << logTI) - 1) >> logTI);
  const size_t lds = recover_lds_bytes(pl.np, pl.K, pl.M, nw32, logTI);
  // the matrix form's staged and register variants are compiled apart, each with its own
  // register count
  const bool staged = recover_staged(pl.np, pl.K, pl.M, nw32, logTI);
#define ZPM_REC(NP_)                                                                           \
  case NP_:                                                                                    \
    if (staged)                                                                                \
      ZPM_LAUNCH((k_recovering_product<NP_, 1>), dim3((unsigned)blocks), dim3(BLOCK), lds, \
                         st, ds.X, L, pl.K, pl.M, pl.nout, nw32, wc, logTI, ds.primes, ds.plan, \
                         out);                                                                 \
    else                                                                                       \
      ZPM_LAUNCH((k_recovering_product<NP_, 0>), dim3((unsigned)blocks), dim3(BLOCK), lds, \
                         st, ds.X, L, pl.K, pl.M, pl.nout, nw32, wc, logTI, ds.primes, ds.plan, \
                         out);                                                                 \
    break;
  switch (pl.np) {
    ZPM_NP_CASES(ZPM_REC)
    default: return hipErrorInvalidValue;
  }
#undef ZPM_REC
  return hipGetLastError();
}

hipError_t launch_check_range(const uint64_t *src, int64_t d, int32_t N, uint32_t *flag,
                              hipStream_t st) {
  if (d <= 0) return hipSuccess;
  const int w = (N + 63) / 64;
  const int tb = (N - 1) & 63;
  if (tb == 63) return hipSuccess;   // N fills the top word: nothing above bit N-1
  const int64_t blocks = (d + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL(k_check_range, dim3((unsigned)blocks), dim3(BLOCK), 0, st, src, d, w, tb, flag);
  return hipGetLastError();
}

hipError_t launch_mul(const Plan &pl, const DevState &ds, const uint64_t *a, const uint64_t *b,
                      uint64_t *c, int32_t wc, int stop_after, hipStream_t st, Profiler *prof) {
  hipError_t e;
  Profiler dummy;
  Profiler &pr = prof ? *prof : dummy;
  // each stage is one kernel launch; a recorded kind gets the launch's own events
  auto timed = [&](int kind, auto &&launch) -> hipError_t {
    hipEvent_t ea = nullptr, eb = nullptr;
    if (!pr.take_pair(kind, &ea, &eb)) return launch();
    t_ev_start = ea;
    t_ev_stop = eb;
    const hipError_t r = launch();
    if (t_ev_start) {   // nothing was launched: the span is empty
      (void)hipEventRecord(ea, st);
      (void)hipEventRecord(eb, st);
      t_ev_start = t_ev_stop = nullptr;
    }
    return r;
  };
  // small products convert both operands in one launch (a square its one operand once)
  const int logTI = pl.log_ti_in;
  const bool pair = !pl.square && xcd_grid((pl.da + (1 << logTI) - 1) >> logTI) +
                                          xcd_grid((pl.db + (1 << logTI) - 1) >> logTI) <=
                                      CONVERT_PAIR_BLOCKS;
  if (pair) {
    e = timed(KK_CONVERT_IN, [&] { return launch_convert_in_pair(pl, ds, a, b, st); });
    if (e != hipSuccess) return e;
  } else {
    e = timed(KK_CONVERT_IN, [&] { return launch_convert_in(pl, ds, a, pl.da, pl.Na, 0, st); });
    if (e != hipSuccess) return e;
    if (!pl.square) {
      e = timed(KK_CONVERT_IN, [&] { return launch_convert_in(pl, ds, b, pl.db, pl.Nb, pl.K, st); });
      if (e != hipSuccess) return e;
    }
  }
  if (stop_after == 1) return hipSuccess;
  for (int cidx = 0; cidx < pl.ncol; ++cidx) {
    e = timed(KK_COL_FWD, [&] { return launch_col(pl, ds, cidx, false, st); });
    if (e != hipSuccess) return e;
  }
  if (stop_after == 2) return hipSuccess;
  e = timed(KK_CONVOLVE, [&] { return launch_convolve(pl, ds, st); });
  if (e != hipSuccess) return e;
  if (stop_after == 3) return hipSuccess;
  for (int cidx = pl.ncol - 1; cidx >= 0; --cidx) {
    e = timed(KK_COL_INV, [&] { return launch_col(pl, ds, cidx, true, st); });
    if (e != hipSuccess) return e;
  }
  if (stop_after == 4) return hipSuccess;
  return timed(KK_RECOVER, [&] { return launch_recover(pl, ds, c, wc, st); });
}

}  // namespace zpm
