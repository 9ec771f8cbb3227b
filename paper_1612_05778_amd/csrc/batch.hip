// Batched products as grouped launches.
//
// Every stage of every product is cut into the same tiles the per-stage kernels use.
// A batch runs level by level (level s = the s-th stage of each product); within a
// level, tiles of the same stage kind and the same compiled variant (prime count or
// limb count) go into one launch, where block b finds its product and tile from a
// list of segments.  Launch order on the stream carries the dependencies between
// levels, so no workgroup ever waits for another.
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "stages.hpp"

namespace zpm {

__device__ __forceinline__ int find_seg(const GroupSeg *__restrict__ segs, int32_t nseg, int64_t b) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].start <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int NP>
__global__ __launch_bounds__(BLOCK) void kg_convert(const JobDev *__restrict__ jobs,
                                                    const GroupSeg *__restrict__ segs, int32_t nseg,
                                                    const PrimeDev *__restrict__ primes) {
  extern __shared__ uint32_t s[];
  const GroupSeg g = segs[find_seg(segs, nseg, blockIdx.x)];
  const JobDev &jb = jobs[g.job];
  const int64_t tile = (int64_t)blockIdx.x - g.start;
  // tiles of a first, then tiles of b (none for a square or a resident operand)
  const bool ob = tile >= jb.tiles_a;
  const int32_t N = ob ? jb.Nb : jb.Na;
  body_convert_in<NP>(s, ob ? tile - jb.tiles_a : tile, ob ? jb.b : jb.a, ob ? jb.db : jb.da, N,
                      (N + 63) / 64, jb.K, jb.M, NP, jb.X, jb.L, ob ? jb.K : 0, jb.log_ti_in,
                      primes, jb.plan);
}

template <int NP>
__global__ __launch_bounds__(BLOCK) void kg_recover(const JobDev *__restrict__ jobs,
                                                    const GroupSeg *__restrict__ segs, int32_t nseg,
                                                    const PrimeDev *__restrict__ primes) {
  extern __shared__ uint64_t S[];
  const GroupSeg g = segs[find_seg(segs, nseg, blockIdx.x)];
  const JobDev &jb = jobs[g.job];
  body_recover<NP>(S, (int64_t)blockIdx.x - g.start, jb.X, jb.L, jb.K, jb.M, jb.nout, jb.nw32,
                   jb.wc, jb.log_ti_out, primes, jb.plan, jb.c);
}

// Blocks are remapped with xcd_tile (as in the single-product column pass) so that
// neighbouring tiles, which share 128-byte lines, run on one XCD.
template <int CLOGN, int CLOGT>
__global__ __launch_bounds__(BLOCK) void kg_col(const JobDev *__restrict__ jobs,
                                                const GroupSeg *__restrict__ segs, int32_t nseg,
                                                int32_t inverse, const PrimeDev *__restrict__ primes,
                                                int64_t nblocks) {
  extern __shared__ uint32_t s[];
  const int64_t b = xcd_tile(nblocks);
  if (b >= nblocks) return;
  const GroupSeg g = segs[find_seg(segs, nseg, b)];
  const JobDev &jb = jobs[g.job];
  const int c = g.pass;
  const bool outer = c == 0;
  const int64_t L = jb.L;
  body_col_pass<CLOGN, CLOGT>(s, b - g.start, jb.X, L, 2 * jb.K, jb.col_logn[c], jb.col_S[c],
                jb.col_logT[c], (outer && !inverse) ? jb.da : L, (outer && !inverse) ? jb.db : L,
                jb.K, (outer && inverse) ? jb.nout : L, inverse, primes,
                ((jb.square || jb.spec) && !inverse) ? jb.K : 2 * jb.K, 0);
}

template <int LOGK, int MODE, int CLOGL1>
__global__ __launch_bounds__(BLOCK) void kg_convolve_reg(const JobDev *__restrict__ jobs,
                                                         const GroupSeg *__restrict__ segs,
                                                         int32_t nseg,
                                                         const PrimeDev *__restrict__ primes) {
  extern __shared__ uint32_t s[];
  const GroupSeg g = segs[find_seg(segs, nseg, blockIdx.x)];
  const JobDev &jb = jobs[g.job];
  const int64_t L = jb.L;
  const bool direct = jb.ncol == 0;
  body_convolve_reg<LOGK, MODE, CLOGL1>(s, (int64_t)blockIdx.x - g.start, jb.X, L, jb.logL1,
                                direct ? jb.da : L, direct ? jb.db : L, direct ? jb.nout : L,
                                primes, jb.plan, jb.spec);
}

template <int CLOGK, int CLOGL1>
__global__ __launch_bounds__(BLOCK) void kg_convolve(const JobDev *__restrict__ jobs,
                                                     const GroupSeg *__restrict__ segs, int32_t nseg,
                                                     const PrimeDev *__restrict__ primes) {
  extern __shared__ uint32_t s[];
  const GroupSeg g = segs[find_seg(segs, nseg, blockIdx.x)];
  const JobDev &jb = jobs[g.job];
  const int64_t L = jb.L;
  const bool direct = jb.ncol == 0;
  int logK = 0;
  while ((1 << logK) < jb.K) ++logK;
  body_convolve<CLOGK, CLOGL1>(s, (int64_t)blockIdx.x - g.start, jb.X, L, jb.K, logK, jb.logL1,
                direct ? jb.da : L, direct ? jb.db : L, direct ? jb.nout : L, primes, jb.plan,
                jb.spec ? CM_WITH_SPECTRUM : jb.square ? CM_SQUARE : CM_PRODUCT, jb.spec);
}

hipError_t launch_group(const Group &gr, const JobDev *jobs, const GroupSeg *segs,
                        const PrimeDev *primes, hipStream_t st) {
  if (gr.blocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)gr.blocks), blk(BLOCK);
  const GroupSeg *sg = segs + gr.seg0;
  const int32_t ns = gr.nseg;
  switch (gr.kind) {
    case SK_CONVERT:
      switch (gr.variant) {
#define ZPM_G(NP_) \
  case NP_: hipLaunchKernelGGL(kg_convert<NP_>, grid, blk, gr.lds, st, jobs, sg, ns, primes); break;
        ZPM_G(1) ZPM_G(2) ZPM_G(3) ZPM_G(4) ZPM_G(5) ZPM_G(6) ZPM_G(7) ZPM_G(8)
        ZPM_G(9) ZPM_G(10) ZPM_G(11) ZPM_G(12) ZPM_G(13) ZPM_G(14) ZPM_G(15) ZPM_G(16)
        ZPM_G(17) ZPM_G(18) ZPM_G(19) ZPM_G(20)
#undef ZPM_G
        default: return hipErrorInvalidValue;
      }
      break;
    case SK_RECOVER:
      switch (gr.variant) {
#define ZPM_G(NP_) \
  case NP_: hipLaunchKernelGGL(kg_recover<NP_>, grid, blk, gr.lds, st, jobs, sg, ns, primes); break;
        ZPM_G(1) ZPM_G(2) ZPM_G(3) ZPM_G(4) ZPM_G(5) ZPM_G(6) ZPM_G(7) ZPM_G(8)
        ZPM_G(9) ZPM_G(10) ZPM_G(11) ZPM_G(12) ZPM_G(13) ZPM_G(14) ZPM_G(15) ZPM_G(16)
        ZPM_G(17) ZPM_G(18) ZPM_G(19) ZPM_G(20)
#undef ZPM_G
        default: return hipErrorInvalidValue;
      }
      break;
    case SK_COL_FWD:
    case SK_COL_INV: {
      // variant: fixed_col_index of the pass shape (0: any shape)
      const dim3 g8((unsigned)(8 * ((gr.blocks + 7) / 8)));
      const int32_t inv = gr.kind == SK_COL_INV ? 1 : 0;
      switch (gr.variant) {
#define ZPM_G(I, LN, LT)                                                                      \
  case I: hipLaunchKernelGGL((kg_col<LN, LT>), g8, blk, gr.lds, st, jobs, sg, ns, inv, primes, gr.blocks); break;
        ZPM_G(0, -1, -1) ZPM_G(1, 5, 6) ZPM_G(2, 6, 5) ZPM_G(3, 7, 4) ZPM_G(4, 8, 3) ZPM_G(5, 9, 3)
        ZPM_G(6, 10, 3) ZPM_G(7, 8, 4) ZPM_G(8, 9, 4) ZPM_G(9, 10, 4)
        ZPM_G(10, 1, 8) ZPM_G(11, 2, 8) ZPM_G(12, 3, 8) ZPM_G(13, 4, 7)
#undef ZPM_G
        default: return hipErrorInvalidValue;
      }
      break;
    }
    case SK_CONVOLVE: {
      // variant: register kernel: log2 K, plus 16 for squares or 128 for products with
      // resident spectra, plus 32 for the full inner factor; LDS kernel: 0 (any K), or
      // 64 + log2 K with its full inner factor
      if (gr.variant >= 64 && gr.variant < 128) {
        switch (gr.variant - 64) {
          case 6: hipLaunchKernelGGL((kg_convolve<6, 5>), grid, blk, gr.lds, st, jobs, sg, ns, primes); break;
          case 7: hipLaunchKernelGGL((kg_convolve<7, 4>), grid, blk, gr.lds, st, jobs, sg, ns, primes); break;
          case 8: hipLaunchKernelGGL((kg_convolve<8, 3>), grid, blk, gr.lds, st, jobs, sg, ns, primes); break;
          default: return hipErrorInvalidValue;
        }
        break;
      }
      const bool sq = (gr.variant & 16) != 0, full = (gr.variant & 32) != 0,
                 ws = (gr.variant & 128) != 0;
      switch (gr.variant & 15) {
#define ZPM_GM(LK_, M_)                                                                                      \
  if (full) hipLaunchKernelGGL((kg_convolve_reg<LK_, M_, 12 - LK_>), grid, blk, gr.lds, st, jobs, sg, ns, primes); \
  else hipLaunchKernelGGL((kg_convolve_reg<LK_, M_, -1>), grid, blk, gr.lds, st, jobs, sg, ns, primes);
#define ZPM_G(LK_)                                                                            \
  case LK_:                                                                                   \
    if (ws) { ZPM_GM(LK_, CM_WITH_SPECTRUM) }                                                  \
    else if (sq) { ZPM_GM(LK_, CM_SQUARE) } else { ZPM_GM(LK_, CM_PRODUCT) }                   \
    break;
        ZPM_G(1) ZPM_G(2) ZPM_G(3) ZPM_G(4)
#undef ZPM_G
#undef ZPM_GM
        case 0: hipLaunchKernelGGL((kg_convolve<-1, -1>), grid, blk, gr.lds, st, jobs, sg, ns, primes); break;
        default: return hipErrorInvalidValue;
      }
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t stage_lds(const Plan &pl, int kind, int pass) {
  switch (kind) {
    case SK_CONVERT: {
      const int w = (std::max(pl.Na, pl.Nb) + 63) / 64;
      const int nchunks = (pl.M + 31) >> 5;
      return sizeof(uint32_t) * (((((size_t)1 << pl.log_ti_in) * (2 * w + 1)) + 1) & ~(size_t)1) +
             sizeof(uint2) * (size_t)nchunks * pl.np;
    }
    case SK_COL_FWD:
    case SK_COL_INV:
      return sizeof(uint32_t) * ((size_t)pl.col_tile[pass] << pl.col[pass].logn);
    case SK_CONVOLVE:
      return pl.conv_reg ? sizeof(uint32_t) * (size_t)(2 * pl.K) * (((size_t)1 << pl.logL1) + 1)
                         : sizeof(uint32_t) * (size_t)4 * pl.K << pl.logL1;
    case SK_RECOVER: {
      const int nw32 = 2 * ((pl.nout_bits + 63) / 64);
      return recover_lds_bytes(pl.np, pl.K, pl.M, nw32, pl.log_ti_out);
    }
    default:
      return 0;
  }
}

bool batch_supports(const Plan &pl) {
  if (pl.np < 1 || pl.np > BATCH_NP_MAX) return false;
  for (int c = 0; c < pl.ncol; ++c)
    if (pl.col_tile[c] < 1 || pl.col_tile[c] > BLOCK) return false;   // steps by BLOCK / T
  if (pl.conv_reg && pl.K > 16) return false;
  return true;
}

}  // namespace zpm
