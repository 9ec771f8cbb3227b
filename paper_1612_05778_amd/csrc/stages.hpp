// Device bodies of the pipeline stages, shared by the per-stage kernels and by the
// grouped batch kernels.  Each body processes one tile (one workgroup's share) and
// takes its LDS buffer and tile index as arguments.  See kernels.hip for the layout
// of the workspace and the order of the stages.
#pragma once
#include <hip/hip_runtime.h>

#include "zpm_internal.hpp"

namespace zpm {

// Read-only tables (twiddle heaps, 2^(32 t) tables) live in device memory.  Pointers
// read from a structure are generic to the compiler, which then emits flat loads; these
// go through the global address space instead, so that the loads are plain global (or,
// where the index is uniform, scalar) reads that do not wait on LDS traffic.
__device__ __forceinline__ uint2 ld_tab(const uint2 *__restrict__ tab, int64_t i) {
  const uint64_t v = ((const __attribute__((address_space(1))) uint64_t *)tab)[i];
  return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}

// ------------------------------------------------------------------------------------
// modular arithmetic on 32-bit words, p < 2^30
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t add_mod(uint32_t a, uint32_t b, uint32_t p) {
  uint32_t s = a + b;
  return min(s, s - p);
}
__device__ __forceinline__ uint32_t sub_mod(uint32_t a, uint32_t b, uint32_t p) {
  uint32_t d = a - b;
  return min(d, d + p);
}
// x * w mod p for a constant w with Shoup companion ws = floor(w 2^32 / p); any x < 2^32.
// x w - q p is written x w + q (2^32 - p), which compiles to one multiply-add.
__device__ __forceinline__ uint32_t mul_shoup(uint32_t x, uint2 w, uint32_t p) {
  const uint32_t q = __umulhi(x, w.y);
  const uint32_t negp = 0u - p;
  const uint32_t r = x * w.x + q * negp;   // in [0, 2p)
  return min(r, r + negp);
}
// a * b * 2^-32 mod p (Montgomery), a, b < p.
__device__ __forceinline__ uint32_t mont_mul(uint32_t a, uint32_t b, uint32_t p, uint32_t pinv) {
  uint32_t lo = a * b, hi = __umulhi(a, b);
  uint32_t m = lo * pinv;
  uint32_t mp = __umulhi(m, p);
  uint32_t r = hi - mp;   // wraps above 2^32 - p when hi < mp, and then r + p < r
  return min(r, r + p);
}

// Lazy forms for the transforms: operands and results in [0, 2p), i.e. reduced only up to
// one p (Harvey's butterflies).  Every prime is below 2^30, so 4p < 2^32: a sum of two
// such values, or u - v + 2p, still fits a word.
__device__ __forceinline__ uint32_t add_lz(uint32_t a, uint32_t b, uint32_t p) {
  const uint32_t s = a + b;                   // [0, 4p)
  return min(s, s - 2 * p);
}
__device__ __forceinline__ uint32_t sub_lz(uint32_t a, uint32_t b, uint32_t p) {
  const uint32_t d = a - b;                   // wraps when a < b, and then d + 2p < d
  return min(d, d + 2 * p);
}
// x w mod p up to one p, in [0, 2p), for any x < 2^32 (Shoup's product without its final
// subtraction).
__device__ __forceinline__ uint32_t mul_shoup_lz(uint32_t x, uint2 w, uint32_t p) {
  const uint32_t q = __umulhi(x, w.y);
  return x * w.x + q * (0u - p);
}
// mul_shoup_lz with -p mod 2^32 given instead of p.
__device__ __forceinline__ uint32_t shoup_neg_lz(uint32_t x, uint2 w, uint32_t negp) {
  return x * w.x + __umulhi(x, w.y) * negp;
}
// a b 2^-32 mod p up to one p, in [0, 2p), for a, b < 2p: a b < 4p^2 < p 2^32, so
// hi - mp lies in (-p, p).
__device__ __forceinline__ uint32_t mont_mul_lz(uint32_t a, uint32_t b, uint32_t p, uint32_t pinv) {
  const uint32_t lo = a * b, hi = __umulhi(a, b);
  const uint32_t m = lo * pinv;
  return hi - __umulhi(m, p) + p;
}
// w_m^e from a heap table (tab[m/2 + e] = w_m^e for e < m/2), any e in [0, m).
__device__ __forceinline__ uint2 heap_root(const uint2 *__restrict__ tab, int64_t m, int64_t e, uint32_t p) {
  const int64_t half = m >> 1;
  if (e < half) return ld_tab(tab, half + e);
  uint2 w = ld_tab(tab, e);    // w_m^(e - m/2) = -w_m^e
  return make_uint2(p - w.x, ~w.y);
}

// ------------------------------------------------------------------------------------
// radix-2^R butterfly groups on transforms held in LDS.
// Transform t (t < ntr = 2^logntr, times nops operand copies) has element e at
// s[(t & (ntr-1)) * ts + (t >> logntr) * off2 + e * es].
// ------------------------------------------------------------------------------------
struct LdsShape {
  int logntr, logn, ts, es, off2, logops;
};
// The same shape fixed at compile time, so that every LDS offset of a group folds into
// the instructions' immediates.
template <int LOGNTR, int LOGN, int TS, int ES, int OFF2 = 0, int LOGOPS = 0>
struct CShape {
  static constexpr int logntr = LOGNTR, logn = LOGN, ts = TS, es = ES, off2 = OFF2,
                       logops = LOGOPS;
};

template <class SH>
__device__ __forceinline__ int lds_base(const SH &sh, int t) {
  return (t & ((1 << sh.logntr) - 1)) * sh.ts + (t >> sh.logntr) * sh.off2;
}

// DIF (Gentleman-Sande) stages with half-sizes h0, h0/2, ..., h0/2^(R-1); output of the
// whole transform is in bit-reversed order.
// LOGH0 >= 0 fixes logh0 at compile time (with a compile-time shape).
template <int R, class SH = LdsShape, int LOGH0 = -1>
__device__ void dif_group(uint32_t *s, const SH &sh, int logh0_rt, const uint2 *__restrict__ tw,
                          uint32_t p) {
  constexpr int NR = 1 << R;
  const int logh0 = LOGH0 >= 0 ? LOGH0 : logh0_rt;
  const int loghl = logh0 - (R - 1);
  const int hl = 1 << loghl;
  const int lgpt = sh.logn - R;                       // groups per transform (log)
  const int total = 1 << (sh.logntr + sh.logops + lgpt);
  // lanes run over transforms when those are adjacent in LDS, or when the element
  // stride inside the group is small (which would put a wave on few banks)
  const bool tfast = sh.ts < sh.es || ((sh.ts & 1) && hl * sh.es < 16 && sh.logntr + sh.logops >= 4);
  for (int g = threadIdx.x; g < total; g += BLOCK) {
    int t, q;
    if (tfast) {
      t = g & ((1 << (sh.logntr + sh.logops)) - 1);
      q = g >> (sh.logntr + sh.logops);
    } else {
      q = g & ((1 << lgpt) - 1);
      t = g >> lgpt;
    }
    const int j = q & (hl - 1);
    const int blk = q >> loghl;
    const int base = lds_base(sh, t) + ((blk << (logh0 + 1)) + j) * sh.es;
    const int step = hl * sh.es;
    uint32_t x[NR];
#pragma unroll
    for (int m = 0; m < NR; ++m) x[m] = s[base + m * step];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int half = NR >> (i + 1);
      const int hsz = 1 << (logh0 - i);
#pragma unroll
      for (int m = 0; m < NR; ++m) {
        if (m & half) continue;
        const uint2 w = ld_tab(tw, hsz + j + (m & (half - 1)) * hl);
        const uint32_t u = x[m], v = x[m + half];
        x[m] = add_lz(u, v, p);
        x[m + half] = mul_shoup_lz(u - v + 2 * p, w, p);
      }
    }
#pragma unroll
    for (int m = 0; m < NR; ++m) s[base + m * step] = x[m];
  }
}

// DIT (Cooley-Tukey) stages with half-sizes h0, 2 h0, ..., h0 2^(R-1); input in
// bit-reversed order, output natural.
template <int R, class SH = LdsShape, int LOGH0 = -1>
__device__ void dit_group(uint32_t *s, const SH &sh, int logh0_rt, const uint2 *__restrict__ tw,
                          uint32_t p) {
  constexpr int NR = 1 << R;
  const int logh0 = LOGH0 >= 0 ? LOGH0 : logh0_rt;
  const int h0 = 1 << logh0;
  const int loghr = logh0 + R - 1;
  const int lgpt = sh.logn - R;
  const int total = 1 << (sh.logntr + sh.logops + lgpt);
  const bool tfast = sh.ts < sh.es || ((sh.ts & 1) && h0 * sh.es < 16 && sh.logntr + sh.logops >= 4);
  for (int g = threadIdx.x; g < total; g += BLOCK) {
    int t, q;
    if (tfast) {
      t = g & ((1 << (sh.logntr + sh.logops)) - 1);
      q = g >> (sh.logntr + sh.logops);
    } else {
      q = g & ((1 << lgpt) - 1);
      t = g >> lgpt;
    }
    const int j = q & (h0 - 1);
    const int blk = q >> logh0;
    const int base = lds_base(sh, t) + ((blk << (loghr + 1)) + j) * sh.es;
    const int step = h0 * sh.es;
    uint32_t x[NR];
#pragma unroll
    for (int m = 0; m < NR; ++m) x[m] = s[base + m * step];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int half = 1 << i;
      const int hsz = h0 << i;
#pragma unroll
      for (int m = 0; m < NR; ++m) {
        if (m & half) continue;
        const uint2 w = ld_tab(tw, hsz + j + (m & (half - 1)) * h0);
        const uint32_t u = x[m];
        const uint32_t v = mul_shoup_lz(x[m + half], w, p);
        x[m] = add_lz(u, v, p);
        x[m + half] = sub_lz(u, v, p);
      }
    }
#pragma unroll
    for (int m = 0; m < NR; ++m) s[base + m * step] = x[m];
  }
}

// Stages per register group: the fewest groups of at most 4 stages (radix 16), as even
// as possible, larger groups first (8 -> 4+4, 9 -> 3+3+3, 7 -> 4+3, 6 -> 3+3).
__device__ __forceinline__ int group_stages(int left) {
  const int ngroups = (left + 3) >> 2;
  return (left + ngroups - 1) / ngroups;
}

// Full forward transform (all logn stages); caller synchronises before and after.
__device__ void lds_dif(uint32_t *s, const LdsShape &sh, const uint2 *__restrict__ tw, uint32_t p) {
  int st = sh.logn;
  while (st > 0) {
    const int r = group_stages(st);
    if (r == 4) dif_group<4>(s, sh, st - 1, tw, p);
    else if (r == 3) dif_group<3>(s, sh, st - 1, tw, p);
    else if (r == 2) dif_group<2>(s, sh, st - 1, tw, p);
    else dif_group<1>(s, sh, st - 1, tw, p);
    st -= r;
    __syncthreads();
  }
}

__device__ void lds_dit(uint32_t *s, const LdsShape &sh, const uint2 *__restrict__ tw, uint32_t p) {
  int done = 0;
  while (done < sh.logn) {
    const int r = group_stages(sh.logn - done);
    if (r == 4) dit_group<4>(s, sh, done, tw, p);
    else if (r == 3) dit_group<3>(s, sh, done, tw, p);
    else if (r == 2) dit_group<2>(s, sh, done, tw, p);
    else dit_group<1>(s, sh, done, tw, p);
    done += r;
    __syncthreads();
  }
}

// Full transforms of a compile-time shape: the groups of lds_dif / lds_dit, each with its
// stages fixed at compile time.  ST: stages left (DIF) / done (DIT).
__device__ constexpr int group_stages_c(int left) {
  return (left + ((left + 3) >> 2) - 1) / ((left + 3) >> 2);
}
template <class SH, int ST = SH::logn>
__device__ __forceinline__ void lds_dif_c(uint32_t *s, const uint2 *__restrict__ tw, uint32_t p) {
  if constexpr (ST > 0) {
    constexpr int R = group_stages_c(ST);
    dif_group<R, SH, ST - 1>(s, SH{}, 0, tw, p);
    __syncthreads();
    lds_dif_c<SH, ST - R>(s, tw, p);
  }
}
template <class SH, int DONE = 0>
__device__ __forceinline__ void lds_dit_c(uint32_t *s, const uint2 *__restrict__ tw, uint32_t p) {
  if constexpr (DONE < SH::logn) {
    constexpr int R = group_stages_c(SH::logn - DONE);
    dit_group<R, SH, DONE>(s, SH{}, 0, tw, p);
    __syncthreads();
    lds_dit_c<SH, DONE + R>(s, tw, p);
  }
}

__device__ __forceinline__ int bitrev(int x, int logn) {
  return logn ? (int)(__brev((unsigned)x) >> (32 - logn)) : 0;
}
__host__ __device__ constexpr int bitrev_c(int x, int logn) {
  int r = 0;
  for (int b = 0; b < logn; ++b) r |= ((x >> b) & 1) << (logn - 1 - b);
  return r;
}

// A raw buffer resource over `bytes` bytes from p (gfx9 word 3: 32-bit data format):
// loads past the end read zero, stores past it are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_col_rsrc(uint32_t *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)bytes, 0x00020000);
}

// Element-wise staging between global memory and LDS: for idx = threadIdx.x, +BLOCK, ...
// below `total`, put(idx, load(idx)).  U loads are issued before their results are
// used, so a thread keeps U global reads in flight instead of one.
template <int U, typename T, typename LD, typename ST>
__device__ __forceinline__ void staged(int total, LD load, ST put) {
  for (int i0 = threadIdx.x; i0 < total; i0 += U * BLOCK) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = i0 + u * BLOCK;
      v[u] = idx < total ? load(idx) : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = i0 + u * BLOCK;
      if (idx < total) put(idx, v[u]);
    }
  }
}

// ------------------------------------------------------------------------------------
// BivariateRepresentation: coefficient i of a (N-bit two's complement, w words) is
// split into K limbs of M bits, a_i = sum_j a_{i,j} 2^(M j) (Section 2).  Lower limbs
// are unsigned M-bit fields; the top limb is the signed top field, so that the split
// needs no carries.  Each limb is reduced mod every prime.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t get32(const uint32_t *row, int nw, uint32_t sgn, int64_t pos) {
  const int64_t q = pos >> 5;
  const int sh = (int)(pos & 31);
  const uint32_t lo = q < nw ? row[q] : sgn;
  if (!sh) return lo;
  const uint32_t hi = q + 1 < nw ? row[q + 1] : sgn;
  return (lo >> sh) | (hi << (32 - sh));
}

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a contiguous run
// of tiles so that neighbouring tiles share that XCD's L2.  The grid has 8 * chunk
// blocks; tiles >= ntiles are idle.
__device__ __forceinline__ int64_t xcd_tile_of(int64_t bid, int64_t ntiles) {
  const int64_t chunk = (ntiles + 7) >> 3;
  return (bid & 7) * chunk + (bid >> 3);
}
__device__ __forceinline__ int64_t xcd_tile(int64_t ntiles) { return xcd_tile_of(blockIdx.x, ntiles); }

// lo += a b over 64 bits, hi += the carry out: the multiply-add's own carry feeds one
// add-with-carry (the compiler would compare and select instead).  Register-only ALU.
__device__ __forceinline__ void mac_carry(uint64_t &lo, uint32_t &hi, uint32_t a, uint32_t b) {
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t"
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc"
      : "+v"(lo), "+v"(hi)
      : "v"(a), "v"(b)
      : "vcc");
}

// NP = np exactly: per-prime accumulators stay in registers, loops fully unrolled.
template <int NP>
__device__ __forceinline__ void body_convert_in(uint32_t *s, int64_t tile_id, const uint64_t *__restrict__ src,
                                int64_t d, int32_t N, int32_t w, int32_t K, int32_t M, int32_t np,
                                uint32_t *__restrict__ X, int64_t L, int32_t col_off, int32_t logTI,
                                const PrimeDev *__restrict__ primes, const PlanDev *__restrict__ pd) {
  const int TI = 1 << logTI;
  const int64_t i0 = tile_id << logTI;
  if (i0 >= d) return;
  const int ti = (int)min<int64_t>(TI, d - i0);
  const int nw = 2 * w;
  const int stride = nw + 1;
  const int nchunks = (M + 31) >> 5;
  // 2^(32 t) mod p_k, [t][k], after the staged tile; read together with the tile
  uint32_t *pw = s + (((ti * stride) + 1) & ~1);
  for (int idx = threadIdx.x; idx < nchunks * np; idx += BLOCK) {
    const int t = idx / np, k = idx - t * np;
    pw[idx] = ld_tab(primes[k].pow32, t).x;
  }
  // stage the tile's words (one contiguous block of ti * w words)
  const uint64_t *tile = src + i0 * w;
  staged<8, uint64_t>(ti * w, [&](int idx) { return tile[idx]; }, [&](int idx, uint64_t v) {
    const int il = idx / w, u = idx - il * w;
    s[il * stride + 2 * u] = (uint32_t)v;
    s[il * stride + 2 * u + 1] = (uint32_t)(v >> 32);
  });
  __syncthreads();
  // sign-extend from bit N-1: bits >= N are not part of the value
  const int tq = (N - 1) >> 5, tb = (N - 1) & 31;
  for (int il = threadIdx.x; il < ti; il += BLOCK) {
    uint32_t *row = s + il * stride;
    const uint32_t top = row[tq];
    const uint32_t sgn = ((top >> tb) & 1u) ? 0xFFFFFFFFu : 0u;
    if (tb < 31) {
      const uint32_t keep = (2u << tb) - 1u;
      row[tq] = (top & keep) | (sgn & ~keep);
    }
    for (int q = tq + 1; q < nw; ++q) row[q] = sgn;
  }
  __syncthreads();
  const uint32_t lastmask = (M & 31) ? ((1u << (M & 31)) - 1u) : 0xFFFFFFFFu;
  const int64_t twoK = 2 * (int64_t)K;
  uint32_t pk[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) pk[k] = primes[k].p;
  for (int idx = threadIdx.x; idx < (K << logTI); idx += BLOCK) {
    const int il = idx & (TI - 1);
    const int j = idx >> logTI;
    if (il >= ti) continue;
    const uint32_t *row = s + il * stride;
    const uint32_t sgn = (uint32_t)((int32_t)row[nw - 1] >> 31);
    const int64_t b = (int64_t)M * j;
    // unsigned value of bits [b, b + M): sum_t chunk_t (2^(32 t) mod p), summed exactly
    // per prime as lo + 2^64 hi (each term is below 2^63), reduced once at the end
    uint64_t lo[NP];
    uint32_t hi[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) { lo[k] = 0; hi[k] = 0; }
    for (int t = 0; t < nchunks; ++t) {
      uint32_t c = get32(row, nw, sgn, b + 32 * (int64_t)t);
      if (t == nchunks - 1) c &= lastmask;
      const uint32_t *pwt = pw + t * NP;
#pragma unroll
      for (int k = 0; k < NP; ++k) mac_carry(lo[k], hi[k], c, pwt[k]);
    }
    // the top limb is signed: subtract 2^M when its top bit (bit M K - 1) is set
    const bool neg_top = (j == K - 1) && ((get32(row, nw, sgn, b + M - 1) & 1u) != 0);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const uint32_t p = pk[k];
      const uint2 one = make_uint2(1u, primes[k].ones);
      const uint2 c32 = make_uint2(primes[k].c32, primes[k].c32s);
      // reduced up to one p, as the transforms take their inputs
      uint32_t r = add_lz(mul_shoup_lz((uint32_t)lo[k], one, p),
                          mul_shoup_lz((uint32_t)(lo[k] >> 32), c32, p), p);
      r = add_lz(r, mul_shoup_lz(hi[k], ld_tab(primes[k].pow32, 2), p), p);   // 2^64 mod p
      if (neg_top) r = sub_lz(r, pd->pow2M[k], p);
      X[((int64_t)k * twoK + col_off + j) * L + i0 + il] = r;
    }
  }
}

// ------------------------------------------------------------------------------------
// Strided column passes of the y-transform (outer factors of a four-step split).
// Index i = inner + S (e + n outer); the pass transforms along e and leaves the
// frequencies in natural order.  Forward: DIF, then multiply frequency k by
// w_{nS}^(inner k).  Inverse: multiply by w_{nS}^(-inner k), then DIT.  Each thread
// meets the frequencies k = e0, e0 + de, ... of one column, so its twiddles form a
// geometric progression kept in Montgomery form (no table gathers), advanced by a Shoup
// product with the constant ratio.
// ------------------------------------------------------------------------------------
// cols: columns transformed per prime, those from col0 on among each prime's 2K (K of
// them when only one operand's limbs need a forward transform: a square, or one
// operand of a product with a resident transform).
// CLOGN / CLOGT >= 0: the pass length and tile width fixed at compile time (they must
// equal logn_rt / logT_rt).
template <int CLOGN = -1, int CLOGT = -1>
__device__ void body_col_pass(uint32_t *s, int64_t bid, uint32_t *__restrict__ X, int64_t L,
                              int32_t twoK, int32_t logn_rt, int64_t S, int32_t logT_rt, int64_t nz_a,
                              int64_t nz_b, int32_t K, int64_t nlimit, int32_t inverse,
                              const PrimeDev *__restrict__ primes, int32_t cols, int32_t col0) {
  constexpr bool fixed = CLOGN >= 0 && CLOGT >= 0;
  const int logn = fixed ? CLOGN : logn_rt, logT = fixed ? CLOGT : logT_rt;
  using CSH = CShape<(CLOGT >= 0 ? CLOGT : 0), (CLOGN >= 0 ? CLOGN : 1), 1,
                     (1 << (CLOGT >= 0 ? CLOGT : 0))>;
  const int n = 1 << logn, T = 1 << logT;
  // L, S, T and cols (K or 2K) are powers of two: the block index splits by shifts
  const int logS = __builtin_ctzll((unsigned long long)S);
  const int logL = __builtin_ctzll((unsigned long long)L);
  const int log_inner = logS - logT;                  // inner tiles per outer index
  const int log_tiles = logL - logn - logT;           // tiles per column
  const int64_t cidx = bid >> log_tiles;
  const int64_t tile = bid & (((int64_t)1 << log_tiles) - 1);
  const int64_t outer = tile >> log_inner;
  const int64_t inner0 = (tile & (((int64_t)1 << log_inner) - 1)) << logT;
  const int log_cols = __builtin_ctz((unsigned)cols);
  const int k = (int)(cidx >> log_cols);
  const int jc = col0 + (int)(cidx & (cols - 1));
  const int64_t col = (int64_t)k * twoK + jc;
  const PrimeDev pr = primes[k];
  const uint32_t p = pr.p;
  const int64_t first = inner0 + S * (int64_t)n * outer;   // y index of (t = 0, e = 0)
  uint32_t *base = X + col * L + first;
  const int64_t nz = inverse ? L : (jc < K ? nz_a : nz_b);
  const int64_t m = (int64_t)n * S;
  const int t = threadIdx.x & (T - 1);
  const int e0 = threadIdx.x >> logT, de = BLOCK >> logT;
  const int64_t inner = inner0 + t;
  const uint2 *tab = inverse ? pr.hi : pr.hf;
  const uint32_t R = pr.c32;   // 2^32 mod p
  // cur: the twiddle in Montgomery form (times 2^32), applied by a Montgomery product;
  // step: the ratio of consecutive twiddles with its Shoup companion, so that the
  // progression is a Shoup product (which keeps the Montgomery form)
  uint32_t cur = mul_shoup(R, heap_root(tab, m, (inner * e0) & (m - 1), p), p);
  const uint2 step = heap_root(tab, m, (inner * de) & (m - 1), p);
  // offsets inside the column stay below L <= 2^21: 32-bit index arithmetic
  const int lim_store = (int)std::min<int64_t>(std::max<int64_t>(nlimit - first, 0), L);
  if constexpr (fixed) {
    // Compile-time shape: every loop fully unrolled, so that the bit-reversed LDS indices
    // are immediate offsets, and global memory reached through buffer instructions over
    // the tile's column.  Element (t, e) of the tile is at byte (t + e S) 4 past `base`;
    // this thread's rows are e0 + i de (i < NI), the staged loops' rows idx / T with
    // idx = threadIdx + k BLOCK, i.e. the same rows.  Bounded accesses keep the whole
    // offset in the per-lane part, which the hardware checks against the buffer's size
    // (loads past it read zero, stores past it are dropped); the others put i's row step
    // in the scalar offset.
    constexpr int LDE = 8 - CLOGT;                  // log2(BLOCK / T)
    constexpr int LI = CLOGN - LDE;
    constexpr int NI = 1 << LI;                     // rows per thread
    constexpr int LG = NI < 32 ? NI : 32;           // loads in flight per thread
    constexpr int G8 = NI < 8 ? NI : 8;             // LDS values per store group
    static_assert(LI >= 1 && (BLOCK >> CLOGT) << LI == (1 << CLOGN), "column pass shape");
    const int voff0 = (t + (e0 << logS)) * 4;
    const int vstep = (de << logS) * 4;
    const uint32_t col_bytes = (uint32_t)(L - first) * 4u;
    uint32_t *srow = s + ((bitrev(e0, LDE) << LI) << CLOGT) + t;   // bitrev(e0 + i de) = that | bitrev(i)
    if (!inverse) {
      // rows past nz (zero limbs) read as zero
      const int64_t nzr = std::min<int64_t>(std::max<int64_t>(nz - first, 0), L - first);
      const __amdgpu_buffer_rsrc_t rin = make_col_rsrc(base, (uint32_t)nzr * 4u);
      if (nzr <= ((int64_t)(1 << (CLOGN - 1)) << logS)) {
        // rows n/2 and up are zero (an operand shorter than half the transform, as in a
        // product's outermost pass): the first DIF stage leaves row e as it is and makes
        // row e + n/2 the row times w_n^e, so only the lower half is read
        constexpr int NH = NI / 2, HN = 1 << (CLOGN - 1);
        uint32_t v[NH];
#pragma unroll
        for (int u = 0; u < NH; ++u)
          v[u] = __builtin_amdgcn_raw_buffer_load_b32(rin, voff0 + u * vstep, 0, 0);
#pragma unroll
        for (int u = 0; u < NH; ++u) {
          const int e = e0 + u * de;                           // below n/2
          s[threadIdx.x + u * BLOCK] = v[u];
          s[threadIdx.x + (u + NH) * BLOCK] = mul_shoup_lz(v[u], ld_tab(pr.hf, HN + e), p);
        }
        __syncthreads();
        lds_dif_c<CSH, CLOGN - 1>(s, pr.hf, p);
      } else {
#pragma unroll
        for (int k0 = 0; k0 < NI; k0 += LG) {
          uint32_t v[LG];
#pragma unroll
          for (int u = 0; u < LG; ++u)
            v[u] = __builtin_amdgcn_raw_buffer_load_b32(rin, voff0 + (k0 + u) * vstep, 0, 0);
#pragma unroll
          for (int u = 0; u < LG; ++u) s[threadIdx.x + (k0 + u) * BLOCK] = v[u];
        }
        __syncthreads();
        lds_dif_c<CSH>(s, pr.hf, p);
      }
      const __amdgpu_buffer_rsrc_t rout = make_col_rsrc(base, col_bytes);
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        const uint32_t v = mont_mul_lz(srow[bitrev_c(i, LI) << CLOGT], cur, p, pr.pinv);
        cur = mul_shoup_lz(cur, step, p);
        __builtin_amdgcn_raw_buffer_store_b32(v, rout, voff0, i * vstep, 0);
      }
    } else {
      const __amdgpu_buffer_rsrc_t rin = make_col_rsrc(base, col_bytes);
#pragma unroll
      for (int i0 = 0; i0 < NI; i0 += LG) {
        uint32_t v[LG];
#pragma unroll
        for (int u = 0; u < LG; ++u)
          v[u] = __builtin_amdgcn_raw_buffer_load_b32(rin, voff0, (i0 + u) * vstep, 0);
#pragma unroll
        for (int u = 0; u < LG; ++u) {
          srow[bitrev_c(i0 + u, LI) << CLOGT] = mont_mul_lz(v[u], cur, p, pr.pinv);
          cur = mul_shoup_lz(cur, step, p);
        }
      }
      __syncthreads();
      lds_dit_c<CSH>(s, pr.hi, p);
      // rows with t + e S at or past lim_store are not stored
      const __amdgpu_buffer_rsrc_t rst = make_col_rsrc(base, (uint32_t)lim_store * 4u);
#pragma unroll
      for (int k0 = 0; k0 < NI; k0 += G8) {
        uint32_t v[G8];
#pragma unroll
        for (int u = 0; u < G8; ++u) v[u] = s[threadIdx.x + (k0 + u) * BLOCK];
#pragma unroll
        for (int u = 0; u < G8; ++u)
          __builtin_amdgcn_raw_buffer_store_b32(v[u], rst, voff0 + (k0 + u) * vstep, 0, 0);
      }
    }
    return;
  }
  // every global access of this thread is in its own column t (BLOCK is a multiple of
  // T), at row offsets e S (e S < L <= 2^21)
  uint32_t *bt = base + t;
  if (!inverse) {
    // row e is below nz iff e < e_lim
    const int64_t rem = nz - first - t;
    const int e_lim = rem <= 0 ? 0 : (int)min<int64_t>((rem + S - 1) >> logS, n);
    staged<8, uint32_t>(n << logT, [&](int idx) {
      const int e = idx >> logT;
      return e < e_lim ? bt[e << logS] : 0u;
    }, [&](int idx, uint32_t v) { s[idx] = v; });
    __syncthreads();
    if constexpr (fixed) lds_dif_c<CSH>(s, pr.hf, p);
    else lds_dif(s, LdsShape{logT, logn, 1, T, 0, 0}, pr.hf, p);
    for (int e = e0; e < n; e += de) {
      const uint32_t v = mont_mul_lz(s[(bitrev(e, logn) << logT) + t], cur, p, pr.pinv);
      cur = mul_shoup_lz(cur, step, p);
      bt[e << logS] = v;
    }
  } else {
    // eight independent loads in flight per thread, then the twiddle progression
    for (int e = e0; e < n; e += 8 * de) {
      uint32_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int ee = e + u * de;
        v[u] = ee < n ? bt[ee << logS] : 0u;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int ee = e + u * de;
        if (ee < n) {
          s[(bitrev(ee, logn) << logT) + t] = mont_mul_lz(v[u], cur, p, pr.pinv);
          cur = mul_shoup_lz(cur, step, p);
        }
      }
    }
    __syncthreads();
    if constexpr (fixed) lds_dit_c<CSH>(s, pr.hi, p);
    else lds_dit(s, LdsShape{logT, logn, 1, T, 0, 0}, pr.hi, p);
    // row e is stored iff t + e S < lim_store
    const int rem = lim_store - t;
    const int e_lim = rem <= 0 ? 0 : min((rem + (int)S - 1) >> logS, n);
    staged<8, uint32_t>(n << logT, [&](int idx) { return s[idx]; }, [&](int idx, uint32_t v) {
      const int e = idx >> logT;
      if (e < e_lim) bt[e << logS] = v;
    });
  }
}

// ------------------------------------------------------------------------------------
// The two convolutions along x for one prime and one block of L1 consecutive y
// positions.  Per y-frequency the limbs a_{.,j} (j < K) are zero-padded to 2K and
// transformed with DIF of length 2K: the first stage multiplies row j by theta^j
// (theta a primitive 2K-th root, the twist of NegacyclicConvolution) and the two
// halves then hold the cyclic (mod x^K - 1) and twisted (mod x^K + 1) spectra.
// After the pointwise product the DIT inverse of length 2K undoes both transforms;
// its last stage applies theta^-j (untwist) and forms c- + c+ and c- - c+, which
// times 1/(2K) are c_{i,j} and c_{i,j+K} (Section 2, C+ and C- through Relation
// (recoveringC)).  The pointwise product is a plain Montgomery product: the
// normalisation by 2^32 / (2K L) waits for the recovery, whose first multiplication
// per residue takes it with the CRT constant.
// ------------------------------------------------------------------------------------
// CLOGK / CLOGL1 >= 0: K and L1 fixed at compile time (== the runtime values).
template <int CLOGK = -1, int CLOGL1 = -1>
__device__ void body_convolve(uint32_t *s, int64_t bid, uint32_t *__restrict__ X, int64_t L,
                              int32_t K_rt, int32_t logK_rt, int32_t logL1_rt, int64_t nz_a,
                              int64_t nz_b, int64_t nlimit, const PrimeDev *__restrict__ primes,
                              const PlanDev *__restrict__ pd, int32_t mode,
                              const uint32_t *__restrict__ spec) {
  constexpr bool fixed = CLOGK >= 0 && CLOGL1 >= 0;
  constexpr int FK = fixed ? CLOGK : 1, FL1 = fixed ? CLOGL1 : 1;   // valid when fixed
  constexpr int FTWOKL1 = (2 << FK) << FL1;
  const int logK = fixed ? CLOGK : logK_rt, logL1 = fixed ? CLOGL1 : logL1_rt;
  const int K = fixed ? (1 << CLOGK) : K_rt;
  const int L1 = 1 << logL1;
  const int64_t nrb = L >> logL1;   // a power of two: the block index splits by shifts
  const int k = (int)(bid >> __builtin_ctzll((unsigned long long)nrb));
  const int64_t rb = bid & (nrb - 1);
  const PrimeDev pr = primes[k];
  const uint32_t p = pr.p;
  const int twoK = 2 * K;
  uint32_t *A = s;                      // 2K rows x L1
  uint32_t *B = s + twoK * L1;          // 2K rows x L1
  uint32_t *base = X + (int64_t)k * twoK * L + rb * L1;
  const int64_t y0 = rb * L1;
  const int logL = __builtin_ctzll((unsigned long long)L);
  // rows are read below nz_a / nz_b and written below nlimit: as positions in the block
  const int lim_b = (int)max<int64_t>(0, min<int64_t>(nz_b - y0, L1));
  const int lim_o = (int)max<int64_t>(0, min<int64_t>(nlimit - y0, L1));
  // A: a's limb rows (b's for CM_SPECTRUM); the upper K rows are the zero padding
  const int src_a = mode == CM_SPECTRUM ? K : 0;
  const int lim_first = mode == CM_SPECTRUM ? lim_b : (int)max<int64_t>(0, min<int64_t>(nz_a - y0, L1));
  staged<8, uint32_t>(K << logL1, [&](int idx) {
    const int j = idx >> logL1, e = idx & (L1 - 1);
    return e < lim_first ? base[((int64_t)(src_a + j) << logL) + e] : 0u;
  }, [&](int idx, uint32_t v) { A[idx] = v; A[(K << logL1) + idx] = 0u; });
  if (mode == CM_PRODUCT) {
    staged<8, uint32_t>(K << logL1, [&](int idx) {
      const int j = idx >> logL1, e = idx & (L1 - 1);
      return e < lim_b ? base[((int64_t)(K + j) << logL) + e] : 0u;
    }, [&](int idx, uint32_t v) { B[idx] = v; B[(K << logL1) + idx] = 0u; });
  } else if (mode == CM_WITH_SPECTRUM) {
    // b's spectra, in the order the forward transforms below leave A in
    const uint32_t *sb = spec + (int64_t)k * twoK * L + rb * L1;
    staged<8, uint32_t>(twoK << logL1, [&](int idx) {
      return sb[(int64_t)(idx >> logL1) * L + (idx & (L1 - 1))];
    }, [&](int idx, uint32_t v) { B[idx] = v; });
  }
  __syncthreads();
  // innermost y factor on the K limb rows of both operands (of one operand otherwise)
  const int ops = mode == CM_PRODUCT ? 1 : 0;
  if constexpr (fixed) {
    if (ops) {
      lds_dif_c<CShape<FK, FL1, (1 << FL1), 1, FTWOKL1, 1>>(s, pr.hf, p);
      lds_dif_c<CShape<FL1, FK + 1, 1, (1 << FL1), FTWOKL1, 1>>(s, pr.hf, p);
    } else {
      lds_dif_c<CShape<FK, FL1, (1 << FL1), 1, FTWOKL1, 0>>(s, pr.hf, p);
      lds_dif_c<CShape<FL1, FK + 1, 1, (1 << FL1), FTWOKL1, 0>>(s, pr.hf, p);
    }
  } else {
    lds_dif(s, LdsShape{logK, logL1, L1, 1, twoK * L1, ops}, pr.hf, p);
    // x: 2K-point transforms down the L1 columns
    lds_dif(s, LdsShape{logL1, logK + 1, 1, L1, twoK * L1, ops}, pr.hf, p);
  }
  if (mode == CM_SPECTRUM) {
    // this block's positions only, all read above: the spectra replace the limbs
    staged<8, uint32_t>(twoK << logL1, [&](int idx) { return A[idx]; }, [&](int idx, uint32_t v) {
      base[(int64_t)(idx >> logL1) * L + (idx & (L1 - 1))] = v;
    });
    return;
  }
  const uint32_t *F = mode == CM_SQUARE ? A : B;
  for (int idx = threadIdx.x; idx < (twoK << logL1); idx += BLOCK)
    A[idx] = mont_mul_lz(A[idx], F[idx], p, pr.pinv);
  __syncthreads();
  if constexpr (fixed) {
    lds_dit_c<CShape<FL1, FK + 1, 1, (1 << FL1)>>(s, pr.hi, p);
    lds_dit_c<CShape<FK + 1, FL1, (1 << FL1), 1>>(s, pr.hi, p);
  } else {
    lds_dit(s, LdsShape{logL1, logK + 1, 1, L1, 0, 0}, pr.hi, p);
    lds_dit(s, LdsShape{logK + 1, logL1, L1, 1, 0, 0}, pr.hi, p);
  }
  staged<8, uint32_t>(twoK << logL1, [&](int idx) { return A[idx]; }, [&](int idx, uint32_t v) {
    const int j = idx >> logL1, e = idx & (L1 - 1);
    if (e < lim_o) base[((int64_t)j << logL) + e] = v;
  });
}

// ------------------------------------------------------------------------------------
// Same convolutions with each 2K-point x-transform held in one thread's registers
// (K <= 32): the column's K limbs of a and of b are transformed, multiplied and
// transformed back without touching LDS.  Twiddle offsets are compile-time.
// ------------------------------------------------------------------------------------
template <int LOGK>
__device__ __forceinline__ void reg_dif(uint32_t (&x)[2 << LOGK], const uint2 *__restrict__ tw,
                                        uint32_t p) {
  constexpr int N2 = 2 << LOGK;
  // first stage: the upper half is zero, so x[j + K] = x[j] theta^j (the twist)
#pragma unroll
  for (int j = 0; j < N2 / 2; ++j) x[j + N2 / 2] = j ? mul_shoup_lz(x[j], ld_tab(tw, N2 / 2 + j), p) : x[j];
#pragma unroll
  for (int h = N2 / 4; h >= 1; h >>= 1) {
#pragma unroll
    for (int blk = 0; blk < N2; blk += 2 * h) {
#pragma unroll
      for (int j = 0; j < h; ++j) {
        const uint32_t u = x[blk + j], v = x[blk + j + h];
        x[blk + j] = add_lz(u, v, p);
        x[blk + j + h] = j ? mul_shoup_lz(u - v + 2 * p, ld_tab(tw, h + j), p) : sub_lz(u, v, p);
      }
    }
  }
}

template <int LOGK>
__device__ __forceinline__ void reg_dit(uint32_t (&x)[2 << LOGK], const uint2 *__restrict__ tw,
                                        uint32_t p) {
  constexpr int N2 = 2 << LOGK;
#pragma unroll
  for (int h = 1; h < N2; h <<= 1) {
#pragma unroll
    for (int blk = 0; blk < N2; blk += 2 * h) {
#pragma unroll
      for (int j = 0; j < h; ++j) {
        const uint32_t u = x[blk + j];
        const uint32_t v = j ? mul_shoup_lz(x[blk + j + h], ld_tab(tw, h + j), p) : x[blk + j + h];
        x[blk + j] = add_lz(u, v, p);
        x[blk + j + h] = sub_lz(u, v, p);
      }
    }
  }
}

// MODE is a ConvMode, fixed at compile time so that each variant keeps only its own
// register footprint (the product's is the largest that matters for occupancy).
// CLOGL1 >= 0: the inner factor L1 = 2^CLOGL1 fixed at compile time (== logL1_rt).
template <int LOGK, int MODE, int CLOGL1 = -1>
__device__ void body_convolve_reg(uint32_t *s, int64_t bid, uint32_t *__restrict__ X, int64_t L,
                                  int32_t logL1_rt, int64_t nz_a, int64_t nz_b, int64_t nlimit,
                                  const PrimeDev *__restrict__ primes,
                                  const PlanDev *__restrict__ pd,
                                  const uint32_t *__restrict__ spec) {
  constexpr int K = 1 << LOGK, K2 = 2 * K;
  const int logL1 = CLOGL1 >= 0 ? CLOGL1 : logL1_rt;
  const int L1 = 1 << logL1, RS = L1 + 1;      // odd row stride: rows fall on distinct banks
  const int64_t nrb = L >> logL1;   // a power of two: the block index splits by shifts
  const int k = (int)(bid >> __builtin_ctzll((unsigned long long)nrb));
  const int64_t rb = bid & (nrb - 1);
  const PrimeDev pr = primes[k];
  const uint32_t p = pr.p;
  uint32_t *base = X + (int64_t)k * K2 * L + rb * L1;
  const int64_t y0 = rb * L1;
  const int L32 = (int)L;   // 2K rows of at most 2^21 words: 32-bit row offsets
  const int logL = __builtin_ctzll((unsigned long long)L);
  // rows are read below nz_a / nz_b and written below nlimit: as positions in the block
  const int lim_a = (int)max<int64_t>(0, min<int64_t>(nz_a - y0, L1));
  const int lim_b = (int)max<int64_t>(0, min<int64_t>(nz_b - y0, L1));
  const int lim_o = (int)max<int64_t>(0, min<int64_t>(nlimit - y0, L1));
  // LDS rows 0..K-1: limbs of a (of b for CM_SPECTRUM); rows K..2K-1: limbs of b
  // (CM_PRODUCT only)
  constexpr bool one = MODE != CM_PRODUCT;
  constexpr int rows = one ? K : K2;
  constexpr int src0 = MODE == CM_SPECTRUM ? K : 0;
  staged<8, uint32_t>(rows << logL1, [&](int idx) {
    const int j = src0 + (idx >> logL1), e = idx & (L1 - 1);
    return e < (j < K ? lim_a : lim_b) ? base[(j << logL) + e] : 0u;
  }, [&](int idx, uint32_t v) { s[(idx >> logL1) * RS + (idx & (L1 - 1))] = v; });
  __syncthreads();
  if constexpr (CLOGL1 >= 0)
    lds_dif_c<CShape<(one ? LOGK : LOGK + 1), (CLOGL1 >= 0 ? CLOGL1 : 1), (1 << (CLOGL1 >= 0 ? CLOGL1 : 1)) + 1, 1>>(
        s, pr.hf, p);
  else
    lds_dif(s, LdsShape{one ? LOGK : LOGK + 1, logL1, RS, 1, 0, 0}, pr.hf, p);
  if constexpr (MODE == CM_SPECTRUM) {
    // b's 2K spectra per position replace its limbs (this block's positions, all read)
    for (int e = threadIdx.x; e < L1; e += BLOCK) {
      uint32_t x[K2];
#pragma unroll
      for (int j = 0; j < K; ++j) x[j] = s[j * RS + e];
      reg_dif<LOGK>(x, pr.hf, p);
#pragma unroll
      for (int j = 0; j < K2; ++j) base[j * L32 + e] = x[j];
    }
    return;
  }
  if constexpr (one) {
    // one forward transform per column, times itself or b's stored spectrum
    const uint32_t *sb = spec + (int64_t)k * K2 * L + rb * L1;
    for (int e = threadIdx.x; e < L1; e += BLOCK) {
      uint32_t a[K2];
#pragma unroll
      for (int j = 0; j < K; ++j) a[j] = s[j * RS + e];
      reg_dif<LOGK>(a, pr.hf, p);
      if constexpr (MODE == CM_SQUARE) {
#pragma unroll
        for (int j = 0; j < K2; ++j) a[j] = mont_mul_lz(a[j], a[j], p, pr.pinv);
      } else {
#pragma unroll
        for (int j = 0; j < K2; ++j)
          a[j] = mont_mul_lz(a[j], sb[j * L32 + e], p, pr.pinv);
      }
      reg_dit<LOGK>(a, pr.hi, p);
#pragma unroll
      for (int j = 0; j < K2; ++j) s[j * RS + e] = a[j];
    }
  }
  if constexpr (!one) for (int e = threadIdx.x; e < L1; e += BLOCK) {
    // the column of a is transformed and parked back in LDS (this thread owns column e)
    // before b is transformed, so that at most 3K values are live in registers
    uint32_t b[K2];
#pragma unroll
    for (int j = 0; j < K; ++j) b[j] = s[(K + j) * RS + e];
    {
      uint32_t a[K2];
#pragma unroll
      for (int j = 0; j < K; ++j) a[j] = s[j * RS + e];
      reg_dif<LOGK>(a, pr.hf, p);
#pragma unroll
      for (int j = 0; j < K2; ++j) s[j * RS + e] = a[j];
    }
    reg_dif<LOGK>(b, pr.hf, p);
#pragma unroll
    for (int j = 0; j < K2; ++j) b[j] = mont_mul_lz(s[j * RS + e], b[j], p, pr.pinv);
    reg_dit<LOGK>(b, pr.hi, p);
#pragma unroll
    for (int j = 0; j < K2; ++j) s[j * RS + e] = b[j];
  }
  __syncthreads();
  if constexpr (CLOGL1 >= 0)
    lds_dit_c<CShape<LOGK + 1, (CLOGL1 >= 0 ? CLOGL1 : 1), (1 << (CLOGL1 >= 0 ? CLOGL1 : 1)) + 1, 1>>(
        s, pr.hi, p);
  else
    lds_dit(s, LdsShape{LOGK + 1, logL1, RS, 1, 0, 0}, pr.hi, p);
  staged<8, uint32_t>(K2 << logL1, [&](int idx) {
    return s[(idx >> logL1) * RS + (idx & (L1 - 1))];
  }, [&](int idx, uint32_t v) {
    const int j = idx >> logL1, e = idx & (L1 - 1);
    if (e < lim_o) base[(j << logL) + e] = v;
  });
}

// ------------------------------------------------------------------------------------
// The same convolutions for larger K (32), one K-point half of each 2K-point
// x-transform at a time in registers.  A zero-padded column's first DIF stage is the
// twist (upper half = lower half times theta^j), after which the two halves are
// independent K-point DIFs; the inverse is two K-point DITs and a joining stage that
// applies theta^-j.  Each thread owns one column of the LDS tile, so halves are parked
// there between steps; at most two halves are live in registers.
// ------------------------------------------------------------------------------------
// Twiddle tables read through the constant address space: the indices are the same for
// every lane, so the loads can be scalar and the twiddles need no vector registers.
typedef const __attribute__((address_space(4))) uint64_t *ctw_ptr;
__device__ __forceinline__ uint2 ctw(ctw_ptr t, int i) {
  const uint64_t w = t[i];   // (w, Shoup companion) as one 64-bit word
  return make_uint2((uint32_t)w, (uint32_t)(w >> 32));
}

template <int LOGN>
__device__ __forceinline__ void reg_half_dif(uint32_t (&x)[1 << LOGN], ctw_ptr tw, uint32_t p) {
  constexpr int N = 1 << LOGN;
#pragma unroll
  for (int h = N / 2; h >= 1; h >>= 1) {
#pragma unroll
    for (int blk = 0; blk < N; blk += 2 * h) {
#pragma unroll
      for (int j = 0; j < h; ++j) {
        const uint32_t u = x[blk + j], v = x[blk + j + h];
        x[blk + j] = add_lz(u, v, p);
        x[blk + j + h] = j ? mul_shoup_lz(u - v + 2 * p, ctw(tw, h + j), p) : sub_lz(u, v, p);
      }
    }
  }
}

template <int LOGN>
__device__ __forceinline__ void reg_half_dit(uint32_t (&x)[1 << LOGN], ctw_ptr tw, uint32_t p) {
  constexpr int N = 1 << LOGN;
#pragma unroll
  for (int h = 1; h < N; h <<= 1) {
#pragma unroll
    for (int blk = 0; blk < N; blk += 2 * h) {
#pragma unroll
      for (int j = 0; j < h; ++j) {
        const uint32_t u = x[blk + j];
        const uint32_t v = j ? mul_shoup_lz(x[blk + j + h], ctw(tw, h + j), p) : x[blk + j + h];
        x[blk + j] = add_lz(u, v, p);
        x[blk + j + h] = sub_lz(u, v, p);
      }
    }
  }
}

// CLOGL1 >= 0: the inner factor L1 = 2^CLOGL1 fixed at compile time (== logL1_rt).
template <int LOGK, int MODE, int CLOGL1 = -1>
__device__ void body_convolve_split(uint32_t *s, int64_t bid, uint32_t *__restrict__ X, int64_t L,
                                    int32_t logL1_rt, int64_t nz_a, int64_t nz_b, int64_t nlimit,
                                    const PrimeDev *__restrict__ primes,
                                    const PlanDev *__restrict__ pd,
                                    const uint32_t *__restrict__ spec) {
  constexpr int K = 1 << LOGK, K2 = 2 * K;
  const int logL1 = CLOGL1 >= 0 ? CLOGL1 : logL1_rt;
  const int L1 = 1 << logL1, RS = L1 + 1;
  const int64_t nrb = L >> logL1;   // a power of two: the block index splits by shifts
  const int k = (int)(bid >> __builtin_ctzll((unsigned long long)nrb));
  const int64_t rb = bid & (nrb - 1);
  const PrimeDev pr = primes[k];
  const uint32_t p = pr.p;
  uint32_t *base = X + (int64_t)k * K2 * L + rb * L1;
  const int64_t y0 = rb * L1;
  const int L32 = (int)L;   // 2K rows of at most 2^21 words: 32-bit row offsets
  const int logL = __builtin_ctzll((unsigned long long)L);
  // rows are read below nz_a / nz_b and written below nlimit: as positions in the block
  const int lim_a = (int)max<int64_t>(0, min<int64_t>(nz_a - y0, L1));
  const int lim_b = (int)max<int64_t>(0, min<int64_t>(nz_b - y0, L1));
  const int lim_o = (int)max<int64_t>(0, min<int64_t>(nlimit - y0, L1));
  constexpr bool one = MODE != CM_PRODUCT;
  constexpr int rows = one ? K : K2;
  constexpr int src0 = MODE == CM_SPECTRUM ? K : 0;
  staged<8, uint32_t>(rows << logL1, [&](int idx) {
    const int j = src0 + (idx >> logL1), e = idx & (L1 - 1);
    return e < (j < K ? lim_a : lim_b) ? base[(j << logL) + e] : 0u;
  }, [&](int idx, uint32_t v) { s[(idx >> logL1) * RS + (idx & (L1 - 1))] = v; });
  __syncthreads();
  if constexpr (CLOGL1 >= 0)
    lds_dif_c<CShape<(one ? LOGK : LOGK + 1), (CLOGL1 >= 0 ? CLOGL1 : 1), (1 << (CLOGL1 >= 0 ? CLOGL1 : 1)) + 1, 1>>(
        s, pr.hf, p);
  else
    lds_dif(s, LdsShape{one ? LOGK : LOGK + 1, logL1, RS, 1, 0, 0}, pr.hf, p);
  ctw_ptr hf = (ctw_ptr)(const void *)pr.hf;
  ctw_ptr hi = (ctw_ptr)(const void *)pr.hi;
  // the twisted half: x_j theta^j, then its K-point DIF (rows K..2K-1 of the spectrum)
  auto twisted = [&](uint32_t (&x)[K]) {
#pragma unroll
    for (int j = 1; j < K; ++j) x[j] = mul_shoup_lz(x[j], ctw(hf, K + j), p);
    reg_half_dif<LOGK>(x, hf, p);
  };
  if constexpr (MODE == CM_SPECTRUM) {
    for (int e = threadIdx.x; e < L1; e += BLOCK) {
      uint32_t x[K];
#pragma unroll
      for (int j = 0; j < K; ++j) x[j] = s[j * RS + e];
      twisted(x);
#pragma unroll
      for (int j = 0; j < K; ++j) base[(K + j) * L32 + e] = x[j];
#pragma unroll
      for (int j = 0; j < K; ++j) x[j] = s[j * RS + e];
      reg_half_dif<LOGK>(x, hf, p);
#pragma unroll
      for (int j = 0; j < K; ++j) base[j * L32 + e] = x[j];
    }
    return;
  }
  const uint32_t *sb = spec + (int64_t)k * K2 * L + rb * L1;
  for (int e = threadIdx.x; e < L1; e += BLOCK) {
    uint32_t x[K];
    if constexpr (MODE == CM_PRODUCT) {
      uint32_t b[K];
#pragma unroll
      for (int j = 0; j < K; ++j) b[j] = s[(K + j) * RS + e];
      // a: twisted half over b's limb rows (b is in registers), then the plain half
#pragma unroll
      for (int j = 0; j < K; ++j) x[j] = s[j * RS + e];
      twisted(x);
#pragma unroll
      for (int j = 0; j < K; ++j) s[(K + j) * RS + e] = x[j];
#pragma unroll
      for (int j = 0; j < K; ++j) x[j] = s[j * RS + e];
      reg_half_dif<LOGK>(x, hf, p);
#pragma unroll
      for (int j = 0; j < K; ++j) s[j * RS + e] = x[j];
      // b: each half times a's, the product replacing a's spectrum
#pragma unroll
      for (int j = 0; j < K; ++j) x[j] = b[j];
      twisted(x);
#pragma unroll
      for (int j = 0; j < K; ++j)
        s[(K + j) * RS + e] = mont_mul_lz(s[(K + j) * RS + e], x[j], p, pr.pinv);
      reg_half_dif<LOGK>(b, hf, p);
#pragma unroll
      for (int j = 0; j < K; ++j) s[j * RS + e] = mont_mul_lz(s[j * RS + e], b[j], p, pr.pinv);
    } else {
      // one operand transformed once: times itself, or times b's stored spectra
#pragma unroll
      for (int j = 0; j < K; ++j) x[j] = s[j * RS + e];
      twisted(x);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const uint32_t f = MODE == CM_SQUARE ? x[j] : sb[(K + j) * L32 + e];
        x[j] = mont_mul_lz(x[j], f, p, pr.pinv);
      }
      uint32_t t[K];
#pragma unroll
      for (int j = 0; j < K; ++j) t[j] = s[j * RS + e];
#pragma unroll
      for (int j = 0; j < K; ++j) s[(K + j) * RS + e] = x[j];
      reg_half_dif<LOGK>(t, hf, p);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const uint32_t f = MODE == CM_SQUARE ? t[j] : sb[j * L32 + e];
        s[j * RS + e] = mont_mul_lz(t[j], f, p, pr.pinv);
      }
    }
    // inverse: the two K-point DITs, then the joining stage with theta^-j
#pragma unroll
    for (int j = 0; j < K; ++j) x[j] = s[j * RS + e];
    reg_half_dit<LOGK>(x, hi, p);
    {
      uint32_t y[K];
#pragma unroll
      for (int j = 0; j < K; ++j) y[j] = s[(K + j) * RS + e];
      reg_half_dit<LOGK>(y, hi, p);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const uint32_t u = x[j];
        const uint32_t v = j ? mul_shoup_lz(y[j], ctw(hi, K + j), p) : y[j];
        s[j * RS + e] = add_lz(u, v, p);
        s[(K + j) * RS + e] = sub_lz(u, v, p);
      }
    }
  }
  __syncthreads();
  if constexpr (CLOGL1 >= 0)
    lds_dit_c<CShape<LOGK + 1, (CLOGL1 >= 0 ? CLOGL1 : 1), (1 << (CLOGL1 >= 0 ? CLOGL1 : 1)) + 1, 1>>(
        s, pr.hi, p);
  else
    lds_dit(s, LdsShape{LOGK + 1, logL1, RS, 1, 0, 0}, pr.hi, p);
  staged<8, uint32_t>(K2 << logL1, [&](int idx) {
    return s[(idx >> logL1) * RS + (idx & (L1 - 1))];
  }, [&](int idx, uint32_t v) {
    const int j = idx >> logL1, e = idx & (L1 - 1);
    if (e < lim_o) base[(j << logL) + e] = v;
  });
}

// ------------------------------------------------------------------------------------
// RecoveringProduct.  For each output coefficient i and each j < 2K-1:
//   c_{i,j} from its np residues by CRT into (-P/2, P/2) (exact because
//   |c_{i,j}| < d K 2^(2M) < P/2 (1 - 2^-12)), as W-word two's complement;
// then c_i = sum_j c_{i,j} 2^(M j) (evaluation at beta = 2^M) by per-word sums of
// shifted windows and a wave-wide carry scan.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int fapply(int code, int y) { return ((code >> (2 * (y + 1))) & 3) - 1; }
__device__ __forceinline__ int fcompose(int g, int f) {   // g after f
  int r = 0;
#pragma unroll
  for (int y = -1; y <= 1; ++y) r |= (fapply(g, fapply(f, y)) + 1) << (2 * (y + 1));
  return r;
}

typedef int crt_i32x4 __attribute__((ext_vector_type(4)));

// The CRT of each c_{i,j} on the int8 matrix cores, added at bit M j into S (np <=
// CRT_MFMA_NP).  c_{i,j} = sum_k y_k (P/p_k) - t P with y_k = u_k - p_k, u_k the lazy
// Shoup product r_k (P/p_k)^{-1} mod p_k in [0, 2 p_k) (so y_k in [-p_k, p_k)), and
// t = round(sum_k y_k / p_k), summed in single precision as round(sum_k u_k / p_k) - np.
// (|c_{i,j}| < P/2 (1 - 2^-12) leaves the rounding of t a margin of 2^-13; the sum's error
// is below 2^-15 for 20 terms below 2: each term's conversion and reciprocal add 2^-23,
// each fused multiply-add rounds its partial sum, below 2 k, to 2^-24.)
// Per wave, rounds of 16 values: value v = lane mod 16,
// and lane group g = lane / 16 holds the terms crt_term(s, g, w) of step s (w < 4): it
// loads and reduces those residues, the four groups add their shares of the quotient sum,
// and the terms' balanced signed bytes form the B operand in registers.  D = A Y with A
// the constants' digit matrix (built on the host in fragment order); its 16-digit tiles T
// give lane group g the digits 4 TN g + 4 T + i of value v.  The lane folds its 4 TN digit
// sums into TN consecutive 32-bit words plus a signed carry, exactly its share of
// c_{i,j}, and adds them, shifted by M j bits, into its row of S (RS words, with room for
// every word a lane group touches; S[-1] exists).  Values past the tile's end add zeros
// to row 0.  With short rows (recover_staged) the terms are formed one value per lane
// and passed to the lane groups through LDS instead.  Each round's residues are loaded two rounds ahead; the first two rounds',
// and the A fragments, before the workgroup's set-up (constants to LDS, S cleared,
// barrier).  cw: per prime (c_k, its Shoup companion, -p_k mod 2^32, 1/p_k as float bits).
template <int NP>
struct CrtMatrix {
  static constexpr int NT = NP + 1;
  static constexpr int NS = (NT + 15) / 16;
  static constexpr int TN = crt_tiles(NP);
  static_assert(NS <= CRT_STEPS && TN <= CRT_TILES, "CRT matrix shape");
  static constexpr int YW = crt_stage_words(NP);
  crt_i32x4 af[TN][NS];
  uint32_t pre[NS][4];                // register form: the next round's residues
  uint32_t pres[NP];                  // staged form: the first value's residues

  // round gr of this wave: values wave 64 + (gr / 4) BLOCK + (gr % 4) 16 + 0..15
  __device__ __forceinline__ static int round_item(int gr, int v) {
    return (threadIdx.x & ~63) + (gr >> 2) * BLOCK + (gr & 3) * 16 + v;
  }
  // the residues of lane group g's terms for one value (zero past the tile)
  __device__ __forceinline__ static void load(uint32_t (&r)[NS][4], const uint32_t *__restrict__ X,
                                              int64_t L, int32_t K, int32_t logTI, int ti,
                                              int64_t i0, int item, int g) {
    const int TI = 1 << logTI;
    const int items = (2 * K - 1) << logTI;
    const bool ok = item < items && (item & (TI - 1)) < ti;
    const int64_t off = (int64_t)(item >> logTI) * L + i0 + (item & (TI - 1));
#pragma unroll
    for (int st = 0; st < NS; ++st)
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int q = crt_term(st, g, w);
        r[st][w] = ok && q < NP ? X[(int64_t)q * 2 * K * L + off] : 0u;
      }
  }

  template <int FORM>
  __device__ __forceinline__ void prefetch(bool staged, const uint32_t *__restrict__ X, int64_t L,
                                           int32_t K, int32_t logTI, int ti, int64_t i0,
                                           const PlanDev *__restrict__ pd) {
    const int lane = threadIdx.x & 63;
    if (FORM == 1 || (FORM < 0 && staged)) {
      const int TI = 1 << logTI;
      const int items = (2 * K - 1) << logTI;
      const int item = threadIdx.x;
      const bool ok = item < items && (item & (TI - 1)) < ti;
      const int64_t off = (int64_t)(item >> logTI) * L + i0 + (item & (TI - 1));
#pragma unroll
      for (int k = 0; k < NP; ++k) pres[k] = ok ? X[(int64_t)k * 2 * K * L + off] : 0u;
    } else if (FORM != 1) {
      load(pre, X, L, K, logTI, ti, i0, round_item(0, lane & 15), lane >> 4);
    }
#pragma unroll
    for (int T = 0; T < TN; ++T)
#pragma unroll
      for (int st = 0; st < NS; ++st) {
        const uint4 q = *reinterpret_cast<const uint4 *>(&pd->crt_afrag[T][st][lane][0]);
        af[T][st] = crt_i32x4{(int)q.x, (int)q.y, (int)q.z, (int)q.w};
      }
  }

  // D = A Y for this round's 16 values (B fragments bw), then each lane's share of
  // c_{i,j} 2^(M j) into row il of S
  __device__ __forceinline__ void product_add(const uint32_t (&bw)[NS][4], uint64_t *S, int32_t RS,
                                              int32_t M, int il, int j, int g) {
    crt_i32x4 acc[TN];
#pragma unroll
    for (int T = 0; T < TN; ++T) acc[T] = crt_i32x4{0, 0, 0, 0};
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const crt_i32x4 bf{(int)bw[st][0], (int)bw[st][1], (int)bw[st][2], (int)bw[st][3]};
#pragma unroll
      for (int T = 0; T < TN; ++T)
        acc[T] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[T][st], bf, acc[T], 0, 0, 0);
    }
    // c_{i,j} 2^(M j) = c_{i,j} 2^s 2^(32 q) with s in 1..32 (q = -1 for j = 0: word -1
    // of a row is the end of the previous row or, for row 0, a spare word, and only
    // receives the zero below the value's first word)
    const int64_t bit = (int64_t)M * j;
    // M j < 2 N, and convert-in's LDS tile keeps N below 2^19 bits: a 32-bit word index
    const int qw = (int)((bit - 1) >> 5);
    const uint32_t rsh = (uint32_t)(32 * (qw + 1) - bit);  // 32 - s, in 0..31
    unsigned long long *Sw =
        reinterpret_cast<unsigned long long *>(S + (int64_t)il * RS + qw + TN * g);
    // the words of sum_i D[4 T + i] 2^(8 i) plus the carry, in 32-bit steps (every
    // digit sum is below 2^21 in magnitude, so t1, t2, t3 fit 31 bits)
    int32_t c = 0;
    uint32_t prev = 0;
#pragma unroll
    for (int T = 0; T < TN; ++T) {
      const int32_t t1 = acc[T][0] + c + (int32_t)((uint32_t)acc[T][1] << 8);
      const int32_t t2 = (t1 >> 16) + acc[T][2];
      const int32_t t3 = t2 + (int32_t)((uint32_t)acc[T][3] << 8);
      const uint32_t wd = __builtin_amdgcn_perm((uint32_t)t3, (uint32_t)t1, 0x05040100u);
      c = t3 >> 16;
      // bits 32 - s .. 63 - s of (wd, prev): the word shifted left by s, with the
      // previous word's top s bits below
      atomicAdd(&Sw[T], (unsigned long long)__builtin_amdgcn_alignbit(wd, prev, rsh));
      prev = wd;
    }
    // the lane's carry out (a signed multiple of 2^(32 TN)) with the last word's top bits
    atomicAdd(&Sw[TN],
              (unsigned long long)((int64_t)(((uint64_t)(int64_t)c << 32) | prev) >> rsh));
  }

  // Staged form: the wave's 64 values' terms go through LDS (Y, YW words per value), one
  // value per lane while the residues are reduced.
  __device__ __forceinline__ void run_staged(uint64_t *S, int32_t RS, uint32_t *Y,
                                             const uint4 *cw, const uint32_t *__restrict__ X,
                                             int64_t L, int32_t K, int32_t M, int32_t logTI,
                                             int ti, int64_t i0) {
    constexpr int CH = 6;             // terms whose constants are read from LDS together
    const int TI = 1 << logTI;
    const int J = 2 * K - 1;
    const int64_t twoK = 2 * (int64_t)K;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, v = lane & 15;
    uint32_t *Yw = Y + wave * 64 * YW;
    const int items = J << logTI;
    for (int base = wave * 64; base < items; base += BLOCK) {   // uniform per wave
      {
        const int item = base + lane;
        const bool ok = item < items && (item & (TI - 1)) < ti;
        const int64_t off = (int64_t)(item >> logTI) * L + i0 + (item & (TI - 1));
        uint32_t y[YW];
        if (base == wave * 64) {
#pragma unroll
          for (int k = 0; k < NP; ++k) y[k] = pres[k];
        } else {
#pragma unroll
          for (int k = 0; k < NP; ++k) y[k] = ok ? X[(int64_t)k * twoK * L + off] : 0u;
        }
        float f = 0.0f;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          if (k % CH == 0) asm volatile("" ::: "memory");   // bounds the constants in flight
          const uint4 c = cw[k];
          const uint32_t u = shoup_neg_lz(y[k], make_uint2(c.x, c.y), c.z);   // [0, 2p)
          f = fmaf((float)u, __uint_as_float(c.w), f);
          // |u - p| < 2^30: the bytes of u - p + 0x80808080 are its balanced digits plus 128
          y[k] = (u + c.z + 0x80808080u) ^ 0x80808080u;
        }
        y[NP] = (uint32_t)(__float2int_rn(f) - NP) & 0xFFu;
#pragma unroll
        for (int k = NP + 1; k < YW; ++k) y[k] = 0;
#pragma unroll
        for (int q = 0; q < YW / 4; ++q)
          *reinterpret_cast<uint4 *>(&Yw[lane * YW + 4 * q]) =
              make_uint4(y[4 * q], y[4 * q + 1], y[4 * q + 2], y[4 * q + 3]);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll 1
      for (int r = 0; r < 4; ++r) {
        const int vi = 16 * r + v;
        const int item = base + vi;
        const bool ok = item < items && (item & (TI - 1)) < ti;
        const int il = ok ? item & (TI - 1) : 0, j = ok ? item >> logTI : 0;
        const uint32_t *yv = Yw + vi * YW;
        uint32_t bw[NS][4];
        {
          uint4 q = make_uint4(0u, 0u, 0u, 0u);
          if (4 * g < YW) q = *reinterpret_cast<const uint4 *>(yv + 4 * g);   // terms 4 g + w
          bw[0][0] = q.x; bw[0][1] = q.y; bw[0][2] = q.z; bw[0][3] = q.w;
        }
#pragma unroll
        for (int st = 1; st < NS; ++st)
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            const int q = crt_term(st, g, w);
            bw[st][w] = q < NT ? yv[q] : 0u;
          }
        product_add(bw, S, RS, M, il, j, g);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
  }

  // Register form: lane group g loads and reduces the residues of its terms for the round's
  // value and builds its share of the B operand in registers.
  __device__ __forceinline__ void run(uint64_t *S, int32_t RS, const uint4 *cw,
                                      const uint32_t *__restrict__ X, int64_t L, int32_t K,
                                      int32_t M, int32_t logTI, int ti, int64_t i0) {
    const int TI = 1 << logTI;
    const int J = 2 * K - 1;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, v = lane & 15;
    const int items = J << logTI;
    // rounds of 16 values; each round's residues are loaded one round ahead
    const int nbase = items > wave * 64 ? (items - wave * 64 + BLOCK - 1) / BLOCK : 0;
    const int nr = 4 * nbase;
#pragma unroll 1
    for (int gr = 0; gr < nr; ++gr) {
        const int item = round_item(gr, v);
        const bool ok = item < items && (item & (TI - 1)) < ti;
        const int il = ok ? item & (TI - 1) : 0, j = ok ? item >> logTI : 0;
        uint32_t res[NS][4];
#pragma unroll
        for (int st = 0; st < NS; ++st)
#pragma unroll
          for (int w = 0; w < 4; ++w) res[st][w] = pre[st][w];
        if (gr + 1 < nr) load(pre, X, L, K, logTI, ti, i0, round_item(gr + 1, v), g);
        uint32_t bw[NS][4];
        float f = 0.0f;
#pragma unroll
        for (int st = 0; st < NS; ++st)
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            const int q = crt_term(st, g, w);
            bw[st][w] = 0u;
            if (q < NP) {
              const uint4 c = cw[q];
              const uint32_t u = shoup_neg_lz(res[st][w], make_uint2(c.x, c.y), c.z);
              f = fmaf((float)u, __uint_as_float(c.w), f);
              // |u - p| < 2^30: the bytes of u - p + 0x80808080 are its balanced digits
              // plus 128
              bw[st][w] = (u + c.z + 0x80808080u) ^ 0x80808080u;
            }
          }
        // the four groups' shares (every lane adds them in the same pairs, so all agree)
        f += __shfl_xor(f, 16, 64);
        f += __shfl_xor(f, 32, 64);
        const uint32_t tb = (uint32_t)(__float2int_rn(f) - NP) & 0xFFu;
#pragma unroll
        for (int st = 0; st < NS; ++st)
#pragma unroll
          for (int w = 0; w < 4; ++w)
            if (crt_term(st, g, w) == NP) bw[st][w] = tb;
        product_add(bw, S, RS, M, il, j, g);
    }
  }
};

// NP = np exactly and W = NP words per CRT value (32 NP >= log2 P + 1 since every
// prime is below 2^30).  Per workgroup: TI consecutive coefficients; S holds their
// output words as 64-bit partial sums.  FORM: the matrix form's staged (1) or register
// (0) variant fixed at compile time, or chosen at run time by recover_staged (-1).
template <int NP, int FORM = -1>
__device__ void body_recover(uint64_t *S, int64_t tile_id, const uint32_t *__restrict__ X,
                             int64_t L, int32_t K, int32_t M, int64_t nout, int32_t nw32,
                             int32_t wc, int32_t logTI, const PrimeDev *__restrict__ primes,
                             const PlanDev *__restrict__ pd, uint64_t *__restrict__ out) {
  constexpr int W = NP;
  constexpr int NT = NP + 1;          // terms of each word: the np residues, then t
  constexpr int NPE = (NT + 1) & ~1;  // terms padded to a pair
  constexpr bool MF = NP <= CRT_MFMA_NP;
  const int TI = 1 << logTI;
  const int J = 2 * K - 1;            // c_{i,2K-1} = 0
  const int64_t twoK = 2 * (int64_t)K;
  const int64_t i0 = tile_id << logTI;
  if (i0 >= nout) return;
  const int ti = (int)min<int64_t>(TI, nout - i0);
  // S: TI rows of RS partial sums (nw32 output words and, in the matrix form, room for
  // every word the CRT's lane groups touch), then either per prime (c_k Shoup pair, -p_k,
  // 1/p_k in single precision) (matrix form), or, as [u][k]
  // (W x NPE words), P/p_k for k < np and, at k = np, 2^(32 W) - P (P is odd, so its
  // negation is ~P + 1 = -P[0], ~P[1], ...), then per prime (c_k Shoup pair, p_k) and 1/p_k
  CrtMatrix<MF ? NP : 1> cm;
  const bool staged = FORM >= 0 ? FORM == 1 : recover_staged(NP, K, M, nw32, logTI);
  if constexpr (MF) cm.template prefetch<FORM>(staged, X, L, K, logTI, ti, i0, pd);
  const int RS = recover_row_words(NP, K, M, nw32);
  uint64_t *const S0 = S;             // a spare word, then the rows
  S = S0 + 1;
  uint32_t *cq = reinterpret_cast<uint32_t *>(S0 + ((((int64_t)RS << logTI) + 2) & ~(int64_t)1));
  uint32_t *ci = cq + (MF ? (staged ? BLOCK * crt_stage_words(NP) : 0) : NPE * W);
  double *cr = reinterpret_cast<double *>(ci + ((3 * NP + 1) & ~1));
  if constexpr (MF) {
    uint4 *cw = reinterpret_cast<uint4 *>(ci);
    for (int idx = threadIdx.x; idx < NP; idx += BLOCK)
      cw[idx] = make_uint4(pd->crt_inv[idx].x, pd->crt_inv[idx].y, 0u - primes[idx].p,
                           __float_as_uint((float)pd->crt_rcp[idx]));
  } else {
    for (int idx = threadIdx.x; idx < NPE * W; idx += BLOCK) {
      const int u = idx / NPE, kk = idx - u * NPE;
      cq[idx] = kk < NP ? pd->crt_q[kk][u]
                        : kk == NP ? (u == 0 ? 0u - pd->crt_p[0] : ~pd->crt_p[u]) : 0u;
    }
    for (int idx = threadIdx.x; idx < NP; idx += BLOCK) {
      ci[3 * idx] = pd->crt_inv[idx].x;
      ci[3 * idx + 1] = pd->crt_inv[idx].y;
      ci[3 * idx + 2] = primes[idx].p;
      cr[idx] = pd->crt_rcp[idx];
    }
  }
  for (int idx = threadIdx.x; idx < ti * RS; idx += BLOCK) S[idx] = 0;
  __syncthreads();
  if constexpr (MF) {
    if (FORM != 0 && staged)
      cm.run_staged(S, RS, cq, reinterpret_cast<const uint4 *>(ci), X, L, K, M, logTI, ti, i0);
    else if (FORM != 1)
      cm.run(S, RS, reinterpret_cast<const uint4 *>(ci), X, L, K, M, logTI, ti, i0);
  } else {
  // ---- CRT of each c_{i,j}, then add c_{i,j} 2^(M j) into the output words ----
  for (int idx = threadIdx.x; idx < (J << logTI); idx += BLOCK) {
    const int il = idx & (TI - 1), j = idx >> logTI;
    if (il >= ti) continue;
    const int64_t i = i0 + il;
    uint32_t cc[NPE];
#pragma unroll
    for (int k = 0; k < NP; ++k) cc[k] = X[((int64_t)k * twoK + j) * L + i];
    double f = 0.0;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      cc[k] = mul_shoup(cc[k], make_uint2(ci[3 * k], ci[3 * k + 1]), ci[3 * k + 2]);
      f += (double)cc[k] * cr[k];
    }
    // c_{i,j} = sum_k c_k (P/p_k) - t P, where sum_k c_k P/p_k = c + t P with |c| < P/2,
    // so t = round(sum_k c_k / p_k).  Adding t (2^(32 W) - P) instead of subtracting t P
    // gives c + t 2^(32 W), whose low W words are c in two's complement: every term is
    // an unsigned product.  The value is produced one 32-bit word u at a time (column
    // sums of the products over 64 bits, the carries out of bit 63 counted in a third
    // word, the bits above the word carried into the next one) and its shifted digits
    // are added into the output words at once.
    cc[NP] = (uint32_t)__double2int_rn(f);
    if (NPE > NT) cc[NPE - 1] = 0;
    const int64_t bit = (int64_t)M * j;
    // M j < 2 N, and convert-in's LDS tile keeps N below 2^19 bits: a 32-bit word index
    const int q0 = (int)(bit >> 5);
    const int sh = (int)(bit & 31);
    uint64_t *Si = S + (int64_t)il * RS;
    uint64_t lo = 0;
    uint32_t prev = 0;
#pragma unroll
    for (int u = 0; u < W; ++u) {
      uint32_t hi = 0;
#pragma unroll
      for (int k = 0; k < NPE; k += 2) {
        const uint2 qq = *reinterpret_cast<const uint2 *>(cq + u * NPE + k);
        // the first term cannot carry out of 64 bits: lo holds below 2^37 (the carry
        // from word u - 1) and the product is below 2^63
        if (k == 0) lo += (uint64_t)cc[0] * qq.x;
        else mac_carry(lo, hi, cc[k], qq.x);
        if (k + 1 < NT) mac_carry(lo, hi, cc[k + 1], qq.y);
      }
      const uint32_t wd = (uint32_t)lo;                 // word u of c_{i,j}, two's complement
      lo = (lo >> 32) | ((uint64_t)hi << 32);           // carry into word u + 1
      const uint32_t dgt = sh ? ((wd << sh) | (prev >> (32 - sh))) : wd;
      prev = wd;
      if (q0 + u < nw32 && dgt) atomicAdd((unsigned long long *)&Si[q0 + u], (unsigned long long)dgt);
    }
    const int64_t top = sh ? (int64_t)((int32_t)prev >> (32 - sh)) : -(int64_t)(prev >> 31);
    if (q0 + W < nw32 && top) atomicAdd((unsigned long long *)&Si[q0 + W], (unsigned long long)top);
  }
  }
  __syncthreads();
  // ---- carries ----
  if (nw32 <= 8 * TI) {
    // short outputs: one lane per coefficient, its words in order (eight LDS reads in
    // flight ahead of the carry chain)
    for (int il = threadIdx.x; il < ti; il += BLOCK) {
      uint64_t *Si = S + (int64_t)il * RS;
      int64_t carry = 0;
      for (int w0 = 0; w0 < nw32; w0 += 8) {
        uint64_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = w0 + u < nw32 ? Si[w0 + u] : 0ull;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int64_t tsum = (int64_t)v[u] + carry;
          if (w0 + u < nw32) Si[w0 + u] = (uint32_t)tsum;
          carry = tsum >> 32;
        }
      }
      const uint64_t fill = ((int32_t)(uint32_t)Si[nw32 - 1] < 0) ? ~0ull : 0ull;
      uint64_t *o = out + (i0 + il) * (int64_t)wc;
      for (int u = 0; u < wc; ++u)
        o[u] = (2 * u + 1 < nw32) ? ((Si[2 * u] & 0xFFFFFFFFull) | (Si[2 * u + 1] << 32)) : fill;
    }
    return;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (nw32 <= 512) {
    // outputs of at most 512 words: one wave per coefficient, an even number (at most 8)
    // of consecutive words per lane held in registers, so that each lane also writes its
    // own output words
    const int per = 2 * ((nw32 + 127) >> 7);
    const int w_lo = min(lane * per, nw32), w_hi = min(w_lo + per, nw32);
    for (int il = wave; il < ti; il += BLOCK / 64) {
      const uint64_t *Si = S + (int64_t)il * RS;
      uint32_t wv[8];
      int64_t carry = 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool in = u < per && w_lo + u < w_hi;
        const int64_t tsum = (in ? (int64_t)Si[w_lo + u] : 0) + carry;
        wv[u] = in ? (uint32_t)tsum : 0u;
        if (in) carry = tsum >> 32;
      }
      // the lane below's carry, then this lane's carry out x in {-1, 0, 1}
      int64_t x = __shfl_up(carry, 1, 64);
      if (lane == 0) x = 0;
      bool allz = true, allo = true;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (u < per && w_lo + u < w_hi) {
          const int64_t tsum = (int64_t)wv[u] + x;
          wv[u] = (uint32_t)tsum;
          x = tsum >> 32;
          allz = allz && wv[u] == 0u;
          allo = allo && wv[u] == 0xFFFFFFFFu;
        }
      }
      // as in the general case below: only when some lane passes a carry on does it
      // ripple through runs of all-zero or all-one lanes
      if (__any(w_lo < w_hi && w_hi < nw32 && x != 0)) {
        int code;
        if (w_lo >= w_hi) {
          code = (0) | (1 << 2) | (2 << 4);
        } else {
          const int gg = (int)x;
          const int fm = gg + (allz ? -1 : 0), f0 = gg, fp = gg + (allo ? 1 : 0);
          code = (fm + 1) | ((f0 + 1) << 2) | ((fp + 1) << 4);
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const int other = __shfl_up(code, off, 64);
          if (lane >= off) code = fcompose(code, other);
        }
        const int prevc = __shfl_up(code, 1, 64);
        int y = lane == 0 ? 0 : fapply(prevc, 0);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (u < per && w_lo + u < w_hi) {
            const int64_t tsum = (int64_t)wv[u] + y;
            wv[u] = (uint32_t)tsum;
            y = (int)(tsum >> 32);
          }
        }
      }
      // the top word's sign fills the output words above the product's width
      const int top_lane = (nw32 - 1) / per;
      uint32_t topv = 0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (w_lo + u == nw32 - 1) topv = wv[u];
      topv = __shfl(topv, top_lane, 64);
      const uint64_t fill = (int32_t)topv < 0 ? ~0ull : 0ull;
      uint64_t *o = out + (i0 + il) * (int64_t)wc;
#pragma unroll
      for (int u = 0; u < 8; u += 2)
        if (u < per && w_lo + u < w_hi && (w_lo >> 1) + (u >> 1) < wc)
          o[(w_lo >> 1) + (u >> 1)] = (uint64_t)wv[u] | ((uint64_t)wv[u + 1] << 32);
      for (int u = (nw32 >> 1) + lane; u < wc; u += 64) o[u] = fill;
    }
    return;
  }
  // long outputs: one wave per coefficient
  const int per = (nw32 + 63) >> 6;
  const int w_lo = min(lane * per, nw32), w_hi = min(w_lo + per, nw32);
  for (int il = wave; il < ti; il += BLOCK / 64) {
    uint64_t *Si = S + (int64_t)il * RS;
    int64_t carry = 0;
    for (int w = w_lo; w < w_hi; ++w) {
      const int64_t tsum = (int64_t)Si[w] + carry;
      Si[w] = (uint32_t)tsum;
      carry = tsum >> 32;
    }
    // pass the local carry to the next lane and normalise
    int64_t cin = __shfl_up(carry, 1, 64);
    if (lane == 0) cin = 0;
    int64_t x = cin;
    bool allz = true, allo = true;
    for (int w = w_lo; w < w_hi; ++w) {
      const int64_t tsum = (int64_t)Si[w] + x;
      Si[w] = (uint32_t)tsum;
      x = tsum >> 32;
      allz = allz && (uint32_t)tsum == 0u;
      allo = allo && (uint32_t)tsum == 0xFFFFFFFFu;
    }
    // x is this lane's carry out in {-1, 0, 1} once its carry in is the lane below's
    // first-level carry.  When every lane that has a lane above it gives 0, no carry
    // moves further and the words are final (the top lane's carry out is the sign and
    // leaves the output).  Otherwise the carries ripple through runs of all-zero or
    // all-one lanes, which the scan resolves.
    if (__any(w_lo < w_hi && w_hi < nw32 && x != 0)) {
      int code;
      if (w_lo >= w_hi) {
        code = (0) | (1 << 2) | (2 << 4);               // identity
      } else {
        const int g = (int)x;                           // in {-1, 0, 1}
        const int fm = g + (allz ? -1 : 0), f0 = g, fp = g + (allo ? 1 : 0);
        code = (fm + 1) | ((f0 + 1) << 2) | ((fp + 1) << 4);
      }
      // inclusive scan of carry-transfer functions across the wave
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int other = __shfl_up(code, off, 64);
        if (lane >= off) code = fcompose(code, other);
      }
      const int prevc = __shfl_up(code, 1, 64);
      int y = lane == 0 ? 0 : fapply(prevc, 0);
      for (int w = w_lo; w < w_hi && y != 0; ++w) {
        const int64_t tsum = (int64_t)Si[w] + y;
        Si[w] = (uint32_t)tsum;
        y = (int)(tsum >> 32);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const uint64_t fill = ((int32_t)(uint32_t)Si[nw32 - 1] < 0) ? ~0ull : 0ull;
    uint64_t *o = out + (i0 + il) * (int64_t)wc;
    for (int u = lane; u < wc; u += 64)
      o[u] = (2 * u + 1 < nw32) ? ((Si[2 * u] & 0xFFFFFFFFull) | (Si[2 * u + 1] << 32)) : fill;
  }
}

}  // namespace zpm
