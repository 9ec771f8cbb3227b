// 64-bit machine-word prime variant (Section 4: one, two or three machine-word Fourier
// primes combined by CRT): host number theory, planner, gfx950 kernels, launcher.
//
// Pipeline of one product (all on the caller's stream):
//   k64_convert      limbs of M bits (Section 2, BivariateRepresentation) reduced mod each
//                    prime, into np x 2K columns of length L (a: 0..K-1, b: K..2K-1);
//   k64_ypass        the y-transform as strided passes of at most 2^9 points, outermost
//                    first, each followed by the four-step twiddles (rows >= d are read
//                    as zero by the first pass);
//   k64_xconv        per y-frequency: 2K-point forward transforms of the zero-padded limb
//                    rows of a and b (the even frequencies are the cyclic convolution's,
//                    the odd ones the theta-twisted negacyclic convolution's, Section 2.1),
//                    pointwise product with the 1/(2K L) scale, 2K-point inverse, which
//                    gives c_{i,j} for j < 2K - 1 directly (Eq. CplusandCminus);
//   k64_ypass        inverse y passes, innermost first (rows >= da + db - 1 not written);
//   k64_recover      Garner's CRT into (-P/2, P/2), then c_i = sum_j c_{i,j} 2^(M j) with
//                    a wave-wide carry scan (RecoveringProduct, Section 2.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/zpm.h"
#include "ctx.hpp"
#include "p64.hpp"
#include "plan.hpp"
#include "profiler.hpp"
#include "stages.hpp"

namespace zpm {

using u128 = unsigned __int128;

// ------------------------------------------------------------------------------------
// host number theory
// ------------------------------------------------------------------------------------
static uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)((u128)a * b % p); }

static uint64_t powmod64(uint64_t a, uint64_t e, uint64_t p) {
  uint64_t r = 1 % p, x = a % p;
  while (e) {
    if (e & 1) r = mulmod64(r, x, p);
    x = mulmod64(x, x, p);
    e >>= 1;
  }
  return r;
}

static uint64_t invmod64(uint64_t a, uint64_t p) { return powmod64(a, p - 2, p); }   // p prime

// Miller-Rabin with the first twelve primes as bases: deterministic below 3.3e24.
static bool is_prime64(uint64_t n) {
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t q : bases)
    if (n % q == 0) return n == q;
  uint64_t d = n - 1;
  int s = 0;
  while (!(d & 1)) { d >>= 1; ++s; }
  for (uint64_t a : bases) {
    uint64_t x = powmod64(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s && comp; ++r) {
      x = mulmod64(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

static W64 shoup64(uint64_t w, uint64_t p) { return W64{w, (uint64_t)(((u128)w << 64) / p)}; }

const Prime64Host *prime64_table() {
  static Prime64Host tab[MAXNP64];
  static std::once_flag once;
  std::call_once(once, [] {
    const uint64_t step = 1ull << LOG2_ROOT64;
    int n = 0;
    for (uint64_t c = ((1ull << 62) - 1) / step; n < MAXNP64 && c > 0; --c) {
      const uint64_t p = c * step + 1;
      if (!is_prime64(p)) continue;
      // for a quadratic non-residue g, g^((p-1)/2^21) has order exactly 2^21
      for (uint64_t g = 2;; ++g) {
        if (powmod64(g, (p - 1) / 2, p) == p - 1) {
          tab[n].root = powmod64(g, (p - 1) >> LOG2_ROOT64, p);
          break;
        }
      }
      tab[n++].p = p;
    }
  });
  return tab;
}

// little-endian multiword helpers (4 x 64 bits)
static void mw4_mul_small(uint64_t *x, uint64_t m) {
  uint64_t carry = 0;
  for (int i = 0; i < 4; ++i) {
    const u128 t = (u128)x[i] * m + carry;
    x[i] = (uint64_t)t;
    carry = (uint64_t)(t >> 64);
  }
}
static int mw4_bitlen(const uint64_t *x) {
  for (int i = 3; i >= 0; --i)
    if (x[i]) return 64 * i + 64 - __builtin_clzll(x[i]);
  return 0;
}
static void prime_product(int np, uint64_t *P) {
  P[0] = 1; P[1] = P[2] = P[3] = 0;
  for (int k = 0; k < np; ++k) mw4_mul_small(P, prime64_table()[k].p);
}

// prod p_k > 4 d K 2^(2M) (the bound of Section 2.2 with the prime product as modulus)
static bool primes64_cover(int np, int64_t d, int64_t K, int32_t M) {
  uint64_t P[4];
  prime_product(np, P);
  const u128 dk = (u128)(uint64_t)d * (uint64_t)K;
  const int shift = 2 * M + 2;
  uint64_t R[4] = {0, 0, 0, 0};
  const int w = shift / 64, b = shift % 64;
  if (w >= 4) return false;
  const uint64_t lo = (uint64_t)dk, hi = (uint64_t)(dk >> 64);
  uint64_t parts[3] = {lo << b, b ? (lo >> (64 - b)) | (hi << b) : hi, b ? hi >> (64 - b) : 0};
  for (int i = 0; i < 3; ++i) {
    if (!parts[i]) continue;
    if (w + i >= 4) return false;
    R[w + i] = parts[i];
  }
  for (int i = 3; i >= 0; --i)
    if (P[i] != R[i]) return P[i] > R[i];
  return false;
}

static int clog2(int64_t x) {
  int r = 0;
  while (((int64_t)1 << r) < x) ++r;
  return r;
}

// ------------------------------------------------------------------------------------
// planner
// ------------------------------------------------------------------------------------
static double cost64(const Plan64 &pl) {
  const double K = pl.K, L = std::ldexp(1.0, pl.logL), np = pl.np;
  const double cols = 2.0 * K;
  // radix-2 butterflies: forward y on 2K columns, inverse y on 2K, three 2K-point
  // x-transforms per y position
  const double bfly = np * (cols * L / 2 * pl.logL * 2 + 3.0 * L * K * std::log2(2 * K));
  double ops = bfly * 40.0 + np * cols * L * 45.0;
  ops += (double)pl.nout * (2 * K - 1) * (np * np * 30.0 + pl.DIG * 12.0);
  double bytes = 8.0 * np * cols * L * 2.0 * (2 * pl.npass + 1);
  bytes += 8.0 * (pl.da * ((pl.Na + 63) / 64) + pl.db * ((pl.Nb + 63) / 64) +
                  pl.nout * ((pl.nout_bits + 63) / 64));
  return ops / 39.3e12 / 0.6 + bytes / 5.0e12 + 4e-6 * (4 + 2 * pl.npass);
}

bool make_plan64(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K_force, int32_t np_force,
                 Plan64 &out, const char **why) {
  static const char *dummy;
  if (!why) why = &dummy;
  *why = nullptr;
  if (da < 1 || db < 1 || Na < 1 || Nb < 1) { *why = "sizes must be positive"; return false; }
  if (np_force < 0 || np_force > MAXNP64) { *why = "np must be 1, 2 or 3"; return false; }
  const int64_t nout = da + db - 1;
  const int logL = clog2(nout);
  if (logL > LOG2_ROOT64) { *why = "da + db - 1 exceeds 2^21"; return false; }
  const int32_t N = std::max(std::max(Na, Nb), 2);
  const int64_t d = std::max(da, db);
  bool found = false;
  Plan64 best;
  for (int logK = 1; (1 << logK) <= K_MAX64; ++logK) {
    const int32_t K = 1 << logK;
    if (K_force && K != K_force) continue;
    if (!K_force && K > 2 * (int64_t)N) break;
    Plan64 pl;
    std::memset(&pl, 0, sizeof(pl));
    pl.da = da; pl.db = db; pl.Na = Na; pl.Nb = Nb; pl.nout = nout;
    pl.nout_bits = out_bits(da, Na, db, Nb);
    pl.K = K;
    pl.M = std::max<int32_t>(2, (N + K - 1) / K);
    if (pl.M > 127) continue;                 // a limb spans at most two 64-bit words
    pl.logL = logL;
    int np = 0;
    for (int t = 1; t <= MAXNP64; ++t) {
      if (np_force && t != np_force) continue;
      if (primes64_cover(t, d, K, pl.M)) { np = t; break; }
    }
    if (!np) continue;
    pl.np = np;
    // y passes: the innermost factors take 2^9 points each, the outermost the rest
    int logn[MAX_PASS64], cnt = 0;
    for (int rem = logL; rem > 0 && cnt < MAX_PASS64; ++cnt) {
      logn[cnt] = std::min(rem, 9);
      rem -= logn[cnt];
    }
    pl.npass = cnt;
    int logS = 0;
    for (int q = 0; q < cnt; ++q) {           // q = 0 innermost
      Pass64 &ps = pl.pass[cnt - 1 - q];
      ps.logn = logn[q];
      ps.logS = logS;
      ps.logT = std::min(4, logS);
      ps.logG = std::min(4 - ps.logT, logL - ps.logn - logS);
      logS += logn[q];
    }
    pl.logTX = std::min(std::min(6, 11 - logK), logL);
    pl.DIG = 2 * np + 1;
    const int64_t J = 2 * (int64_t)K - 1;
    int lt = 3;
    while (lt > 0 && (J << lt) * pl.DIG > 2 * LDS64) --lt;
    pl.logTI = lt;
    uint64_t P[4];
    prime_product(np, P);
    pl.log2P = mw4_bitlen(P);
    pl.ws_words = (int64_t)np * 2 * K << logL;
    pl.cost = cost64(pl);
    if (!found || pl.cost < best.cost) { best = pl; found = true; }
  }
  if (!found) { *why = "no feasible (K, M, np) with at most three 62-bit primes"; return false; }
  out = best;
  return true;
}

// ------------------------------------------------------------------------------------
// device arithmetic modulo p < 2^62
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t add64(uint64_t a, uint64_t b, uint64_t p) {
  const uint64_t s = a + b;
  return s >= p ? s - p : s;
}
__device__ __forceinline__ uint64_t sub64(uint64_t a, uint64_t b, uint64_t p) {
  const uint64_t d = a - b;
  return a < b ? d + p : d;
}
// x w mod p for a constant w < p with companion floor(w 2^64 / p); any x < 2^64
__device__ __forceinline__ uint64_t mulsh64(uint64_t x, W64 w, uint64_t p) {
  const uint64_t q = __umul64hi(x, w.s);
  const uint64_t r = x * w.w - q * p;   // in [0, 2p)
  return r >= p ? r - p : r;
}
// a b 2^-64 mod p (Montgomery), a, b < p
__device__ __forceinline__ uint64_t mont64(uint64_t a, uint64_t b, uint64_t p, uint64_t pinv) {
  const uint64_t lo = a * b, hi = __umul64hi(a, b);
  const uint64_t m = lo * pinv;
  const uint64_t mp = __umul64hi(m, p);   // m p = lo mod 2^64, so no borrow below
  return hi >= mp ? hi - mp : hi - mp + p;
}
// Twiddle heaps live in device memory; their pointers come from the per-prime constants
// and are generic to the compiler, so they are read through the global address space
// (global or scalar loads instead of flat ones).
__device__ __forceinline__ W64 ld_tab64(const W64 *__restrict__ tab, int64_t i) {
  const auto *g = (const __attribute__((address_space(1))) uint64_t *)tab;
  return W64{g[2 * i], g[2 * i + 1]};
}

// w_m^e from a heap table (tab[m/2 + e] = w_m^e for e < m/2), e in [0, m), m >= 2
__device__ __forceinline__ W64 heap_root64(const W64 *__restrict__ tab, int64_t m, int64_t e, uint64_t p) {
  const int64_t half = m >> 1;
  if (e < half) return ld_tab64(tab, half + e);
  const W64 w = ld_tab64(tab, e);   // w_m^(e - m/2) = -w_m^e
  return W64{p - w.w, ~w.s};
}

// Radix-2^R groups of DIF / DIT stages on transforms in LDS, in the layout of
// LdsShape (transform t, element e at lds_base(t) + e es).
template <int R, class SH = LdsShape, int LOGH0 = -1>
__device__ void dif64_group(uint64_t *s, const SH &sh, int logh0_rt, const W64 *__restrict__ tw,
                            uint64_t p) {
  constexpr int NR = 1 << R;
  const int logh0 = LOGH0 >= 0 ? LOGH0 : logh0_rt;
  const int loghl = logh0 - (R - 1);
  const int hl = 1 << loghl;
  const int lgpt = sh.logn - R;
  const int total = 1 << (sh.logntr + sh.logops + lgpt);
  const bool tfast = sh.ts < sh.es;
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
    uint64_t x[NR];
#pragma unroll
    for (int m = 0; m < NR; ++m) x[m] = s[base + m * step];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int half = NR >> (i + 1);
      const int hsz = 1 << (logh0 - i);
#pragma unroll
      for (int m = 0; m < NR; ++m) {
        if (m & half) continue;
        const W64 w = ld_tab64(tw, hsz + j + (m & (half - 1)) * hl);
        const uint64_t u = x[m], v = x[m + half];
        x[m] = add64(u, v, p);
        x[m + half] = mulsh64(u - v + p, w, p);
      }
    }
#pragma unroll
    for (int m = 0; m < NR; ++m) s[base + m * step] = x[m];
  }
}

template <int R, class SH = LdsShape, int LOGH0 = -1>
__device__ void dit64_group(uint64_t *s, const SH &sh, int logh0_rt, const W64 *__restrict__ tw,
                            uint64_t p) {
  constexpr int NR = 1 << R;
  const int logh0 = LOGH0 >= 0 ? LOGH0 : logh0_rt;
  const int h0 = 1 << logh0;
  const int loghr = logh0 + R - 1;
  const int lgpt = sh.logn - R;
  const int total = 1 << (sh.logntr + sh.logops + lgpt);
  const bool tfast = sh.ts < sh.es;
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
    uint64_t x[NR];
#pragma unroll
    for (int m = 0; m < NR; ++m) x[m] = s[base + m * step];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int half = 1 << i;
      const int hsz = h0 << i;
#pragma unroll
      for (int m = 0; m < NR; ++m) {
        if (m & half) continue;
        const W64 w = ld_tab64(tw, hsz + j + (m & (half - 1)) * h0);
        const uint64_t u = x[m];
        const uint64_t v = mulsh64(x[m + half], w, p);
        x[m] = add64(u, v, p);
        x[m + half] = sub64(u, v, p);
      }
    }
#pragma unroll
    for (int m = 0; m < NR; ++m) s[base + m * step] = x[m];
  }
}

// the fewest groups of at most 3 stages (radix 8: eight 64-bit values per thread)
__device__ __forceinline__ int group_stages64(int left) {
  const int ngroups = (left + 2) / 3;
  return (left + ngroups - 1) / ngroups;
}

// Full transforms; the caller synchronises before; each group ends with a barrier.
__device__ void lds64_dif(uint64_t *s, const LdsShape &sh, const W64 *__restrict__ tw, uint64_t p) {
  int st = sh.logn;
  while (st > 0) {
    const int r = group_stages64(st);
    if (r == 3) dif64_group<3>(s, sh, st - 1, tw, p);
    else if (r == 2) dif64_group<2>(s, sh, st - 1, tw, p);
    else dif64_group<1>(s, sh, st - 1, tw, p);
    st -= r;
    __syncthreads();
  }
}
__device__ void lds64_dit(uint64_t *s, const LdsShape &sh, const W64 *__restrict__ tw, uint64_t p) {
  int done = 0;
  while (done < sh.logn) {
    const int r = group_stages64(sh.logn - done);
    if (r == 3) dit64_group<3>(s, sh, done, tw, p);
    else if (r == 2) dit64_group<2>(s, sh, done, tw, p);
    else dit64_group<1>(s, sh, done, tw, p);
    done += r;
    __syncthreads();
  }
}

// The same transforms for a compile-time shape (CShape), every group's stages fixed.
__device__ constexpr int group_stages64_c(int left) { return (left + (left + 2) / 3 - 1) / ((left + 2) / 3); }
template <class SH, int ST = SH::logn>
__device__ __forceinline__ void lds64_dif_c(uint64_t *s, const W64 *__restrict__ tw, uint64_t p) {
  if constexpr (ST > 0) {
    constexpr int R = group_stages64_c(ST);
    dif64_group<R, SH, ST - 1>(s, SH{}, 0, tw, p);
    __syncthreads();
    lds64_dif_c<SH, ST - R>(s, tw, p);
  }
}
template <class SH, int DONE = 0>
__device__ __forceinline__ void lds64_dit_c(uint64_t *s, const W64 *__restrict__ tw, uint64_t p) {
  if constexpr (DONE < SH::logn) {
    constexpr int R = group_stages64_c(SH::logn - DONE);
    dit64_group<R, SH, DONE>(s, SH{}, 0, tw, p);
    __syncthreads();
    lds64_dit_c<SH, DONE + R>(s, tw, p);
  }
}

// ------------------------------------------------------------------------------------
// BivariateRepresentation: a workgroup takes 64 coefficients and all their K limbs;
// a wave reads one limb of 64 coefficients and writes 64 consecutive residues per prime.
// ------------------------------------------------------------------------------------
template <int NP>
__global__ __launch_bounds__(BLOCK) void k64_convert(const uint64_t *__restrict__ x, int64_t d,
                                                     int32_t N, int32_t w, int32_t K, int32_t M,
                                                     const Prime64Dev *__restrict__ primes,
                                                     const Plan64Dev *__restrict__ pd,
                                                     uint64_t *__restrict__ X, int64_t L,
                                                     int32_t col_off) {
  const int64_t i = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  if (i >= d) return;   // no barriers below
  const uint64_t *xi = x + i * w;
  const int topw = (N - 1) >> 6, topb = (N - 1) & 63;
  const bool neg = (xi[topw] >> topb) & 1;
  // word q of the value sign-extended from bit N - 1
  auto word = [&](int64_t q) -> uint64_t {
    if (q < topw) return xi[q];
    if (q > topw) return neg ? ~0ull : 0ull;
    const uint64_t v = xi[q];
    if (topb == 63) return v;
    const uint64_t keep = (2ull << topb) - 1;
    return neg ? (v | ~keep) : (v & keep);
  };
  auto bits = [&](int64_t b) -> uint64_t {   // bits [b, b + 64)
    const int64_t q = b >> 6;
    const int s = (int)(b & 63);
    const uint64_t lo = word(q);
    return s ? (lo >> s) | (word(q + 1) << (64 - s)) : lo;
  };
  const int64_t twoK = 2 * (int64_t)K;
  const uint64_t mlo = M >= 64 ? ~0ull : ((1ull << M) - 1);
  const uint64_t mhi = M > 64 ? ((1ull << (M - 64)) - 1) : 0;
  uint64_t pk[NP];
  W64 one[NP], c64[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    pk[k] = primes[k].p;
    one[k] = primes[k].one;
    c64[k] = primes[k].c64;
  }
  for (int j = threadIdx.x >> 6; j < K; j += BLOCK / 64) {
    const int64_t b = (int64_t)M * j;
    const uint64_t lo = bits(b) & mlo;
    const uint64_t hi = M > 64 ? bits(b + 64) & mhi : 0;
    // the top limb is signed: its bit M - 1 weighs -2^(M-1)
    const bool neg_top = j == K - 1 && ((bits(b + M - 1) & 1) != 0);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      uint64_t r = mulsh64(lo, one[k], pk[k]);
      if (M > 64) r = add64(r, mulsh64(hi, c64[k], pk[k]), pk[k]);
      if (neg_top) r = sub64(r, pd->pow2M[k], pk[k]);
      X[((int64_t)k * twoK + col_off + j) * L + i] = r;
    }
  }
}

// ------------------------------------------------------------------------------------
// One strided pass of the y-transform over columns 0..cols-1 of every prime.
// Index i = inner + S (e + n outer); a workgroup holds T inner x G outer transforms
// (T G n <= 8192 words).  Forward: DIF along e, then frequency k of inner index u is
// multiplied by w_{nS}^(u k) and stored in natural order.  Inverse: multiplied by
// w_{nS}^(-u k), then DIT.  Rows i >= nz read as zero (first forward pass), rows
// i >= nlimit are not stored (last inverse pass).
// ------------------------------------------------------------------------------------
// CLOGN, CLOGT, CLOGG >= 0: the workgroup's shape fixed at compile time (== the runtime
// values); -1: any shape.
template <int INV, int CLOGN, int CLOGT, int CLOGG>
__global__ __launch_bounds__(BLOCK) void k64_ypass(uint64_t *__restrict__ X, int64_t L, int32_t twoK,
                                                   int32_t cols, int32_t logn_rt, int32_t logS,
                                                   int32_t logT_rt, int32_t logG_rt, int64_t nz_a,
                                                   int64_t nz_b, int32_t K, int64_t nlimit,
                                                   const Prime64Dev *__restrict__ primes) {
  __shared__ uint64_t s[LDS64];
  constexpr bool fixed = CLOGN >= 0;
  constexpr int FN = fixed ? CLOGN : 1, FT = fixed ? CLOGT : 0, FG = fixed ? CLOGG : 0;
  using CSH = CShape<FT, FN, 1, (1 << FT), (1 << FN) << FT, FG>;
  const int logn = fixed ? CLOGN : logn_rt, logT = fixed ? CLOGT : logT_rt,
            logG = fixed ? CLOGG : logG_rt;
  const int n = 1 << logn, T = 1 << logT;
  const int64_t S = (int64_t)1 << logS;
  const int64_t inner_tiles = S >> logT;
  const int64_t tiles = inner_tiles * ((L >> (logn + logS)) >> logG);
  const int64_t bid = blockIdx.x;
  // tiles, inner_tiles and cols (K or 2K) are powers of two: split by shifts
  const int64_t cidx = bid >> __builtin_ctzll((unsigned long long)tiles), tile = bid & (tiles - 1);
  const int k = (int)(cidx >> __builtin_ctz((unsigned)cols)), jc = (int)(cidx & (cols - 1));
  const int64_t inner0 = (tile & (inner_tiles - 1)) << logT;
  const int64_t outer0 = (tile >> (logS - logT)) << logG;
  const Prime64Dev pr = primes[k];
  const uint64_t p = pr.p;
  uint64_t *base = X + ((int64_t)k * twoK + jc) * L;
  const int64_t nz = INV ? L : (jc < K ? nz_a : nz_b);
  const int total = n << (logT + logG);
  const int64_t m = (int64_t)n << logS;
  auto gidx = [&](int idx) -> int64_t {
    const int tt = idx & (T - 1), e = (idx >> logT) & (n - 1), g = idx >> (logT + logn);
    return inner0 + tt + S * (e + (int64_t)n * (outer0 + g));
  };
  // LDS slot of frequency e of transform (tt, g) after a DIF (bit-reversed order)
  auto slot_rev = [&](int idx) -> int {
    const int tt = idx & (T - 1), e = (idx >> logT) & (n - 1), g = idx >> (logT + logn);
    return (((g << logn) + bitrev(e, logn)) << logT) + tt;
  };
  const LdsShape sh{logT, logn, 1, T, n << logT, logG};
  if (!INV) {
    staged<4, uint64_t>(total, [&](int idx) {
      const int64_t i = gidx(idx);
      return i < nz ? base[i] : 0ull;
    }, [&](int idx, uint64_t v) { s[idx] = v; });
    __syncthreads();
    if constexpr (fixed) lds64_dif_c<CSH>(s, pr.hf, p);
    else lds64_dif(s, sh, pr.hf, p);
    for (int idx = threadIdx.x; idx < total; idx += BLOCK) {
      uint64_t v = s[slot_rev(idx)];
      if (logS) {
        const int64_t u = inner0 + (idx & (T - 1));
        const int64_t e = (idx >> logT) & (n - 1);
        v = mulsh64(v, heap_root64(pr.hf, m, (u * e) & (m - 1), p), p);
      }
      base[gidx(idx)] = v;
    }
  } else {
    staged<4, uint64_t>(total, [&](int idx) {
      uint64_t v = base[gidx(idx)];
      if (logS) {
        const int64_t u = inner0 + (idx & (T - 1));
        const int64_t e = (idx >> logT) & (n - 1);
        v = mulsh64(v, heap_root64(pr.hi, m, (u * e) & (m - 1), p), p);
      }
      return v;
    }, [&](int idx, uint64_t v) { s[slot_rev(idx)] = v; });
    __syncthreads();
    if constexpr (fixed) lds64_dit_c<CSH>(s, pr.hi, p);
    else lds64_dit(s, sh, pr.hi, p);
    for (int idx = threadIdx.x; idx < total; idx += BLOCK) {
      const int64_t i = gidx(idx);
      if (i < nlimit) base[i] = s[idx];
    }
  }
}

// ------------------------------------------------------------------------------------
// x part of the convolution for TX consecutive y-frequencies of one prime: 2K-point
// DIF of the zero-padded limb rows of a and b, pointwise Montgomery product with the
// scale 2^64 / (2 K L), 2K-point DIT; row j of the result is c_{., j} (row 2K - 1 is 0).
// SQ: b is a (one forward transform).
// ------------------------------------------------------------------------------------
// CLOGK, CLOGTX >= 0: K and the tile fixed at compile time; -1: any.
template <int SQ, int CLOGK, int CLOGTX>
__global__ __launch_bounds__(BLOCK) void k64_xconv(uint64_t *__restrict__ X, int64_t L, int32_t logK_rt,
                                                   int32_t logTX_rt, const Prime64Dev *__restrict__ primes,
                                                   const Plan64Dev *__restrict__ pd) {
  __shared__ uint64_t s[LDS64];
  constexpr bool fixed = CLOGK >= 0;
  constexpr int FK = fixed ? CLOGK : 1, FX = fixed ? CLOGTX : 0;
  const int logK = fixed ? CLOGK : logK_rt, logTX = fixed ? CLOGTX : logTX_rt;
  const int K = 1 << logK, twoK = 2 * K, TX = 1 << logTX;
  const int64_t tiles = L >> logTX;
  const int k = (int)((int64_t)blockIdx.x >> __builtin_ctzll((unsigned long long)tiles));
  const int64_t y0 = ((int64_t)blockIdx.x & (tiles - 1)) << logTX;
  const Prime64Dev pr = primes[k];
  const uint64_t p = pr.p;
  uint64_t *base = X + (int64_t)k * twoK * L + y0;
  const int rows = SQ ? K : twoK;   // limb rows: a's 0..K-1, then b's K..2K-1
  const int L32 = (int)L;           // L <= 2^21
  // operand op's row j goes to LDS row op 2K + j; rows op 2K + K + j are zero
  staged<4, uint64_t>(rows << logTX, [&](int idx) {
    return base[(idx >> logTX) * L32 + (idx & (TX - 1))];
  }, [&](int idx, uint64_t v) {
    const int r = idx >> logTX, tt = idx & (TX - 1);
    const int op = r >> logK, j = r & (K - 1);
    s[((op * twoK + j) << logTX) + tt] = v;
    s[((op * twoK + K + j) << logTX) + tt] = 0;
  });
  __syncthreads();
  if constexpr (fixed)
    lds64_dif_c<CShape<FX, FK + 1, 1, (1 << FX), (2 << FK) << FX, SQ ? 0 : 1>>(s, pr.hf, p);
  else
    lds64_dif(s, LdsShape{logTX, logK + 1, 1, TX, twoK << logTX, SQ ? 0 : 1}, pr.hf, p);
  const W64 sc = pd->scale[k];
  for (int idx = threadIdx.x; idx < (twoK << logTX); idx += BLOCK) {
    const uint64_t u = s[idx];
    const uint64_t v = SQ ? u : s[(twoK << logTX) + idx];
    s[idx] = mulsh64(mont64(u, v, p, pr.pinv), sc, p);
  }
  __syncthreads();
  if constexpr (fixed)
    lds64_dit_c<CShape<FX, FK + 1, 1, (1 << FX)>>(s, pr.hi, p);
  else
    lds64_dit(s, LdsShape{logTX, logK + 1, 1, TX, 0, 0}, pr.hi, p);
  for (int idx = threadIdx.x; idx < (twoK << logTX); idx += BLOCK)
    base[(idx >> logTX) * L32 + (idx & (TX - 1))] = s[idx];
}

// ------------------------------------------------------------------------------------
// RecoveringProduct for TI consecutive coefficients.
// Phase 1: each c_{i,j} (j < 2K - 1) from its residues by Garner's mixed-radix CRT,
//   lifted to (-P/2, P/2) (exact: |c_{i,j}| < P/4), shifted left by (M j) mod 32 and
//   kept as DIG = 2 np + 1 digits of two's complement in LDS.
// Phase 2: one wave per coefficient.  Lane l owns the 32-bit output digits
//   [l per, (l+1) per); digit q sums the digits of every c_{i,j} whose window covers
//   it (window of c_{i,j} starts at digit floor(M j / 32)), and -1 one digit above the
//   window of each negative c_{i,j}; then the lanes' carries are resolved by a scan.
// ------------------------------------------------------------------------------------
__device__ void wave_carry_resolve(uint32_t *dst, int lo, int hi, int64_t carry, int lane) {
  // each lane's digits are normalised; add the previous lane's carry out
  int64_t cin = __shfl_up(carry, 1, 64);
  if (lane == 0) cin = 0;
  int64_t x = cin;
  bool allz = true, allo = true;
  for (int q = lo; q < hi; ++q) {
    const int64_t t = (int64_t)dst[q] + x;
    dst[q] = (uint32_t)t;
    x = t >> 32;
    allz = allz && (uint32_t)t == 0u;
    allo = allo && (uint32_t)t == 0xFFFFFFFFu;
  }
  // carry out is now in {-1, 0, 1}; code the lane's map carry-in -> carry-out on
  // {-1, 0, 1} and compose the maps of the lanes below by an inclusive scan
  int code;
  if (lo >= hi) {
    code = 0 | (1 << 2) | (2 << 4);   // identity
  } else {
    const int g = (int)x;
    code = (g + (allz ? -1 : 0) + 1) | ((g + 1) << 2) | ((g + (allo ? 1 : 0) + 1) << 4);
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int other = __shfl_up(code, off, 64);
    if (lane >= off) code = fcompose(code, other);
  }
  const int prevc = __shfl_up(code, 1, 64);
  int y = lane == 0 ? 0 : fapply(prevc, 0);
  for (int q = lo; q < hi && y != 0; ++q) {
    const int64_t t = (int64_t)dst[q] + y;
    dst[q] = (uint32_t)t;
    y = (int)(t >> 32);
  }
}

template <int NP>
__global__ __launch_bounds__(BLOCK) void k64_recover(const uint64_t *__restrict__ X, int64_t L,
                                                     int32_t K, int32_t M, int64_t nout, int32_t logTI,
                                                     const Prime64Dev *__restrict__ primes,
                                                     const Plan64Dev *__restrict__ pd,
                                                     uint64_t *__restrict__ c, int32_t wc) {
  constexpr int DIG = 2 * NP + 1;
  __shared__ uint32_t dig[2 * LDS64];
  const int J = 2 * K - 1, TI = 1 << logTI;
  const int64_t i0 = (int64_t)blockIdx.x << logTI;
  const int64_t twoK = 2 * (int64_t)K;
  uint64_t pk[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) pk[k] = primes[k].p;
  const uint64_t Ph0 = pd->Phalf[0], Ph1 = pd->Phalf[1], Ph2 = pd->Phalf[2];
  const uint64_t P0 = pd->P[0], P1 = pd->P[1], P2 = pd->P[2];
  for (int q = threadIdx.x; q < (J << logTI); q += BLOCK) {
    const int il = q & (TI - 1), j = q >> logTI;
    const int64_t i = i0 + il;
    if (i >= nout) continue;
    uint64_t r[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) r[k] = X[((int64_t)k * twoK + j) * L + i];
    uint64_t v0 = r[0], v1 = 0, v2 = 0;
    if (NP >= 2) {
      // x1 = (r1 - r0) p0^{-1} mod p1;  v = r0 + p0 x1
      const uint64_t p1 = pk[1];
      const uint64_t x1 = mulsh64(sub64(r[1], mulsh64(r[0], primes[1].one, p1), p1), pd->inv01, p1);
      const uint64_t lo = pk[0] * x1, hi = __umul64hi(pk[0], x1);
      v0 = r[0] + lo;
      v1 = hi + (v0 < lo ? 1 : 0);
      if (NP >= 3) {
        // x2 = (r2 - v mod p2) (p0 p1)^{-1} mod p2;  v += p0 p1 x2
        const uint64_t p2 = pk[2];
        const uint64_t vm = add64(mulsh64(r[0], primes[2].one, p2), mulsh64(x1, pd->p0_mod2, p2), p2);
        const uint64_t x2 = mulsh64(sub64(r[2], vm, p2), pd->inv012, p2);
        const uint64_t a0 = pd->p01[0] * x2, a1 = __umul64hi(pd->p01[0], x2);
        const uint64_t b1 = pd->p01[1] * x2, b2 = __umul64hi(pd->p01[1], x2);
        const uint64_t t1 = a1 + b1;
        const uint64_t c2 = t1 < a1 ? 1 : 0;
        const uint64_t n0 = v0 + a0;
        const uint64_t cy = n0 < v0 ? 1 : 0;
        uint64_t n1 = v1 + t1;
        uint64_t cy1 = n1 < v1 ? 1 : 0;
        n1 += cy;
        cy1 += n1 < cy ? 1 : 0;
        v0 = n0;
        v1 = n1;
        v2 = b2 + c2 + cy1;
      }
    }
    // symmetric representative: v > (P - 1) / 2 stands for v - P
    const bool gt = v2 != Ph2 ? v2 > Ph2 : (v1 != Ph1 ? v1 > Ph1 : v0 > Ph0);
    uint64_t v3 = 0;
    if (gt) {
      const uint64_t d0 = v0 - P0;
      const uint64_t bw0 = v0 < P0 ? 1 : 0;
      const uint64_t d1 = v1 - P1 - bw0;
      const uint64_t bw1 = (v1 < P1 || (v1 - P1) < bw0) ? 1 : 0;
      v2 = v2 - P2 - bw1;
      v1 = d1;
      v0 = d0;
      v3 = ~0ull;
    }
    const int sh = (int)(((int64_t)M * j) & 31);
    uint64_t ww[4] = {v0, v1, v2, v3};
    if (sh) {
      ww[3] = (v3 << sh) | (v2 >> (64 - sh));
      ww[2] = (v2 << sh) | (v1 >> (64 - sh));
      ww[1] = (v1 << sh) | (v0 >> (64 - sh));
      ww[0] = v0 << sh;
    }
    uint32_t *dst = dig + (il * J + j) * DIG;
#pragma unroll
    for (int u = 0; u < DIG; ++u) dst[u] = (uint32_t)(ww[u >> 1] >> (32 * (u & 1)));
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nd = 2 * wc;
  const int per = ((nd + 127) / 128) * 2;
  const int lo = min(lane * per, nd), hi = min(lo + per, nd);
  for (int il = wave; il < TI; il += BLOCK / 64) {
    const int64_t i = i0 + il;
    if (i >= nout) break;   // uniform per wave
    const uint32_t *dg = dig + il * J * DIG;
    uint32_t *out = reinterpret_cast<uint32_t *>(c + i * wc);
    int64_t carry = 0;
    for (int q = lo; q < hi; ++q) {
      int64_t acc = carry;
      const int64_t qlo = 32 * (int64_t)(q - DIG);
      const int jlo = qlo <= 0 ? 0 : (int)((qlo + M - 1) / M);
      const int jhi = (int)min<int64_t>(J - 1, (32 * (int64_t)q + 31) / M);
      for (int j = jlo; j <= jhi; ++j) {
        const int u = q - (int)(((int64_t)M * j) >> 5);   // 0 <= u <= DIG
        if (u < DIG) acc += dg[j * DIG + u];
        else if ((int32_t)dg[j * DIG + DIG - 1] < 0) acc -= 1;
      }
      out[q] = (uint32_t)acc;
      carry = acc >> 32;
    }
    wave_carry_resolve(out, lo, hi, carry, lane);
  }
}

// ------------------------------------------------------------------------------------
// context state and launcher
// ------------------------------------------------------------------------------------
struct P64State {
  Prime64Dev *primes = nullptr;   // MAXNP64 entries
  W64 *heaps = nullptr;           // prime k: forward heap at (2k) H, inverse at (2k+1) H
  int64_t H = 0;
  std::map<std::tuple<int, int, int, int>, Plan64Dev *> consts;   // (np, K, logL, M)
  uint64_t *ws = nullptr;
  int64_t ws_words = 0;
};

static int ensure_tables64(P64State &S, int64_t H) {
  if (S.heaps && S.H >= H) return ZPM_OK;
  H = std::max<int64_t>(H, 2);
  const Prime64Host *tab = prime64_table();
  std::vector<W64> host((size_t)2 * MAXNP64 * H, W64{0, 0});
  for (int k = 0; k < MAXNP64; ++k) {
    const uint64_t p = tab[k].p;
    W64 *hf = host.data() + (size_t)(2 * k) * H, *hi = hf + H;
    for (int64_t h = 1; h < H; h <<= 1) {
      // w_{2h} = root^(2^21 / (2h))
      const uint64_t w = powmod64(tab[k].root, ((uint64_t)1 << LOG2_ROOT64) / (2 * h), p);
      const uint64_t wi = invmod64(w, p);
      uint64_t a = 1, b = 1;
      for (int64_t j = 0; j < h; ++j) {
        hf[h + j] = shoup64(a, p);
        hi[h + j] = shoup64(b, p);
        a = mulmod64(a, w, p);
        b = mulmod64(b, wi, p);
      }
    }
  }
  W64 *heaps = nullptr;
  if (hipMalloc(&heaps, host.size() * sizeof(W64)) != hipSuccess) return ZPM_ENOMEM;
  if (hipMemcpy(heaps, host.data(), host.size() * sizeof(W64), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(heaps);
    return ZPM_EDEVICE;
  }
  Prime64Dev pd[MAXNP64];
  for (int k = 0; k < MAXNP64; ++k) {
    const uint64_t p = tab[k].p;
    uint64_t inv = p;   // Newton: p^{-1} mod 2^64 (3 -> 96 correct bits)
    for (int it = 0; it < 5; ++it) inv *= 2 - p * inv;
    pd[k].p = p;
    pd[k].pinv = inv;
    pd[k].one = shoup64(1, p);
    pd[k].c64 = shoup64((uint64_t)(((u128)1 << 64) % p), p);
    pd[k].hf = heaps + (size_t)(2 * k) * H;
    pd[k].hi = heaps + (size_t)(2 * k + 1) * H;
  }
  if (!S.primes && hipMalloc(&S.primes, sizeof(pd)) != hipSuccess) {
    (void)hipFree(heaps);
    return ZPM_ENOMEM;
  }
  // the old tables may still be read by queued work
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(S.primes, pd, sizeof(pd), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(heaps);
    return ZPM_EDEVICE;
  }
  if (S.heaps) (void)hipFree(S.heaps);
  S.heaps = heaps;
  S.H = H;
  return ZPM_OK;
}

static int plan_consts64(P64State &S, const Plan64 &pl, Plan64Dev **out) {
  const auto key = std::make_tuple(pl.np, pl.K, pl.logL, pl.M);
  auto it = S.consts.find(key);
  if (it != S.consts.end()) { *out = it->second; return ZPM_OK; }
  const Prime64Host *tab = prime64_table();
  Plan64Dev h;
  std::memset(&h, 0, sizeof(h));
  const uint64_t len = (uint64_t)2 * pl.K << pl.logL;
  for (int k = 0; k < pl.np; ++k) {
    const uint64_t p = tab[k].p;
    const uint64_t c64 = (uint64_t)(((u128)1 << 64) % p);
    h.scale[k] = shoup64(mulmod64(c64, invmod64(len % p, p), p), p);
    h.pow2M[k] = powmod64(2, (uint64_t)pl.M, p);
  }
  if (pl.np >= 2) {
    const uint64_t p0 = tab[0].p, p1 = tab[1].p;
    h.inv01 = shoup64(invmod64(p0 % p1, p1), p1);
    const u128 q = (u128)p0 * p1;
    h.p01[0] = (uint64_t)q;
    h.p01[1] = (uint64_t)(q >> 64);
  }
  if (pl.np >= 3) {
    const uint64_t p0 = tab[0].p, p1 = tab[1].p, p2 = tab[2].p;
    h.p0_mod2 = shoup64(p0 % p2, p2);
    h.inv012 = shoup64(invmod64(mulmod64(p0 % p2, p1 % p2, p2), p2), p2);
  }
  uint64_t P[4];
  prime_product(pl.np, P);
  for (int i = 0; i < 3; ++i) {
    h.P[i] = P[i];
    h.Phalf[i] = (P[i] >> 1) | (i < 2 ? P[i + 1] << 63 : 0);   // P odd: (P - 1) / 2 = P >> 1
  }
  Plan64Dev *d = nullptr;
  if (hipMalloc(&d, sizeof(h)) != hipSuccess) return ZPM_ENOMEM;
  if (hipMemcpy(d, &h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return ZPM_EDEVICE;
  }
  S.consts[key] = d;
  *out = d;
  return ZPM_OK;
}

static int ensure_ws64(P64State &S, int64_t words) {
  if (words <= S.ws_words) return ZPM_OK;
  if (hipDeviceSynchronize() != hipSuccess) return ZPM_EDEVICE;
  if (S.ws) (void)hipFree(S.ws);
  S.ws = nullptr;
  S.ws_words = 0;
  if (hipMalloc(&S.ws, (size_t)words * 8) != hipSuccess) return ZPM_ENOMEM;
  S.ws_words = words;
  return ZPM_OK;
}

template <int NP>
static void launch_convert(const Plan64 &pl, const P64State &S, const Plan64Dev *pd, const uint64_t *x,
                           int64_t d, int32_t N, uint64_t *X, int32_t col_off, hipStream_t st) {
  const int64_t L = (int64_t)1 << pl.logL;
  hipLaunchKernelGGL(k64_convert<NP>, dim3((unsigned)((d + 63) / 64)), dim3(BLOCK), 0, st, x, d, N,
                     (N + 63) / 64, pl.K, pl.M, S.primes, pd, X, L, col_off);
}

template <int NP>
static void launch_recover(const Plan64 &pl, const P64State &S, const Plan64Dev *pd, const uint64_t *X,
                           uint64_t *c, int32_t wc, hipStream_t st) {
  const int64_t L = (int64_t)1 << pl.logL;
  const int64_t blocks = (pl.nout + (1 << pl.logTI) - 1) >> pl.logTI;
  hipLaunchKernelGGL(k64_recover<NP>, dim3((unsigned)blocks), dim3(BLOCK), 0, st, X, L, pl.K, pl.M,
                     pl.nout, pl.logTI, S.primes, pd, c, wc);
}

static void launch_pass(const Plan64 &pl, const P64State &S, uint64_t *X, int q, bool inverse, int cols,
                        hipStream_t st) {
  const Pass64 &ps = pl.pass[q];
  const int64_t L = (int64_t)1 << pl.logL;
  const int64_t tiles = ((int64_t)1 << (ps.logS - ps.logT)) * ((L >> (ps.logn + ps.logS)) >> ps.logG);
  const int64_t blocks = (int64_t)pl.np * cols * tiles;
  const int64_t nz_a = q == 0 ? pl.da : L, nz_b = q == 0 ? (pl.square ? pl.da : pl.db) : L;
  const int64_t nlimit = q == 0 ? pl.nout : L;
  // the shapes of the planner's passes for L = 2^17 ... 2^21: the innermost 2^9-point
  // pass (16 transforms per workgroup) and outer passes of 2^8 and 2^9 points on
  // 16-column tiles
  const int shape = (ps.logn == 9 && ps.logT == 0 && ps.logG == 4)   ? 1
                    : (ps.logn == 8 && ps.logT == 4 && ps.logG == 0) ? 2
                    : (ps.logn == 9 && ps.logT == 4 && ps.logG == 0) ? 3
                                                                     : 0;
#define ZPM_YP(INV_, LN, LT, LG)                                                              \
  hipLaunchKernelGGL((k64_ypass<INV_, LN, LT, LG>), dim3((unsigned)blocks), dim3(BLOCK), 0, st, X, L, \
                     2 * pl.K, cols, ps.logn, ps.logS, ps.logT, ps.logG, INV_ ? L : nz_a,      \
                     INV_ ? L : nz_b, pl.K, INV_ ? nlimit : L, S.primes)
#define ZPM_YP_ALL(INV_)                          \
  switch (shape) {                                \
    case 1: ZPM_YP(INV_, 9, 0, 4); break;         \
    case 2: ZPM_YP(INV_, 8, 4, 0); break;         \
    case 3: ZPM_YP(INV_, 9, 4, 0); break;         \
    default: ZPM_YP(INV_, -1, -1, -1); break;     \
  }
  if (!inverse) {
    ZPM_YP_ALL(0)
  } else {
    ZPM_YP_ALL(1)
  }
#undef ZPM_YP_ALL
#undef ZPM_YP
}

int mul_p64(Ctx &cx, const Plan64 &pl, const uint64_t *a, const uint64_t *b, uint64_t *c, int32_t wc,
            hipStream_t st) {
  if (!cx.p64) cx.p64 = new P64State();
  P64State &S = *cx.p64;
  const int64_t L = (int64_t)1 << pl.logL;
  // launch shapes the kernels rely on
  if (pl.np < 1 || pl.np > MAXNP64 || pl.K < 2 || pl.K > K_MAX64 || (pl.K & (pl.K - 1)) ||
      pl.logTX > pl.logL || ((2 * (int64_t)pl.K) << (pl.logTX + 1)) > LDS64 ||
      (int64_t)(2 * pl.K - 1) * pl.DIG << pl.logTI > 2 * LDS64 || pl.DIG != 2 * pl.np + 1)
    return ZPM_EINVAL;
  for (int q = 0; q < pl.npass; ++q) {
    const Pass64 &ps = pl.pass[q];
    if (ps.logn < 1 || ps.logn > 9 || ps.logT > ps.logS || ps.logT + ps.logG > 4 ||
        ps.logn + ps.logS + ps.logG > pl.logL)
      return ZPM_EINVAL;
  }
  int rc;
  if ((rc = ensure_tables64(S, std::max<int64_t>(L, 2 * (int64_t)pl.K))) != ZPM_OK) return rc;
  Plan64Dev *pd = nullptr;
  if ((rc = plan_consts64(S, pl, &pd)) != ZPM_OK) return rc;
  if ((rc = ensure_ws64(S, pl.ws_words)) != ZPM_OK) return rc;
  uint64_t *X = S.ws;
  Profiler &prof = cx.prof;
  prof.begin(KK_P64_CONVERT, st);
  for (int op = 0; op < (pl.square ? 1 : 2); ++op) {
    const uint64_t *x = op ? b : a;
    const int64_t d = op ? pl.db : pl.da;
    const int32_t N = op ? pl.Nb : pl.Na;
    const int32_t off = op ? pl.K : 0;
    if (pl.np == 1) launch_convert<1>(pl, S, pd, x, d, N, X, off, st);
    else if (pl.np == 2) launch_convert<2>(pl, S, pd, x, d, N, X, off, st);
    else launch_convert<3>(pl, S, pd, x, d, N, X, off, st);
  }
  prof.end(st);
  const int fcols = pl.square ? pl.K : 2 * pl.K;
  if (pl.npass) {
    prof.begin(KK_P64_YFWD, st);
    for (int q = 0; q < pl.npass; ++q) launch_pass(pl, S, X, q, false, fcols, st);
    prof.end(st);
  }
  prof.begin(KK_P64_X, st);
  const int64_t xblocks = (int64_t)pl.np * (L >> pl.logTX);
  // K = 64 and 128 with their widest tiles have compile-time kernels
  const int lk = __builtin_ctz(pl.K);
  const int xshape = (lk == 6 && pl.logTX == 5) ? 1 : (lk == 7 && pl.logTX == 4) ? 2 : 0;
#define ZPM_XC(SQ_, LK_, LT_)                                                                 \
  hipLaunchKernelGGL((k64_xconv<SQ_, LK_, LT_>), dim3((unsigned)xblocks), dim3(BLOCK), 0, st, X, L, \
                     lk, pl.logTX, S.primes, pd)
#define ZPM_XC_ALL(SQ_)                          \
  switch (xshape) {                              \
    case 1: ZPM_XC(SQ_, 6, 5); break;            \
    case 2: ZPM_XC(SQ_, 7, 4); break;            \
    default: ZPM_XC(SQ_, -1, -1); break;         \
  }
  if (pl.square) {
    ZPM_XC_ALL(1)
  } else {
    ZPM_XC_ALL(0)
  }
#undef ZPM_XC_ALL
#undef ZPM_XC
  prof.end(st);
  if (pl.npass) {
    prof.begin(KK_P64_YINV, st);
    for (int q = pl.npass - 1; q >= 0; --q) launch_pass(pl, S, X, q, true, 2 * pl.K, st);
    prof.end(st);
  }
  prof.begin(KK_P64_RECOVER, st);
  if (pl.np == 1) launch_recover<1>(pl, S, pd, X, c, wc, st);
  else if (pl.np == 2) launch_recover<2>(pl, S, pd, X, c, wc, st);
  else launch_recover<3>(pl, S, pd, X, c, wc, st);
  prof.end(st);
  return hipGetLastError() == hipSuccess ? ZPM_OK : ZPM_EDEVICE;
}

void p64_release(Ctx &cx) {
  if (!cx.p64) return;
  P64State &S = *cx.p64;
  (void)hipSetDevice(cx.device);
  (void)hipDeviceSynchronize();
  if (S.ws) (void)hipFree(S.ws);
  if (S.heaps) (void)hipFree(S.heaps);
  if (S.primes) (void)hipFree(S.primes);
  for (auto &kv : S.consts) (void)hipFree(kv.second);
  delete cx.p64;
  cx.p64 = nullptr;
}

}  // namespace zpm
