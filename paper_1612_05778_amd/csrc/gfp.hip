// One big generalized Fermat prime p = r^k + 1 (Section 3.1, Relation (FurerHypothesis)
// and the table of generalized Fermat primes; Section 5): planner, host number theory,
// gfx950 kernels and the launch sequence.
//
// Element layout: k int32 digits, balanced in radix r (|d| <= r/2 + 64 after every
// normalisation), value sum d_l r^l mod p.  Workspace: column j in [0, 2K), position i in
// [0, L), element at ((j L + i) k + l).  Columns j < K hold limb j of a, columns K + j
// limb j of b; after the x-kernel column j holds c_{i,j} (y still transformed), and after
// the inverse y-passes c_{i,j} mod p itself.
//
// Two data layouts inside the kernels:
//   digit per lane   -- a group of k lanes holds one transform instance, lane l holding
//                       digit l of each of its elements in registers.  Butterflies are
//                       lane-local adds, a product by r^e is a cross-lane rotation
//                       (ds_bpermute) with the wrapped digits negated;
//   element per lane -- for generic products a thread holds all k digits of one element
//                       (through LDS) and forms the negacyclic digit convolution with
//                       32 x 32 -> 64-bit multiply-adds, then carries in radix r.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "../../include/zpm.h"
#include "ctx.hpp"
#include "gfp.hpp"

namespace zpm {

// ------------------------------------------------------------------------------------
// primes
// ------------------------------------------------------------------------------------
template <int KD>
struct GfpR;
template <>
struct GfpR<8> {
  static constexpr int32_t R = (1 << 29) - (1 << 25);
  static constexpr int S1 = 25, G1 = -1, S2 = 0, G2 = 0, W = 8;
};
template <>
struct GfpR<16> {
  static constexpr int32_t R = (1 << 29) - (1 << 9) - (1 << 7);
  static constexpr int S1 = 9, G1 = -1, S2 = 7, G2 = -1, W = 15;
};
template <>
struct GfpR<32> {
  static constexpr int32_t R = (1 << 29) - (1 << 14) - (1 << 13);
  static constexpr int S1 = 14, G1 = -1, S2 = 13, G2 = -1, W = 30;
};

// bit length of r^k + 1 and the 32-bit words of a signed value below it in magnitude
static void prime_sizes(GfpPrime &P) {
  std::vector<uint32_t> x(64, 0);
  x[0] = 1;
  for (int t = 0; t < P.k; ++t) {
    uint64_t c = 0;
    for (auto &w : x) {
      const uint64_t v = (uint64_t)w * (uint32_t)P.r + c;
      w = (uint32_t)v;
      c = v >> 32;
    }
  }
  x[0] += 1;   // r^k is even: no carry
  int bl = 0;
  for (int i = 63; i >= 0; --i)
    if (x[i]) {
      bl = 32 * i + 32 - __builtin_clz(x[i]);
      break;
    }
  P.log2p = bl;
  P.W = (bl + 1 + 31) / 32;
}

const GfpPrime *gfp_prime_table() {
  static GfpPrime T[GFP_NPRIMES] = {
      {8, GfpR<8>::R, GfpR<8>::S1, GfpR<8>::G1, GfpR<8>::S2, GfpR<8>::G2, 0, 0},
      {16, GfpR<16>::R, GfpR<16>::S1, GfpR<16>::G1, GfpR<16>::S2, GfpR<16>::G2, 0, 0},
      {32, GfpR<32>::R, GfpR<32>::S1, GfpR<32>::G1, GfpR<32>::S2, GfpR<32>::G2, 0, 0},
  };
  static bool init = [] {
    for (auto &P : T) prime_sizes(P);
    return true;
  }();
  (void)init;
  return T;
}

static int gfp_W(int k) { return k == 8 ? GfpR<8>::W : k == 16 ? GfpR<16>::W : GfpR<32>::W; }

// ------------------------------------------------------------------------------------
// host arithmetic in radix r (tables and roots; slow and simple)
// ------------------------------------------------------------------------------------
typedef __int128 i128;

struct HE {
  int64_t d[GFP_KMAX];
};

static i128 rdiv_nearest(i128 t, i128 r) {   // floor((t + r/2) / r)
  const i128 num = t + r / 2;
  i128 q = num / r;
  if (num % r < 0) q -= 1;
  return q;
}

// z (k digits) -> balanced digits in [-r/2, r/2); the carry out of the top digit wraps
// into digit 0 negated (r^k = -1)
static HE h_norm(const GfpPrime &P, i128 *z) {
  const i128 r = P.r;
  i128 c = 0;
  for (int pass = 0; pass < 16; ++pass) {
    for (int l = 0; l < P.k; ++l) {
      const i128 t = z[l] + c;
      const i128 q = rdiv_nearest(t, r);
      z[l] = t - q * r;
      c = q;
    }
    if (c == 0) break;
    c = -c;
  }
  HE o;
  std::memset(&o, 0, sizeof(o));
  for (int l = 0; l < P.k; ++l) o.d[l] = (int64_t)z[l];
  return o;
}

static HE h_from(const GfpPrime &P, int64_t v) {
  i128 z[GFP_KMAX] = {0};
  z[0] = v;
  return h_norm(P, z);
}

static HE h_rpow(const GfpPrime &P, int e) {   // r^e, e in [0, 2k)
  HE o;
  std::memset(&o, 0, sizeof(o));
  o.d[e % P.k] = (e / P.k) & 1 ? -1 : 1;
  return o;
}

static HE h_mul(const GfpPrime &P, const HE &x, const HE &y) {
  i128 z[GFP_KMAX] = {0};
  const int k = P.k;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      const i128 t = (i128)x.d[i] * y.d[j];
      if (i + j < k) z[i + j] += t;
      else z[i + j - k] -= t;
    }
  return h_norm(P, z);
}

static bool h_eq(const GfpPrime &P, const HE &x, const HE &y) {
  i128 z[GFP_KMAX] = {0};
  for (int l = 0; l < P.k; ++l) z[l] = (i128)x.d[l] - y.d[l];
  const HE n = h_norm(P, z);
  for (int l = 0; l < P.k; ++l)
    if (n.d[l]) return false;
  return true;
}

static HE h_pow(const GfpPrime &P, HE x, uint64_t e) {
  HE y = h_from(P, 1);
  while (e) {
    if (e & 1) y = h_mul(P, y, x);
    x = h_mul(P, x, x);
    e >>= 1;
  }
  return y;
}

static HE h_sq_times(const GfpPrime &P, HE x, int64_t n) {
  for (int64_t i = 0; i < n; ++i) x = h_mul(P, x, x);
  return x;
}

static int v2(int64_t x) { return __builtin_ctzll((uint64_t)x); }

// A generator of the 2-Sylow subgroup (order 2^(a k), a = v2(r)): z^(u^k) for the first
// quadratic non-residue z, r = 2^a u.
static HE sylow2_generator(const GfpPrime &P) {
  const int a = v2(P.r);
  const int64_t u = P.r >> a;
  const HE minus1 = h_from(P, -1);
  for (int64_t z = 3; z < 1000; ++z) {
    HE y = h_from(P, z);
    for (int t = 0; t < P.k; ++t) y = h_pow(P, y, (uint64_t)u);
    if (h_eq(P, h_sq_times(P, y, (int64_t)a * P.k - 1), minus1)) return y;
  }
  return h_from(P, 0);   // not reached for the primes of the table
}

static bool root_of(const GfpPrime &P, int logL, HE &out) {
  const int a = v2(P.r);
  const int64_t L = (int64_t)1 << logL;
  if (logL > a * P.k) return false;
  if (L <= 2 * P.k) {
    out = h_rpow(P, (int)((2 * P.k / L) % (2 * P.k)));
    return true;
  }
  const HE g = sylow2_generator(P);
  const HE w0 = h_sq_times(P, g, (int64_t)a * P.k - logL);   // order L
  int lk2 = 0;
  while ((1 << lk2) < 2 * P.k) ++lk2;
  const HE t = h_sq_times(P, w0, logL - lk2);                  // order 2k: r^m, m odd
  int m = -1;
  for (int e = 1; e < 2 * P.k; e += 2)
    if (h_eq(P, t, h_rpow(P, e))) {
      m = e;
      break;
    }
  if (m < 0) return false;
  uint64_t inv = (uint64_t)m;   // m^{-1} mod 2^64 (Newton), then mod L
  for (int it = 0; it < 6; ++it) inv *= 2 - (uint64_t)m * inv;
  out = h_pow(P, w0, inv & (uint64_t)(L - 1));
  return h_eq(P, h_sq_times(P, out, logL - lk2), h_rpow(P, 1));
}

// (2^e)^{-1} mod p.  From r = 2^a u and r^k = -1: 2^(2ak) u^(2k) = 1, so
// 2^{-1} = 2^(2ak - 1) u^(2k).
static HE inv_pow2(const GfpPrime &P, int e) {
  const int a = v2(P.r);
  const int64_t u = P.r >> a;
  const HE two = h_from(P, 2);
  const HE inv2 = h_mul(P, h_pow(P, two, (uint64_t)(2 * a * P.k - 1)),
                        h_pow(P, h_from(P, u), (uint64_t)(2 * P.k)));
  return h_pow(P, inv2, (uint64_t)e);
}

bool gfp_root(int prime, int logL, int32_t *digits) {
  if (prime < 0 || prime >= GFP_NPRIMES || logL < 0 || logL > GFP_LOG2_LMAX) return false;
  const GfpPrime &P = gfp_prime_table()[prime];
  HE w;
  if (!root_of(P, logL, w)) return false;
  for (int l = 0; l < P.k; ++l) digits[l] = (int32_t)w.d[l];
  return true;
}

// ------------------------------------------------------------------------------------
// planner
// ------------------------------------------------------------------------------------
constexpr int GFP_TMAX = 32;   // 16-bit chunks of a limb (M <= 512)
constexpr int GFP_WMAX = 32;

static int clog2(int64_t x) {
  int r = 0;
  while (((int64_t)1 << r) < x) ++r;
  return r;
}

bool make_plan_gfp(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K_force,
                   int32_t prime_force, PlanGfp &out) {
  if (da < 1 || db < 1 || Na < 1 || Nb < 1) return false;
  const int64_t d = std::max(da, db);
  const int32_t N = std::max(Na, Nb);
  const int64_t nout = da + db - 1;
  const int logL = clog2(nout);
  if (logL > GFP_LOG2_LMAX) return false;
  const GfpPrime *T = gfp_prime_table();
  bool found = false;
  for (int pi = 0; pi < GFP_NPRIMES; ++pi) {
    if (prime_force >= 0 && pi != prime_force) continue;
    const GfpPrime &P = T[pi];
    for (int lk = 1; (1 << lk) <= P.k; ++lk) {
      const int K = 1 << lk;
      if (K_force && K != K_force) continue;
      const int32_t M = std::max<int32_t>(2, (N + K - 1) / K);
      // p > 4 d K 2^(2M) (Relation (recoveryModulo)): p >= 2^(log2p - 1)
      if (2 + clog2(d) + lk + 2 * M > P.log2p - 1) continue;
      const int T16 = (M + 15) / 16;
      if (T16 > GFP_TMAX) continue;
      PlanGfp pl;
      std::memset(&pl, 0, sizeof(pl));
      pl.da = da;
      pl.db = db;
      pl.Na = Na;
      pl.Nb = Nb;
      pl.nout = nout;
      pl.nout_bits = zpm_out_bits(da, Na, db, Nb);
      pl.prime = pi;
      pl.k = P.k;
      pl.K = K;
      pl.M = M;
      pl.logL = logL;
      // y-passes of at most 2k points (roots r^(2k/n)) and at most 32: a 64-point pass
      // keeps 64 digit registers per lane across its twiddle products and spills; as even
      // as possible, outermost first
      const int maxln = std::min(clog2(2 * P.k), 5);
      pl.npass = (logL + maxln - 1) / maxln;
      if (pl.npass > GFP_MAX_PASS) continue;
      for (int q = 0; q < pl.npass; ++q)
        pl.pass_logn[q] = logL / pl.npass + (q < logL % pl.npass ? 1 : 0);
      pl.T16 = T16;
      pl.W = P.W;
      pl.ws_words = (int64_t)2 * K * P.k << logL;
      // work model: generic products (k^2 multiply-adds each) in the twiddles between
      // y-passes and the pointwise step, rotations and adds in the passes, the lift
      const double nel = 2.0 * K * (double)((int64_t)1 << logL);
      const double prods = (pl.npass > 1 ? 2.0 * (pl.npass - 1) : 0.0) + 0.5;
      pl.cost = nel * (prods * P.k * P.k + 6.0 * P.k * (logL + 2 * (lk + 1)) + 5.0 * P.k * P.W) +
                2.0 * (double)d * K * T16 * P.k;
      if (!found || pl.cost < out.cost) {
        out = pl;
        found = true;
      }
    }
  }
  return found;
}

// ------------------------------------------------------------------------------------
// device arithmetic
// ------------------------------------------------------------------------------------
constexpr int GB = 256;   // threads per workgroup

// Per-plan constants.
struct GfpConstDev {
  int32_t Pa[GFP_TMAX * GFP_KMAX];   // 2^(16 t) mod p
  int32_t Pb[GFP_TMAX * GFP_KMAX];   // 2^(16 t) (2 K L)^{-1} mod p
  int32_t scale[GFP_KMAX];           // (2 K L)^{-1} mod p
  uint32_t pbin[GFP_WMAX];           // p, little-endian words
  double rpow[GFP_KMAX];             // r^l
  double phalf;                      // p / 2
};

__device__ __forceinline__ int32_t lane_from(int32_t v, int src) {
  return __builtin_amdgcn_ds_bpermute(src << 2, v);
}

// round(v / R) for |v| < 2R + 2^9 (the digits after two butterfly stages)
template <int KD>
__device__ __forceinline__ int32_t qround32(int32_t v) {
  constexpr uint32_t R = (uint32_t)GfpR<KD>::R;
  const uint32_t u = (uint32_t)v + (R >> 1) + 4u * R;   // in [0, 2^32) as an integer
  return (int32_t)(u / R) - 4;
}

// q with |t - q R| <= R/2, for |t| < 2^62
template <int KD>
__device__ __forceinline__ int64_t qround64(int64_t t) {
  constexpr int64_t R = GfpR<KD>::R;
  int64_t q = (int64_t)rint((double)t * (1.0 / (double)R));
  const int64_t rem = t - q * R;
  if (rem > (R >> 1)) ++q;
  else if (rem < -(R >> 1)) --q;
  return q;
}

// d = x y mod p: negacyclic convolution of the digit vectors (r^k = -1), then carries
// in radix r.  Inputs |digit| <= R/2 + 64: each sum stays below 2^62.  d must not alias
// x or y.
template <int KD>
__device__ __forceinline__ void gmul(const int32_t (&x)[KD], const int32_t (&y)[KD],
                                     int32_t (&d)[KD]) {
  constexpr int64_t R = GfpR<KD>::R;
  int64_t c = 0;
#pragma unroll
  for (int m = 0; m < KD; ++m) {
    int64_t sp = 0, sn = 0;
#pragma unroll
    for (int i = 0; i <= m; ++i) sp += (int64_t)x[i] * y[m - i];
#pragma unroll
    for (int i = m + 1; i < KD; ++i) sn += (int64_t)x[i] * y[m - i + KD];
    const int64_t t = sp - sn + c;
    const int64_t q = qround64<KD>(t);
    d[m] = (int32_t)(t - q * R);
    c = q;
  }
  // the carry out of the top digit times r^k = -carry, into digit 0
  const int64_t t = (int64_t)d[0] - c;
  const int64_t q = qround64<KD>(t);
  d[0] = (int32_t)(t - q * R);
  d[1] += (int32_t)q;
}

// v r^E (E in [0, 2 KD)) in the digit-per-lane layout: lane l of the group (first lane
// `base` of the wave) takes digit l - E, negated when it wrapped past the top.
template <int KD>
__device__ __forceinline__ int32_t rot(int32_t v, int E, int l, int base) {
  const int e = E % KD;
  const bool neg = ((E / KD) & 1) != 0;
  int32_t w = v;
  if (e != 0) w = lane_from(v, base + ((l - e) & (KD - 1)));
  const bool flip = (e != 0 && l < e) != neg;
  return flip ? -w : w;
}

// carries of one step in the digit-per-lane layout: |v| < 2R + 2^9 -> |v| <= R/2 + 3
template <int KD, int N>
__device__ __forceinline__ void lnorm(int32_t (&v)[N], int l, int base) {
  constexpr int32_t R = GfpR<KD>::R;
  const int src = base + ((l - 1) & (KD - 1));
#pragma unroll
  for (int e = 0; e < N; ++e) {
    const int32_t q = qround32<KD>(v[e]);
    v[e] -= q * R;
    const int32_t qin = lane_from(q, src);
    v[e] += (l == 0) ? -qin : qin;
  }
}

// Forward transform of N = 2^LN points with root r^(2 KD / N): natural order in,
// bit-reversed order out.  ZHI: the upper half is zero (its first stage is the twist).
template <int KD, int LN, bool ZHI>
__device__ __forceinline__ void dif(int32_t (&v)[1 << LN], int l, int base) {
  constexpr int N = 1 << LN;
  constexpr int U = 2 * KD / N;
#pragma unroll
  for (int s = 0; s < LN; ++s) {
    const int h = N >> (s + 1);
#pragma unroll
    for (int b = 0; b < N; b += 2 * h)
#pragma unroll
      for (int j = 0; j < h; ++j) {
        const int32_t x = v[b + j], y = v[b + j + h];
        if (ZHI && s == 0) {
          v[b + j + h] = rot<KD>(x, j * U, l, base);
        } else {
          v[b + j] = x + y;
          v[b + j + h] = rot<KD>(x - y, ((j << s) * U) % (2 * KD), l, base);
        }
      }
    if ((s & 1) || s == LN - 1) lnorm<KD>(v, l, base);
  }
}

// Inverse transform (root r^(-2 KD / N), unscaled): bit-reversed order in, natural out.
template <int KD, int LN>
__device__ __forceinline__ void dit_inv(int32_t (&v)[1 << LN], int l, int base) {
  constexpr int N = 1 << LN;
  constexpr int U = 2 * KD / N;
#pragma unroll
  for (int s = 0; s < LN; ++s) {
    const int h = 1 << s;
#pragma unroll
    for (int b = 0; b < N; b += 2 * h)
#pragma unroll
      for (int j = 0; j < h; ++j) {
        const int e = (j * (N / (2 * h)) * U) % (2 * KD);
        const int32_t x = v[b + j];
        const int32_t y = rot<KD>(v[b + j + h], (2 * KD - e) % (2 * KD), l, base);
        v[b + j] = x + y;
        v[b + j + h] = x - y;
      }
    if ((s & 1) || s == LN - 1) lnorm<KD>(v, l, base);
  }
}

template <int LN>
__device__ __forceinline__ int brev(int e) {
  return LN ? (int)(__brev((unsigned)e) >> (32 - LN)) : 0;
}
static constexpr int brev_c(int e, int ln) {
  int r = 0;
  for (int i = 0; i < ln; ++i) r |= ((e >> i) & 1) << (ln - 1 - i);
  return r;
}

template <int KD>
__device__ __forceinline__ void lds_load(const int32_t *p, int32_t (&x)[KD]) {
#pragma unroll
  for (int l = 0; l < KD; l += 4) {
    const int4 q = *reinterpret_cast<const int4 *>(p + l);
    x[l] = q.x;
    x[l + 1] = q.y;
    x[l + 2] = q.z;
    x[l + 3] = q.w;
  }
}
template <int KD>
__device__ __forceinline__ void lds_store(int32_t *p, const int32_t (&x)[KD]) {
#pragma unroll
  for (int l = 0; l < KD; l += 4) *reinterpret_cast<int4 *>(p + l) = make_int4(x[l], x[l + 1], x[l + 2], x[l + 3]);
}

// ------------------------------------------------------------------------------------
// kernels
// ------------------------------------------------------------------------------------

// Bits [bit, bit + 16) of coefficient s (w words), sign-extended from bit N - 1.
__device__ __forceinline__ uint32_t bits16(const uint64_t *s, int32_t w, int32_t N, int64_t bit) {
  const uint32_t sign = ((s[(N - 1) >> 6] >> ((N - 1) & 63)) & 1) ? 0xFFFFu : 0u;
  if (bit >= N) return sign;
  const int q = (int)(bit >> 6), o = (int)(bit & 63);
  const uint64_t lo = s[q];
  const uint64_t hi = (q + 1 < w) ? s[q + 1] : 0;
  uint32_t v = (uint32_t)((o ? (lo >> o) | (hi << (64 - o)) : lo) & 0xFFFFu);
  if (bit + 16 > N) {
    const uint32_t m = (1u << (N - bit)) - 1;
    v = (v & m) | (sign & ~m);
  }
  return v;
}

// BivariateRepresentation (Section 2): limb j of coefficient i, bits [jM, jM + M)
// (the top limb signed), as sum_t chunk_t 2^(16 t) mod p with the table P.
template <int KD>
__global__ __launch_bounds__(GB) void kg_convert(const uint64_t *__restrict__ src, int64_t d,
                                                 int32_t N, int32_t w, int32_t K, int32_t M,
                                                 int32_t T16, int32_t *__restrict__ X,
                                                 int32_t logL, int32_t col_off,
                                                 const int32_t *__restrict__ P) {
  const int64_t i = (int64_t)blockIdx.x * GB + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= d) return;
  const uint64_t *s = src + i * w;
  int64_t z[KD];
#pragma unroll
  for (int l = 0; l < KD; ++l) z[l] = 0;
  for (int t = 0; t < T16; ++t) {
    const int nb = min(16, M - 16 * t);
    uint32_t ch = bits16(s, w, N, (int64_t)j * M + 16 * t);
    int32_t c;
    if (nb < 16) ch &= (1u << nb) - 1;
    if (j == K - 1 && t == T16 - 1) c = (int32_t)(ch << (32 - nb)) >> (32 - nb);   // signed top limb
    else c = (int32_t)ch;
#pragma unroll
    for (int l = 0; l < KD; ++l) z[l] += (int64_t)c * P[t * KD + l];
  }
  // carries in radix r (|z| < 2^50)
  constexpr int64_t R = GfpR<KD>::R;
  int32_t o[KD];
  int64_t c = 0;
#pragma unroll
  for (int l = 0; l < KD; ++l) {
    const int64_t t = z[l] + c;
    const int64_t q = qround64<KD>(t);
    o[l] = (int32_t)(t - q * R);
    c = q;
  }
  {
    const int64_t t = (int64_t)o[0] - c;
    const int64_t q = qround64<KD>(t);
    o[0] = (int32_t)(t - q * R);
    o[1] += (int32_t)q;
  }
  int32_t *dst = X + ((((int64_t)(col_off + j)) << logL) + i) * KD;
#pragma unroll
  for (int l = 0; l < KD; l += 4) *reinterpret_cast<int4 *>(dst + l) = make_int4(o[l], o[l + 1], o[l + 2], o[l + 3]);
}

// tw[t] = hi[t >> sh] lo[t & (2^sh - 1)] = omega^t
template <int KD>
__global__ __launch_bounds__(GB) void kg_twiddles(int32_t *__restrict__ tw, int64_t L, int32_t sh,
                                                  const int32_t *__restrict__ hi,
                                                  const int32_t *__restrict__ lo) {
  const int64_t t = (int64_t)blockIdx.x * GB + threadIdx.x;
  if (t >= L) return;
  int32_t x[KD], y[KD], o[KD];
#pragma unroll
  for (int l = 0; l < KD; ++l) {
    x[l] = hi[(t >> sh) * KD + l];
    y[l] = lo[(t & (((int64_t)1 << sh) - 1)) * KD + l];
  }
  gmul<KD>(x, y, o);
#pragma unroll
  for (int l = 0; l < KD; ++l) tw[t * KD + l] = o[l];
}

// One strided pass of the y-transform (Section 3.3's FFTs along y, four-step): position
// i = inner + S (e + n outer), transform of n = 2^LN points along e with root r^(2k/n),
// then (forward, S > 1) the twiddle omega_{nS}^(f inner) on frequency f; the inverse
// applies the conjugate twiddle first and the inverse transform after.  A k-lane group
// holds one (column, outer, inner) instance.
template <int KD, int LN, int INV>
__global__ __launch_bounds__(GB) void kg_ypass(int32_t *__restrict__ X, int32_t logL, int32_t logS,
                                               int64_t ninst, int32_t col0, int32_t K,
                                               int64_t nz_a, int64_t nz_b, int64_t nlimit,
                                               const int32_t *__restrict__ tw, int32_t twsh) {
  constexpr int N = 1 << LN, G = GB / KD, ES = KD + 4;
  constexpr int ROUNDS = (N + KD - 1) / KD;
  __shared__ __align__(16) int32_t lds[GB * ES];
  const int tid = threadIdx.x, g = tid / KD, l = tid % KD;
  const int base = (tid & 63) & ~(KD - 1);
  const int64_t inst = (int64_t)blockIdx.x * G + g;
  const bool live = inst < ninst;
  const int lpc = logL - LN;
  const int64_t col = (inst >> lpc) + col0;
  const int64_t rem = inst & (((int64_t)1 << lpc) - 1);
  const int64_t inner = rem & (((int64_t)1 << logS) - 1);
  const int64_t outer = rem >> logS;
  const int64_t pos0 = inner + (outer << (logS + LN));
  int32_t *colp = X + (col << logL) * KD + l;
  const int64_t nz = col < K ? nz_a : nz_b;   // rows at and above it are zero (first pass)
  int32_t v[N];
#pragma unroll
  for (int e = 0; e < N; ++e) {
    const int64_t pos = pos0 + ((int64_t)(INV ? brev_c(e, LN) : e) << logS);
    v[e] = (live && (INV || pos < nz)) ? colp[pos * KD] : 0;
  }
  const int64_t L = (int64_t)1 << logL;
  const int tsh = logL - LN - logS;
  // twiddles: register e holds frequency f = bitrev(e); element-per-lane through LDS
  auto twiddle = [&](bool conj) {
#pragma unroll
    for (int rho = 0; rho < ROUNDS; ++rho) {
#pragma unroll
      for (int el = 0; el < KD; ++el)
        if (rho * KD + el < N) lds[(g * KD + el) * ES + l] = v[rho * KD + el];
      __syncthreads();
      const int e = rho * KD + l;
      if (live && e < N) {
        int32_t x[KD], w[KD], y[KD];
        lds_load<KD>(lds + tid * ES, x);
        int64_t t = ((int64_t)brev<LN>(e) * inner) << tsh;
        if (conj) t = (L - t) & (L - 1);
        const int32_t *wp = tw + (t << twsh) * KD;
#pragma unroll
        for (int q = 0; q < KD; q += 4) {
          const int4 u = *reinterpret_cast<const int4 *>(wp + q);
          w[q] = u.x;
          w[q + 1] = u.y;
          w[q + 2] = u.z;
          w[q + 3] = u.w;
        }
        gmul<KD>(x, w, y);
        lds_store<KD>(lds + tid * ES, y);
      }
      __syncthreads();
#pragma unroll
      for (int el = 0; el < KD; ++el)
        if (rho * KD + el < N) v[rho * KD + el] = lds[(g * KD + el) * ES + l];
      __syncthreads();
    }
  };
  const bool tw_on = logS > 0;
  if (INV && tw_on) twiddle(true);
  if (!INV) dif<KD, LN, false>(v, l, base);
  else dit_inv<KD, LN>(v, l, base);
  if (!INV && tw_on) twiddle(false);
#pragma unroll
  for (int e = 0; e < N; ++e) {
    const int64_t pos = pos0 + ((int64_t)(INV ? e : brev_c(e, LN)) << logS);
    if (live && (!INV || pos < nlimit)) colp[pos * KD] = v[e];
  }
}

// Per y-frequency position: 2K-point transforms of a's and b's zero-padded limb rows
// with root theta = r^(k/K) (their first stage is the twist of NegacyclicConvolution;
// even frequencies are CyclicConvolution's), pointwise products, and the inverse, which
// leaves c_{i,j} for j < 2K (the halves (c- + c+)/2 and (c- - c+)/2 of Section 2.1).
template <int KD, int LK, int SQ>
__global__ __launch_bounds__(GB) void kg_xconv(int32_t *__restrict__ X, int32_t logL,
                                               const int32_t *__restrict__ scale) {
  constexpr int K = 1 << LK, N = 2 * K, G = GB / KD, ES = KD + 4;
  constexpr int ROUNDS = (N + KD - 1) / KD;
  __shared__ __align__(16) int32_t lds[GB * ES];
  const int tid = threadIdx.x, g = tid / KD, l = tid % KD;
  const int base = (tid & 63) & ~(KD - 1);
  const int64_t L = (int64_t)1 << logL;
  const int64_t pos = (int64_t)blockIdx.x * G + g;
  const bool live = pos < L;
  int32_t a[N], b[N];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    a[j] = live ? X[(((int64_t)j << logL) + pos) * KD + l] : 0;
    a[j + K] = 0;
    if (!SQ) {
      b[j] = live ? X[(((int64_t)(K + j) << logL) + pos) * KD + l] : 0;
      b[j + K] = 0;
    }
  }
  dif<KD, LK + 1, true>(a, l, base);
  if (!SQ) dif<KD, LK + 1, true>(b, l, base);
#pragma unroll
  for (int rho = 0; rho < ROUNDS; ++rho) {
    const int e = rho * KD + l;
    const bool act = live && e < N;
    int32_t x[KD], y[KD], o[KD];
#pragma unroll
    for (int el = 0; el < KD; ++el)
      if (rho * KD + el < N) lds[(g * KD + el) * ES + l] = a[rho * KD + el];
    __syncthreads();
    if (act) lds_load<KD>(lds + tid * ES, x);
    __syncthreads();
    if (!SQ) {
#pragma unroll
      for (int el = 0; el < KD; ++el)
        if (rho * KD + el < N) lds[(g * KD + el) * ES + l] = b[rho * KD + el];
      __syncthreads();
      if (act) lds_load<KD>(lds + tid * ES, y);
    } else {
#pragma unroll
      for (int q = 0; q < KD; ++q) y[q] = x[q];
    }
    if (act) {
      gmul<KD>(x, y, o);
      if (SQ) {   // a square's one operand was converted unscaled: (2 K L)^{-1} here
#pragma unroll
        for (int q = 0; q < KD; ++q) y[q] = scale[q];
        gmul<KD>(o, y, x);
        lds_store<KD>(lds + tid * ES, x);
      } else {
        lds_store<KD>(lds + tid * ES, o);
      }
    }
    __syncthreads();
#pragma unroll
    for (int el = 0; el < KD; ++el)
      if (rho * KD + el < N) a[rho * KD + el] = lds[(g * KD + el) * ES + l];
    __syncthreads();
  }
  dit_inv<KD, LK + 1>(a, l, base);
  if (live) {
#pragma unroll
    for (int j = 0; j < N; ++j) X[(((int64_t)j << logL) + pos) * KD + l] = a[j];
  }
}

// 32-bit word q of a W-word two's complement value (sign words above)
__device__ __forceinline__ uint32_t wordx(const uint32_t *v, int W, int q) {
  return q < W ? v[q] : (uint32_t)((int32_t)v[W - 1] >> 31);
}

// RecoveringProduct (Section 2.2) with one prime: each c_{i,j} mod p is lifted to the
// integer in (-p/2, p/2) (exact, since |c_{i,j}| < p/4), then c_i = sum_j c_{i,j} 2^(Mj)
// with carries.  One wave per output coefficient.
template <int KD>
__global__ __launch_bounds__(64) void kg_recover(const int32_t *__restrict__ X, int32_t logL,
                                                 int32_t K, int32_t M, int64_t nout, int32_t nw32,
                                                 int32_t wc, const GfpConstDev *__restrict__ cst,
                                                 uint64_t *__restrict__ out) {
  constexpr int W = GfpR<KD>::W;
  constexpr int S1 = GfpR<KD>::S1, G1 = GfpR<KD>::G1, S2 = GfpR<KD>::S2, G2 = GfpR<KD>::G2;
  extern __shared__ uint32_t sm[];
  const int lane = threadIdx.x;
  const int64_t i = blockIdx.x;
  if (i >= nout) return;
  uint32_t *vals = sm;                                     // 2K x W words
  uint64_t *sums = reinterpret_cast<uint64_t *>(sm + ((2 * K * W + 1) & ~1));   // nw32
  if (lane < 2 * K) {
    int32_t dg[KD];
    const int32_t *src = X + ((((int64_t)lane) << logL) + i) * KD;
#pragma unroll
    for (int l = 0; l < KD; l += 4) {
      const int4 u = *reinterpret_cast<const int4 *>(src + l);
      dg[l] = u.x;
      dg[l + 1] = u.y;
      dg[l + 2] = u.z;
      dg[l + 3] = u.w;
    }
    double vf = 0;
#pragma unroll
    for (int l = 0; l < KD; ++l) vf += (double)dg[l] * cst->rpow[l];
    const int q = vf > cst->phalf ? 1 : (vf < -cst->phalf ? -1 : 0);
    // Horner in binary: V = V r + d_l, r = 2^29 + G1 2^S1 + G2 2^S2
    uint32_t V[W];
#pragma unroll
    for (int w = 0; w < W; ++w) V[w] = (uint32_t)(dg[KD - 1] >> 31);
    V[0] = (uint32_t)dg[KD - 1];
#pragma unroll
    for (int s = 1; s < KD; ++s) {
      const int dl = dg[KD - 1 - s];
      // |V| < r^(s+1): the words that can be nonzero now (the rest hold the sign)
      const int wl = min(W, (29 * (s + 1) + 1 + 31) / 32 + 1);
      int64_t carry = dl;
      uint32_t prev = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        if (w < wl) {
          const uint32_t cur = V[w];
          const uint32_t t29 = (cur << 29) | (w ? prev >> 3 : 0);
          const uint32_t ta = (cur << S1) | (w ? prev >> (32 - S1) : 0);
          int64_t acc = (int64_t)t29 + G1 * (int64_t)ta + carry;
          if constexpr (G2 != 0) {
            const uint32_t tb = (cur << S2) | (w ? prev >> (32 - S2) : 0);
            acc += G2 * (int64_t)tb;
          }
          prev = cur;
          V[w] = (uint32_t)acc;
          carry = acc >> 32;
        } else if (w == wl) {
          V[w] = (uint32_t)((int32_t)V[w - 1] >> 31);
        }
      }
    }
    if (q) {   // V - q p
      int64_t carry = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const int64_t acc = (int64_t)V[w] - q * (int64_t)cst->pbin[w] + carry;
        V[w] = (uint32_t)acc;
        carry = acc >> 32;
      }
    }
#pragma unroll
    for (int w = 0; w < W; ++w) vals[lane * W + w] = V[w];
  }
  __syncthreads();
  // column sums of the shifted values (unsigned 32-bit slices of the sign-extended terms)
  for (int col = lane; col < nw32; col += 64) {
    uint64_t s = 0;
    for (int j = 0; j < 2 * K; ++j) {
      const int64_t o = (int64_t)32 * col - (int64_t)M * j;   // bit of c_{i,j} at this column
      if (o <= -32) continue;
      const uint32_t *v = vals + j * W;
      uint32_t sl;
      if (o < 0) {
        sl = v[0] << (-o);
      } else {
        const int qw = (int)(o >> 5), sh = (int)(o & 31);
        const uint32_t lo = wordx(v, W, qw);
        sl = sh ? (lo >> sh) | (wordx(v, W, qw + 1) << (32 - sh)) : lo;
      }
      s += sl;
    }
    sums[col] = s;
  }
  __syncthreads();
  if (lane == 0) {
    uint64_t carry = 0;
    for (int col = 0; col < nw32; ++col) {
      const uint64_t t = sums[col] + carry;
      sums[col] = (uint32_t)t;
      carry = t >> 32;
    }
  }
  __syncthreads();
  const int nw64 = nw32 / 2;
  const uint64_t sgn = ((sums[nw32 - 1] >> 31) & 1) ? ~(uint64_t)0 : 0;
  uint64_t *o = out + i * wc;
  for (int u = lane; u < wc; u += 64) o[u] = u < nw64 ? (sums[2 * u] | (sums[2 * u + 1] << 32)) : sgn;
}

// ------------------------------------------------------------------------------------
// context state, tables, launch sequence
// ------------------------------------------------------------------------------------
struct GfpState {
  int32_t *tw[GFP_NPRIMES] = {nullptr, nullptr, nullptr};   // omega^t, t < 2^logLtab
  int logLtab[GFP_NPRIMES] = {-1, -1, -1};
  std::map<std::tuple<int, int, int>, GfpConstDev *> consts;   // (prime, K, logL)
  int32_t *ws = nullptr;
  int64_t ws_words = 0;
};

template <int KD>
static void launch_twiddles(int32_t *tw, int64_t L, int sh, const int32_t *hi, const int32_t *lo,
                            hipStream_t st) {
  hipLaunchKernelGGL(kg_twiddles<KD>, dim3((unsigned)((L + GB - 1) / GB)), dim3(GB), 0, st, tw, L, sh,
                     hi, lo);
}

static int ensure_twiddles(GfpState &S, int prime, int logL) {
  if (S.logLtab[prime] >= logL) return ZPM_OK;
  const GfpPrime &P = gfp_prime_table()[prime];
  const int lt = std::max(logL, 1);
  HE w;
  if (!root_of(P, lt, w)) return ZPM_EUNSUPPORTED;
  const int64_t L = (int64_t)1 << lt;
  const int sh = (lt + 1) / 2;
  const int64_t nlo = (int64_t)1 << sh, nhi = L >> sh;
  std::vector<int32_t> host((size_t)(nlo + nhi) * P.k);
  HE x = h_from(P, 1);
  for (int64_t t = 0; t < nlo; ++t) {
    for (int l = 0; l < P.k; ++l) host[(size_t)t * P.k + l] = (int32_t)x.d[l];
    x = h_mul(P, x, w);
  }
  const HE step = x;   // omega^(2^sh)
  x = h_from(P, 1);
  for (int64_t t = 0; t < nhi; ++t) {
    for (int l = 0; l < P.k; ++l) host[(size_t)(nlo + t) * P.k + l] = (int32_t)x.d[l];
    x = h_mul(P, x, step);
  }
  int32_t *tab = nullptr, *tmp = nullptr;
  if (hipMalloc(&tab, (size_t)L * P.k * 4) != hipSuccess) return ZPM_ENOMEM;
  if (hipMalloc(&tmp, host.size() * 4) != hipSuccess) {
    (void)hipFree(tab);
    return ZPM_ENOMEM;
  }
  if (hipMemcpy(tmp, host.data(), host.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(tab);
    (void)hipFree(tmp);
    return ZPM_EDEVICE;
  }
  const int32_t *lo = tmp, *hi = tmp + (size_t)nlo * P.k;
  if (P.k == 8) launch_twiddles<8>(tab, L, sh, hi, lo, nullptr);
  else if (P.k == 16) launch_twiddles<16>(tab, L, sh, hi, lo, nullptr);
  else launch_twiddles<32>(tab, L, sh, hi, lo, nullptr);
  // the old table may still be read by queued work
  if (hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(tab);
    (void)hipFree(tmp);
    return ZPM_EDEVICE;
  }
  (void)hipFree(tmp);
  if (S.tw[prime]) (void)hipFree(S.tw[prime]);
  S.tw[prime] = tab;
  S.logLtab[prime] = lt;
  return ZPM_OK;
}

static int plan_consts_gfp(GfpState &S, const PlanGfp &pl, GfpConstDev **out) {
  const auto key = std::make_tuple(pl.prime, pl.K, pl.logL);
  auto it = S.consts.find(key);
  if (it != S.consts.end()) {
    *out = it->second;
    return ZPM_OK;
  }
  const GfpPrime &P = gfp_prime_table()[pl.prime];
  GfpConstDev h;
  std::memset(&h, 0, sizeof(h));
  int lk = 0;
  while ((1 << lk) < pl.K) ++lk;
  const HE s = inv_pow2(P, 1 + lk + pl.logL);   // (2 K L)^{-1}
  for (int l = 0; l < P.k; ++l) h.scale[l] = (int32_t)s.d[l];
  const HE c16 = h_from(P, 65536);
  HE x = h_from(P, 1);
  for (int t = 0; t < GFP_TMAX; ++t) {
    const HE xs = h_mul(P, x, s);
    for (int l = 0; l < P.k; ++l) {
      h.Pa[t * P.k + l] = (int32_t)x.d[l];
      h.Pb[t * P.k + l] = (int32_t)xs.d[l];
    }
    x = h_mul(P, x, c16);
  }
  std::vector<uint32_t> pw(GFP_WMAX + 2, 0);
  pw[0] = 1;
  for (int t = 0; t < P.k; ++t) {
    uint64_t c = 0;
    for (auto &w : pw) {
      const uint64_t v = (uint64_t)w * (uint32_t)P.r + c;
      w = (uint32_t)v;
      c = v >> 32;
    }
  }
  pw[0] += 1;
  for (int w = 0; w < GFP_WMAX; ++w) h.pbin[w] = pw[w];
  for (int l = 0; l < P.k; ++l) h.rpow[l] = std::pow((double)P.r, (double)l);
  h.phalf = 0.5 * std::pow((double)P.r, (double)P.k);
  GfpConstDev *d = nullptr;
  if (hipMalloc(&d, sizeof(h)) != hipSuccess) return ZPM_ENOMEM;
  if (hipMemcpy(d, &h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return ZPM_EDEVICE;
  }
  S.consts[key] = d;
  *out = d;
  return ZPM_OK;
}

static int ensure_ws_gfp(GfpState &S, int64_t words) {
  if (words <= S.ws_words) return ZPM_OK;
  if (hipDeviceSynchronize() != hipSuccess) return ZPM_EDEVICE;
  if (S.ws) (void)hipFree(S.ws);
  S.ws = nullptr;
  S.ws_words = 0;
  if (hipMalloc(&S.ws, (size_t)words * 4) != hipSuccess) return ZPM_ENOMEM;
  S.ws_words = words;
  return ZPM_OK;
}

template <int KD, int INV>
static bool launch_pass_kd(const PlanGfp &pl, GfpState &S, int q, int cols, hipStream_t st) {
  const int ln = pl.pass_logn[q];
  int logS = 0;
  for (int t = q + 1; t < pl.npass; ++t) logS += pl.pass_logn[t];
  const int64_t L = (int64_t)1 << pl.logL;
  const int64_t ninst = (int64_t)cols * (L >> ln);
  const int G = GB / KD;
  const dim3 grid((unsigned)((ninst + G - 1) / G));
  const int64_t nz_a = q == 0 ? pl.da : L, nz_b = q == 0 ? pl.db : L;
  const int64_t nlimit = q == 0 ? pl.nout : L;
  const int twsh = S.logLtab[pl.prime] - pl.logL;
  int32_t *X = S.ws;
  const int32_t *tw = S.tw[pl.prime];
#define ZPM_GP(LN_)                                                                           \
  case LN_:                                                                                   \
    if constexpr ((1 << LN_) <= 2 * KD)                                                       \
      hipLaunchKernelGGL((kg_ypass<KD, LN_, INV>), grid, dim3(GB), 0, st, X, pl.logL, logS,   \
                         ninst, 0, pl.K, nz_a, nz_b, nlimit, tw, twsh);                       \
    else                                                                                      \
      return false;                                                                           \
    break;
  switch (ln) {
    ZPM_GP(1) ZPM_GP(2) ZPM_GP(3) ZPM_GP(4) ZPM_GP(5) ZPM_GP(6)
    default: return false;
  }
#undef ZPM_GP
  return true;
}

template <int KD>
static bool launch_all(const PlanGfp &pl, GfpState &S, const GfpConstDev *cd, const uint64_t *a,
                       const uint64_t *b, uint64_t *c, int32_t wc, hipStream_t st, Profiler &prof) {
  const int64_t L = (int64_t)1 << pl.logL;
  int32_t *X = S.ws;
  const char *cb = reinterpret_cast<const char *>(cd);   // device address
  const int32_t *Pa = reinterpret_cast<const int32_t *>(cb + offsetof(GfpConstDev, Pa));
  const int32_t *Pb = reinterpret_cast<const int32_t *>(cb + offsetof(GfpConstDev, Pb));
  const int32_t *sc = reinterpret_cast<const int32_t *>(cb + offsetof(GfpConstDev, scale));
  prof.begin(KK_GFP_CONVERT, st);
  for (int op = 0; op < (pl.square ? 1 : 2); ++op) {
    const uint64_t *x = op ? b : a;
    const int64_t d = op ? pl.db : pl.da;
    const int32_t N = op ? pl.Nb : pl.Na;
    // b's limbs carry the scale (2 K L)^{-1} of the inverse transforms (a square's
    // operand is converted unscaled and scaled in the x-kernel)
    hipLaunchKernelGGL(kg_convert<KD>, dim3((unsigned)((d + GB - 1) / GB), (unsigned)pl.K), dim3(GB), 0,
                       st, x, d, N, (N + 63) / 64, pl.K, pl.M, pl.T16, X, pl.logL, op ? pl.K : 0,
                       op ? Pb : Pa);
  }
  prof.end(st);
  prof.begin(KK_GFP_YFWD, st);
  for (int q = 0; q < pl.npass; ++q)
    if (!launch_pass_kd<KD, 0>(pl, S, q, pl.square ? pl.K : 2 * pl.K, st)) return false;
  prof.end(st);
  prof.begin(KK_GFP_X, st);
  const int G = GB / KD;
  const dim3 xg((unsigned)((L + G - 1) / G));
  int lk = 0;
  while ((1 << lk) < pl.K) ++lk;
#define ZPM_GX(LK_)                                                                                \
  case LK_:                                                                                        \
    if constexpr ((1 << LK_) <= KD) {                                                              \
      if (pl.square) hipLaunchKernelGGL((kg_xconv<KD, LK_, 1>), xg, dim3(GB), 0, st, X, pl.logL, sc); \
      else hipLaunchKernelGGL((kg_xconv<KD, LK_, 0>), xg, dim3(GB), 0, st, X, pl.logL, sc);           \
    } else {                                                                                       \
      return false;                                                                                \
    }                                                                                              \
    break;
  switch (lk) {
    ZPM_GX(1) ZPM_GX(2) ZPM_GX(3) ZPM_GX(4) ZPM_GX(5)
    default: return false;
  }
#undef ZPM_GX
  prof.end(st);
  prof.begin(KK_GFP_YINV, st);
  for (int q = pl.npass - 1; q >= 0; --q)
    if (!launch_pass_kd<KD, 1>(pl, S, q, 2 * pl.K, st)) return false;
  prof.end(st);
  prof.begin(KK_GFP_RECOVER, st);
  const int nw32 = 2 * ((pl.nout_bits + 63) / 64);
  const size_t lds = 4 * (size_t)((2 * pl.K * pl.W + 1) & ~1) + 8 * (size_t)nw32;
  hipLaunchKernelGGL(kg_recover<KD>, dim3((unsigned)pl.nout), dim3(64), lds, st, X, pl.logL, pl.K,
                     pl.M, pl.nout, nw32, wc, cd, c);
  prof.end(st);
  return true;
}

int mul_gfp(Ctx &cx, const PlanGfp &pl, const uint64_t *a, const uint64_t *b, uint64_t *c,
            int32_t wc, hipStream_t st) {
  if (!cx.gfp) cx.gfp = new GfpState();
  GfpState &S = *cx.gfp;
  const GfpPrime &P = gfp_prime_table()[pl.prime];
  // shapes the kernels rely on
  if (pl.k != P.k || gfp_W(P.k) != P.W || pl.W != P.W || pl.K < 2 || pl.K > P.k ||
      (pl.K & (pl.K - 1)) || pl.T16 < 1 || pl.T16 > GFP_TMAX || pl.logL > GFP_LOG2_LMAX)
    return ZPM_EINVAL;
  int sum = 0;
  for (int q = 0; q < pl.npass; ++q) {
    if (pl.pass_logn[q] < 1 || (1 << pl.pass_logn[q]) > 2 * P.k || pl.pass_logn[q] > 6) return ZPM_EINVAL;
    sum += pl.pass_logn[q];
  }
  if (sum != pl.logL) return ZPM_EINVAL;
  const int nw32 = 2 * ((pl.nout_bits + 63) / 64);
  if (4 * (size_t)((2 * pl.K * pl.W + 1) & ~1) + 8 * (size_t)nw32 > 65536) return ZPM_EUNSUPPORTED;
  int rc;
  if ((rc = ensure_twiddles(S, pl.prime, pl.logL)) != ZPM_OK) return rc;
  GfpConstDev *cd = nullptr;
  if ((rc = plan_consts_gfp(S, pl, &cd)) != ZPM_OK) return rc;
  if ((rc = ensure_ws_gfp(S, pl.ws_words)) != ZPM_OK) return rc;
  bool ok;
  if (P.k == 8) ok = launch_all<8>(pl, S, cd, a, b, c, wc, st, cx.prof);
  else if (P.k == 16) ok = launch_all<16>(pl, S, cd, a, b, c, wc, st, cx.prof);
  else ok = launch_all<32>(pl, S, cd, a, b, c, wc, st, cx.prof);
  if (!ok) return ZPM_EINVAL;
  return hipGetLastError() == hipSuccess ? ZPM_OK : ZPM_EDEVICE;
}

void gfp_release(Ctx &cx) {
  if (!cx.gfp) return;
  GfpState &S = *cx.gfp;
  (void)hipSetDevice(cx.device);
  (void)hipDeviceSynchronize();
  if (S.ws) (void)hipFree(S.ws);
  for (auto *t : S.tw)
    if (t) (void)hipFree(t);
  for (auto &kv : S.consts) (void)hipFree(kv.second);
  delete cx.gfp;
  cx.gfp = nullptr;
}

}  // namespace zpm
