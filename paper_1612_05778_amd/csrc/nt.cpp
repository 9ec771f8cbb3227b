// Host number theory for the word-size prime variant (Section 4: machine-word
// Fourier primes combined by the Chinese remaindering algorithm).
//
// * Fourier primes p < 2^30 with 2^21 | p - 1 (Section 2.1, root-of-unity
//   condition), found by deterministic Miller-Rabin, largest first.
// * A primitive 2^21-th root of unity per prime; every transform length used
//   takes its roots as powers of it, so all tables agree.
// * Shoup companions floor(w 2^32 / p) for constant multipliers.
// * CRT constants for recovering c_{i,j} in (-P/2, P/2) from its residues.
#include "nt.hpp"

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>
#include <cstdlib>

namespace zpm {

uint32_t mulmod(uint32_t a, uint32_t b, uint32_t p) { return (uint32_t)((uint64_t)a * b % p); }

uint32_t powmod(uint32_t a, uint64_t e, uint32_t p) {
  uint64_t r = 1 % p, x = a % p;
  while (e) {
    if (e & 1) r = r * x % p;
    x = x * x % p;
    e >>= 1;
  }
  return (uint32_t)r;
}

uint32_t invmod(uint32_t a, uint32_t p) { return powmod(a, p - 2, p); }   // p prime

uint32_t shoup(uint32_t w, uint32_t p) { return (uint32_t)(((uint64_t)w << 32) / p); }

static bool miller_rabin(uint32_t n) {
  if (n < 2) return false;
  for (uint32_t q : {2u, 3u, 5u, 7u, 11u, 13u}) {
    if (n % q == 0) return n == q;
  }
  uint32_t d = n - 1;
  int s = 0;
  while (!(d & 1)) { d >>= 1; ++s; }
  // bases 2, 7, 61 are deterministic for n < 4759123141
  for (uint32_t a : {2u, 7u, 61u}) {
    if (a % n == 0) continue;
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = x * x % n;
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

bool is_prime(uint32_t n) { return miller_rabin(n); }

// A generator of (Z/p)^*: g with g^((p-1)/q) != 1 for every prime q | p - 1.
static uint32_t generator(uint32_t p) {
  uint32_t m = p - 1;
  uint32_t fac[32];
  int nf = 0;
  uint32_t t = m;
  for (uint32_t q = 2; (uint64_t)q * q <= t; ++q) {
    if (t % q == 0) {
      fac[nf++] = q;
      while (t % q == 0) t /= q;
    }
  }
  if (t > 1) fac[nf++] = t;
  for (uint32_t g = 2; g < p; ++g) {
    bool ok = true;
    for (int i = 0; i < nf && ok; ++i) ok = powmod(g, m / fac[i], p) != 1;
    if (ok) return g;
  }
  return 0;
}

const std::vector<PrimeHost> &prime_table() {
  static std::vector<PrimeHost> table;
  static std::once_flag once;
  std::call_once(once, [] {
    const uint32_t step = 1u << LOG2_ROOT_ORDER;
    // below 2^30: the transforms keep values in [0, 2p) and sums of two in [0, 4p)
    for (uint64_t k = ((1ull << PRIME_BITS) - 1) / step; k >= 1 && (int)table.size() < MAXNP; --k) {
      uint64_t p = k * step + 1;
      if (p >= (1ull << PRIME_BITS) || !is_prime((uint32_t)p)) continue;
      PrimeHost h;
      h.p = (uint32_t)p;
      uint32_t g = generator(h.p);
      h.root = powmod(g, (p - 1) >> LOG2_ROOT_ORDER, h.p);   // order exactly 2^21
      // p^{-1} mod 2^32 by Newton iteration
      uint32_t inv = h.p;
      for (int i = 0; i < 5; ++i) inv *= 2u - h.p * inv;
      h.pinv = inv;
      h.c32 = (uint32_t)((1ull << 32) % p);
      h.c32s = shoup(h.c32, h.p);
      h.ones = shoup(1, h.p);
      table.push_back(h);
    }
  });
  return table;
}

// Root of order 2^e (e <= 21) for prime index k: root^(2^(21-e)).
uint32_t root_of_order(int k, int e) {
  const PrimeHost &h = prime_table()[k];
  return powmod(h.root, 1ull << (LOG2_ROOT_ORDER - e), h.p);
}

void fill_heap(int k, int H, uint2 *hf, uint2 *hi) {
  // hf[h + j] = w_{2h}^j, hi[h + j] = w_{2h}^{-j} for h = 1, 2, ..., H/2 and j < h.
  const uint32_t p = prime_table()[k].p;
  hf[0] = make_uint2(0, 0);
  hi[0] = make_uint2(0, 0);
  for (int lh = 0; (1 << lh) < H; ++lh) {
    int h = 1 << lh;
    uint32_t w = root_of_order(k, lh + 1);
    uint32_t wi = invmod(w, p);
    uint32_t x = 1, xi = 1;
    for (int j = 0; j < h; ++j) {
      hf[h + j] = make_uint2(x, shoup(x, p));
      hi[h + j] = make_uint2(xi, shoup(xi, p));
      x = mulmod(x, w, p);
      xi = mulmod(xi, wi, p);
    }
  }
}

// ---- small multi-word helpers on little-endian 32-bit words ----
static void mw_mul_small(uint32_t *x, int n, uint32_t m) {
  uint64_t c = 0;
  for (int i = 0; i < n; ++i) {
    uint64_t t = (uint64_t)x[i] * m + c;
    x[i] = (uint32_t)t;
    c = t >> 32;
  }
}

static uint32_t mw_mod_small(const uint32_t *x, int n, uint32_t p) {
  uint64_t r = 0;
  for (int i = n - 1; i >= 0; --i) r = ((r << 32) | x[i]) % p;
  return (uint32_t)r;
}

int bitlen_product(int np) {
  uint32_t P[MAXW + 1];
  std::memset(P, 0, sizeof(P));
  P[0] = 1;
  for (int k = 0; k < np; ++k) mw_mul_small(P, MAXW + 1, prime_table()[k].p);
  for (int i = MAXW; i >= 0; --i) {
    if (P[i]) return 32 * i + (32 - __builtin_clz(P[i]));
  }
  return 0;
}

// True if P = prod_{k<np} p_k > 2 d K 2^(2M) (1 + 2^-12), with d = min(da, db).
// Relation (recoveryModulo) bounds the prime by 4 d K 2^(2M) because it must hold
// c+_{i,j} and c-_{i,j} (each below 2 d K 2^(2M) in magnitude) in its symmetric range.
// Here the halving (c+ + c-) / 2 and (c- - c+) / 2 is done modulo each prime before the
// Chinese remaindering, which therefore recovers c_{i,j} itself: a sum of at most
// min(da, db) K products of limbs below 2^M in magnitude, so |c_{i,j}| < d K 2^(2M) and
// P > 2 |c_{i,j}| suffices for (-P/2, P/2).  The factor 1 + 2^-12 keeps |c_{i,j}| / P at
// least 2^-13 below 1/2, the margin the recovery's floating-point quotient needs.
bool primes_cover(int np, int64_t d, int64_t K, int64_t M) {
  const int n = MAXW + 1;
  uint32_t R[MAXW + 1];
  std::memset(R, 0, sizeof(R));
  const uint64_t dk = (uint64_t)d * (uint64_t)K;      // callers keep d K < 2^62
  // 4096 P > 4097 d K 2^(2M+1)
  const int64_t shift = 2 * M + 1;
  const int64_t w = shift / 32;
  const unsigned __int128 t = ((unsigned __int128)dk * 4097u) << (shift % 32);   // < 2^107
  for (int i = 0; i < 4; ++i) {
    uint32_t part = (uint32_t)(t >> (32 * i));
    if (!part) continue;
    if (w + i >= n) return false;                     // rhs beyond what MAXNP primes reach
    R[w + i] = part;
  }
  uint32_t P[MAXW + 1];
  std::memset(P, 0, sizeof(P));
  P[0] = 1;
  for (int k = 0; k < np; ++k) mw_mul_small(P, n, prime_table()[k].p);
  mw_mul_small(P, n, 4096u);
  for (int i = n - 1; i >= 0; --i) {
    if (P[i] != R[i]) return P[i] > R[i];
  }
  return false;   // strict inequality required
}

// Balanced base-256 digits d_n in [-128, 127] of x = sign * |x| (|x| little-endian 32-bit
// words), nd of them; false if x does not fit.  For x < 0 the digits of |x| are taken in
// [-127, 128] and negated.
static bool balanced_bytes(const uint32_t *mag, int nw, int sign, int nd, int8_t *out) {
  int carry = 0;
  for (int n = 0; n < nd; ++n) {
    const int byte = n < 4 * nw ? (int)((mag[n >> 2] >> (8 * (n & 3))) & 255u) : 0;
    int v = byte + carry;
    const bool wrap = sign > 0 ? v >= 128 : v > 128;
    carry = wrap ? 1 : 0;
    if (wrap) v -= 256;
    out[n] = (int8_t)(sign > 0 ? v : -v);
  }
  if (carry) return false;
  for (int n = nd; n < 4 * nw; ++n)
    if ((mag[n >> 2] >> (8 * (n & 3))) & 255u) return false;
  return true;
}

// The CRT sum c = sum_k y_k (P / p_k) - t P as an int8 matrix product.  Each term (y_k
// centred in (-p_k/2, p_k/2), and t, |t| <= np/2) is split into balanced signed bytes,
// one slot per byte a < 4 (t uses a = 0 only), placed in the B operand as crt_term
// says; each constant P/p_k and -P is written in balanced bytes too, and
// A[n][(term, a)] = digit n - a of the term's constant, so that
// c = sum_n 2^(8n) sum_slot A[n][slot] y_slot.  Rows are placed so that
// lane group g of the product's output holds digits 4 TN g + 4 T + i (tile T, row i),
// i.e. the consecutive words TN g .. TN g + TN - 1 of the value.
static void crt_matrix_constants(int np, const uint32_t *P, const uint32_t (*Q)[MAXW],
                                 PlanDev &pd) {
  static_assert(crt_tiles(CRT_MFMA_NP) <= CRT_TILES, "CRT tiles");
  static_assert((CRT_MFMA_NP + 1 + 15) / 16 <= CRT_STEPS, "CRT steps");
  std::memset(pd.crt_afrag, 0, sizeof(pd.crt_afrag));
  if (np > CRT_MFMA_NP) return;
  const int TN = crt_tiles(np), ND = 16 * TN;
  std::vector<int8_t> dig((size_t)(np + 1) * ND, 0);
  // a constant's digit b meets byte a < 4 at row b + a: its digits must end 3 rows early
  for (int k = 0; k < np; ++k)
    if (!balanced_bytes(Q[k], MAXW, 1, ND - 3, &dig[(size_t)k * ND])) std::abort();
  if (!balanced_bytes(P, MAXW, -1, ND, &dig[(size_t)np * ND])) std::abort();
  // slot (s, g, 4 w + a): byte a of term crt_term(s, g, w)
  auto A = [&](int n, int term, int a) -> int {
    if (term > np || (term == np && a != 0) || n - a < 0) return 0;
    return dig[(size_t)term * ND + (n - a)];
  };
  auto row_digit = [&](int T, int m) { return 4 * TN * (m >> 2) + 4 * T + (m & 3); };
  for (int T = 0; T < TN; ++T)
    for (int st = 0; st < CRT_STEPS; ++st)
      for (int lane = 0; lane < 64; ++lane) {
        const int n = row_digit(T, lane & 15);
        for (int b = 0; b < 16; ++b) {
          const int term = crt_term(st, lane >> 4, b >> 2);
          pd.crt_afrag[T][st][lane][b >> 2] |= (uint32_t)(uint8_t)(int8_t)A(n, term, b & 3)
                                               << (8 * (b & 3));
        }
      }
}

void crt_constants(int np, PlanDev &pd) {
  const auto &T = prime_table();
  uint32_t P[MAXW];
  std::memset(P, 0, sizeof(P));
  P[0] = 1;
  for (int k = 0; k < np; ++k) mw_mul_small(P, MAXW, T[k].p);
  std::memcpy(pd.crt_p, P, sizeof(P));
  for (int k = 0; k < np; ++k) {
    uint32_t Q[MAXW];
    std::memset(Q, 0, sizeof(Q));
    Q[0] = 1;
    for (int t = 0; t < np; ++t)
      if (t != k) mw_mul_small(Q, MAXW, T[t].p);
    std::memcpy(pd.crt_q[k], Q, sizeof(Q));
    uint32_t qk = mw_mod_small(Q, MAXW, T[k].p);
    uint32_t inv = invmod(qk, T[k].p);
    pd.crt_inv[k] = make_uint2(inv, shoup(inv, T[k].p));
    pd.crt_rcp[k] = 1.0 / (double)T[k].p;
  }
  crt_matrix_constants(np, pd.crt_p, pd.crt_q, pd);
}

void scale_constants(int np, int K, int M, int logL, PlanDev &pd) {
  const auto &T = prime_table();
  for (int k = 0; k < np; ++k) {
    uint32_t p = T[k].p;
    // The transforms are left unscaled and the pointwise product is a Montgomery
    // product, so the row kernels leave c_{i,j} (2K L) 2^-32 mod p.  The normalisation
    // 2^32 (2K L)^{-1} is folded into the recovery's first constant, (P/p_k)^{-1}
    // (crt_constants must have run).
    uint64_t n = ((uint64_t)(2 * K) << logL) % p;
    uint32_t s = mulmod(invmod((uint32_t)n, p), T[k].c32, p);
    pd.scale[k] = make_uint2(s, shoup(s, p));
    const uint32_t ci = mulmod(pd.crt_inv[k].x, s, p);
    pd.crt_inv[k] = make_uint2(ci, shoup(ci, p));
    pd.pow2M[k] = powmod(2, (uint64_t)M, p);
  }
}

}  // namespace zpm
