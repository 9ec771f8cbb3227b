// Variant with one big generalized Fermat prime (Section 3.1: a single prime p in
// place of several machine-word primes and CRT, with p a generalized Fermat number
// r^k + 1 so that r is a 2k-th root of unity and products by its powers are cheap,
// Relation (FurerHypothesis); Section 5 names this as the variant the paper's own
// implementation had not yet built).
//
// An element of Z/pZ is k balanced digits in radix r (value sum d_l r^l), each digit a
// 32-bit lane word.  Because r^k = -1, multiplying by r^e is a rotation of the digits
// by e places with the wrapped ones negated: the x-transforms (length 2K <= 2k, root
// theta = r^(k/K)) and every y-pass of length n <= 2k (root r^(2k/n)) take no
// multiplications; generic products in Z/pZ (negacyclic digit convolutions) appear
// only in the twiddles between y-passes and in the pointwise products.
//
// The primes have a radix r < 2^29 with at most three terms, so that a digit product
// fits a 32 x 32 -> 64-bit multiply-add and multiplying by r is two or three shifts:
//   k =  8: r = 2^29 - 2^25,         p ~ 2^232
//   k = 16: r = 2^29 - 2^9 - 2^7,    p ~ 2^464
//   k = 32: r = 2^29 - 2^14 - 2^13,  p ~ 2^928
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zpm {

constexpr int GFP_NPRIMES = 3;
constexpr int GFP_KMAX = 32;         // digits of the largest prime
constexpr int GFP_LOG2_LMAX = 21;    // y-transform length limit (twiddle table L k words)
constexpr int GFP_MAX_PASS = 6;

// p = r^k + 1, r = 2^29 + g1 2^s1 + g2 2^s2 (g2 = 0: two terms).
struct GfpPrime {
  int32_t k;
  int32_t r;
  int32_t s1, g1, s2, g2;
  int32_t W;        // 32-bit words of a signed value of absolute value below p
  int32_t log2p;    // bit length of p
};
const GfpPrime *gfp_prime_table();   // GFP_NPRIMES entries, k ascending

struct PlanGfp {
  int64_t da, db, nout;
  int32_t Na, Nb, nout_bits;
  int32_t prime;      // index into gfp_prime_table()
  int32_t k;          // digits of the prime
  int32_t K, M;       // K limbs of M bits (K <= k, so theta = r^(k/K))
  int32_t logL;       // cyclic length along y
  int32_t npass;
  int32_t pass_logn[GFP_MAX_PASS];   // y-pass lengths, outermost first (each <= 2k points)
  int32_t T16;        // 16-bit chunks per limb in the conversion
  int32_t W;
  int32_t square;
  int64_t ws_words;   // 2K L k int32 digits
  double cost;
};

bool make_plan_gfp(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K_force,
                   int32_t prime_force, PlanGfp &out);

// Host number theory.  omega: the root of order L = 2^logL used by the y-transforms,
// normalised to balanced digits; omega^(L/2k) = r when L >= 2k, omega = r^(2k/L)
// otherwise, so that every y-pass of n <= 2k points has root r^(2k/n).
bool gfp_root(int prime, int logL, int32_t *digits);

struct Ctx;
struct GfpState;
int mul_gfp(Ctx &cx, const PlanGfp &pl, const uint64_t *a, const uint64_t *b, uint64_t *c,
            int32_t wc, hipStream_t st);
void gfp_release(Ctx &cx);

}  // namespace zpm
