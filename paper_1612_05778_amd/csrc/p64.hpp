// Variant with 64-bit machine-word Fourier primes (Section 4: the modulus is one
// machine-word prime, or the product of two or three of them combined by the Chinese
// remaindering algorithm; the paper's own implementation uses two).  The method is
// unchanged: K limbs of M bits, a 2K x L two-dimensional cyclic convolution of the
// zero-padded limb arrays (whose even and odd x-frequencies are the cyclic and the
// twisted negacyclic parts of Section 2.1), CRT, evaluation at 2^M with carries.
//
// Residues are 64-bit words modulo primes p < 2^62; gfx950 has no 64-bit multiplier,
// so each modular product is built from 32-bit multiplies.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zpm {

constexpr int MAXNP64 = 3;            // one, two or three machine-word primes
constexpr int LOG2_ROOT64 = 21;       // every prime has a primitive 2^21-th root
constexpr int K_MAX64 = 512;
constexpr int MAX_PASS64 = 3;
constexpr int LDS64 = 8192;           // 64-bit words of LDS per workgroup (64 KiB)

// A constant multiplier and its Shoup companion floor(w 2^64 / p).
struct W64 {
  uint64_t w, s;
};

struct Prime64Dev {
  uint64_t p;
  uint64_t pinv;     // p^{-1} mod 2^64 (Montgomery)
  W64 one;           // (1, floor(2^64 / p)): reduces any 64-bit word
  W64 c64;           // 2^64 mod p
  const W64 *hf;     // hf[h + j] = w_{2h}^j, w a primitive 2h-th root (heap order)
  const W64 *hi;     // hi[h + j] = w_{2h}^{-j}
};

// Per-plan constants.
struct Plan64Dev {
  W64 scale[MAXNP64];     // 2^64 (2 K L)^{-1} mod p_k: undoes the Montgomery factor and scales
  uint64_t pow2M[MAXNP64];
  // Garner's mixed-radix CRT: c = x0 + p0 x1 + p0 p1 x2
  W64 inv01;              // p0^{-1} mod p1
  W64 p0_mod2;            // p0 mod p2
  W64 inv012;             // (p0 p1)^{-1} mod p2
  uint64_t p01[2];        // p0 p1
  uint64_t P[3];          // product of the np primes
  uint64_t Phalf[3];      // (P - 1) / 2
};

// One strided pass of the y-transform: index i = inner + S (e + n outer), transform
// along e (n = 2^logn); a workgroup takes T inner indices and G outer ones.
struct Pass64 {
  int32_t logn, logS, logT, logG;
};

struct Plan64 {
  int64_t da, db, nout;
  int32_t Na, Nb, nout_bits;
  int32_t K, M, np;
  int32_t logL;
  int32_t npass;
  Pass64 pass[MAX_PASS64];   // outermost first
  int32_t logTX;             // y positions per workgroup of the x-kernel
  int32_t logTI;             // coefficients per workgroup of the recovery
  int32_t DIG;               // 32-bit digits of a shifted CRT value (2 np + 1)
  int32_t log2P;
  int32_t square;
  int64_t ws_words;          // np 2K L 64-bit words
  double cost;
};

struct Prime64Host {
  uint64_t p, root;   // root: primitive 2^21-th root of unity mod p
};
// The MAXNP64 largest primes p < 2^62 with 2^21 | p - 1, largest first.
const Prime64Host *prime64_table();

bool make_plan64(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K_force, int32_t np_force,
                 Plan64 &out, const char **why);

struct Ctx;
struct P64State;
// c = a * b with the 64-bit prime variant (pl from make_plan64; pl.square when b is a).
int mul_p64(Ctx &cx, const Plan64 &pl, const uint64_t *a, const uint64_t *b, uint64_t *c,
            int32_t wc, hipStream_t st);
void p64_release(Ctx &cx);

}  // namespace zpm
