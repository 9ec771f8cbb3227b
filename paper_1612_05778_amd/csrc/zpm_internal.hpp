// Internal structures shared by the host planner and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace zpm {

// Word-size Fourier primes p < 2^30 with 2^LOG2_ROOT_ORDER | p - 1 (Section 2.1,
// Relation (HavingAppropriatePrimitiveRootsOfUnity): the transform lengths along
// y and the 2K-th root theta along x must divide p - 1).
constexpr int PRIME_BITS = 30;          // every prime is below 2^PRIME_BITS
constexpr int MAXNP = 48;               // largest prime count a plan may use
constexpr int LOG2_ROOT_ORDER = 21;     // every prime has a primitive 2^21-th root
constexpr int MAXW = 48;                // 32-bit words of a CRT value (> 31*MAXNP + 2 bits)
constexpr int BLOCK = 256;              // threads per workgroup of every kernel
constexpr int LDS_WORDS = 16384;        // 64 KiB of LDS staging per workgroup
constexpr int MAX_COL_PASSES = 4;
// The recovery's CRT runs on int8 matrix cores up to this prime count: np + 1 terms of 4
// bytes in CRT_STEPS steps of 64 slots, values of up to 16 CRT_TILES signed bytes.
constexpr int CRT_MFMA_NP = 20;
constexpr int CRT_STEPS = 2;
constexpr int CRT_TILES = 6;
// The CRT term (y_q for q < np, t for q = np, none above) whose four bytes lane group g
// supplies as word w of the matrix product's step s: terms 0..15 in step 0, four per
// group, then 16, 17, ... spread over the groups first.
__host__ __device__ constexpr int crt_term(int s, int g, int w) {
  return s == 0 ? 4 * g + w : 16 + g + 4 * w;
}
// 16-digit tiles of one CRT value, each lane group of the matrix product holding one
// 32-bit word of each: 4 TN words >= the bytes of P plus the three bytes of the offsets.
constexpr int crt_tiles(int np) { return (4 * np + 8 + 15) / 16; }

// Prime counts with compiled kernels (per-prime loops are unrolled at compile time);
// a plan's prime count is rounded up to one of these.
constexpr int NP_SET[] = {1,  2,  3,  4,  5,  6,  7,  8,  9,  10, 11, 12, 13, 14, 15, 16,
                          17, 18, 19, 20, 21, 22, 23, 24, 26, 28, 30, 32, 36, 40, 44, 48};
inline int np_compiled(int np) {
  for (int v : NP_SET)
    if (v >= np) return v;
  return 0;
}

// Per-prime constants resident on the device.
struct PrimeDev {
  uint32_t p;          // the prime
  uint32_t pinv;       // p^{-1} mod 2^32 (Montgomery)
  uint32_t c32, c32s;  // 2^32 mod p and its Shoup companion floor(c32 * 2^32 / p)
  uint32_t ones;       // floor(2^32 / p): Shoup companion of 1 (plain reduction)
  uint32_t pad[3];
  const uint2 *hf;     // forward heap: hf[h + j] = (w^j, shoup) with w a primitive 2h-th root
  const uint2 *hi;     // inverse heap: hi[h + j] = (w^-j, shoup)
  const uint2 *pow32;  // pow32[t] = (2^(32 t) mod p, shoup)
};

// Per-plan constants (np primes, transform sizes) resident on the device.
struct PlanDev {
  uint2 scale[MAXNP];      // Montgomery-corrected 1/(2K L): 2^32 (2 K L)^{-1} mod p, Shoup pair
                           // (already folded into crt_inv; kept for inspection)
  uint32_t pow2M[MAXNP];   // 2^M mod p (weight of the sign bit of the top limb)
  uint2 crt_inv[MAXNP];    // (P/p_k)^{-1} scale_k mod p_k, Shoup pair: the CRT constant times
                           // the transforms' normalisation
  double crt_rcp[MAXNP];   // 1/p_k
  uint32_t crt_q[MAXNP][MAXW];  // P/p_k, little-endian 32-bit words
  uint32_t crt_p[MAXW];         // P
  // The CRT sum as an int8 matrix product (np <= CRT_MFMA_NP): the A operand, digits n
  // by byte slots (term, a), in each lane's fragment order (tile T of 16 digits, step s
  // of 64 slots, lane, 16 signed bytes).
  uint32_t crt_afrag[CRT_TILES][CRT_STEPS][64][4];
};

// A factor of the y-transform done by a strided column pass: index
// i = inner + S (e + n outer), transform along e (length n = 2^logn).
struct ColPass {
  int32_t logn;
  int64_t S;      // stride of e, in elements
};

// What a row-convolution block computes:
//   CM_PRODUCT        a * b from both operands' limb rows;
//   CM_SQUARE         a * a from a's rows, transformed once;
//   CM_SPECTRUM       only the forward transforms of b's rows (rows K..2K-1), whose 2K
//                     spectra per position are written back over rows 0..2K-1;
//   CM_WITH_SPECTRUM  a * b from a's rows and b's spectra written earlier by
//                     CM_SPECTRUM for the same plan.
enum ConvMode : int32_t { CM_PRODUCT = 0, CM_SQUARE = 1, CM_SPECTRUM = 2, CM_WITH_SPECTRUM = 3 };

// 64-bit partial sums per coefficient row of a recovery workgroup: the nw32 output words
// and, in the CRT's matrix form, the words past them that its lane groups may touch
// (value j starts at word floor(M j / 32); lane group 3's carry lands 4 TN words on).
// Those extra words collect nothing the output needs.
__host__ __device__ inline int recover_row_words(int np, int K, int M, int nw32) {
  if (np > CRT_MFMA_NP) return nw32;
  const int need = (int)(((int64_t)M * (2 * K - 2)) >> 5) + 4 * crt_tiles(np) + 1;
  return need > nw32 ? need : nw32;
}

// LDS of one recovery workgroup: a spare word, 2^log_ti coefficient rows of partial sums
// (rounded to 16 bytes), then either the staged terms (staged matrix form) and 4 words of
// constants per prime (matrix form), or the CRT's word table and 3 words and a double per
// prime.
// Words each value stages in LDS in the recovery's staged matrix form: its np terms and
// t, rounded to a 16-byte fragment.
__host__ __device__ constexpr int crt_stage_words(int np) { return 4 * ((np + 4) / 4); }

// The matrix-form recovery stages each wave's 64 values' terms in LDS (one value per
// lane while the residues are reduced) when the rows and the staging fit in 40 KiB, so
// that four workgroups share a CU; with longer rows each lane group builds its share of
// the terms in registers instead.
__host__ __device__ inline bool recover_staged(int np, int K, int M, int nw32, int log_ti) {
  if (np > CRT_MFMA_NP) return false;
  const int64_t rows = 8 * ((((int64_t)recover_row_words(np, K, M, nw32) << log_ti) + 2) & ~(int64_t)1);
  return rows + 4 * (int64_t)BLOCK * crt_stage_words(np) <= 40 * 1024;
}

inline size_t recover_lds_bytes(int np, int K, int M, int nw32, int log_ti) {
  // a spare word before the rows, rounded to 16 bytes
  size_t b = sizeof(uint64_t) * ((((size_t)recover_row_words(np, K, M, nw32) << log_ti) + 2) & ~(size_t)1);
  if (recover_staged(np, K, M, nw32, log_ti))
    b += sizeof(uint32_t) * (size_t)BLOCK * crt_stage_words(np);
  if (np <= CRT_MFMA_NP) return b + sizeof(uint32_t) * 4 * (size_t)np;
  b += sizeof(uint32_t) * (size_t)((np + 2) & ~1) * np;
  return b + sizeof(uint32_t) * ((3 * np + 1) & ~1) + sizeof(double) * np;
}

struct Plan {
  // caller-visible problem
  int64_t da, db;
  int32_t Na, Nb;
  int64_t nout;        // da + db - 1
  int32_t nout_bits;   // two's complement width that holds every c_i
  // method parameters (Section 2: N = K M, beta = 2^M; Section 2.1: primes)
  int32_t K, M, np;
  int32_t logL;        // L = 2^logL >= da + db - 1, the cyclic length along y
  int32_t logL1;       // innermost y factor handled inside the fused convolution kernel
  int32_t conv_reg;    // 1: x-transforms in registers (K <= 32), 0: in LDS
  int32_t square;      // 1: a and b are one operand, transformed once (c = a^2)
  int32_t spec;        // 1: b's spectra are resident (an operand's); only a is converted
                       //    and transformed, the row kernel takes b's spectra as they are
  int32_t ncol;        // number of strided column passes (outermost first)
  ColPass col[MAX_COL_PASSES];
  int32_t col_tile[MAX_COL_PASSES];  // inner indices per workgroup of each column pass
  int32_t W;           // 32-bit words of each CRT value c_{i,j} (= np)
  int32_t log2P;       // floor(log2(P)) + 1
  int32_t log_ti_in;   // log2 coefficients per workgroup in convert-in
  int32_t log_ti_out;  // log2 coefficients per workgroup in recovery
  int64_t ws_words;    // workspace size in 32-bit words: np * 2K * L
  double cost;         // planner's cost estimate (arbitrary units)
};

}  // namespace zpm
