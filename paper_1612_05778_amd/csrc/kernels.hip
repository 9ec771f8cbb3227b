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

#include "kernels.hpp"

namespace zpm {

// ------------------------------------------------------------------------------------
// modular arithmetic on 32-bit words, p < 2^31
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
__device__ __forceinline__ uint32_t mul_shoup(uint32_t x, uint2 w, uint32_t p) {
  uint32_t q = __umulhi(x, w.y);
  uint32_t r = x * w.x - q * p;   // in [0, 2p)
  return min(r, r - p);
}
// a * b * 2^-32 mod p (Montgomery), a, b < p.
__device__ __forceinline__ uint32_t mont_mul(uint32_t a, uint32_t b, uint32_t p, uint32_t pinv) {
  uint32_t lo = a * b, hi = __umulhi(a, b);
  uint32_t m = lo * pinv;
  uint32_t mp = __umulhi(m, p);
  uint32_t r = hi - mp;
  return hi < mp ? r + p : r;
}
// w_m^e from a heap table (tab[m/2 + e] = w_m^e for e < m/2), any e in [0, m).
__device__ __forceinline__ uint2 heap_root(const uint2 *__restrict__ tab, int64_t m, int64_t e, uint32_t p) {
  const int64_t half = m >> 1;
  if (e < half) return tab[half + e];
  uint2 w = tab[e];            // w_m^(e - m/2) = -w_m^e
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

__device__ __forceinline__ int lds_base(const LdsShape &sh, int t) {
  return (t & ((1 << sh.logntr) - 1)) * sh.ts + (t >> sh.logntr) * sh.off2;
}

// DIF (Gentleman-Sande) stages with half-sizes h0, h0/2, ..., h0/2^(R-1); output of the
// whole transform is in bit-reversed order.
template <int R>
__device__ void dif_group(uint32_t *s, const LdsShape &sh, int logh0, const uint2 *__restrict__ tw,
                          uint32_t p) {
  constexpr int NR = 1 << R;
  const int loghl = logh0 - (R - 1);
  const int hl = 1 << loghl;
  const int lgpt = sh.logn - R;                       // groups per transform (log)
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
        const uint2 w = tw[hsz + j + (m & (half - 1)) * hl];
        const uint32_t u = x[m], v = x[m + half];
        x[m] = add_mod(u, v, p);
        x[m + half] = mul_shoup(u - v + p, w, p);
      }
    }
#pragma unroll
    for (int m = 0; m < NR; ++m) s[base + m * step] = x[m];
  }
}

// DIT (Cooley-Tukey) stages with half-sizes h0, 2 h0, ..., h0 2^(R-1); input in
// bit-reversed order, output natural.
template <int R>
__device__ void dit_group(uint32_t *s, const LdsShape &sh, int logh0, const uint2 *__restrict__ tw,
                          uint32_t p) {
  constexpr int NR = 1 << R;
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
        const uint2 w = tw[hsz + j + (m & (half - 1)) * h0];
        const uint32_t u = x[m];
        const uint32_t v = mul_shoup(x[m + half], w, p);
        x[m] = add_mod(u, v, p);
        x[m + half] = sub_mod(u, v, p);
      }
    }
#pragma unroll
    for (int m = 0; m < NR; ++m) s[base + m * step] = x[m];
  }
}

// Full forward transform (all logn stages); caller synchronises before and after.
__device__ void lds_dif(uint32_t *s, const LdsShape &sh, const uint2 *__restrict__ tw, uint32_t p) {
  int st = sh.logn;
  while (st > 0) {
    const int r = st >= 3 ? 3 : st;
    if (r == 3) dif_group<3>(s, sh, st - 1, tw, p);
    else if (r == 2) dif_group<2>(s, sh, st - 1, tw, p);
    else dif_group<1>(s, sh, st - 1, tw, p);
    st -= r;
    __syncthreads();
  }
}

__device__ void lds_dit(uint32_t *s, const LdsShape &sh, const uint2 *__restrict__ tw, uint32_t p) {
  int done = 0;
  while (done < sh.logn) {
    const int left = sh.logn - done;
    const int r = left >= 3 ? 3 : left;
    if (r == 3) dit_group<3>(s, sh, done, tw, p);
    else if (r == 2) dit_group<2>(s, sh, done, tw, p);
    else dit_group<1>(s, sh, done, tw, p);
    done += r;
    __syncthreads();
  }
}

__device__ __forceinline__ int bitrev(int x, int logn) {
  return logn ? (int)(__brev((unsigned)x) >> (32 - logn)) : 0;
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

__global__ __launch_bounds__(BLOCK) void k_bivariate_representation(
    const uint64_t *__restrict__ src, int64_t d, int32_t N, int32_t w, int32_t K, int32_t M,
    int32_t np, uint32_t *__restrict__ X, int64_t L, int32_t col_off, int32_t TI,
    const PrimeDev *__restrict__ primes, const PlanDev *__restrict__ pd) {
  extern __shared__ uint32_t s[];
  const int64_t i0 = (int64_t)blockIdx.x * TI;
  const int ti = (int)min<int64_t>(TI, d - i0);
  const int nw = 2 * w;
  const int stride = nw + 1;
  // stage the tile's words (one contiguous block of ti * w words)
  const uint64_t *tile = src + i0 * w;
  for (int idx = threadIdx.x; idx < ti * w; idx += BLOCK) {
    const int il = idx / w, u = idx - il * w;
    const uint64_t v = tile[idx];
    s[il * stride + 2 * u] = (uint32_t)v;
    s[il * stride + 2 * u + 1] = (uint32_t)(v >> 32);
  }
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
  const int nchunks = (M + 31) >> 5;
  const uint32_t lastmask = (M & 31) ? ((1u << (M & 31)) - 1u) : 0xFFFFFFFFu;
  const int64_t twoK = 2 * (int64_t)K;
  for (int idx = threadIdx.x; idx < ti * K; idx += BLOCK) {
    const int il = idx % ti;
    const int j = idx / ti;
    const uint32_t *row = s + il * stride;
    const uint32_t sgn = (uint32_t)((int32_t)row[nw - 1] >> 31);
    const int64_t b = (int64_t)M * j;
    const bool neg_top = (j == K - 1) && ((get32(row, nw, sgn, b + M - 1) & 1u) != 0);
    for (int k = 0; k < np; ++k) {
      const PrimeDev pr = primes[k];
      const uint2 c32 = make_uint2(pr.c32, pr.c32s);
      const uint2 one = make_uint2(1u, pr.ones);
      uint32_t r = 0;
      for (int t = nchunks - 1; t >= 0; --t) {
        uint32_t c = get32(row, nw, sgn, b + 32 * (int64_t)t);
        if (t == nchunks - 1) c &= lastmask;
        r = add_mod(mul_shoup(r, c32, pr.p), mul_shoup(c, one, pr.p), pr.p);
      }
      if (neg_top) r = sub_mod(r, pd->pow2M[k], pr.p);
      X[((int64_t)k * twoK + col_off + j) * L + i0 + il] = r;
    }
  }
}

// ------------------------------------------------------------------------------------
// Strided column passes of the y-transform (outer factors of a four-step split).
// Index i = inner + S (e + n outer); the pass transforms along e.  Forward: DIF,
// then multiply position e (frequency k = bitrev(e)) by w_{nS}^(inner k).
// Inverse: multiply by w_{nS}^(-inner k), then DIT.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_col_pass(
    uint32_t *__restrict__ X, int64_t L, int32_t twoK, int32_t logn, int64_t S, int32_t logT,
    int64_t nz_a, int64_t nz_b, int32_t K, int64_t nlimit, int32_t inverse,
    const PrimeDev *__restrict__ primes) {
  extern __shared__ uint32_t s[];
  const int n = 1 << logn, T = 1 << logT;
  const int64_t inner_tiles = S >> logT;
  const int64_t outers = L / ((int64_t)n * S);
  const int64_t tiles = inner_tiles * outers;
  const int64_t col = blockIdx.x / tiles;
  const int64_t tile = blockIdx.x - col * tiles;
  const int64_t outer = tile / inner_tiles;
  const int64_t inner0 = (tile - outer * inner_tiles) << logT;
  const int k = (int)(col / twoK);
  const int jc = (int)(col - (int64_t)k * twoK);
  const PrimeDev pr = primes[k];
  const uint32_t p = pr.p;
  uint32_t *base = X + col * L + inner0 + S * (int64_t)n * outer;
  const int64_t nz = inverse ? L : (jc < K ? nz_a : nz_b);
  const int64_t first = inner0 + S * (int64_t)n * outer;   // index of (t=0, e=0)
  const int64_t m = (int64_t)n * S;
  for (int idx = threadIdx.x; idx < (n << logT); idx += BLOCK) {
    const int t = idx & (T - 1), e = idx >> logT;
    const int64_t off = t + S * (int64_t)e;
    uint32_t v = (first + off < nz) ? base[off] : 0u;
    if (inverse) {
      const int64_t ex = (inner0 + t) * (int64_t)bitrev(e, logn);
      v = mul_shoup(v, heap_root(pr.hi, m, ex, p), p);
    }
    s[idx] = v;
  }
  __syncthreads();
  LdsShape sh{logT, logn, 1, T, 0, 0};
  if (inverse) lds_dit(s, sh, pr.hi, p);
  else lds_dif(s, sh, pr.hf, p);
  for (int idx = threadIdx.x; idx < (n << logT); idx += BLOCK) {
    const int t = idx & (T - 1), e = idx >> logT;
    const int64_t off = t + S * (int64_t)e;
    uint32_t v = s[idx];
    if (!inverse) {
      const int64_t ex = (inner0 + t) * (int64_t)bitrev(e, logn);
      v = mul_shoup(v, heap_root(pr.hf, m, ex, p), p);
      base[off] = v;
    } else if (first + off < nlimit) {
      base[off] = v;
    }
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
// after the 1/(2K) in the scale constant are c_{i,j} and c_{i,j+K} (Section 2,
// C+ and C- through Relation (recoveringC)).
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_convolve_rows(
    uint32_t *__restrict__ X, int64_t L, int32_t K, int32_t logK, int32_t logL1, int64_t nz_a,
    int64_t nz_b, int64_t nlimit, const PrimeDev *__restrict__ primes,
    const PlanDev *__restrict__ pd) {
  extern __shared__ uint32_t s[];
  const int L1 = 1 << logL1;
  const int64_t nrb = L >> logL1;
  const int k = (int)(blockIdx.x / nrb);
  const int64_t rb = blockIdx.x - (int64_t)k * nrb;
  const PrimeDev pr = primes[k];
  const uint32_t p = pr.p;
  const int twoK = 2 * K;
  uint32_t *A = s;                      // 2K rows x L1
  uint32_t *B = s + twoK * L1;          // 2K rows x L1
  uint32_t *base = X + (int64_t)k * twoK * L + rb * L1;
  const int64_t y0 = rb * L1;
  for (int idx = threadIdx.x; idx < (K << logL1); idx += BLOCK) {
    const int j = idx >> logL1, e = idx & (L1 - 1);
    const int64_t i = y0 + e;
    A[idx] = (i < nz_a) ? base[(int64_t)j * L + e] : 0u;
    B[idx] = (i < nz_b) ? base[(int64_t)(K + j) * L + e] : 0u;
    A[(K << logL1) + idx] = 0u;
    B[(K << logL1) + idx] = 0u;
  }
  __syncthreads();
  // innermost y factor on the K limb rows of both operands
  lds_dif(s, LdsShape{logK, logL1, L1, 1, twoK * L1, 1}, pr.hf, p);
  // x: 2K-point transforms down the L1 columns of both operands
  lds_dif(s, LdsShape{logL1, logK + 1, 1, L1, twoK * L1, 1}, pr.hf, p);
  const uint2 sc = pd->scale[k];
  for (int idx = threadIdx.x; idx < (twoK << logL1); idx += BLOCK)
    A[idx] = mul_shoup(mont_mul(A[idx], B[idx], p, pr.pinv), sc, p);
  __syncthreads();
  lds_dit(s, LdsShape{logL1, logK + 1, 1, L1, 0, 0}, pr.hi, p);
  lds_dit(s, LdsShape{logK + 1, logL1, L1, 1, 0, 0}, pr.hi, p);
  for (int idx = threadIdx.x; idx < (twoK << logL1); idx += BLOCK) {
    const int j = idx >> logL1, e = idx & (L1 - 1);
    if (y0 + e < nlimit) base[(int64_t)j * L + e] = A[idx];
  }
}

// ------------------------------------------------------------------------------------
// RecoveringProduct.  For each output coefficient i and each j < 2K-1:
//   c_{i,j} from its np residues by CRT into (-P/2, P/2) (exact because
//   |c_{i,j}| < d K 2^(2M) < P/4), as W-word two's complement;
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

template <int WT>
__global__ __launch_bounds__(BLOCK) void k_recovering_product(
    const uint32_t *__restrict__ X, int64_t L, int32_t K, int32_t M, int32_t np, int32_t W,
    int64_t nout, int32_t nw32, int32_t wc, int32_t TI, const PrimeDev *__restrict__ primes,
    const PlanDev *__restrict__ pd, uint64_t *__restrict__ out) {
  extern __shared__ uint32_t s[];
  const int J = 2 * K - 1;
  const int64_t twoK = 2 * (int64_t)K;
  const int64_t i0 = (int64_t)blockIdx.x * TI;
  const int ti = (int)min<int64_t>(TI, nout - i0);
  uint32_t *V = s;                          // ti x J x W
  uint32_t *rows = s + (int64_t)TI * J * W;  // 4 waves x nw32
  // ---- CRT ----
  for (int idx = threadIdx.x; idx < ti * J; idx += BLOCK) {
    const int il = idx % ti, j = idx / ti;
    const int64_t i = i0 + il;
    uint32_t acc[WT];
#pragma unroll
    for (int u = 0; u < WT; ++u) acc[u] = 0;
    double f = 0.0;
    for (int k = 0; k < np; ++k) {
      const uint32_t p = primes[k].p;
      const uint32_t r = X[((int64_t)k * twoK + j) * L + i];
      const uint32_t c = mul_shoup(r, pd->crt_inv[k], p);
      f += (double)c * pd->crt_rcp[k];
      const uint32_t *q = pd->crt_q[k];
      uint64_t carry = 0;
#pragma unroll
      for (int u = 0; u < WT; ++u) {
        if (u < W) {
          const uint64_t t = (uint64_t)c * q[u] + acc[u] + carry;
          acc[u] = (uint32_t)t;
          carry = t >> 32;
        }
      }
    }
    // sum_k c_k P/p_k = c + t P with |c| < P/4, so t = round(sum_k c_k / p_k)
    const uint32_t t = (uint32_t)__double2int_rn(f);
    uint64_t borrow = 0;
#pragma unroll
    for (int u = 0; u < WT; ++u) {
      if (u < W) {
        const uint64_t sub = (uint64_t)t * pd->crt_p[u] + borrow;
        const uint32_t lo = (uint32_t)sub;
        borrow = (sub >> 32) + (acc[u] < lo ? 1 : 0);
        acc[u] = acc[u] - lo;
      }
    }
    uint32_t *dst = V + ((int64_t)il * J + j) * W;
#pragma unroll
    for (int u = 0; u < WT; ++u)
      if (u < W) dst[u] = acc[u];
  }
  __syncthreads();
  // ---- evaluation at 2^M and carries, one wave per coefficient ----
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t *row = rows + wave * nw32;
  const int per = (nw32 + 63) >> 6;
  const int w_lo = min(lane * per, nw32), w_hi = min(w_lo + per, nw32);
  const int64_t topbits = 32 * (int64_t)W;
  for (int il = wave; il < ti; il += BLOCK / 64) {
    const uint32_t *Vi = V + (int64_t)il * J * W;
    int64_t carry = 0;
    for (int w = w_lo; w < w_hi; ++w) {
      const int64_t wb = 32 * (int64_t)w;
      int64_t S = 0;
      const int64_t jl = wb - topbits > 0 ? (wb - topbits) / M : 0;
      const int64_t jh = min<int64_t>(J - 1, (wb + 31) / M);
      for (int64_t j = jl; j <= jh; ++j) {
        const uint32_t *v = Vi + j * W;
        const int64_t pos = wb - (int64_t)M * j;
        uint32_t win = 0;
        if (pos >= topbits || pos <= -32) {
          win = 0;
        } else if (pos >= 0) {
          const int q = (int)(pos >> 5), sh = (int)(pos & 31);
          const uint32_t lo = v[q];
          const uint32_t hi = (q + 1 < W) ? v[q + 1] : 0u;
          win = sh ? ((lo >> sh) | (hi << (32 - sh))) : lo;
        } else {
          win = v[0] << (int)(-pos);
        }
        S += win;
        if ((int32_t)v[W - 1] < 0 && ((topbits + (int64_t)M * j) >> 5) == w)
          S -= (int64_t)1 << ((topbits + (int64_t)M * j) & 31);
      }
      const int64_t tsum = S + carry;
      row[w] = (uint32_t)tsum;
      carry = tsum >> 32;
    }
    // pass the local carry to the next lane and normalise
    int64_t cin = __shfl_up(carry, 1, 64);
    if (lane == 0) cin = 0;
    int64_t x = cin;
    bool allz = true, allo = true;
    for (int w = w_lo; w < w_hi; ++w) {
      const int64_t tsum = (int64_t)row[w] + x;
      row[w] = (uint32_t)tsum;
      x = tsum >> 32;
      allz = allz && row[w] == 0u;
      allo = allo && row[w] == 0xFFFFFFFFu;
    }
    int code;
    if (w_lo >= w_hi) {
      code = (0) | (1 << 2) | (2 << 4);                 // identity
    } else {
      const int g = (int)x;                             // in {-1, 0, 1}
      const int fm = g + (allz ? -1 : 0), f0 = g, fp = g + (allo ? 1 : 0);
      code = (fm + 1) | ((f0 + 1) << 2) | ((fp + 1) << 4);
    }
    // inclusive scan of carry-transfer functions across the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int other = __shfl_up(code, off, 64);
      if (lane >= off) code = fcompose(code, other);
    }
    int prev = __shfl_up(code, 1, 64);
    int y = lane == 0 ? 0 : fapply(prev, 0);
    for (int w = w_lo; w < w_hi && y != 0; ++w) {
      const int64_t tsum = (int64_t)row[w] + y;
      row[w] = (uint32_t)tsum;
      y = (int)(tsum >> 32);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const uint64_t fill = ((int32_t)row[nw32 - 1] < 0) ? ~0ull : 0ull;
    uint64_t *o = out + (i0 + il) * (int64_t)wc;
    for (int u = lane; u < wc; u += 64) {
      o[u] = (2 * u + 1 < nw32) ? ((uint64_t)row[2 * u] | ((uint64_t)row[2 * u + 1] << 32)) : fill;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
}

// ------------------------------------------------------------------------------------
// host launchers
// ------------------------------------------------------------------------------------
static inline int ilog2(int64_t x) {
  int r = 0;
  while (((int64_t)1 << (r + 1)) <= x) ++r;
  return r;
}

hipError_t launch_convert_in(const Plan &pl, const DevState &ds, const uint64_t *src, int64_t d,
                             int32_t N, int32_t col_off, hipStream_t st) {
  const int w = (N + 63) / 64;
  const int TI = pl.ti_in;
  const int64_t blocks = (d + TI - 1) / TI;
  const size_t lds = sizeof(uint32_t) * (size_t)TI * (2 * w + 1);
  hipLaunchKernelGGL(k_bivariate_representation, dim3((unsigned)blocks), dim3(BLOCK), lds, st, src,
                     d, N, w, pl.K, pl.M, pl.np, ds.X, (int64_t)1 << pl.logL, col_off, TI, ds.primes,
                     ds.plan);
  return hipGetLastError();
}

hipError_t launch_col(const Plan &pl, const DevState &ds, int c, bool inverse, hipStream_t st) {
  const int64_t L = (int64_t)1 << pl.logL;
  const int logn = pl.col[c].logn;
  const int64_t S = pl.col[c].S;
  const int T = pl.col_tile[c];
  const int logT = ilog2(T);
  const int64_t tiles = (S >> logT) * (L / (((int64_t)1 << logn) * S));
  const int64_t blocks = tiles * pl.np * 2 * pl.K;
  const size_t lds = sizeof(uint32_t) * ((size_t)T << logn);
  const int64_t nz_a = (c == 0 && !inverse) ? pl.da : L;
  const int64_t nz_b = (c == 0 && !inverse) ? pl.db : L;
  const int64_t nlimit = (c == 0 && inverse) ? pl.nout : L;
  hipLaunchKernelGGL(k_col_pass, dim3((unsigned)blocks), dim3(BLOCK), lds, st, ds.X, L, 2 * pl.K,
                     logn, S, logT, nz_a, nz_b, pl.K, nlimit, inverse ? 1 : 0, ds.primes);
  return hipGetLastError();
}

hipError_t launch_convolve(const Plan &pl, const DevState &ds, hipStream_t st) {
  const int64_t L = (int64_t)1 << pl.logL;
  const int64_t blocks = (int64_t)pl.np * (L >> pl.logL1);
  const size_t lds = sizeof(uint32_t) * (size_t)4 * pl.K << pl.logL1;
  const bool direct = pl.ncol == 0;
  hipLaunchKernelGGL(k_convolve_rows, dim3((unsigned)blocks), dim3(BLOCK), lds, st, ds.X, L, pl.K,
                     ilog2(pl.K), pl.logL1, direct ? pl.da : L, direct ? pl.db : L,
                     direct ? pl.nout : L, ds.primes, ds.plan);
  return hipGetLastError();
}

hipError_t launch_recover(const Plan &pl, const DevState &ds, uint64_t *out, int32_t wc,
                          hipStream_t st) {
  const int64_t L = (int64_t)1 << pl.logL;
  const int nw32 = 2 * ((pl.nout_bits + 63) / 64);
  const int TI = pl.ti_out;
  const int64_t blocks = (pl.nout + TI - 1) / TI;
  const size_t lds = sizeof(uint32_t) * ((size_t)TI * (2 * pl.K - 1) * pl.W + 4 * (size_t)nw32);
#define ZPM_REC(WT_)                                                                              \
  hipLaunchKernelGGL(k_recovering_product<WT_>, dim3((unsigned)blocks), dim3(BLOCK), lds, st,    \
                     ds.X, L, pl.K, pl.M, pl.np, pl.W, pl.nout, nw32, wc, TI, ds.primes, ds.plan, \
                     out)
  if (pl.W <= 4) ZPM_REC(4);
  else if (pl.W <= 8) ZPM_REC(8);
  else if (pl.W <= 12) ZPM_REC(12);
  else if (pl.W <= 16) ZPM_REC(16);
  else if (pl.W <= 24) ZPM_REC(24);
  else if (pl.W <= 32) ZPM_REC(32);
  else ZPM_REC(48);
#undef ZPM_REC
  return hipGetLastError();
}

hipError_t launch_mul(const Plan &pl, const DevState &ds, const uint64_t *a, const uint64_t *b,
                      uint64_t *c, int32_t wc, int stop_after, hipStream_t st, Profiler *prof) {
  hipError_t e;
  Profiler dummy;
  Profiler &pr = prof ? *prof : dummy;
  pr.begin(KK_CONVERT_IN, st);
  e = launch_convert_in(pl, ds, a, pl.da, pl.Na, 0, st);
  pr.end(st);
  if (e != hipSuccess) return e;
  pr.begin(KK_CONVERT_IN, st);
  e = launch_convert_in(pl, ds, b, pl.db, pl.Nb, pl.K, st);
  pr.end(st);
  if (e != hipSuccess) return e;
  if (stop_after == 1) return hipSuccess;
  for (int cidx = 0; cidx < pl.ncol; ++cidx) {
    pr.begin(KK_COL_FWD, st);
    e = launch_col(pl, ds, cidx, false, st);
    pr.end(st);
    if (e != hipSuccess) return e;
  }
  if (stop_after == 2) return hipSuccess;
  pr.begin(KK_CONVOLVE, st);
  e = launch_convolve(pl, ds, st);
  pr.end(st);
  if (e != hipSuccess) return e;
  if (stop_after == 3) return hipSuccess;
  for (int cidx = pl.ncol - 1; cidx >= 0; --cidx) {
    pr.begin(KK_COL_INV, st);
    e = launch_col(pl, ds, cidx, true, st);
    pr.end(st);
    if (e != hipSuccess) return e;
  }
  if (stop_after == 4) return hipSuccess;
  pr.begin(KK_RECOVER, st);
  e = launch_recover(pl, ds, c, wc, st);
  pr.end(st);
  return e;
}

}  // namespace zpm
