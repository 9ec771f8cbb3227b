// Balancing by Kronecker substitution (Section 1: when N is not in Theta(d log d), a
// forward and backward Kronecker substitution replaces (a, b) by a pair of polynomials
// for which it is).  Here it serves coefficients too wide for one product: each
// coefficient x_i is cut into s chunks of w bits (w a multiple of 64),
//   x_i = sum_{t < s} x_{i,t} 2^(w t),   lower chunks unsigned, the top chunk signed,
// and y is replaced by z^S with S = s_a + s_b - 1, so that
//   a'(z) = sum_i sum_t a_{i,t} z^(S i + t)   (and b' alike)
// has coefficients of w + 1 bits.  Since t + u < S for the chunk indices of a and b,
// the product's coefficient S k + r is the coefficient of 2^(w r) in c_k, so
//   c_k = sum_{r < S} c'_{S k + r} 2^(w r),
// which the join kernel evaluates with carries.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/zpm.h"
#include "ctx.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "stages.hpp"

namespace zpm {

// x'_r for r = S i + t: chunk t of x_i (t < s) as wq + 1 words of two's complement,
// zero for t >= s.  Chunks below the top one lie below bit N - 1, so only the top
// chunk sees the sign: bits >= N of x_i are replaced by copies of bit N - 1.
__global__ __launch_bounds__(BLOCK) void k_kron_split(const uint64_t *__restrict__ x, int64_t d,
                                                      int32_t N, int32_t win, int32_t s, int32_t S,
                                                      int32_t wq, uint64_t *__restrict__ xo,
                                                      int64_t dout) {
  const int32_t wo = wq + 1;
  const int64_t total = dout * wo;
  const int top_w = (N - 1) >> 6, top_b = (N - 1) & 63;
  for (int64_t g = (int64_t)blockIdx.x * BLOCK + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * BLOCK) {
    const int64_t r = g / wo;
    const int u = (int)(g - r * wo);
    const int64_t i = r / S;
    const int t = (int)(r - i * S);
    uint64_t v = 0;
    if (i < d && t < s) {
      const uint64_t *xi = x + i * win;
      const bool neg = (xi[top_w] >> top_b) & 1;
      const int64_t gw = (int64_t)t * wq + u;       // input word of this output word
      if (u == wq) {
        v = (t == s - 1 && neg) ? ~0ull : 0ull;     // extension word
      } else if (gw < top_w) {
        v = xi[gw];
      } else if (gw == top_w) {
        v = xi[gw];
        if (top_b < 63) {
          const uint64_t keep = (2ull << top_b) - 1;
          v = neg ? (v | ~keep) : (v & keep);
        }
      } else {
        v = neg ? ~0ull : 0ull;
      }
    }
    xo[g] = v;
  }
}

// c_k = sum_{r < S} c'_{S k + r} 2^(64 wq r) modulo 2^(64 wc) (c_k fits in wc words).
// One wave per output coefficient.  Lane l owns the 32-bit digits [l per, (l+1) per)
// of c_k (per even, so whole output words) and writes them in place in c:
//   pass 1: digit sums (at most three overlapping c' plus their sign extensions)
//           with the lane's own carry propagation;
//   pass 2: the previous lane's outgoing carry is added; the lane's outgoing carry is
//           then in {-1, 0, 1}, and so is its response to a further carry in {-1, 0, 1};
//   pass 3: an inclusive scan of those carry-transfer functions gives each lane its
//           final incoming carry.
__global__ __launch_bounds__(BLOCK) void k_kron_join(const uint64_t *__restrict__ cp, int32_t wcp,
                                                     int32_t S, int32_t wq, int64_t nout,
                                                     uint64_t *__restrict__ c, int32_t wc) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * (BLOCK / 64) + wave;
  if (k >= nout) return;                     // uniform per wave
  const int nd = 2 * wc;                     // digits of c_k
  const int U = 2 * wcp;                     // digits of each c'
  const int D = 2 * wq;                      // digit shift from r to r + 1
  const int per = ((nd + 127) / 128) * 2;
  const int lo = min(lane * per, nd), hi = min(lo + per, nd);
  const uint32_t *src = reinterpret_cast<const uint32_t *>(cp + k * (int64_t)S * wcp);
  uint32_t *dst = reinterpret_cast<uint32_t *>(c + k * (int64_t)wc);
  int64_t carry = 0;
  for (int q = lo; q < hi; ++q) {
    int64_t acc = carry;
    const int rmin = q >= U ? (q - U + D) / D : 0;          // r with 0 <= q - r D < U
    const int rmax = min(S - 1, q / D);
    for (int r = rmin; r <= rmax; ++r) acc += src[(int64_t)r * U + (q - r * D)];
    // a negative c'_r is its U digits minus 2^(32 U): -1 at digit r D + U
    if (q >= U && (q - U) % D == 0) {
      const int r = (q - U) / D;
      if (r < S && (int32_t)src[(int64_t)r * U + U - 1] < 0) acc -= 1;
    }
    dst[q] = (uint32_t)acc;
    carry = acc >> 32;
  }
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
  int code;
  if (lo >= hi) {
    code = (0) | (1 << 2) | (2 << 4);        // identity
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

bool kron_plan(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t chunk_bits, KronPlan *out) {
  if (da < 1 || db < 1 || Na < 1 || Nb < 1 || chunk_bits < 0 || (chunk_bits & 63)) return false;
  bool found = false;
  KronPlan best;
  for (int32_t w = 256; w <= 16384; w *= 2) {
    if (chunk_bits && w != chunk_bits) continue;
    KronPlan kp;
    kp.w = w;
    kp.wq = w / 64;
    kp.sa = (Na + w - 1) / w;
    kp.sb = (Nb + w - 1) / w;
    kp.S = kp.sa + kp.sb - 1;
    kp.da2 = (int64_t)kp.S * (da - 1) + kp.sa;
    kp.db2 = (int64_t)kp.S * (db - 1) + kp.sb;
    kp.nout2 = kp.da2 + kp.db2 - 1;
    kp.N2 = w + 1;
    kp.wc2 = (out_bits(kp.da2, kp.N2, kp.db2, kp.N2) + 63) / 64;
    const char *why = nullptr;
    if (!make_plan(kp.da2, kp.N2, kp.db2, kp.N2, 0, 0, kp.inner, &why, nullptr)) continue;
    // the inner product plus the split and join passes over the chunked operands
    kp.cost = kp.inner.cost +
              8.0 * ((double)(kp.da2 + kp.db2) * (kp.wq + 1) + 2.0 * kp.nout2 * kp.wc2) / 5.0e12;
    if (!found || kp.cost < best.cost) {
      best = kp;
      found = true;
    }
  }
  if (found) *out = best;
  return found;
}

static hipError_t launch_split(const uint64_t *x, int64_t d, int32_t N, int32_t s, const KronPlan &kp,
                               uint64_t *xo, int64_t dout, hipStream_t st) {
  const int64_t total = dout * (kp.wq + 1);
  const int64_t blocks = std::min<int64_t>((total + BLOCK - 1) / BLOCK, 65536);
  hipLaunchKernelGGL(k_kron_split, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(BLOCK), 0, st,
                     x, d, N, (N + 63) / 64, s, kp.S, kp.wq, xo, dout);
  return hipGetLastError();
}

int Ctx::ensure_kbuf(int64_t words) {
  if (words <= kbuf_words) return ZPM_OK;
  if (reserved) return ZPM_ENOMEM;   // beyond the reservation: no reallocation
  if (hipDeviceSynchronize() != hipSuccess) return ZPM_EDEVICE;
  if (kbuf) (void)hipFree(kbuf);
  kbuf = nullptr;
  kbuf_words = 0;
  if (hipMalloc(&kbuf, (size_t)words * 8) != hipSuccess) return ZPM_ENOMEM;
  kbuf_words = words;
  return ZPM_OK;
}

int Ctx::mul_kronecker(const uint64_t *a, int64_t da, int32_t Na, const uint64_t *b, int64_t db,
                       int32_t Nb, uint64_t *c, int32_t wc, int32_t chunk_bits, hipStream_t st) {
  KronPlan kp;
  if (!kron_plan(da, Na, db, Nb, chunk_bits, &kp)) return ZPM_EUNSUPPORTED;
  const bool square = a == b && da == db && Na == Nb;
  const int64_t w2 = kp.wq + 1;
  const int64_t na = kp.da2 * w2, nb = square ? 0 : kp.db2 * w2, nc = kp.nout2 * kp.wc2;
  int rc;
  if ((rc = ensure_kbuf(na + nb + nc)) != ZPM_OK) return rc;
  uint64_t *ap = kbuf, *bp = square ? kbuf : kbuf + na, *cpp = kbuf + na + nb;
  Plan pl = kp.inner;
  pl.square = square ? 1 : 0;
  DevState ds;
  if ((rc = prepare(pl, &ds, st)) != ZPM_OK) return rc;
  if (launch_split(a, da, Na, kp.sa, kp, ap, kp.da2, st) != hipSuccess) return ZPM_EDEVICE;
  if (!square && launch_split(b, db, Nb, kp.sb, kp, bp, kp.db2, st) != hipSuccess) return ZPM_EDEVICE;
  if (launch_mul(pl, ds, ap, bp, cpp, kp.wc2, 0, st, &prof) != hipSuccess) return ZPM_EDEVICE;
  const int64_t nout = da + db - 1;
  const int64_t blocks = (nout + BLOCK / 64 - 1) / (BLOCK / 64);
  hipLaunchKernelGGL(k_kron_join, dim3((unsigned)blocks), dim3(BLOCK), 0, st, cpp, kp.wc2, kp.S,
                     kp.wq, nout, c, wc);
  return hipGetLastError() == hipSuccess ? ZPM_OK : ZPM_EDEVICE;
}

}  // namespace zpm
