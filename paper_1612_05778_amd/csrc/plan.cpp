// Planner: the DetermineBase and RecoveryPrime steps of the algorithm of
// Section 2.3, made into a table-free search.
//
// For every power-of-two K (K >= 2) the limb width is M = max(2, ceil(N/K)) so
// that K M >= N (Relation (minimalConditionsForN) with N padded up to K M; sign
// extension keeps the value).  The prime count np is the smallest whose product
// exceeds 2 d K 2^(2M) (1 + 2^-12) with d = min(da, db): Relation (recoveryModulo) with
// the product of the primes playing the role of p (Section 4), halved because the
// recovery reconstructs c_{i,j} rather than c+_{i,j} and c-_{i,j} (primes_cover
// states why).  The transform length along y is the power
// of two L >= da + db - 1, and L and 2K must divide p - 1 (Section 2.1).
//
// Among the feasible K the planner keeps the one with the lowest modelled time,
// from the butterfly count of the row-column transforms (Section 3.3: K
// transforms of length L along y, 2L convolutions of length K along x, for the
// cyclic and the negacyclic product) plus CRT and memory traffic.  This follows
// the remark of Section 4 that the word-prime variant gains from a large M.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "nt.hpp"
#include "plan.hpp"

namespace zpm {

static int ceil_log2(int64_t x) {
  int r = 0;
  while (((int64_t)1 << r) < x) ++r;
  return r;
}

int32_t out_bits(int64_t da, int32_t Na, int64_t db, int32_t Nb) {
  // |c_i| <= min(da, db) 2^(Na+Nb-2), Relation (citighterbound) with the exact term count
  int64_t t = std::min(da, db);
  if (t <= 0) return 1;
  int bl = 0;
  while (((int64_t)1 << bl) <= t) ++bl;   // bit length of t
  return Na + Nb - 1 + bl;
}

// Split of the y-transform: innermost factor L1 inside the fused kernel, the rest
// into strided column passes of length <= 2^10 each.
// Widest column tile of a strided pass (inner indices per workgroup); ZPM_COL_TILE
// overrides the default of 16.  Tiles sharing 128-byte lines run next to each other on
// one XCD, so narrow tiles cost no extra HBM traffic; 16 columns (64-byte runs) suit the
// inverse passes, which read every row, better than 8.
static int64_t col_tile_max() {
  static const int64_t v = [] {
    const char *e = std::getenv("ZPM_COL_TILE");
    const long x = e ? std::atol(e) : 0;
    return (int64_t)(x >= 1 && x <= 64 && !(x & (x - 1)) ? x : 16);
  }();
  return v;
}

static bool split_y(Plan &pl, int reg_k_max, int col_tile, int l1_cap = 64) {
  const int logK = ceil_log2(pl.K);
  int logcap = 0;
  pl.conv_reg = pl.K <= reg_k_max ? 1 : 0;
  if (pl.conv_reg) {
    // 2K rows of L1 + 1 words (x-transforms in registers)
    while (2ll * pl.K * ((1ll << (logcap + 1)) + 1) <= LDS_WORDS) ++logcap;
  } else {
    // two 2K x L1 tiles: 4 K L1 <= LDS_WORDS
    while ((4ll << (logK + logcap + 1)) <= LDS_WORDS) ++logcap;
    if ((4ll << (logK + logcap)) > LDS_WORDS) return false;     // K too large even for L1 = 1
    // tiles of half that (32 KiB) where L1 allows: five workgroups share a CU's LDS
    // instead of two, which hides the LDS latency of the x-transforms
    if (logcap >= 1) --logcap;
  }
  pl.logL1 = std::min(pl.logL, std::min(logcap, l1_cap));
  int rest = pl.logL - pl.logL1;
  int npass = (rest + 9) / 10;
  if (npass > MAX_COL_PASSES) return false;
  pl.ncol = npass;
  int64_t S = (int64_t)1 << pl.logL;
  for (int c = 0; c < npass; ++c) {
    int take = rest / (npass - c);   // outermost passes get the smaller share
    rest -= take;
    pl.col[c].logn = take;
    S >>= take;
    pl.col[c].S = S;
    // inner indices per workgroup: T * n <= LDS_WORDS, T <= S, and T <= BLOCK (each
    // thread owns one inner index and steps through the frequencies by BLOCK / T);
    // short passes get wider tiles so that a workgroup holds up to 2048 elements
    int64_t want = std::max<int64_t>(col_tile > 0 ? col_tile : col_tile_max(), 2048 >> take);
    want = std::min<int64_t>(want, BLOCK);
    int64_t T = std::min<int64_t>(S, std::min<int64_t>(want, LDS_WORDS >> take));
    pl.col_tile[c] = (int32_t)std::max<int64_t>(T, 1);
  }
  return true;
}

static bool finish(Plan &pl) {
  pl.log2P = bitlen_product(pl.np);
  pl.W = pl.np;                      // >= (log2P + 1) / 32: every prime is below 2^30
  if (pl.W > MAXW) return false;
  const int wa = (pl.Na + 63) / 64, wb = (pl.Nb + 63) / 64;
  const int wmax = std::max(wa, wb);
  // convert-in: stage TI coefficients (2w+1 words each) in LDS; the smallest tile whose
  // K TI limbs still give every thread of the workgroup one, but not below 16
  // coefficients where LDS allows: each residue row gets TI consecutive words per
  // workgroup, and shorter runs than 64 bytes slow the writes down (large K)
  const int pw_words = 2 * ((pl.M + 31) / 32) * pl.np + 2;   // staged 2^(32t) mod p table
  int lt = 6;
  while (lt > 0 && ((((2 * wmax + 1) << lt) + pw_words > LDS_WORDS) ||
                    (lt > 4 && ((int64_t)pl.K << (lt - 1)) >= BLOCK)))
    --lt;
  if (((2 * wmax + 1) << lt) + pw_words > LDS_WORDS) return false;
  pl.log_ti_in = lt;
  // recovery: TI coefficients x nw32 64-bit partial sums (<= 48 KiB) and at most 1024
  // items; then the smallest tile that still gives the workgroup at least 192 of its 256
  // threads' worth of items, so that more workgroups share a CU's LDS, but not below 4
  // coefficients: a tile's residue loads take TI consecutive words of each row, and
  // narrower tiles waste most of each line (wide outputs, large K)
  const int64_t J = 2 * (int64_t)pl.K - 1;
  const int64_t nw32 = 2 * (int64_t)((pl.nout_bits + 63) / 64);
  lt = 6;
  while (lt > 0 && ((nw32 << lt) * 2 > 12288 || (J << lt) > 1024)) --lt;
  while (lt > 2 && (J << (lt - 1)) >= 192) --lt;
  // the CRT's matrix form may touch 4 TN + 1 words past a row: such a recovery may take
  // more than 64 KiB (up to 96 of the 160 KiB a gfx950 workgroup can address)
  const size_t lds_cap = pl.np <= CRT_MFMA_NP ? 96 * 1024 : 4 * (size_t)LDS_WORDS;
  if (recover_lds_bytes(pl.np, pl.K, pl.M, (int)nw32, lt) > lds_cap) return false;
  pl.log_ti_out = lt;
  pl.ws_words = (int64_t)pl.np * 2 * pl.K << pl.logL;
  return true;
}

static double model_cost(const Plan &pl) {
  // butterflies of the row-column transforms (forward on both operands, inverse
  // on the product) and the pointwise products, in units of one radix-2 butterfly
  const double K = pl.K, L = std::ldexp(1.0, pl.logL), np = pl.np;
  const double logK2 = std::log2(2.0 * K);
  double bfly = np * (K * L * pl.logL            // forward y, two operands, K columns each
                      + K * L * pl.logL           // inverse y, 2K columns
                      + 3.0 * L * K * logK2       // forward x (two operands) + inverse x
                      + 2.0 * K * L);             // pointwise
  double alu = bfly * 10.0;
  const double J = 2.0 * K - 1.0;
  // CRT per value c_{i,j}: on the matrix cores up to CRT_MFMA_NP primes (its residue
  // products, staging, digit folding and carries), else np W word multiply-adds
  const double crt = pl.np <= CRT_MFMA_NP ? 17.0 * np + 450.0 : np * 4.0 + (np + 1.0) * pl.W * 3.0;
  alu += (double)pl.nout * J * crt;
  double words = np * 2.0 * K * L;
  double bytes = 4.0 * words * 2.0 * (1 + pl.ncol * 1.5) + 4.0 * words;   // passes over the spectra
  bytes += 8.0 * (pl.da * ((pl.Na + 63) / 64) + pl.db * ((pl.Nb + 63) / 64) +
                  pl.nout * ((pl.nout_bits + 63) / 64));
  double t_alu = alu / 39.3e12, t_mem = bytes / 5.0e12;
  // strided passes with tiles narrower than 32 bytes waste part of each request
  for (int c = 0; c < pl.ncol; ++c)
    if (pl.col_tile[c] < 8) t_mem *= 8.0 / pl.col_tile[c];
  return t_alu + t_mem + 4e-6 * (4 + 3 * pl.ncol);
}

int32_t size_class(int64_t da, int32_t Na, int64_t db, int32_t Nb) {
  const int32_t N = std::max(std::max(Na, Nb), 2);
  return (ceil_log2(da + db - 1) << 8) | ceil_log2((N + 31) / 32);
}

bool make_plan(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K_force, int32_t np_force,
               Plan &out, const char **why, const PlanLimits *lim) {
  static const PlanLimits deflim;
  if (!lim) lim = &deflim;
  static const char *dummy;
  if (!why) why = &dummy;
  *why = nullptr;
  if (da < 1 || db < 1 || Na < 1 || Nb < 1) { *why = "sizes must be positive"; return false; }
  const int64_t nout = da + db - 1;
  const int logL = ceil_log2(nout);
  if (logL > LOG2_ROOT_ORDER) { *why = "da + db - 1 exceeds 2^21"; return false; }
  const int32_t N = std::max(std::max(Na, Nb), 2);
  const int64_t d = std::min(da, db);   // terms of each c_{i,j}: at most min(da, db) K
  bool found = false;
  Plan best;
  for (int logK = 1; logK <= 20; ++logK) {
    const int32_t K = 1 << logK;
    if (K_force && K != K_force) continue;
    if (K > lim->k_max) break;
    if (!K_force && K > 2 * (int64_t)N) break;     // limbs of 2 bits or less: no point going further
    if (logK + 1 > LOG2_ROOT_ORDER) break;
    Plan pl;
    std::memset(&pl, 0, sizeof(pl));
    pl.da = da; pl.db = db; pl.Na = Na; pl.Nb = Nb;
    pl.nout = nout;
    pl.nout_bits = out_bits(da, Na, db, Nb);
    pl.K = K;
    pl.M = std::max<int32_t>(2, (N + K - 1) / K);
    pl.logL = logL;
    if ((double)d * K > 4e18) continue;
    int np = 0;
    if (np_force) {
      if (np_force > MAXNP || np_compiled(np_force) != np_force ||
          !primes_cover(np_force, d, K, pl.M))
        continue;
      np = np_force;
    } else {
      for (int t = 1; t <= lim->np_max; ++t)
        if (primes_cover(t, d, K, pl.M)) { np = t; break; }
      if (!np) continue;
      np = np_compiled(np);
      if (np > lim->np_max) continue;
    }
    pl.np = np;
    if (!split_y(pl, lim->reg_k_max, lim->col_tile) || !finish(pl)) continue;
    pl.cost = model_cost(pl);
    if (!found || pl.cost < best.cost) { best = pl; found = true; }
  }
  if (!found) { *why = "no feasible (K, M, np) for these sizes"; return false; }
  // A small product's fused row kernel runs one workgroup per prime and inner block of
  // L1 rows: with a long inner factor that is a handful of workgroups, each working
  // through log2 L1 LDS stages, while the rest of the chip idles.  For a product that
  // runs alone, shorten the inner factor (K unchanged) until there are enough workgroups;
  // the column pass that takes the difference costs two short launches.  Only deep inner
  // transforms gain: at 2^9 or less, or with K >= 8, the pass costs more than it saves.
  // A forced K or np keeps the cost model's split.
  if (lim->row_groups_min > 0 && !K_force && !np_force && best.conv_reg && best.ncol <= 1 &&
      best.logL1 >= 10) {
    int cap = best.logL1;
    while (cap > 5 && ((int64_t)best.np << (best.logL - cap)) < lim->row_groups_min) --cap;
    Plan alt = best;
    if (cap < best.logL1 && split_y(alt, lim->reg_k_max, lim->col_tile, cap) && alt.ncol <= 1 &&
        finish(alt)) {
      alt.cost = model_cost(alt);
      best = alt;
    }
  }
  out = best;
  return true;
}

}  // namespace zpm
