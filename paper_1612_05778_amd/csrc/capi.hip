// C-ABI of the zpm library: context, planner queries and the multiply entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/zpm.h"
#include "ctx.hpp"
#include "kernels.hpp"
#include "p64.hpp"
#include "gfp.hpp"
#include "nt.hpp"
#include "plan.hpp"

using namespace zpm;

static void fill_info(const Plan &pl, zpm_plan_info *o) {
  std::memset(o, 0, sizeof(*o));
  o->da = pl.da; o->db = pl.db; o->Na = pl.Na; o->Nb = pl.Nb;
  o->K = pl.K; o->M = pl.M; o->np = pl.np;
  o->log2_L = pl.logL; o->log2_L1 = pl.logL1; o->ncol = pl.ncol;
  for (int c = 0; c < pl.ncol && c < 4; ++c) {
    o->col_log2n[c] = pl.col[c].logn;
    o->col_tile[c] = pl.col_tile[c];
  }
  o->W = pl.W; o->log2P = pl.log2P; o->nout_bits = pl.nout_bits;
  o->workspace_bytes = pl.ws_words * 4;
}

namespace zpm {

int Ctx::ensure_tables(int np, int64_t H, int64_t TP) {
  H = std::max<int64_t>(H, 2);
  TP = std::max<int64_t>(TP, 64);
  if (np <= np_built && H <= H_built && TP <= TP_built) return ZPM_OK;
  if (reserved) return ZPM_ENOMEM;   // beyond the reservation: no reallocation
  const int np2 = std::max(np, np_built);
  const int64_t H2 = std::max(H, H_built);
  const int64_t TP2 = std::max(TP, TP_built);
  const int64_t per = 2 * H2 + TP2;          // forward heap, inverse heap, powers of 2^32
  if (hipDeviceSynchronize() != hipSuccess) return ZPM_EDEVICE;
  std::vector<uint2> host((size_t)np2 * per);
  const auto &PT = prime_table();
  for (int k = 0; k < np2; ++k) {
    uint2 *blk = &host[(size_t)k * per];
    fill_heap(k, (int)H2, blk, blk + H2);
    const uint32_t p = PT[k].p;
    uint32_t x = 1;
    for (int64_t t = 0; t < TP2; ++t) {
      blk[2 * H2 + t] = make_uint2(x, shoup(x, p));
      x = mulmod(x, PT[k].c32, p);
    }
  }
  uint2 *dev = nullptr;
  if (hipMalloc(&dev, host.size() * sizeof(uint2)) != hipSuccess) return ZPM_ENOMEM;
  if (hipMemcpy(dev, host.data(), host.size() * sizeof(uint2), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(dev);
    return ZPM_EDEVICE;
  }
  if (heaps) (void)hipFree(heaps);
  heaps = dev;
  np_built = np2;
  H_built = H2;
  TP_built = TP2;
  std::vector<PrimeDev> pd(MAXNP);
  const auto &T = prime_table();
  for (int k = 0; k < MAXNP; ++k) {
    std::memset(&pd[k], 0, sizeof(PrimeDev));
    pd[k].p = T[k].p;
    pd[k].pinv = T[k].pinv;
    pd[k].c32 = T[k].c32;
    pd[k].c32s = T[k].c32s;
    pd[k].ones = T[k].ones;
    if (k < np2) {
      pd[k].hf = heaps + (size_t)k * per;
      pd[k].hi = heaps + (size_t)k * per + H2;
      pd[k].pow32 = heaps + (size_t)k * per + 2 * H2;
    }
  }
  if (hipMemcpy(primes, pd.data(), sizeof(PrimeDev) * MAXNP, hipMemcpyHostToDevice) != hipSuccess)
    return ZPM_EDEVICE;
  return ZPM_OK;
}

int Ctx::plan_consts(const Plan &pl, PlanDev **out, hipStream_t st) {
  auto key = std::make_tuple(pl.np, pl.K, pl.M, pl.logL);
  auto it = consts.find(key);
  if (it != consts.end()) { *out = it->second; return ZPM_OK; }
  PlanDev h;
  std::memset(&h, 0, sizeof(h));
  crt_constants(pl.np, h);
  scale_constants(pl.np, pl.K, pl.M, pl.logL, h);
  if (reserved) {
    // a reserved slot: its pinned copy is written once and uploaded on the caller's
    // stream, ahead of the kernels that read it
    if (pool_used >= pool_cap) return ZPM_ENOMEM;
    const int slot = pool_used;
    pool_h[slot] = h;
    if (hipMemcpyAsync(pool_d + slot, pool_h + slot, sizeof(PlanDev), hipMemcpyHostToDevice, st) !=
        hipSuccess)
      return ZPM_EDEVICE;
    ++pool_used;
    consts[key] = pool_d + slot;
    *out = pool_d + slot;
    return ZPM_OK;
  }
  PlanDev *d = nullptr;
  if (hipMalloc(&d, sizeof(PlanDev)) != hipSuccess) return ZPM_ENOMEM;
  if (hipMemcpy(d, &h, sizeof(PlanDev), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return ZPM_EDEVICE;
  }
  consts[key] = d;
  consts_owned.push_back(d);
  *out = d;
  return ZPM_OK;
}

int Ctx::ensure_ws(int64_t words) {
  if (words <= ws_words) return ZPM_OK;
  if (reserved) return ZPM_ENOMEM;
  if (hipDeviceSynchronize() != hipSuccess) return ZPM_EDEVICE;
  if (ws) (void)hipFree(ws);
  ws = nullptr;
  ws_words = 0;
  if (hipMalloc(&ws, (size_t)words * 4) != hipSuccess) return ZPM_ENOMEM;
  ws_words = words;
  return ZPM_OK;
}

int Ctx::get_plan(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K, int32_t np,
                  Plan *out, bool alone) {
  // -2: plans of products alone, -3: of resident operands
  auto key = std::make_tuple(da, Na, db, Nb, K, np, (int32_t)(alone ? -2 : -3));
  auto it = plans.find(key);
  if (it != plans.end()) { *out = it->second; return ZPM_OK; }
  Plan pl;
  const char *why = nullptr;
  PlanLimits lim;
  lim.row_groups_min = alone ? ROW_GROUPS_MIN : 0;
  if (!make_plan(da, Na, db, Nb, K, np, pl, &why, &lim)) return ZPM_EUNSUPPORTED;
  if (plans.size() > 65536) plans.clear();
  plans[key] = pl;
  *out = pl;
  return ZPM_OK;
}

int Ctx::prepare(const Plan &pl, DevState *ds, hipStream_t st) {
  int rc;
  const int64_t H = std::max<int64_t>((int64_t)1 << pl.logL, 2 * (int64_t)pl.K);
  if ((rc = ensure_tables(pl.np, H, (pl.M + 31) / 32 + 1)) != ZPM_OK) return rc;
  PlanDev *pd = nullptr;
  if ((rc = plan_consts(pl, &pd, st)) != ZPM_OK) return rc;
  if ((rc = ensure_ws(pl.ws_words)) != ZPM_OK) return rc;
  ds->X = ws;
  ds->primes = primes;
  ds->plan = pd;
  return ZPM_OK;
}

int Ctx::reserve(size_t ws_bytes, int64_t max_len, int32_t max_bits, int32_t max_plans) {
  int rc;
  if (hipDeviceSynchronize() != hipSuccess) return ZPM_EDEVICE;
  reserved = false;   // growth below is allowed
  // twiddle heaps of every prime for transforms up to the next power of two of max_len
  // and for every 2K-point x-transform (K <= 2 max_bits, K <= 1024), and the 2^(32 t)
  // tables for limbs of up to max_bits / 2 bits
  int64_t H = 2;
  while (H < max_len) H <<= 1;
  int64_t twoK = 4;
  while (twoK < 4 * (int64_t)max_bits && twoK < 2048) twoK <<= 1;
  H = std::max(H, twoK);
  const int64_t TP = ((int64_t)max_bits / 2 + 1 + 31) / 32 + 2;
  if ((rc = ensure_tables(MAXNP, H, TP)) != ZPM_OK) return rc;
  if ((rc = ensure_ws((int64_t)((ws_bytes + 3) / 4))) != ZPM_OK) return rc;
  const int cap = max_plans > 0 ? max_plans : 256;
  if (cap > pool_cap - pool_used) {
    // a new pool; slots handed out earlier stay where they are (kept until destruction)
    PlanDev *d = nullptr, *h = nullptr;
    if (hipMalloc(&d, sizeof(PlanDev) * (size_t)cap) != hipSuccess) return ZPM_ENOMEM;
    if (hipHostMalloc(&h, sizeof(PlanDev) * (size_t)cap, hipHostMallocDefault) != hipSuccess) {
      (void)hipFree(d);
      return ZPM_ENOMEM;
    }
    if (pool_d) pool_old.emplace_back(pool_d, pool_h);
    pool_d = d;
    pool_h = h;
    pool_cap = cap;
    pool_used = 0;
  }
  reserved = true;
  return ZPM_OK;
}

int Ctx::check_range(const uint64_t *src, int64_t d, int32_t N, hipStream_t st) {
  if (!check_inputs || d <= 0 || ((N - 1) & 63) == 63) return ZPM_OK;
  if (hipMemsetAsync(flag_d, 0, sizeof(uint32_t), st) != hipSuccess) return ZPM_EDEVICE;
  if (launch_check_range(src, d, N, flag_d, st) != hipSuccess) return ZPM_EDEVICE;
  if (hipMemcpyAsync(flag_h, flag_d, sizeof(uint32_t), hipMemcpyDeviceToHost, st) != hipSuccess)
    return ZPM_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return ZPM_EDEVICE;
  return *flag_h ? ZPM_ERANGE : ZPM_OK;
}

Ctx::~Ctx() {
  p64_release(*this);
  gfp_release(*this);
  if (!primes) return;   // a host-only context (planning) owns no device resources
  (void)hipSetDevice(device);
  (void)hipDeviceSynchronize();
  batch_eager.release();
  batch_graph.release();
  if (capture_stream) (void)hipStreamDestroy(capture_stream);
  if (ws) (void)hipFree(ws);
  if (kbuf) (void)hipFree(kbuf);
  if (heaps) (void)hipFree(heaps);
  if (primes) (void)hipFree(primes);
  for (PlanDev *d : consts_owned) (void)hipFree(d);
  pool_old.emplace_back(pool_d, pool_h);
  for (auto &ph : pool_old) {
    if (ph.first) (void)hipFree(ph.first);
    if (ph.second) (void)hipHostFree(ph.second);
  }
  if (flag_d) (void)hipFree(flag_d);
  if (flag_h) (void)hipHostFree(flag_h);
}

}  // namespace zpm

namespace zpm {

Plan operand_plan(const zpm_operand &op, int64_t da, int32_t Na) {
  Plan pl = op.pl;
  pl.da = da;
  pl.Na = Na;
  pl.nout = da + op.db - 1;
  pl.nout_bits = out_bits(da, Na, op.db, op.Nb);
  pl.square = 0;
  pl.spec = 1;
  return pl;
}

int operand_product(Ctx &cx, const zpm_operand &op, const Plan &pl, const uint64_t *a, uint64_t *c,
                    int32_t wc, uint32_t *ws, hipStream_t st) {
  int rc;
  PlanDev *pd = nullptr;
  if ((rc = cx.plan_consts(pl, &pd, st)) != ZPM_OK) return rc;
  DevState ds;
  ds.X = ws;
  ds.primes = cx.primes;
  ds.plan = pd;
  // a's limbs into rows 0..K-1 and their forward column passes; the row kernel takes
  // b's spectra as they are
  bool ok = launch_convert_in(pl, ds, a, pl.da, pl.Na, 0, st) == hipSuccess;
  for (int k = 0; ok && k < pl.ncol; ++k) ok = launch_col(pl, ds, k, false, st, pl.K, 0) == hipSuccess;
  ok = ok && launch_convolve(pl, ds, st, CM_WITH_SPECTRUM, op.spec) == hipSuccess;
  for (int k = pl.ncol - 1; ok && k >= 0; --k) ok = launch_col(pl, ds, k, true, st) == hipSuccess;
  ok = ok && launch_recover(pl, ds, c, wc, st) == hipSuccess;
  return ok ? ZPM_OK : ZPM_EDEVICE;
}

}  // namespace zpm

extern "C" {

int zpm_version(void) { return 100; }

const char *zpm_strerror(int err) {
  switch (err) {
    case ZPM_OK: return "ok";
    case ZPM_EINVAL: return "invalid argument";
    case ZPM_ENOMEM: return "device allocation failed";
    case ZPM_EDEVICE: return "HIP device or runtime error";
    case ZPM_ERANGE: return "input coefficient outside the declared N-bit range";
    case ZPM_EUNSUPPORTED: return "sizes not supported by the prime table";
    case ZPM_ENOTIMPL: return "not implemented by this library";
    case ZPM_EBUSY: return "no capacity right now";
    case ZPM_ENOTFOUND: return "unknown ticket";
    case ZPM_ETOOBIG: return "product exceeds the fixed no-allocation scratch array";
    default: return "unknown error";
  }
}

int32_t zpm_out_bits(int64_t da, int32_t Na, int64_t db, int32_t Nb) {
  if (da < 1 || db < 1 || Na < 1 || Nb < 1) return 0;
  return out_bits(da, Na, db, Nb);
}

int zpm_plan(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K, int32_t np,
             zpm_plan_info *out) {
  if (!out || da < 1 || db < 1 || Na < 1 || Nb < 1 || K < 0 || np < 0) return ZPM_EINVAL;
  Plan pl;
  const char *why = nullptr;
  PlanLimits lim;
  lim.row_groups_min = ROW_GROUPS_MIN;     // the plan zpm_mul takes
  if (!make_plan(da, Na, db, Nb, K, np, pl, &why, &lim)) return ZPM_EUNSUPPORTED;
  fill_info(pl, out);
  return ZPM_OK;
}

int zpm_prime(int32_t k, uint32_t *p, uint32_t *root) {
  if (k < 0 || k >= MAXNP || !p || !root) return ZPM_EINVAL;
  const auto &T = prime_table();
  if (k >= (int)T.size()) return ZPM_EINVAL;
  *p = T[k].p;
  *root = T[k].root;
  return ZPM_OK;
}

int zpm_crt_matrix(int32_t np, int8_t *out, int64_t cap, int32_t *tiles) {
  if (np < 1 || np > CRT_MFMA_NP || !out || !tiles) return ZPM_EINVAL;
  const int TN = crt_tiles(np);
  const int64_t bytes = (int64_t)TN * CRT_STEPS * 64 * 16;
  if (cap < bytes) return ZPM_EINVAL;
  PlanDev h;
  std::memset(&h, 0, sizeof(h));
  crt_constants(np, h);
  std::memcpy(out, h.crt_afrag, (size_t)bytes);   // tiles are the array's leading index
  *tiles = TN;
  return ZPM_OK;
}

int zpm_device_limits(int device, int32_t *ncu, int64_t *lds_per_block, int64_t *lds_per_cu) {
  if (!ncu || !lds_per_block || !lds_per_cu) return ZPM_EINVAL;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return ZPM_EDEVICE;
  *ncu = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess)
    return ZPM_EDEVICE;
  *lds_per_block = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) !=
      hipSuccess)
    return ZPM_EDEVICE;
  *lds_per_cu = v;
  return ZPM_OK;
}

int zpm_create(zpm_ctx **out, int device) {
  if (!out) return ZPM_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return ZPM_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return ZPM_EDEVICE;
  Ctx *c = new (std::nothrow) Ctx();
  if (!c) return ZPM_ENOMEM;
  c->device = device;
  if (prime_table().size() < (size_t)MAXNP) { delete c; return ZPM_EUNSUPPORTED; }
  if (hipMalloc(&c->primes, sizeof(PrimeDev) * MAXNP) != hipSuccess) { delete c; return ZPM_ENOMEM; }
  if (hipMalloc(&c->flag_d, sizeof(uint32_t)) != hipSuccess ||
      hipHostMalloc(&c->flag_h, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return ZPM_ENOMEM;
  }
  if (noalloc_init(device) != hipSuccess) { delete c; return ZPM_EDEVICE; }
  const char *chk = std::getenv("ZPM_CHECK_INPUTS");
  c->check_inputs = (chk && chk[0] == '1') ? 1 : 0;
  *out = reinterpret_cast<zpm_ctx *>(c);
  return ZPM_OK;
}

void zpm_destroy(zpm_ctx *ctx) { delete reinterpret_cast<Ctx *>(ctx); }

int zpm_reserve(zpm_ctx *ctx, size_t workspace_bytes, int64_t max_len, int32_t max_bits,
                int32_t max_plans) {
  if (!ctx || max_len < 1 || max_bits < 1 || max_plans < 0) return ZPM_EINVAL;
  if (max_len > ((int64_t)1 << LOG2_ROOT_ORDER)) return ZPM_EUNSUPPORTED;
  Ctx *cx = reinterpret_cast<Ctx *>(ctx);
  std::lock_guard<std::mutex> lock(cx->mu);
  if (hipSetDevice(cx->device) != hipSuccess) return ZPM_EDEVICE;
  return cx->reserve(workspace_bytes, max_len, max_bits, max_plans);
}

int zpm_set_option(zpm_ctx *ctx, int32_t option, int64_t value) {
  if (!ctx) return ZPM_EINVAL;
  Ctx *cx = reinterpret_cast<Ctx *>(ctx);
  std::lock_guard<std::mutex> lock(cx->mu);
  switch (option) {
    case ZPM_OPT_CHECK_INPUTS:
      if (value != 0 && value != 1) return ZPM_EINVAL;
      cx->check_inputs = (int)value;
      return ZPM_OK;
    default: return ZPM_EINVAL;
  }
}

static int check_mul_args(const uint64_t *a, int64_t da, int32_t Na, const uint64_t *b, int64_t db,
                          int32_t Nb, uint64_t *c, int32_t wc) {
  if (da < 0 || db < 0 || Na < 1 || Nb < 1) return ZPM_EINVAL;
  if (da == 0 || db == 0) return ZPM_OK;
  if (!a || !b || !c) return ZPM_EINVAL;
  const int32_t nb = out_bits(da, Na, db, Nb);
  if (wc < (nb + 63) / 64) return ZPM_EINVAL;
  // the output must not overlap either input
  const uint64_t *c_end = c + (size_t)(da + db - 1) * wc;
  const uint64_t *a_end = a + (size_t)da * ((Na + 63) / 64);
  const uint64_t *b_end = b + (size_t)db * ((Nb + 63) / 64);
  if (c < a_end && a < c_end) return ZPM_EINVAL;
  if (c < b_end && b < c_end) return ZPM_EINVAL;
  return ZPM_OK;
}

int zpm_mul_ex(zpm_ctx *ctx, const uint64_t *a, int64_t da, int32_t Na, const uint64_t *b,
               int64_t db, int32_t Nb, uint64_t *c, int32_t wc, int32_t K, int32_t np,
               int32_t stop_after, uint32_t *ws_out, void *stream) {
  if (!ctx || K < 0 || np < 0 || stop_after < 0 || stop_after > 4) return ZPM_EINVAL;
  if (stop_after && !ws_out) return ZPM_EINVAL;
  int rc = check_mul_args(a, da, Na, b, db, Nb, c, wc);
  if (rc != ZPM_OK) return rc;
  if (da == 0 || db == 0) return ZPM_OK;
  Ctx *cx = reinterpret_cast<Ctx *>(ctx);
  std::lock_guard<std::mutex> lock(cx->mu);
  if (hipSetDevice(cx->device) != hipSuccess) return ZPM_EDEVICE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if ((rc = cx->check_range(a, da, Na, st)) != ZPM_OK) return rc;
  if ((rc = cx->check_range(b, db, Nb, st)) != ZPM_OK) return rc;
  Plan pl;
  if ((rc = cx->get_plan(da, Na, db, Nb, K, np, &pl)) != ZPM_OK) {
    // coefficients too wide for one product: Kronecker reshaping, when nothing is forced
    if (rc != ZPM_EUNSUPPORTED || K || np || stop_after) return rc;
    return cx->mul_kronecker(a, da, Na, b, db, Nb, c, wc, 0, st);
  }
  // c = a^2 when one operand is passed twice: it is converted and transformed once
  // (stage dumps keep the documented layout with both operands' rows)
  pl.square = (a == b && da == db && Na == Nb && !stop_after) ? 1 : 0;
  DevState ds;
  if ((rc = cx->prepare(pl, &ds, st)) != ZPM_OK) return rc;
  if (launch_mul(pl, ds, a, b, c, wc, stop_after, st, &cx->prof) != hipSuccess) return ZPM_EDEVICE;
  if (stop_after) {
    if (hipMemcpyAsync(ws_out, ds.X, (size_t)pl.ws_words * 4, hipMemcpyDeviceToDevice, st) !=
        hipSuccess)
      return ZPM_EDEVICE;
  }
  return ZPM_OK;
}

int zpm_mul(zpm_ctx *ctx, const uint64_t *a, int64_t da, int32_t Na, const uint64_t *b, int64_t db,
            int32_t Nb, uint64_t *c, int32_t wc, void *stream) {
  return zpm_mul_ex(ctx, a, da, Na, b, db, Nb, c, wc, 0, 0, 0, nullptr, stream);
}

int zpm_profile_begin_kinds(zpm_ctx *ctx, uint32_t kinds) {
  if (!ctx) return ZPM_EINVAL;
  Ctx *cx = reinterpret_cast<Ctx *>(ctx);
  std::lock_guard<std::mutex> lock(cx->mu);
  cx->prof.reset();
  cx->prof.mask = kinds;
  cx->prof.on = true;
  return ZPM_OK;
}

int zpm_profile_begin(zpm_ctx *ctx) { return zpm_profile_begin_kinds(ctx, ~0u); }

int zpm_profile_end(zpm_ctx *ctx, zpm_kernel_time *out, int32_t max_out, int32_t *n_out) {
  if (!ctx || !n_out || (max_out > 0 && !out)) return ZPM_EINVAL;
  Ctx *cx = reinterpret_cast<Ctx *>(ctx);
  std::lock_guard<std::mutex> lock(cx->mu);
  static const char *names[KK_COUNT] = {"bivariate_representation", "col_pass_fwd",
                                        "convolve_rows", "col_pass_inv",
                                        "recovering_product", "batch",
                                        "p64_convert_in", "p64_y_fwd", "p64_x_convolve",
                                        "p64_y_inv", "p64_recover", "gfp_convert_in",
                                        "gfp_y_fwd", "gfp_x_convolve", "gfp_y_inv",
                                        "gfp_recover"};
  double ms[KK_COUNT] = {0};
  int64_t cnt[KK_COUNT] = {0};
  int rc = ZPM_OK;
  for (auto &r : cx->prof.recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) { rc = ZPM_EDEVICE; break; }
    float t = 0;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) { rc = ZPM_EDEVICE; break; }
    ms[r.kind] += t;
    cnt[r.kind] += 1;
  }
  cx->prof.on = false;
  cx->prof.reset();
  int n = 0;
  for (int k = 0; k < KK_COUNT; ++k) {
    if (!cnt[k]) continue;
    if (n < max_out) {
      std::memset(&out[n], 0, sizeof(zpm_kernel_time));
      std::strncpy(out[n].name, names[k], sizeof(out[n].name) - 1);
      out[n].launches = cnt[k];
      out[n].total_ms = ms[k];
    }
    ++n;
  }
  *n_out = n;
  return rc;
}

int zpm_mul_kronecker(zpm_ctx *ctx, const uint64_t *a, int64_t da, int32_t Na, const uint64_t *b,
                      int64_t db, int32_t Nb, uint64_t *c, int32_t wc, int32_t chunk_bits,
                      void *stream) {
  if (!ctx || chunk_bits < 0 || (chunk_bits & 63)) return ZPM_EINVAL;
  int rc = check_mul_args(a, da, Na, b, db, Nb, c, wc);
  if (rc != ZPM_OK) return rc;
  if (da == 0 || db == 0) return ZPM_OK;
  Ctx *cx = reinterpret_cast<Ctx *>(ctx);
  std::lock_guard<std::mutex> lock(cx->mu);
  if (hipSetDevice(cx->device) != hipSuccess) return ZPM_EDEVICE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if ((rc = cx->check_range(a, da, Na, st)) != ZPM_OK) return rc;
  if ((rc = cx->check_range(b, db, Nb, st)) != ZPM_OK) return rc;
  return cx->mul_kronecker(a, da, Na, b, db, Nb, c, wc, chunk_bits, st);
}

int zpm_kronecker_plan(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t chunk_bits,
                       zpm_kron_info *out) {
  if (!out || da < 1 || db < 1 || Na < 1 || Nb < 1 || chunk_bits < 0 || (chunk_bits & 63))
    return ZPM_EINVAL;
  KronPlan kp;
  if (!kron_plan(da, Na, db, Nb, chunk_bits, &kp)) return ZPM_EUNSUPPORTED;
  out->chunk_bits = kp.w;
  out->s_a = kp.sa;
  out->s_b = kp.sb;
  out->S = kp.S;
  out->da2 = kp.da2;
  out->db2 = kp.db2;
  out->N2 = kp.N2;
  out->wc2 = kp.wc2;
  fill_info(kp.inner, &out->inner);
  return ZPM_OK;
}

static void fill_info64(const Plan64 &pl, zpm_p64_info *out) {
  std::memset(out, 0, sizeof(*out));
  out->da = pl.da;
  out->db = pl.db;
  out->Na = pl.Na;
  out->Nb = pl.Nb;
  out->K = pl.K;
  out->M = pl.M;
  out->np = pl.np;
  out->log2_L = pl.logL;
  out->npass = pl.npass;
  for (int q = 0; q < pl.npass; ++q) out->pass_log2n[q] = pl.pass[q].logn;
  out->log2_tx = pl.logTX;
  out->log2_ti = pl.logTI;
  out->log2P = pl.log2P;
  out->nout_bits = pl.nout_bits;
  out->workspace_bytes = pl.ws_words * 8;
}

int zpm_plan_p64(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K, int32_t np,
                 zpm_p64_info *out) {
  if (!out || K < 0 || np < 0 || da < 1 || db < 1 || Na < 1 || Nb < 1) return ZPM_EINVAL;
  Plan64 pl;
  if (!make_plan64(da, Na, db, Nb, K, np, pl, nullptr)) return ZPM_EUNSUPPORTED;
  fill_info64(pl, out);
  return ZPM_OK;
}

int zpm_prime64(int32_t k, uint64_t *p, uint64_t *root) {
  if (k < 0 || k >= MAXNP64 || !p || !root) return ZPM_EINVAL;
  *p = prime64_table()[k].p;
  *root = prime64_table()[k].root;
  return ZPM_OK;
}

int zpm_mul_p64(zpm_ctx *ctx, const uint64_t *a, int64_t da, int32_t Na, const uint64_t *b, int64_t db,
                int32_t Nb, uint64_t *c, int32_t wc, int32_t K, int32_t np, void *stream) {
  if (!ctx || K < 0 || np < 0) return ZPM_EINVAL;
  int rc = check_mul_args(a, da, Na, b, db, Nb, c, wc);
  if (rc != ZPM_OK) return rc;
  if (da == 0 || db == 0) return ZPM_OK;
  Plan64 pl;
  if (!make_plan64(da, Na, db, Nb, K, np, pl, nullptr)) return ZPM_EUNSUPPORTED;
  pl.square = (a == b && da == db && Na == Nb) ? 1 : 0;
  Ctx *cx = reinterpret_cast<Ctx *>(ctx);
  std::lock_guard<std::mutex> lock(cx->mu);
  if (hipSetDevice(cx->device) != hipSuccess) return ZPM_EDEVICE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if ((rc = cx->check_range(a, da, Na, st)) != ZPM_OK) return rc;
  if ((rc = cx->check_range(b, db, Nb, st)) != ZPM_OK) return rc;
  return mul_p64(*cx, pl, a, b, c, wc, st);
}

int zpm_operand_create(zpm_ctx *ctx, const uint64_t *b, int64_t db, int32_t Nb, int64_t da_max,
                       int32_t Na_max, int32_t K, zpm_operand **out, void *stream) {
  if (!ctx || !b || !out || db < 1 || Nb < 1 || da_max < 1 || Na_max < 1 || K < 0)
    return ZPM_EINVAL;
  *out = nullptr;
  Ctx *cx = reinterpret_cast<Ctx *>(ctx);
  std::lock_guard<std::mutex> lock(cx->mu);
  if (hipSetDevice(cx->device) != hipSuccess) return ZPM_EDEVICE;
  int rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if ((rc = cx->check_range(b, db, Nb, st)) != ZPM_OK) return rc;
  Plan pl;
  if ((rc = cx->get_plan(da_max, Na_max, db, Nb, K, 0, &pl, false)) != ZPM_OK) return rc;
  const int64_t H = std::max<int64_t>((int64_t)1 << pl.logL, 2 * (int64_t)pl.K);
  if ((rc = cx->ensure_tables(pl.np, H, (pl.M + 31) / 32 + 1)) != ZPM_OK) return rc;
  PlanDev *pd = nullptr;
  if ((rc = cx->plan_consts(pl, &pd, st)) != ZPM_OK) return rc;
  zpm_operand *op = new zpm_operand();
  op->cx = cx;
  op->pl = pl;
  op->b = b;
  op->db = db;
  op->Nb = Nb;
  op->da_max = da_max;
  op->Na_max = Na_max;
  if (hipMalloc(&op->spec, (size_t)pl.ws_words * 4) != hipSuccess) {
    delete op;
    return ZPM_ENOMEM;
  }
  DevState ds;
  ds.X = op->spec;
  ds.primes = cx->primes;
  ds.plan = pd;
  // b's limbs into rows K..2K-1, their forward column passes, then the spectra
  bool ok = launch_convert_in(pl, ds, b, db, Nb, pl.K, st) == hipSuccess;
  for (int c = 0; ok && c < pl.ncol; ++c) ok = launch_col(pl, ds, c, false, st, pl.K, pl.K) == hipSuccess;
  ok = ok && launch_convolve(pl, ds, st, CM_SPECTRUM) == hipSuccess;
  if (!ok) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(op->spec);
    delete op;
    return ZPM_EDEVICE;
  }
  *out = op;
  return ZPM_OK;
}

int zpm_mul_operand(zpm_ctx *ctx, const uint64_t *a, int64_t da, int32_t Na, const zpm_operand *op,
                    uint64_t *c, int32_t wc, void *stream) {
  if (!ctx || !op || reinterpret_cast<Ctx *>(ctx) != op->cx) return ZPM_EINVAL;
  if (da > op->da_max || Na > op->Na_max) return ZPM_EINVAL;
  int rc = check_mul_args(a, da, Na, op->b, op->db, op->Nb, c, wc);
  if (rc != ZPM_OK) return rc;
  if (da == 0) return ZPM_OK;
  Ctx *cx = op->cx;
  std::lock_guard<std::mutex> lock(cx->mu);
  if (hipSetDevice(cx->device) != hipSuccess) return ZPM_EDEVICE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if ((rc = cx->check_range(a, da, Na, st)) != ZPM_OK) return rc;
  // the operand's plan, for this a: K, M, np and L are fixed by the bounds
  const Plan pl = operand_plan(*op, da, Na);
  if ((rc = cx->ensure_ws(pl.ws_words)) != ZPM_OK) return rc;
  return operand_product(*cx, *op, pl, a, c, wc, cx->ws, st);
}

int zpm_mul_operand_batch(zpm_ctx *ctx, const zpm_operand_job *jobs, int64_t n, int32_t flags,
                          void *stream) {
  if (!ctx || n < 0 || (n > 0 && !jobs)) return ZPM_EINVAL;
  if (flags != 0 && flags != ZPM_BATCH_GRAPH && flags != ZPM_BATCH_PERSISTENT) return ZPM_EINVAL;
  Ctx *cx = reinterpret_cast<Ctx *>(ctx);
  std::vector<zpm_job> js((size_t)n);
  std::vector<Plan> pls((size_t)n);
  std::vector<const uint32_t *> specs((size_t)n, nullptr);
  for (int64_t i = 0; i < n; ++i) {
    const zpm_operand_job &o = jobs[i];
    if (!o.op || o.op->cx != cx || o.da > o.op->da_max || o.Na > o.op->Na_max) return ZPM_EINVAL;
    int rc = check_mul_args(o.a, o.da, o.Na, o.op->b, o.op->db, o.op->Nb, o.c, o.wc);
    if (rc != ZPM_OK) return rc;
    zpm_job &j = js[(size_t)i];
    j.a = o.a; j.da = o.da; j.Na = o.Na;
    j.b = o.op->b; j.db = o.op->db; j.Nb = o.op->Nb;
    j.c = o.c; j.wc = o.wc;
    if (o.da == 0) continue;
    pls[(size_t)i] = operand_plan(*o.op, o.da, o.Na);
    specs[(size_t)i] = o.op->spec;
  }
  std::lock_guard<std::mutex> lock(cx->mu);
  if (hipSetDevice(cx->device) != hipSuccess) return ZPM_EDEVICE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (int64_t i = 0; cx->check_inputs && i < n; ++i) {
    if (js[(size_t)i].da <= 0) continue;
    const int rc = cx->check_range(js[(size_t)i].a, js[(size_t)i].da, js[(size_t)i].Na, st);
    if (rc != ZPM_OK) return rc;
  }
  return cx->mul_batch(js.data(), n, flags, 0, st, 0, pls.data(), specs.data());
}

int zpm_operand_info(const zpm_operand *op, zpm_plan_info *out) {
  if (!op || !out) return ZPM_EINVAL;
  fill_info(op->pl, out);
  return ZPM_OK;
}

void zpm_operand_destroy(zpm_operand *op) {
  if (!op) return;
  (void)hipSetDevice(op->cx->device);
  if (op->spec) (void)hipFree(op->spec);
  delete op;
}

static void fill_info_gfp(const PlanGfp &pl, zpm_gfp_info *out) {
  std::memset(out, 0, sizeof(*out));
  out->da = pl.da;
  out->db = pl.db;
  out->Na = pl.Na;
  out->Nb = pl.Nb;
  out->k = pl.k;
  out->r = gfp_prime_table()[pl.prime].r;
  out->K = pl.K;
  out->M = pl.M;
  out->log2_L = pl.logL;
  out->npass = pl.npass;
  for (int q = 0; q < pl.npass && q < 6; ++q) out->pass_log2n[q] = pl.pass_logn[q];
  out->log2p = gfp_prime_table()[pl.prime].log2p;
  out->nout_bits = pl.nout_bits;
  out->workspace_bytes = pl.ws_words * 4;
}

static int gfp_prime_index(int32_t k) {
  if (k == 0) return -1;
  for (int i = 0; i < GFP_NPRIMES; ++i)
    if (gfp_prime_table()[i].k == k) return i;
  return -2;
}

int zpm_gfp_prime(int32_t k, int32_t *r, int32_t *log2p) {
  const int i = gfp_prime_index(k);
  if (i < 0 || !r || !log2p) return ZPM_EINVAL;
  *r = gfp_prime_table()[i].r;
  *log2p = gfp_prime_table()[i].log2p;
  return ZPM_OK;
}

int zpm_gfp_root(int32_t k, int32_t log2_L, int32_t *digits) {
  const int i = gfp_prime_index(k);
  if (i < 0 || !digits || log2_L < 0 || log2_L > GFP_LOG2_LMAX) return ZPM_EINVAL;
  return gfp_root(i, log2_L, digits) ? ZPM_OK : ZPM_EUNSUPPORTED;
}

int zpm_plan_gfp(int64_t da, int32_t Na, int64_t db, int32_t Nb, int32_t K, int32_t k,
                 zpm_gfp_info *out) {
  if (!out || K < 0 || da < 1 || db < 1 || Na < 1 || Nb < 1) return ZPM_EINVAL;
  const int pi = gfp_prime_index(k);
  if (pi == -2) return ZPM_EINVAL;
  PlanGfp pl;
  if (!make_plan_gfp(da, Na, db, Nb, K, pi, pl)) return ZPM_EUNSUPPORTED;
  fill_info_gfp(pl, out);
  return ZPM_OK;
}

int zpm_mul_gfp(zpm_ctx *ctx, const uint64_t *a, int64_t da, int32_t Na, const uint64_t *b,
                int64_t db, int32_t Nb, uint64_t *c, int32_t wc, int32_t K, int32_t k,
                void *stream) {
  if (!ctx || K < 0) return ZPM_EINVAL;
  const int pi = gfp_prime_index(k);
  if (pi == -2) return ZPM_EINVAL;
  int rc = check_mul_args(a, da, Na, b, db, Nb, c, wc);
  if (rc != ZPM_OK) return rc;
  if (da == 0 || db == 0) return ZPM_OK;
  PlanGfp pl;
  if (!make_plan_gfp(da, Na, db, Nb, K, pi, pl)) return ZPM_EUNSUPPORTED;
  pl.square = (a == b && da == db && Na == Nb) ? 1 : 0;
  Ctx *cx = reinterpret_cast<Ctx *>(ctx);
  std::lock_guard<std::mutex> lock(cx->mu);
  if (hipSetDevice(cx->device) != hipSuccess) return ZPM_EDEVICE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if ((rc = cx->check_range(a, da, Na, st)) != ZPM_OK) return rc;
  if ((rc = cx->check_range(b, db, Nb, st)) != ZPM_OK) return rc;
  return mul_gfp(*cx, pl, a, b, c, wc, st);
}

int zpm_sync(zpm_ctx *ctx, void *stream) {
  if (!ctx) return ZPM_EINVAL;
  Ctx *cx = reinterpret_cast<Ctx *>(ctx);
  if (hipSetDevice(cx->device) != hipSuccess) return ZPM_EDEVICE;
  if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return ZPM_EDEVICE;
  if (hipGetLastError() != hipSuccess) return ZPM_EDEVICE;
  return ZPM_OK;
}

}  // extern "C"
