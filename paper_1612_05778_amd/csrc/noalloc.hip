// Products that allocate nothing: zpm_mul with its residue workspace in a fixed
// device array instead of the context's allocated buffer.
//
// The array `scratch` below is a device symbol.  In host code its name is only a
// host-side stand-in, not a device address: every host use goes through the address
// that hipGetSymbolAddress returns for the current device, taken once per device when
// a context is created there (zpm_create calls noalloc_init).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "../../include/zpm.h"
#include "ctx.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace zpm {

// 64 MiB of 32-bit residues: np * 2K * L words of one product.
constexpr int64_t SCRATCH_WORDS = (int64_t)1 << 24;
static __device__ __align__(256) uint32_t scratch[SCRATCH_WORDS];

constexpr int MAX_DEVICES = 64;
static std::mutex g_mu;
static uint32_t *g_ptr[MAX_DEVICES];   // device address of `scratch` on each device
static hipError_t g_rc[MAX_DEVICES];
static bool g_done[MAX_DEVICES];

// Takes the address of `scratch` on `device`, which must be the current device.  Runs
// the lookup once per device; later calls return the first result.
hipError_t noalloc_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_done[device]) {
    void *p = nullptr;
    g_rc[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_ptr[device] = g_rc[device] == hipSuccess ? static_cast<uint32_t *>(p) : nullptr;
    g_done[device] = true;
  }
  return g_rc[device];
}

static uint32_t *scratch_ptr(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_done[device] ? g_ptr[device] : nullptr;
}

}  // namespace zpm

using namespace zpm;

extern "C" {

int64_t zpm_noalloc_max_bytes(void) { return SCRATCH_WORDS * 4; }

int zpm_mul_noalloc(zpm_ctx *ctx, const uint64_t *a, int64_t da, int32_t Na, const uint64_t *b,
                    int64_t db, int32_t Nb, uint64_t *c, int32_t wc, void *stream) {
  if (!ctx || da < 0 || db < 0 || Na < 1 || Nb < 1) return ZPM_EINVAL;
  if (da == 0 || db == 0) return ZPM_OK;
  if (!a || !b || !c) return ZPM_EINVAL;
  if (wc < (out_bits(da, Na, db, Nb) + 63) / 64) return ZPM_EINVAL;
  const uint64_t *c_end = c + (size_t)(da + db - 1) * wc;
  if (c < a + (size_t)da * ((Na + 63) / 64) && a < c_end) return ZPM_EINVAL;
  if (c < b + (size_t)db * ((Nb + 63) / 64) && b < c_end) return ZPM_EINVAL;
  Ctx *cx = reinterpret_cast<Ctx *>(ctx);
  std::lock_guard<std::mutex> lock(cx->mu);
  if (hipSetDevice(cx->device) != hipSuccess) return ZPM_EDEVICE;
  uint32_t *ws = scratch_ptr(cx->device);
  if (!ws) return ZPM_EDEVICE;
  int rc;
  Plan pl;
  if ((rc = cx->get_plan(da, Na, db, Nb, 0, 0, &pl)) != ZPM_OK) {
    // coefficients too wide for a direct plan: zpm_mul reshapes them (Kronecker), which
    // needs a buffer of its own; not provided here
    KronPlan kp;
    if (rc == ZPM_EUNSUPPORTED && kron_plan(da, Na, db, Nb, 0, &kp)) return ZPM_ENOTIMPL;
    return rc;
  }
  if (pl.ws_words > SCRATCH_WORDS) return ZPM_ETOOBIG;
  pl.square = (a == b && da == db && Na == Nb) ? 1 : 0;
  // tables and plan constants must already be resident (zpm_reserve, or earlier
  // products of this plan): building them would allocate
  const int64_t H = std::max<int64_t>((int64_t)1 << pl.logL, 2 * (int64_t)pl.K);
  const int64_t TP = std::max<int64_t>((pl.M + 31) / 32 + 1, 64);
  if (pl.np > cx->np_built || std::max<int64_t>(H, 2) > cx->H_built || TP > cx->TP_built)
    return ZPM_ENOMEM;
  const bool have_consts =
      cx->consts.count(std::make_tuple(pl.np, pl.K, pl.M, pl.logL)) != 0;
  if (!have_consts && !cx->reserved) return ZPM_ENOMEM;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  DevState ds;
  PlanDev *pd = nullptr;
  if ((rc = cx->plan_consts(pl, &pd, st)) != ZPM_OK) return rc;
  ds.X = ws;
  ds.primes = cx->primes;
  ds.plan = pd;
  if (launch_mul(pl, ds, a, b, c, wc, 0, st, &cx->prof) != hipSuccess) return ZPM_EDEVICE;
  return ZPM_OK;
}

}  // extern "C"
