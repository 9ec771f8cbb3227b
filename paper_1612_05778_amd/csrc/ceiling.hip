// Attainable rate of the transforms' modular butterfly on one device: every thread keeps
// eight independent (u, v) pairs modulo a 30-bit Fourier prime in registers and applies
// the forward-transform butterfly u, v -> u + v, (u - v) w (the add_lz / mul_shoup_lz pair
// of the transform kernels, values in [0, 2p)) to each, with no memory traffic.  Reported beside the ALU
// peak derived from the chip's lane count and clock.
#include <hip/hip_runtime.h>

#include "../../include/zpm.h"
#include "nt.hpp"
#include "stages.hpp"

namespace zpm {

__global__ __launch_bounds__(BLOCK) void k_bfly_ceiling(uint32_t p, uint2 w, int32_t iters,
                                                        uint32_t *__restrict__ sink) {
  const uint32_t id = blockIdx.x * BLOCK + threadIdx.x;
  uint32_t u[8], v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    u[j] = (id * 8 + j) % p;
    v[j] = (id * 13 + 7 * j + 1) % p;
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t a = add_lz(u[j], v[j], p);
      const uint32_t b = mul_shoup_lz(u[j] - v[j] + 2 * p, w, p);
      u[j] = a;
      v[j] = b;
    }
  }
  uint32_t acc = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) acc ^= u[j] ^ v[j];
  sink[id] = acc;
}

}  // namespace zpm

using namespace zpm;

extern "C" int zpm_butterfly_ceiling(int device, int32_t iters, double *bfly_per_s) {
  if (!bfly_per_s || iters < 1) return ZPM_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return ZPM_EDEVICE;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return ZPM_EDEVICE;
  const int blocks = 8 * ncu;   // eight 256-thread workgroups per compute unit
  uint32_t *sink = nullptr;
  if (hipMalloc(&sink, sizeof(uint32_t) * BLOCK * blocks) != hipSuccess) return ZPM_ENOMEM;
  const auto &T = prime_table();
  const uint32_t p = T[0].p;
  const uint32_t wv = T[0].root % p;
  const uint2 w = make_uint2(wv, shoup(wv, p));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = ZPM_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = ZPM_EDEVICE;
  float ms = 0;
  if (rc == ZPM_OK) {
    hipLaunchKernelGGL(k_bfly_ceiling, dim3(blocks), dim3(BLOCK), 0, nullptr, p, w, iters, sink);
    (void)hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(k_bfly_ceiling, dim3(blocks), dim3(BLOCK), 0, nullptr, p, w, iters, sink);
    (void)hipEventRecord(e1, nullptr);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
        hipGetLastError() != hipSuccess)
      rc = ZPM_EDEVICE;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  if (rc != ZPM_OK) return rc;
  *bfly_per_s = (double)blocks * BLOCK * 8.0 * iters / (ms / 1e3);
  return ZPM_OK;
}
