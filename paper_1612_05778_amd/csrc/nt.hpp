// Host number theory: Fourier primes, roots of unity, Shoup companions, CRT constants.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <vector>

#include "zpm_internal.hpp"

namespace zpm {

struct PrimeHost {
  uint32_t p;
  uint32_t root;   // primitive 2^LOG2_ROOT_ORDER-th root of unity mod p
  uint32_t pinv;   // p^{-1} mod 2^32
  uint32_t c32, c32s, ones;
};

uint32_t mulmod(uint32_t a, uint32_t b, uint32_t p);
uint32_t powmod(uint32_t a, uint64_t e, uint32_t p);
uint32_t invmod(uint32_t a, uint32_t p);
uint32_t shoup(uint32_t w, uint32_t p);
bool is_prime(uint32_t n);

// MAXNP primes, largest first.
const std::vector<PrimeHost> &prime_table();
uint32_t root_of_order(int k, int e);
// hf/hi have H entries: roots for every transform length up to H.
void fill_heap(int k, int H, uint2 *hf, uint2 *hi);
int bitlen_product(int np);
bool primes_cover(int np, int64_t d, int64_t K, int64_t M);
void crt_constants(int np, PlanDev &pd);
// after crt_constants: also folds the transforms' normalisation into crt_inv
void scale_constants(int np, int K, int M, int logL, PlanDev &pd);

}  // namespace zpm
