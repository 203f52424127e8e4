// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), from its published
// definition: ten rounds of two 32x32->64-bit products with the Weyl key
// schedule.  Site-proposal uniforms use counter (site, slice, sweep, pass),
// key (seed low, seed high) and u = (w0 * 2^21 + (w1 >> 11)) * 2^-53.
#pragma once
#include <stdint.h>

struct philox_out { uint32_t w[4]; };

__host__ __device__ __forceinline__ philox_out philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                              uint32_t c3, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    uint64_t p0 = (uint64_t)M0 * c0;
    uint64_t p1 = (uint64_t)M1 * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  philox_out o;
  o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
  return o;
}

__host__ __device__ __forceinline__ double philox_u53(uint32_t w0, uint32_t w1) {
  return ((double)w0 * 2097152.0 + (double)(w1 >> 11)) * (1.0 / 9007199254740992.0);
}

__host__ __device__ __forceinline__ double site_uniform(uint64_t seed, uint64_t sweep, int pass, int slice,
                                                       int site) {
  philox_out o = philox4x32_10((uint32_t)site, (uint32_t)slice, (uint32_t)sweep, (uint32_t)pass,
                               (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  return philox_u53(o.w[0], o.w[1]);
}
