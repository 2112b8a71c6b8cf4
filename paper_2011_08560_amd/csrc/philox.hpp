// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11), device version.
// One round maps (c0,c1,c2,c3) with key (k0,k1) to
//   (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));
// the key grows by the Weyl constants before every round after the first.
// On gfx950 the 32x32->64 product is one full-rate v_mad_u64_u32; counter words
// that are uniform across the wave stay in scalar registers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace nfm {

struct u32x4 {
  uint32_t v[4];
};

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)M0 * c0;
    const uint64_t p1 = (uint64_t)M1 * c2;
    // three-input xors as single v_bitop3 (truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += W0;
    k1 += W1;
  }
  u32x4 r;
  r.v[0] = c0;
  r.v[1] = c1;
  r.v[2] = c2;
  r.v[3] = c3;
  return r;
}

// The same generator for counters whose words 0..2 are uniform across the wave and word 3
// varies (the acceptance and tempering streams): rounds 0-2 xor at most one varying word into
// uniform ones (a scalar xor, then one vector xor) and leave the uniform products to the scalar
// unit; from round 3 (c2's side) and round 4 (c0's side) on two varying words meet, one
// three-input v_bitop3. The keys stay uniform.
__device__ __forceinline__ u32x4 philox4x32_10_u(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                 uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
    const uint32_t n0 = round >= 4 ? __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96)
                                   : (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = round >= 3 ? __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96)
                                   : (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += W0;
    k1 += W1;
  }
  u32x4 r;
  r.v[0] = c0;
  r.v[1] = c1;
  r.v[2] = c2;
  r.v[3] = c3;
  return r;
}

// The same generator with the ten round keys precomputed in vector registers.
struct PhiloxKeysV {
  uint32_t k0[10], k1[10];
};

__device__ __forceinline__ PhiloxKeysV philox_round_keys_v(uint32_t k0, uint32_t k1) {
  PhiloxKeysV kv;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t a = k0 + (uint32_t)r * 0x9E3779B9u, b = k1 + (uint32_t)r * 0xBB67AE85u;
    asm volatile("v_mov_b32 %0, %1" : "=v"(kv.k0[r]) : "s"(a));
    asm volatile("v_mov_b32 %0, %1" : "=v"(kv.k1[r]) : "s"(b));
  }
  return kv;
}

__device__ __forceinline__ u32x4 philox4x32_10_vk(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                  const PhiloxKeysV& kv) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)M0 * c0;
    const uint64_t p1 = (uint64_t)M1 * c2;
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, kv.k0[round], 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, kv.k1[round], 0x96);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
  u32x4 r;
  r.v[0] = c0;
  r.v[1] = c1;
  r.v[2] = c2;
  r.v[3] = c3;
  return r;
}

// Stepwise form, for interleaving a generator call with other work: rounds [R0, R1) of a call
// whose state is s (initially the counter).
struct PhiloxRun {
  uint32_t c0, c1, c2, c3;
};

// Rounds R0..R1-1 (R1 <= 3) of a counter whose words 0..2 are uniform across the wave at round
// 0: the uniform products and xors stay on the scalar unit (uniform round keys), as in
// philox4x32_10_u.
template <int R0, int R1>
__device__ __forceinline__ void philox_rounds_u(PhiloxRun& s, uint32_t key0, uint32_t key1) {
  static_assert(R1 <= 3, "from round 3 on two varying words meet");
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int round = R0; round < R1; ++round) {
    const uint64_t p0 = (uint64_t)M0 * s.c0;
    const uint64_t p1 = (uint64_t)M1 * s.c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ s.c1 ^ (key0 + (uint32_t)round * W0);
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ s.c3 ^ (key1 + (uint32_t)round * W1);
    s.c1 = (uint32_t)p1;
    s.c3 = (uint32_t)p0;
    s.c0 = n0;
    s.c2 = n2;
  }
}

template <int R0, int R1>
__device__ __forceinline__ void philox_rounds(PhiloxRun& s, const PhiloxKeysV& kv) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
#pragma unroll
  for (int round = R0; round < R1; ++round) {
    const uint64_t p0 = (uint64_t)M0 * s.c0;
    const uint64_t p1 = (uint64_t)M1 * s.c2;
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), s.c1, kv.k0[round], 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), s.c3, kv.k1[round], 0x96);
    s.c1 = (uint32_t)p1;
    s.c3 = (uint32_t)p0;
    s.c0 = n0;
    s.c2 = n2;
  }
}

}  // namespace nfm
