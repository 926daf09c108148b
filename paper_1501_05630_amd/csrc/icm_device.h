// Device helpers shared by the HIP kernels of the library (the fused sweep
// kernel and the site-percolation kernel): the Philox4x32-10 generator and
// its stream ids, wave64 lane helpers, and union-find on an LDS parent array.
#pragma once
#include <hip/hip_runtime.h>

#include "icm_internal.h"

namespace icm {

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64
// multiplies by the Philox constants with the key added through xor; the key is
// bumped by the golden-ratio Weyl increments between rounds.
// ----------------------------------------------------------------------------
struct Words4 {
  uint32_t w[4];
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                                uint32_t key0, uint32_t key1) {
  // The round keys are recomputed by scalar adds at every call: opaque to the
  // optimiser here, so it does not hold all twenty of them in scalar registers
  // across the sweep loop.
  asm volatile("" : "+s"(key0), "+s"(key1));
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t m0 = (uint64_t)0xD2511F53u * x0;
    const uint64_t m1 = (uint64_t)0xCD9E8D57u * x2;
    // three-way xor in one v_bitop3_b32 (truth table 0x96)
    const uint32_t y0 = __builtin_amdgcn_bitop3_b32((uint32_t)(m1 >> 32), x1, key0, 0x96);
    const uint32_t y2 = __builtin_amdgcn_bitop3_b32((uint32_t)(m0 >> 32), x3, key1, 0x96);
    x1 = (uint32_t)m1;
    x3 = (uint32_t)m0;
    x0 = y0;
    x2 = y2;
    key0 += 0x9E3779B9u;
    key1 += 0xBB67AE85u;
  }
  Words4 r;
  r.w[0] = x0; r.w[1] = x1; r.w[2] = x2; r.w[3] = x3;
  return r;
}

__device__ __forceinline__ uint64_t philox_m0(uint32_t x0) { return (uint64_t)0xD2511F53u * x0; }

// The same function of (x0, x1, x2, x3, key) when x1, x2, x3 and the key are
// the same in every lane of the wave and only x0 differs: the parts of the
// first three rounds that depend on the uniform words alone go to the scalar
// unit (readfirstlane keeps them there), leaving 73 vector operations for two
// blocks with the same x0 instead of 81.  m0 = x0 times the first multiplier
// (64-bit, philox_m0), which a caller drawing several blocks for one x0 forms
// once.
__device__ __forceinline__ Words4 philox4x32_10_lane(uint64_t m0, uint32_t x1, uint32_t x2, uint32_t x3,
                                                     uint32_t key0, uint32_t key1) {
  asm volatile("" : "+s"(key0), "+s"(key1));
  // round 1: y0 = hi(M1 x2) ^ x1 ^ k0 is uniform, y2 = hi(m0) ^ x3 ^ k1 is not
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
  const uint32_t u0 = __builtin_amdgcn_readfirstlane((uint32_t)(p1 >> 32) ^ x1 ^ key0);
  const uint32_t u1 = (uint32_t)p1;
  uint32_t v2 = (uint32_t)(m0 >> 32) ^ __builtin_amdgcn_readfirstlane(x3 ^ key1);
  const uint32_t v3 = (uint32_t)m0;
  key0 += 0x9E3779B9u;
  key1 += 0xBB67AE85u;
  // round 2: M0 u0 is uniform
  const uint64_t p0 = (uint64_t)0xD2511F53u * u0;
  const uint64_t q1 = (uint64_t)0xCD9E8D57u * v2;
  uint32_t x0 = (uint32_t)(q1 >> 32) ^ __builtin_amdgcn_readfirstlane(u1 ^ key0);
  v2 = v3 ^ __builtin_amdgcn_readfirstlane((uint32_t)(p0 >> 32) ^ key1);
  x1 = (uint32_t)q1;
  const uint32_t u3 = (uint32_t)p0;
  key0 += 0x9E3779B9u;
  key1 += 0xBB67AE85u;
  // round 3: the word carried in position 3 is still uniform
  {
    const uint64_t a = (uint64_t)0xD2511F53u * x0;
    const uint64_t b = (uint64_t)0xCD9E8D57u * v2;
    x0 = __builtin_amdgcn_bitop3_b32((uint32_t)(b >> 32), x1, key0, 0x96);
    v2 = (uint32_t)(a >> 32) ^ __builtin_amdgcn_readfirstlane(u3 ^ key1);
    x1 = (uint32_t)b;
    x3 = (uint32_t)a;
    key0 += 0x9E3779B9u;
    key1 += 0xBB67AE85u;
  }
  x2 = v2;
#pragma unroll
  for (int round = 3; round < 10; ++round) {
    const uint64_t a = (uint64_t)0xD2511F53u * x0;
    const uint64_t b = (uint64_t)0xCD9E8D57u * x2;
    const uint32_t y0 = __builtin_amdgcn_bitop3_b32((uint32_t)(b >> 32), x1, key0, 0x96);
    const uint32_t y2 = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), x3, key1, 0x96);
    x1 = (uint32_t)b;
    x3 = (uint32_t)a;
    x0 = y0;
    x2 = y2;
    key0 += 0x9E3779B9u;
    key1 += 0xBB67AE85u;
  }
  Words4 r;
  r.w[0] = x0; r.w[1] = x1; r.w[2] = x2; r.w[3] = x3;
  return r;
}

enum : uint32_t { kStreamMetro = 0, kStreamInit = 1, kStreamIcm = 2, kStreamPt = 3, kStreamPerc = 4 };

// ----------------------------------------------------------------------------
// wavefront helpers (wave64)
// ----------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
// wave index, known to the compiler as uniform (kept in a scalar register)
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Orders this wave's LDS accesses around the call (lanes of one wave exchange
// data through LDS between phases).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ----------------------------------------------------------------------------
// union-find on an LDS parent array (parent[x] <= x; roots satisfy parent[x] == x)
// ----------------------------------------------------------------------------
// SCOPE: the lanes that share the array (one wave, or a whole workgroup).
template <int SCOPE = __HIP_MEMORY_SCOPE_WAVEFRONT>
__device__ __forceinline__ int uf_load(int* parent, int x) {
  return __hip_atomic_load(&parent[x], __ATOMIC_RELAXED, SCOPE);
}

template <int SCOPE = __HIP_MEMORY_SCOPE_WAVEFRONT>
__device__ __forceinline__ int uf_find(int* parent, int x) {
  int p = uf_load<SCOPE>(parent, x);
  while (p != x) {
    x = p;
    p = uf_load<SCOPE>(parent, x);
  }
  return x;
}

// Hooks the larger root under the smaller one with atomicMin; when the target
// stopped being a root meanwhile, continues with the value it pointed to, so
// no link is ever lost.  Component roots end up at their minimum site index.
template <int SCOPE = __HIP_MEMORY_SCOPE_WAVEFRONT>
__device__ __forceinline__ void uf_union(int* parent, int a, int b) {
  while (true) {
    a = uf_find<SCOPE>(parent, a);
    b = uf_find<SCOPE>(parent, b);
    if (a == b) return;
    if (a > b) { int t = a; a = b; b = t; }
    const int old = __hip_atomic_fetch_min(&parent[b], a, __ATOMIC_RELAXED, SCOPE);
    if (old == b) return;
    b = old;
  }
}

}  // namespace icm
