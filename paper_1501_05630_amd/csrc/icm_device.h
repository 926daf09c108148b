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
