// HIP kernel and launcher for site percolation on the simulated graphs, for
// gfx950.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "icm_device.h"

namespace icm {

// ----------------------------------------------------------------------------
// Site percolation (the chimera threshold study of the Supplemental Material):
// each sample occupies every site independently with probability p and
// reports the size of its largest cluster of occupied sites.  One workgroup of
// WAVES waves per sample (a grid-stride loop over samples): site i is occupied
// iff word i mod 4 of Philox(sample, i / 4, 0, 4) is below floor(p 2^32);
// union-find over the bonds between occupied sites (hooking to the smaller
// root), the component sizes by LDS atomics at the roots, then a maximum.
// LDS: parent and size arrays of N ints and one int per wave.
// ----------------------------------------------------------------------------
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int y = __shfl_xor(v, o, 64);
    v = y > v ? y : v;
  }
  return v;
}

template <int WAVES>
__device__ __forceinline__ void perc_sync() {
  if (WAVES == 1) wave_sync();
  else __syncthreads();
}

// A site's DEG neighbours are fetched together (from the cached table) before
// its unions, so their latencies overlap.
template <int WAVES, int DEG>
__global__ void __launch_bounds__(64 * WAVES) percolation_kernel(const uint16_t* __restrict__ nbr, int N,
                                                                 unsigned long long thr, uint32_t sample0,
                                                                 uint32_t n_samples, uint32_t seed, uint32_t key,
                                                                 int32_t* __restrict__ smax) {
  constexpr int SC = WAVES == 1 ? __HIP_MEMORY_SCOPE_WAVEFRONT : __HIP_MEMORY_SCOPE_WORKGROUP;
  constexpr int NT = 64 * WAVES;
  extern __shared__ __align__(16) unsigned char lds[];
  int* parent = (int*)lds;  // -1: empty site
  int* size = parent + N;
  int* wmax = size + N;     // [WAVES], WAVES <= 16
  const int tid = threadIdx.x;
  for (uint32_t s = blockIdx.x; s < n_samples; s += gridDim.x) {
    const uint32_t sample = sample0 + s;
    for (int q = tid; 4 * q < N; q += NT) {
      const Words4 u = philox4x32_10(sample, (uint32_t)q, 0u, kStreamPerc, seed, key);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = 4 * q + b;
        if (i < N) {
          parent[i] = (unsigned long long)u.w[b] < thr ? i : -1;
          size[i] = 0;
        }
      }
    }
    perc_sync<WAVES>();
    // each bond once, from its smaller end; an empty site never changes, an
    // occupied one always holds a site index
    for (int i = tid; i < N; i += NT) {
      if (uf_load<SC>(parent, i) < 0) continue;
      int jn[DEG];
#pragma unroll
      for (int d = 0; d < DEG; ++d) jn[d] = nbr[i * DEG + d];
#pragma unroll
      for (int d = 0; d < DEG; ++d) {
        const int j = jn[d];
        if (j > i && uf_load<SC>(parent, j) >= 0) uf_union<SC>(parent, i, j);
      }
    }
    perc_sync<WAVES>();
    for (int i = tid; i < N; i += NT)
      if (uf_load<SC>(parent, i) >= 0) atomicAdd(&size[uf_find<SC>(parent, i)], 1);
    perc_sync<WAVES>();
    int m = 0;
    for (int i = tid; i < N; i += NT) m = size[i] > m ? size[i] : m;
    m = wave_max(m);
    if (WAVES == 1) {
      if (tid == 0) smax[s] = m;
    } else {
      if ((tid & 63) == 0) wmax[tid >> 6] = m;
      __syncthreads();
      if (tid == 0) {
        int best = wmax[0];
        for (int w = 1; w < WAVES; ++w) best = wmax[w] > best ? wmax[w] : best;
        smax[s] = best;
      }
    }
    perc_sync<WAVES>();
  }
}

}  // namespace icm

extern "C" {

int icmk_set_percolation_lds_limit(size_t bytes) {
  hipError_t e = hipSuccess;
  const void* perc[10] = {(const void*)icm::percolation_kernel<1, 4>,  (const void*)icm::percolation_kernel<1, 6>,
                          (const void*)icm::percolation_kernel<2, 4>,  (const void*)icm::percolation_kernel<2, 6>,
                          (const void*)icm::percolation_kernel<4, 4>,  (const void*)icm::percolation_kernel<4, 6>,
                          (const void*)icm::percolation_kernel<8, 4>,  (const void*)icm::percolation_kernel<8, 6>,
                          (const void*)icm::percolation_kernel<16, 4>, (const void*)icm::percolation_kernel<16, 6>};
  for (int x = 0; x < 10; ++x) {
    hipError_t r = hipFuncSetAttribute(perc[x], hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (r != hipSuccess) e = r;
  }
  return (int)e;
}

size_t icmk_percolation_lds(int N) { return 8u * (size_t)N + 64u; }

// n_cus compute units with lds_cu bytes of LDS each: the grid is what fits
// resident at once (samples are dealt over it by the grid-stride loop).  The
// waves per workgroup (1, 2, 4, 8 or 16) are the fewest with which the
// workgroups that fit a compute unit's LDS hold 32 waves (8 per SIMD, to hide
// LDS latency); large N fits one workgroup and takes sixteen.
int icmk_launch_percolation(const uint16_t* nbr, int N, int deg, unsigned long long thr, uint32_t sample0,
                            uint32_t n_samples, uint32_t seed, uint32_t key, int32_t* smax, int n_cus,
                            size_t lds_cu, hipStream_t stream) {
  if (n_samples == 0) return 0;
  if (N < 1 || N > icm::kMaxPercSites || n_cus < 1 || (deg != 4 && deg != 6)) return (int)hipErrorInvalidValue;
  const size_t lds = icmk_percolation_lds(N);
  if (lds > lds_cu) return (int)hipErrorInvalidValue;
  const int fit = (int)(lds_cu / lds);
  int waves = 1;
  while (waves < 16 && waves * fit < 32) waves *= 2;
  const int per_cu = std::max(1, std::min(32 / waves, (int)(lds_cu / lds)));
  const uint32_t nb = (uint32_t)(n_cus * per_cu);
  const uint32_t g = n_samples < nb ? n_samples : nb;
#define ICM_PERC(W, D)                                                                                   \
  hipLaunchKernelGGL((icm::percolation_kernel<W, D>), dim3(g), dim3(64 * W), lds, stream, nbr, N, thr,   \
                     sample0, n_samples, seed, key, smax)
  switch (waves) {
    case 1: if (deg == 4) ICM_PERC(1, 4); else ICM_PERC(1, 6); break;
    case 2: if (deg == 4) ICM_PERC(2, 4); else ICM_PERC(2, 6); break;
    case 4: if (deg == 4) ICM_PERC(4, 4); else ICM_PERC(4, 6); break;
    case 8: if (deg == 4) ICM_PERC(8, 4); else ICM_PERC(8, 6); break;
    default: if (deg == 4) ICM_PERC(16, 4); else ICM_PERC(16, 6); break;
  }
#undef ICM_PERC
  return (int)hipGetLastError();
}

}  // extern "C"
