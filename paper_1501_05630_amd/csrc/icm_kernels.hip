// HIP kernels for parallel tempering + isoenergetic cluster moves on gfx950.
//
// The fused sweep-block kernel runs, for every work unit (one disorder
// instance with all its temperatures and replicas), n simulation steps of the
// paper's isoenergetic cluster algorithm (steps 1, 2a, 2b, 3) with the unit
// resident in LDS (spins bit-packed, 32 walkers per word):
//   step 1   checkerboard Metropolis: each thread updates the four walkers of
//            one Philox quad at one site with one Philox block;
//   step 2a  spin reversal recorded as a per-walker gauge bit;
//   step 2b  one wavefront per cluster move: q-mask by bit compare, n_minus by
//            popcount + DPP wave reduction, seed by ballot counts, the seed's
//            cluster grown breadth-first with the frontier compacted by ballot +
//            mbcnt, flipped in both replicas, the energy updated exactly from the
//            bonds that leave the cluster; for the label readout the full
//            component labelling by union-find (LDS atomicMin hooking, pointer
//            jumping);
//   step 3   parallel tempering: one lane per chain scans the neighbouring
//            temperature pairs in ascending order.
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

enum : uint32_t { kStreamMetro = 0, kStreamInit = 1, kStreamIcm = 2, kStreamPt = 3 };

// ----------------------------------------------------------------------------
// wavefront helpers (wave64)
// ----------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// Sum over the 64 lanes of a wave (all lanes active), returned to every lane.
// DPP: butterfly inside each quad, then half-row and row mirrors give every
// lane its 16-lane row sum; the four row sums are read back with readlane.
__device__ __forceinline__ int dpp_row_sum(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);  // row_mirror
  return v;
}

__device__ __forceinline__ int wave_sum(int v) {
  v = dpp_row_sum(v);
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
         __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Exact for values on a common fixed grid (every partial sum is representable).
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

__device__ __forceinline__ int wave_exclusive_scan(int v) {
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane_id() >= o) x += y;
  }
  return x - v;
}

// Orders this wave's LDS accesses around the call (lanes of one wave exchange
// data through LDS between ICM phases).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ double uniform_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ----------------------------------------------------------------------------
// Metropolis acceptance for float couplings.  dE is exact (2^-32 grid); the
// decision is u * 2^-32 < exp(-beta dE) in double.  A float estimate settles
// all but a ~1e-4 band around the boundary: p32 = 2^(-dE * beta log2 e) has a
// relative error below 2^-18 for every exponent that matters, so with a 2^-14
// margin the fast accept/reject can only be taken when the double comparison
// gives the same answer; the band falls back to the double evaluation.
// ----------------------------------------------------------------------------
// Out of line: taken for ~1e-4 of the attempts, and inlining it would keep the
// double exp's constants in registers across the whole sweep loop.
__device__ __noinline__ bool accept_exact(uint32_t u, double dE, double beta) {
  return (double)u * 0x1p-32 < exp(-(beta * dE));
}

__device__ __forceinline__ bool accept_float(uint32_t u, double dE, double beta, float bl2e) {
  if (dE <= 0.0) return true;
  const float p = __builtin_amdgcn_exp2f(-((float)dE * bl2e));
  const float uf = (float)(u >> 8) * 0x1p-24f;  // exact; true u/2^32 lies in [uf, uf + 2^-24)
  if (uf > p * (1.0f + 0x1p-14f)) return false;
  if (uf + 0x1p-24f <= p * (1.0f - 0x1p-14f)) return true;
  return accept_exact(u, dE, beta);
}

// ----------------------------------------------------------------------------
// union-find on an LDS parent array (parent[x] <= x; roots satisfy parent[x] == x)
// ----------------------------------------------------------------------------
__device__ __forceinline__ int uf_load(int* parent, int x) {
  return __hip_atomic_load(&parent[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

__device__ __forceinline__ int uf_find(int* parent, int x) {
  int p = uf_load(parent, x);
  while (p != x) {
    x = p;
    p = uf_load(parent, x);
  }
  return x;
}

// Hooks the larger root under the smaller one with atomicMin; when the target
// stopped being a root meanwhile, continues with the value it pointed to, so
// no link is ever lost.  Component roots end up at their minimum site index.
__device__ __forceinline__ void uf_union(int* parent, int a, int b) {
  while (true) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a > b) { int t = a; a = b; b = t; }
    const int old = __hip_atomic_fetch_min(&parent[b], a, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WAVEFRONT);
    if (old == b) return;
    b = old;
  }
}

template <int JK>
struct EnergyT;
template <>
struct EnergyT<0> { using T = int; };
template <>
struct EnergyT<1> { using T = double; };

__device__ __forceinline__ uint32_t bit_of(uint32_t word, int pos) { return (word >> pos) & 1u; }

// Spin (+1/-1) of byte b of an int8 quad word.
__device__ __forceinline__ int spin_of(uint32_t word, int b) {
  return (int)(int8_t)(uint8_t)(word >> (8 * b));
}

// ----------------------------------------------------------------------------
// The fused sweep-block kernel.  JK: 0 = int8 couplings, 1 = float couplings.
// DEG: neighbour slots (4 for square2d, 6 otherwise).  One workgroup runs one
// unit; its spins live bit-packed in LDS for the whole block of sweeps.
// ----------------------------------------------------------------------------
template <int JK, int DEG, int TL>
__global__ void __launch_bounds__(1024) sweep_block_kernel(const UnitDesc* __restrict__ units,
                                                          uint32_t n_sweeps, int icm_slots) {
  using E_t = typename EnergyT<JK>::T;
  extern __shared__ __align__(16) unsigned char lds[];
  const UnitDesc U = units[blockIdx.x];
  const int N = U.N, Nc = U.Nc, W = U.W, Wq = U.Wq, K = U.K, R = U.R, Kc = U.Kc, HM = U.HM;
  const int Wp = 4 * Wq, G = bit_words(Wq);
  const LdsLayout lay = lds_layout(N, DEG, Wq, K, R, HM, JK, icm_slots, TL,
                                   (U.flags & kFlagRecord) ? 1 : 0, Kc);

  uint32_t* sp = (uint32_t*)(lds + lay.sp);
  // TL: tables in LDS; otherwise read-only global memory (cached in L1/L2)
  const uint16_t* nbr = TL ? (const uint16_t*)(lds + lay.nbr) : U.nbr;
  const uint16_t* clist = TL ? (const uint16_t*)(lds + lay.clist) : U.clist;
  const int8_t* cj = TL ? (const int8_t*)(lds + lay.coup) : (const int8_t*)U.coup;
  const float* cf = TL ? (const float*)(lds + lay.coup) : (const float*)U.coup;
  int* tau = (int*)(lds + lay.tau);
  int* at = (int*)(lds + lay.at);
  int* gauge = (int*)(lds + lay.gauge);
  E_t* energy = (E_t*)(lds + lay.energy);
  uint32_t* thr = (uint32_t*)(lds + lay.thr);
  double* beta = (double*)(lds + lay.beta);
  float* bl2e = (float*)(lds + lay.bl2e);
  uint32_t* ptu = (uint32_t*)(lds + lay.ptu);
  uint32_t* icmu = (uint32_t*)(lds + lay.icmu);
  unsigned long long* stats = (unsigned long long*)(lds + lay.stats);

  const int tid = threadIdx.x, nthr = blockDim.x;
  // ---- load the unit into LDS; int8 quad words -> bit-packed words ----
  for (int x = tid; x < G * N; x += nthr) {
    const int g = x / N, i = x - g * N;
    uint32_t bits = 0;
    for (int qq = 0; qq < 8; ++qq) {
      const int q = 8 * g + qq;
      if (q >= Wq) break;
      const uint32_t w = U.spins[(size_t)q * N + i];
      // byte 0x01 = up, 0xFF = down: bit 7 of each byte is the down flag
      const uint32_t d = (w >> 7) & 0x01010101u;
      bits |= ((d & 1u) | ((d >> 7) & 2u) | ((d >> 14) & 4u) | ((d >> 21) & 8u)) << (4 * qq);
    }
    sp[x] = bits;
  }
  if (TL) {
    uint16_t* nbr_w = (uint16_t*)(lds + lay.nbr);
    uint16_t* clist_w = (uint16_t*)(lds + lay.clist);
    for (int x = tid; x < N * DEG; x += nthr) nbr_w[x] = U.nbr[x];
    for (int x = tid; x < N; x += nthr) clist_w[x] = U.clist[x];
    if (JK) {
      float* cf_w = (float*)(lds + lay.coup);
      for (int x = tid; x < N * DEG; x += nthr) cf_w[x] = ((const float*)U.coup)[x];
    } else {
      int8_t* cj_w = (int8_t*)(lds + lay.coup);
      for (int x = tid; x < N * DEG; x += nthr) cj_w[x] = ((const int8_t*)U.coup)[x];
    }
  }
  if (!JK)
    for (int x = tid; x < K * HM; x += nthr) thr[x] = U.thr[x];
  for (int x = tid; x < Wp; x += nthr) {
    tau[x] = U.tau[x];
    gauge[x] = U.gauge[x];
    if (JK) energy[x] = (E_t)((double)U.energy[x] * 0x1p-32);
    else energy[x] = (E_t)U.energy[x];
  }
  for (int x = tid; x < K * R; x += nthr) at[x] = U.at[x];
  for (int x = tid; x < K; x += nthr) { beta[x] = U.beta[x]; bl2e[x] = U.bl2e[x]; }
  for (int x = tid; x < kNumStats; x += nthr) stats[x] = 0;
  __syncthreads();

  const uint32_t t0 = *U.sweep;
  const uint32_t flags = U.flags, seed = U.seed, key = U.key;
  const int lane = lane_id(), wave = wave_id(), nwaves = nthr >> 6;
  unsigned long long metro_acc = 0;  // wave-uniform counter, flushed at the end

  for (uint32_t s = 0; s < n_sweeps; ++s) {
    const uint32_t t = t0 + s;
    // The random numbers of PT and ICM do not depend on the state: draw them
    // now, in parallel; the barriers of the sweep order them before their use.
    if (flags & kFlagPt)
      for (int x = tid; x < (K - 1) * R; x += nthr) {
        const int k = x / R, r = x - k * R;
        ptu[x] = philox4x32_10((uint32_t)k, t, (uint32_t)r, kStreamPt, seed, key).w[0];
      }
    for (int x = tid; x < Kc * (R >> 1); x += nthr)
      icmu[x] = philox4x32_10((uint32_t)x, t, 0u, kStreamIcm, seed, key).w[0];
    if (flags & kFlagSkipMetro) __syncthreads();
    // ---------------- step 1: Metropolis sweep, colour 0 then colour 1 ----------
    if (!(flags & kFlagSkipMetro)) {
      for (int c = 0; c < 2; ++c) {
        const int nchunk = (Nc + 63) >> 6;
        const int ntasks = Wq * nchunk;
        const int tb = (int)(((long long)ntasks * wave) / nwaves);
        const int te = (int)(((long long)ntasks * (wave + 1)) / nwaves);
        int cur_q = -1;
        E_t acc[4] = {0, 0, 0, 0};
        int tq[4] = {K, K, K, K};
        int rowb[4] = {0, 0, 0, 0};
        double bq[4] = {0, 0, 0, 0};
        float lq[4] = {0, 0, 0, 0};
        int q = tb / nchunk, chunk = tb - q * nchunk;
        for (int task = tb; task < te; ++task, (++chunk == nchunk ? (chunk = 0, ++q) : 0)) {
          if (q != cur_q) {
            if (cur_q >= 0) {
#pragma unroll
              for (int b = 0; b < 4; ++b) {
                const E_t v = wave_sum(acc[b]);
                if (lane == b && v != (E_t)0) atomicAdd(&energy[4 * cur_q + b], v);
                acc[b] = 0;
              }
            }
            cur_q = q;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              tq[b] = uniform(4 * q + b < W ? tau[4 * q + b] : K);
              if (tq[b] < K) {
                if (JK) {
                  bq[b] = uniform_d(beta[tq[b]]);
                  lq[b] = __int_as_float(uniform(__float_as_int(bl2e[tq[b]])));
                } else {
                  rowb[b] = tq[b] * HM;
                }
              }
            }
          }
          const int j = chunk * 64 + lane;
          if (j < Nc) {
            const int g = q >> 3, sh = 4 * (q & 7);
            uint32_t* row = sp + g * N;
            const int i = clist[c * Nc + j];
            const uint32_t own = row[i] >> sh;
            uint32_t nw[DEG];
#pragma unroll
            for (int d = 0; d < DEG; ++d) nw[d] = row[nbr[i * DEG + d]] >> sh;
            const Words4 u = philox4x32_10((uint32_t)i, t, (uint32_t)q, kStreamMetro, seed, key);
            uint32_t flip = 0;
            if (JK) {
              // h = sum_d J_d s_d with s_d = 1 - 2 bit_d: h = sum J - 2 sum_d J_d bit_d (exact)
              double Jd[DEG];
              double Jsum = 0.0;
#pragma unroll
              for (int d = 0; d < DEG; ++d) { Jd[d] = (double)cf[i * DEG + d]; Jsum += Jd[d]; }
#pragma unroll
              for (int b = 0; b < 4; ++b) {
                if (tq[b] >= K) continue;
                double m = 0.0;
#pragma unroll
                for (int d = 0; d < DEG; ++d) m += Jd[d] * (double)bit_of(nw[d], b);
                const double h = Jsum - 2.0 * m;
                const double dE = bit_of(own, b) ? -2.0 * h : 2.0 * h;
                if (accept_float(u.w[b], dE, bq[b], lq[b])) {
                  flip |= 1u << b;
                  acc[b] += (E_t)dE;
                }
              }
            } else {
              int Ji[DEG];
              int Jsum = 0;
#pragma unroll
              for (int d = 0; d < DEG; ++d) { Ji[d] = cj[i * DEG + d]; Jsum += Ji[d]; }
#pragma unroll
              for (int b = 0; b < 4; ++b) {
                if (tq[b] >= K) continue;
                int m = 0;
#pragma unroll
                for (int d = 0; d < DEG; ++d) m += Ji[d] * (int)bit_of(nw[d], b);
                const int h = Jsum - 2 * m;
                const int e = bit_of(own, b) ? -h : h;  // dE = 2e
                if (e <= 0 || u.w[b] < thr[rowb[b] + e]) {
                  flip |= 1u << b;
                  acc[b] += (E_t)(2 * e);
                }
              }
            }
            if (flip) atomicXor(&row[i], flip << sh);
            metro_acc += (unsigned long long)__popcll(__ballot(flip & 1u)) +
                         (unsigned long long)__popcll(__ballot(flip & 2u)) +
                         (unsigned long long)__popcll(__ballot(flip & 4u)) +
                         (unsigned long long)__popcll(__ballot(flip & 8u));
          }
        }
        if (cur_q >= 0) {
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const E_t v = wave_sum(acc[b]);
            if (lane == b && v != (E_t)0) atomicAdd(&energy[4 * cur_q + b], v);
          }
        }
        __syncthreads();
      }
    }

    // ---------------- steps 2a + 2b: isoenergetic cluster moves ----------------
    // icm_slots moves are in flight per workgroup: each ICM wave sets up P moves
    // one after the other with the full wave (mask, 2a, seed), then grows their
    // clusters concurrently in P lane groups of 64/P lanes, then updates energies
    // and flips.  Site i is owned by lane i % 64 as bit i / 64 of its mask word,
    // so ascending site order is (bit, lane) order and ballot s is mask words 2s,
    // 2s+1.
    if (Kc > 0) {
      const int half = R >> 1;
      const int nmoves = Kc * half;
      const int P = icm_slots >= 4 * nwaves ? 4 : (icm_slots >= 2 * nwaves ? 2 : 1);
      const int iwaves = (icm_slots / P) < nwaves ? (icm_slots / P) : nwaves;
      if (wave < iwaves) {
        const int spl = (N + 63) >> 6;  // mask bits per lane
        const int nvis = (N + 31) >> 5;
        const int lpm = 64 / P;         // lanes per move in the BFS
        const int grp = lane / lpm, li = lane - grp * lpm;
        const int nown = N > lane ? (N - lane + 63) >> 6 : 0;  // sites owned by this lane
        const unsigned long long own_mask = nown >= 64 ? ~0ull : ((1ull << nown) - 1ull);
        const unsigned long long gmask = lpm == 64 ? ~0ull : ((1ull << lpm) - 1ull);
        const unsigned long long lt_in_grp = (li == 0) ? 0ull : (((1ull << li) - 1ull) << (grp * lpm));
        for (int mbase = wave * P; mbase < nmoves; mbase += iwaves * P) {
          // ---- set-up, one move at a time with the full wave ----
          int mv_g[4], a_g[4], b_g[4], n_g[4];
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            mv_g[g] = -1; a_g[g] = 0; b_g[g] = 0; n_g[g] = 0;
            if (g >= P || mbase + g >= nmoves) continue;
            const int mv = mbase + g, slot = wave * P + g;
            uint16_t* queue = (uint16_t*)(lds + lay.queue) + slot * N;
            uint32_t* visited = (uint32_t*)(lds + lay.visited) + slot * nvis;
            uint32_t* mask32 = (uint32_t*)(lds + lay.mask) + slot * nvis;
            int* parent = (int*)(lds + lay.parent) + slot * N;
            const int k = mv / half, p = mv - k * half;
            const int a = at[k * R + 2 * p], b = at[k * R + 2 * p + 1];
            const uint32_t* rowa = sp + (a >> 5) * N;
            const uint32_t* rowb = sp + (b >> 5) * N;
            const int pa = a & 31, pb = b & 31;
            const uint32_t gx = (uint32_t)(gauge[a] ^ gauge[b]);
            // site overlap q_i = -1  <=>  the two replicas differ at i
            unsigned long long m = 0;
            for (int s2 = 0; s2 < nown; ++s2) {
              const int i = s2 * 64 + lane;
              const uint32_t diff = bit_of(rowa[i], pa) ^ bit_of(rowb[i], pb) ^ gx;
              m |= (unsigned long long)diff << s2;
            }
            int n = wave_sum((int)__popcll(m));
            const bool twoa = (flags & kFlag2a) && 2 * n > N;
            if (twoa) {  // step 2a: reverse the second replica
              m = ~m & own_mask;
              n = N - n;
              if (lane == 0) gauge[b] ^= 1;
            }
            int seedsite = -1;
            if (n > 0) {
              // step 2b: the idx-th q = -1 site in ascending order seeds the cluster;
              // visited starts as the complement of the mask
              int rem = (int)(((unsigned long long)icmu[mv] * (unsigned long long)n) >> 32);
              for (int s2 = 0; s2 < spl; ++s2) {
                unsigned long long bal = __ballot((m >> s2) & 1ull);
                if (lane == 0) {
                  mask32[2 * s2] = (uint32_t)bal;
                  visited[2 * s2] = ~(uint32_t)bal;
                  if (2 * s2 + 1 < nvis) {
                    mask32[2 * s2 + 1] = (uint32_t)(bal >> 32);
                    visited[2 * s2 + 1] = ~(uint32_t)(bal >> 32);
                  }
                }
                const int c2 = __popcll(bal);
                if (rem >= 0 && rem < c2) {
                  for (; rem > 0; --rem) bal &= bal - 1ull;
                  seedsite = s2 * 64 + (int)__builtin_ctzll(bal);
                  rem = -1;
                } else if (rem >= 0) {
                  rem -= c2;
                }
              }
              seedsite = uniform(seedsite);
              wave_sync();
              if (lane == 0) {
                visited[seedsite >> 5] |= 1u << (seedsite & 31);
                queue[0] = (uint16_t)seedsite;
              }
              if ((flags & kFlagRecord) && s + 1 == n_sweeps) {
                // full labelling for the readout: union-find over the q = -1
                // subgraph, roots hooked towards the smaller index, path compression
                for (int s2 = 0; s2 < nown; ++s2)
                  if ((m >> s2) & 1ull) parent[s2 * 64 + lane] = s2 * 64 + lane;
                wave_sync();
                for (unsigned long long mm = m; mm; mm &= mm - 1ull) {
                  const int i = (int)__builtin_ctzll(mm) * 64 + lane;
#pragma unroll
                  for (int d = 0; d < DEG; ++d) {
                    const int jn = nbr[i * DEG + d];
                    if (jn > i && ((mask32[jn >> 5] >> (jn & 31)) & 1u)) uf_union(parent, i, jn);
                  }
                }
                wave_sync();
                for (unsigned long long mm = m; mm; mm &= mm - 1ull) {
                  const int i = (int)__builtin_ctzll(mm) * 64 + lane;
                  const int r0 = uf_find(parent, i);
                  __hip_atomic_store(&parent[i], r0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                }
              }
            }
            if ((flags & kFlagRecord) && s + 1 == n_sweeps) {
              wave_sync();
              int* lab = U.labels + (size_t)mv * N;
              for (int s2 = 0; s2 < nown; ++s2) {
                const int i = s2 * 64 + lane;
                lab[i] = (n > 0 && ((m >> s2) & 1ull)) ? uf_load(parent, i) : -1;
              }
              if (lane == 0) {
                U.seeds[mv] = seedsite;
                U.seeds[nmoves + mv] = n;
              }
            }
            if (lane == 0) {
              atomicAdd(&stats[kStatIcmMoves], 1ull);
              if (twoa) atomicAdd(&stats[kStat2a], 1ull);
              if (n > 0) atomicAdd(&stats[kStatIcmNontrivial], 1ull);
            }
            mv_g[g] = mv; a_g[g] = a; b_g[g] = b; n_g[g] = n;
          }
          wave_sync();
          // ---- the P clusters grow concurrently, one lane group each ----
          const int my_mv = grp == 0 ? mv_g[0] : grp == 1 ? mv_g[1] : grp == 2 ? mv_g[2] : mv_g[3];
          const int my_n = grp == 0 ? n_g[0] : grp == 1 ? n_g[1] : grp == 2 ? n_g[2] : n_g[3];
          const int my_a = grp == 0 ? a_g[0] : grp == 1 ? a_g[1] : grp == 2 ? a_g[2] : a_g[3];
          const int my_b = grp == 0 ? b_g[0] : grp == 1 ? b_g[1] : grp == 2 ? b_g[2] : b_g[3];
          const int slot = wave * P + grp;
          uint16_t* queue = (uint16_t*)(lds + lay.queue) + slot * N;
          uint32_t* visited = (uint32_t*)(lds + lay.visited) + slot * nvis;
          const uint32_t* mask32 = (const uint32_t*)(lds + lay.mask) + slot * nvis;
          int head = 0, tail = (my_mv >= 0 && my_n > 0) ? 1 : 0;
          while (__ballot(head < tail)) {
            const int cnt = (tail - head) < lpm ? (tail - head) : lpm;
            const bool act = li < cnt;
            int jn[DEG];
            bool claim[DEG];
            if (act) {
              const int i = queue[head + li];
#pragma unroll
              for (int d = 0; d < DEG; ++d) jn[d] = nbr[i * DEG + d];
#pragma unroll
              for (int d = 0; d < DEG; ++d) {
                const uint32_t bitm = 1u << (jn[d] & 31);
                claim[d] = !(atomicOr(&visited[jn[d] >> 5], bitm) & bitm);
              }
            } else {
#pragma unroll
              for (int d = 0; d < DEG; ++d) { jn[d] = 0; claim[d] = false; }
            }
            head += cnt > 0 ? cnt : 0;
#pragma unroll
            for (int d = 0; d < DEG; ++d) {
              const unsigned long long bal = __ballot(claim[d]);
              const unsigned long long gb = (bal >> (grp * lpm)) & gmask;
              const int pos = tail + __popcll(bal & lt_in_grp);
              if (claim[d]) queue[pos] = (uint16_t)jn[d];
              tail += __popcll(gb);
            }
            wave_sync();
          }
          // ---- bonds leaving the cluster change sign in replica a (every q = -1
          // neighbour of the cluster is in it, so they are the bonds to q = +1
          // sites); then the cluster flips in both replicas ----
          E_t dEa = 0;
          if (my_mv >= 0) {
            uint32_t* rowa = sp + (my_a >> 5) * N;
            uint32_t* rowb = sp + (my_b >> 5) * N;
            const int pa = my_a & 31, pb = my_b & 31;
            for (int x = li; x < tail; x += lpm) {
              const int i = queue[x];
              const uint32_t bi = bit_of(rowa[i], pa);
#pragma unroll
              for (int d = 0; d < DEG; ++d) {
                const int j2 = nbr[i * DEG + d];
                if (!((mask32[j2 >> 5] >> (j2 & 31)) & 1u)) {
                  const int sgn = (bi ^ bit_of(rowa[j2], pa)) ? -1 : 1;  // s_a,i s_a,j
                  if (JK) dEa += (E_t)((double)cf[i * DEG + d] * (double)sgn);
                  else dEa += (E_t)(cj[i * DEG + d] * sgn);
                }
              }
              if (rowa == rowb) {
                atomicXor(&rowa[i], (1u << pa) | (1u << pb));
              } else {
                atomicXor(&rowa[i], 1u << pa);
                atomicXor(&rowb[i], 1u << pb);
              }
            }
          }
          // per-group sums: DPP row sums are 16-lane sums, groups are 1, 2 or 4 rows
          E_t rows[4];
          {
            E_t v = dEa;
            if (JK) {
              double dv = (double)v;
              dv += dpp_d<0xB1>(dv); dv += dpp_d<0x4E>(dv); dv += dpp_d<0x141>(dv); dv += dpp_d<0x140>(dv);
#pragma unroll
              for (int r2 = 0; r2 < 4; ++r2) rows[r2] = (E_t)readlane_d(dv, 16 * r2);
            } else {
              int iv = (int)v;
              iv = dpp_row_sum(iv);
#pragma unroll
              for (int r2 = 0; r2 < 4; ++r2) rows[r2] = (E_t)__builtin_amdgcn_readlane(iv, 16 * r2);
            }
          }
          if (lane == 0) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
              if (g >= P || mv_g[g] < 0 || n_g[g] == 0) continue;
              E_t sum = 0;
              for (int r2 = g * (4 / P); r2 < (g + 1) * (4 / P); ++r2) sum += rows[r2];
              energy[a_g[g]] += (E_t)2 * sum;
              energy[b_g[g]] -= (E_t)2 * sum;
            }
          }
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            if (g >= P) continue;
            const int tg = __builtin_amdgcn_readlane(tail, g * lpm);
            if (lane == 0 && mv_g[g] >= 0 && n_g[g] > 0)
              atomicAdd(&stats[kStatIcmSites], (unsigned long long)tg);
          }
          wave_sync();
        }
      }
    }
    __syncthreads();

    // ---------------- step 3: parallel tempering ---------------------------------
    if (flags & kFlagPt) {
      if (wave == 0) {
        const int r = lane;
        int acc_pt = 0;
        for (int k = 0; r < R && k + 1 < K; ++k) {
          const int x = at[k * R + r], y = at[(k + 1) * R + r];
          bool accept;
          const uint32_t u = ptu[k * R + r];
          if (JK) {
            const double D = (double)energy[y] - (double)energy[x];
            accept = D <= 0.0 || (double)u * 0x1p-32 < exp(-((beta[k] - beta[k + 1]) * D));
          } else {
            const int D = (int)energy[y] - (int)energy[x];
            accept = D <= 0 || (D <= U.ptlen && u < U.ptthr[k * U.ptlen + (D - 1)]);
          }
          if (accept) {
            at[k * R + r] = y;
            at[(k + 1) * R + r] = x;
            tau[x] = k + 1;
            tau[y] = k;
            ++acc_pt;
          }
        }
        const int tot = wave_sum(acc_pt);
        if (lane == 0) {
          stats[kStatPtAttempts] += (unsigned long long)(K - 1) * R;
          stats[kStatPtAccepts] += (unsigned long long)tot;
        }
      }
      __syncthreads();
    }
  }

  // ---- store the unit back (bit-packed -> int8 quad words) ----
  if (lane == 0 && metro_acc) atomicAdd(&stats[kStatMetroAcc], metro_acc);
  __syncthreads();
  for (int x = tid; x < Wq * N; x += nthr) {
    const int q = x / N, i = x - q * N;
    const uint32_t nib = (sp[(q >> 3) * N + i] >> (4 * (q & 7))) & 0xFu;
    uint32_t w = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) w |= (((nib >> b) & 1u) ? 0xFFu : 0x01u) << (8 * b);
    U.spins[x] = w;
  }
  for (int x = tid; x < Wp; x += nthr) {
    U.tau[x] = tau[x];
    U.gauge[x] = (uint8_t)gauge[x];
    if (JK) U.energy[x] = (int64_t)((double)energy[x] * 0x1p32);
    else U.energy[x] = (int64_t)energy[x];
  }
  for (int x = tid; x < K * R; x += nthr) U.at[x] = at[x];
  if (tid == 0) {
    stats[kStatSweeps] = n_sweeps;
    *U.sweep = t0 + n_sweeps;
  }
  __syncthreads();
  for (int x = tid; x < kNumStats; x += nthr) U.stats[x] += stats[x];
}

// ----------------------------------------------------------------------------
// Hot start: spin = -1 iff bit 31 of the walker's INIT word is set.
// grid: (ceil(Wq*N/256), 1), one thread per quad-word.
// ----------------------------------------------------------------------------
__global__ void init_spins_kernel(uint32_t* spins, int N, int Wq, int W, uint32_t seed, uint32_t key) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= Wq * N) return;
  const int q = x / N, i = x - q * N;
  const Words4 u = philox4x32_10((uint32_t)i, 0u, (uint32_t)q, kStreamInit, seed, key);
  uint32_t word = 0;
  for (int b = 0; b < 4; ++b) {
    const uint32_t sb = (4 * q + b < W && (u.w[b] >> 31)) ? 0xFFu : 0x01u;
    word |= sb << (8 * b);
  }
  spins[x] = word;
}

// Scatter of caller states [W][N] (walker-major, walker w = k*R + r) into the
// quad-word layout.
__global__ void scatter_spins_kernel(uint32_t* spins, const int8_t* src, int N, int Wq, int W) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= Wq * N) return;
  const int q = x / N, i = x - q * N;
  uint32_t word = 0;
  for (int b = 0; b < 4; ++b) {
    const int w = 4 * q + b;
    const uint32_t sb = (w < W && src[(size_t)w * N + i] < 0) ? 0xFFu : 0x01u;
    word |= sb << (8 * b);
  }
  spins[x] = word;
}

// Energy of every walker from scratch: each bond is seen from both ends, so the
// slot sum is halved (exact: integer, or float couplings on the 2^-32 grid summed
// as int64 after scaling).  grid: (Wp), block 256.
template <int JK>
__global__ void energy_kernel(const uint32_t* spins, const uint16_t* nbr, const void* coup, int N,
                              int deg, int64_t* energy) {
  const int w = blockIdx.x, q = w >> 2, b = w & 3;
  __shared__ long long part[256];
  long long acc = 0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const int si = spin_of(spins[(size_t)q * N + i], b);
    for (int d = 0; d < deg; ++d) {
      const int j = nbr[i * deg + d];
      const int sj = spin_of(spins[(size_t)q * N + j], b);
      long long Jraw;
      if (JK) Jraw = (long long)((double)((const float*)coup)[i * deg + d] * 0x1p32);
      else Jraw = ((const int8_t*)coup)[i * deg + d];
      acc -= Jraw * si * sj;
    }
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) energy[w] = part[0] / 2;
}

}  // namespace icm

// ----------------------------------------------------------------------------
// launch wrappers used by the host runtime
// ----------------------------------------------------------------------------
extern "C" {

int icmk_launch_sweep(const icm::UnitDesc* d_units, int n_units, int jkind, int deg, int tables,
                      uint32_t n_sweeps, int threads, int icm_slots, size_t lds_bytes,
                      hipStream_t stream) {
  if (n_units <= 0) return 0;
  dim3 grid(n_units), block(threads);
#define ICM_LAUNCH(JK, DEG, TL)                                                            \
  hipLaunchKernelGGL((icm::sweep_block_kernel<JK, DEG, TL>), grid, block, lds_bytes, stream, \
                     d_units, n_sweeps, icm_slots)
  const int sel = (jkind ? 4 : 0) + (deg == 6 ? 2 : 0) + (tables ? 1 : 0);
  switch (sel) {
    case 0: ICM_LAUNCH(0, 4, 0); break;
    case 1: ICM_LAUNCH(0, 4, 1); break;
    case 2: ICM_LAUNCH(0, 6, 0); break;
    case 3: ICM_LAUNCH(0, 6, 1); break;
    case 4: ICM_LAUNCH(1, 4, 0); break;
    case 5: ICM_LAUNCH(1, 4, 1); break;
    case 6: ICM_LAUNCH(1, 6, 0); break;
    case 7: ICM_LAUNCH(1, 6, 1); break;
    default: return (int)hipErrorInvalidValue;
  }
#undef ICM_LAUNCH
  if (deg != 4 && deg != 6) return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

int icmk_set_lds_limit(size_t bytes) {
  hipError_t e = hipSuccess;
  const void* fns[8] = {
      (const void*)icm::sweep_block_kernel<0, 4, 0>, (const void*)icm::sweep_block_kernel<0, 4, 1>,
      (const void*)icm::sweep_block_kernel<0, 6, 0>, (const void*)icm::sweep_block_kernel<0, 6, 1>,
      (const void*)icm::sweep_block_kernel<1, 4, 0>, (const void*)icm::sweep_block_kernel<1, 4, 1>,
      (const void*)icm::sweep_block_kernel<1, 6, 0>, (const void*)icm::sweep_block_kernel<1, 6, 1>};
  for (int x = 0; x < 8; ++x) {
    hipError_t r = hipFuncSetAttribute(fns[x], hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (r != hipSuccess) e = r;
  }
  return (int)e;
}

int icmk_launch_init(uint32_t* spins, int N, int Wq, int W, uint32_t seed, uint32_t key,
                     hipStream_t stream) {
  const int n = Wq * N;
  hipLaunchKernelGGL(icm::init_spins_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, spins, N,
                     Wq, W, seed, key);
  return (int)hipGetLastError();
}

int icmk_launch_scatter(uint32_t* spins, const int8_t* src, int N, int Wq, int W,
                        hipStream_t stream) {
  const int n = Wq * N;
  hipLaunchKernelGGL(icm::scatter_spins_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, spins,
                     src, N, Wq, W);
  return (int)hipGetLastError();
}

int icmk_launch_energy(const uint32_t* spins, const uint16_t* nbr, const void* coup, int N, int deg,
                       int Wp, int jkind, int64_t* energy, hipStream_t stream) {
  if (jkind)
    hipLaunchKernelGGL(icm::energy_kernel<1>, dim3(Wp), dim3(256), 0, stream, spins, nbr, coup, N,
                       deg, energy);
  else
    hipLaunchKernelGGL(icm::energy_kernel<0>, dim3(Wp), dim3(256), 0, stream, spins, nbr, coup, N,
                       deg, energy);
  return (int)hipGetLastError();
}

}  // extern "C"
