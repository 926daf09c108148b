// HIP kernels for parallel tempering + isoenergetic cluster moves on gfx950.
//
// The fused sweep-block kernel runs, for every work unit (one disorder
// instance with all its temperatures and replicas), n simulation steps of the
// paper's isoenergetic cluster algorithm (steps 1, 2a, 2b, 3) with the unit
// resident in LDS (spins bit-packed, 32 walkers per word):
//   step 1   checkerboard Metropolis: a lane's task is one site and the
//            walkers of one or two Philox quads; the field of each walker from
//            the xor of the site's word with its neighbour words (24-bit
//            integer multiply-adds for float couplings, byte dot products for
//            int8 couplings); float couplings decide by a float estimate, and
//            the rare calls it cannot make are redone exactly in double;
//   step 2a  spin reversal recorded as a per-walker gauge bit;
//   step 2b  on the walker-major view of the spins (in-place 32x32 bit
//            transposes), a lane group per move: q-mask words by xor,
//            n_minus by popcounts, the seed by a scan, the seed's cluster grown
//            as a bitset flood fill (a whole frontier per level), flipped in
//            both replicas by word xor, the energy change from the bonds that
//            leave the cluster; union-find labelling only for the label
//            readout;
//   step 3   parallel tempering: one lane per chain scans the neighbouring
//            temperature pairs in ascending order (long ladders decide every
//            pair the scan can meet up front, in parallel).

#include <hip/hip_runtime.h>

#include <algorithm>

#include "icm_device.h"

namespace icm {


// ----------------------------------------------------------------------------
// wavefront helpers (wave64)
// ----------------------------------------------------------------------------

// Sum over the 64 lanes of a wave (all lanes active), returned to every lane.
// DPP: butterfly inside each quad, then half-row and row mirrors give every
// lane its 16-lane row sum; the four row sums are read back with readlane.
__device__ __forceinline__ int dpp_row_sum(int v) {
  v += __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);   // quad_perm [1,0,3,2]
  v += __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);   // quad_perm [2,3,0,1]
  v += __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);  // row_half_mirror
  v += __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true);  // row_mirror
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
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
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

// Prefix sums over the wave by DPP: shifts by 1, 2, 4, 8 within each 16-lane
// row (zeros shifted in) give the rows' inclusive scans, then each row's last
// lane is broadcast into the rows after it (row_bcast 15 and 31).
__device__ __forceinline__ int wave_exclusive_scan(int v) {
  int x = v;
  x += __builtin_amdgcn_mov_dpp(x, 0x111, 0xF, 0xF, true);  // row_shr:1
  x += __builtin_amdgcn_mov_dpp(x, 0x112, 0xF, 0xF, true);  // row_shr:2
  x += __builtin_amdgcn_mov_dpp(x, 0x114, 0xF, 0xF, true);  // row_shr:4
  x += __builtin_amdgcn_mov_dpp(x, 0x118, 0xF, 0xF, true);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
  return x - v;
}

// NV per-lane values v[0..NV-1] (NV a power of two) summed over the wave at
// once: each butterfly stage halves the values a lane holds (it keeps the sum
// for one half of the indices and hands the other half to its partner), so
// after log2 NV stages lane l holds the sum over its NV-lane group for index
// l mod NV (transpose_stages), which the remaining stages complete over the
// wave (wave_rest).  transpose_sum returns, in every lane, the wave total for
// index lane mod NV.  Exact for integers and for doubles holding integers.
template <int NV, typename T>
__device__ __forceinline__ T transpose_stages(T (&v)[NV]) {
  const int lane = lane_id();
#pragma unroll
  for (int s = 0; (1 << s) < NV; ++s) {
    const int m = 1 << s;
    const bool hi = (lane & m) != 0;
#pragma unroll
    for (int j = 0; j < (NV >> (s + 1)); ++j) {
      const T keep = hi ? v[2 * j + 1] : v[2 * j];
      const T send = hi ? v[2 * j] : v[2 * j + 1];
      v[j] = keep + __shfl_xor(send, m, 64);
    }
  }
  return v[0];
}

template <int NV, typename T>
__device__ __forceinline__ T wave_rest(T r) {
#pragma unroll
  for (int m = NV; m < 64; m <<= 1) r += __shfl_xor(r, m, 64);
  return r;
}

template <int NV, typename T>
__device__ __forceinline__ T transpose_sum(T (&v)[NV]) {
  return wave_rest<NV>(transpose_stages<NV>(v));
}

// The transposed stages for integers by DPP inside 16-lane rows, no LDS
// permute: partners at lane distance 1 and 2 (quad permutes), then 8 (row
// rotate by 8).  Stage s pairs lanes that differ in bit m_s = 1, 2, 8 of the
// lane id; after the stages NV = 2, 4, 8 needs, lane l holds the sum over its
// NV-lane group (the lanes that differ from l in those bits) of index
// dpp_index<NV>(l): bit 0, bit 1 and bit 3 of l as the index's bits 0, 1, 2.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}

template <int NV>
__device__ __forceinline__ int dpp_index(int lane) {
  return (lane & (NV > 2 ? 3 : 1)) | (NV > 4 ? (lane >> 1) & 4 : 0);
}

template <int NV>
__device__ __forceinline__ int dpp_transpose_stages(int (&v)[NV]) {
  static_assert(NV == 2 || NV == 4 || NV == 8, "two, four or eight values per lane");
  const int lane = lane_id();
  {
    const bool hi = (lane & 1) != 0;
#pragma unroll
    for (int j = 0; j < NV / 2; ++j) {
      const int a = v[2 * j] + dpp_i<0xB1>(v[2 * j]);              // quad_perm [1,0,3,2]
      const int b = v[2 * j + 1] + dpp_i<0xB1>(v[2 * j + 1]);
      v[j] = hi ? b : a;
    }
  }
  if constexpr (NV >= 4) {
    const bool hi = (lane & 2) != 0;
#pragma unroll
    for (int j = 0; j < NV / 4; ++j) {
      const int a = v[2 * j] + dpp_i<0x4E>(v[2 * j]);              // quad_perm [2,3,0,1]
      const int b = v[2 * j + 1] + dpp_i<0x4E>(v[2 * j + 1]);
      v[j] = hi ? b : a;
    }
  }
  if constexpr (NV == 8) {
    const bool hi = (lane & 8) != 0;
    const int a = v[0] + dpp_i<0x128>(v[0]);                       // row_ror:8
    const int b = v[1] + dpp_i<0x128>(v[1]);
    v[0] = hi ? b : a;
  }
  return v[0];
}


__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// The lane index as a value the optimiser cannot see through: per-lane
// constants derived from it inside one phase of the sweep (the PT scan's
// addresses) are then formed in that phase instead of being hoisted out of
// the sweep loop, where they would hold registers for the whole kernel and be
// spilled (their reloads sat on the scan's serial chain).
__device__ __forceinline__ int phase_lane() {
  int l = (int)(threadIdx.x & 63u);
  asm volatile("" : "+v"(l));
  return l;
}

__device__ __forceinline__ double uniform_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ----------------------------------------------------------------------------
// Metropolis acceptance for float couplings.  dE is exact (coupling grid); the
// decision is u * 2^-32 < exp(-beta dE) in double.  A float estimate settles
// all but a ~1e-4 band around the boundary: P = 2^(32 - dE * beta log2 e)
// (the 2^32 scale folded into the exponent of one fma) has a relative error
// below 2^-18 wherever 1 <= P <= 2^32, and float(u) is within a relative
// 2^-24 of u; with a 2^-14 margin on both sides the fast accept/reject is only
// taken where the double comparison gives the same answer (for P < 1 only
// u = 0 can be accepted, and that case reaches the double test whenever P
// underflows).  The band falls back to the double evaluation.
// ----------------------------------------------------------------------------
// Out of line: taken for ~1e-4 of the attempts, and inlining it would keep the
// double exp's constants in registers across the whole sweep loop.
__device__ __noinline__ bool accept_exact(uint32_t u, double dE, double beta) {
  return (double)u * 0x1p-32 < exp(-(beta * dE));
}

__device__ __forceinline__ bool accept_float(uint32_t u, double dE, double beta, float bl2e) {
  if (dE <= 0.0) return true;
  const float P = __builtin_amdgcn_exp2f(__builtin_fmaf(-(float)dE, bl2e, 32.0f));
  const float uf = (float)u;
  if (uf > P * (1.0f + 0x1p-14f)) return false;
  if (uf < P * (1.0f - 0x1p-14f)) return true;
  return accept_exact(u, dE, beta);
}

// The same decision for an integer field: dE = e 2^(1 - jexp) (e = s_i h in
// units of the coupling grid); lq2 = float(beta log2 e) 2^(1 - jexp), jq2 =
// 2^(1 - jexp).  float(e) is within a relative 2^-24 of e, which the margin
// covers as before; the exact test sees the same double dE as the oracle.
__device__ __forceinline__ bool accept_int_field(uint32_t u, int e, double beta, float lq2, double jq2) {
  if (e <= 0) return true;
  const float P = __builtin_amdgcn_exp2f(__builtin_fmaf(-(float)e, lq2, 32.0f));
  const float uf = (float)u;
  if (uf > P * (1.0f + 0x1p-14f)) return false;
  if (uf < P * (1.0f - 0x1p-14f)) return true;
  return accept_exact(u, (double)e * jq2, beta);
}


// The same sum for int8 couplings from their bit planes (pl: the jpl plane
// words of this word and slot, two's complement): sum over a bit set M of J
// is sum_k w_k popc(M & plane_k), w_k = 2^k and -2^(jpl-1) for the sign
// plane; a handful of operations whatever the number of bits.
__device__ __forceinline__ int boundary_sum_planes(uint32_t bb, uint32_t anti, const uint32_t* pl, int jpl) {
  const uint32_t mp = bb & ~anti, mm = bb & anti;
  int s = 0;
  for (int k = 0; k < jpl; ++k) {
    const uint32_t p = pl[k];
    const int c = (int)__popc(mp & p) - (int)__popc(mm & p);
    s += c * (k + 1 == jpl ? -(1 << k) : (1 << k));
  }
  return s;
}

template <int JK>
struct EnergyT;
template <>
struct EnergyT<0> { using T = int; };
template <>
struct EnergyT<1> { using T = double; };

// Adds a wave's accepted energy changes to the WPT walkers' energies: acc[b] is
// a lane's sum of e = s_i h_i over its accepted flips of walker b (dE = 2 e in
// field units; float couplings: units of 2^-jexp, and |acc| < 2^31 because a
// lane takes at most 32 sites of a colour).  Integer sums throughout.  narrow
// (float couplings): a lane took at most nchunk sites with nchunk DEG WPT <
// 256, so |acc| < 2^31 / WPT (|e| < DEG 2^23) and the WPT-lane group sums of
// the butterfly stages still fit an int; the groups are then added into the
// double energies one by one (LDS atomics, exact in any order).
template <int JK, int WPT>
__device__ __forceinline__ void flush_energy(int (&acc)[WPT], typename EnergyT<JK>::T* en, int jexp,
                                             bool narrow) {
  const int lane = lane_id();
  if constexpr (JK) {
    if (narrow) {
      // the WPT-lane group sums by DPP, then every lane adds its group's sum
      // (WPT = 8: eight lanes per walker); each addition is exact (integer
      // multiples of 2^(1 - jexp) below 2^53 ulps), so their order is free
      const int g = dpp_transpose_stages<WPT>(acc);
      if (g != 0) atomicAdd(&en[dpp_index<WPT>(lane)], ldexp((double)g, 1 - jexp));
    } else {
      double v[WPT];  // integers below 2^53: exact in any order
#pragma unroll
      for (int b = 0; b < WPT; ++b) v[b] = (double)acc[b];
      const double tot = transpose_sum<WPT>(v);
      if (lane < WPT && tot != 0.0) atomicAdd(&en[lane], ldexp(tot, 1 - jexp));
    }
  } else {
    // four-lane group sums by DPP, then the four groups of each 16-lane row
    // (rotations by 4 and 8 keep a lane's index), and one lane per row and
    // walker adds the row's sum
    int v = dpp_transpose_stages<WPT>(acc);
    if constexpr (WPT == 4) {
      v += dpp_i<0x124>(v);  // row_ror:4
      v += dpp_i<0x128>(v);  // row_ror:8
      if ((lane & 12) == 0 && v != 0) atomicAdd(&en[lane & 3], 2 * v);
    } else {
      if (v != 0) atomicAdd(&en[dpp_index<WPT>(lane)], 2 * v);
    }
  }
}

__device__ __forceinline__ uint32_t bit_of(uint32_t word, int pos) { return (word >> pos) & 1u; }

// acc + a b for signed 24-bit a and b (one v_mad_i32_i24; the compiler would
// turn a multiply by a 0/-1 value into selects)
__device__ __forceinline__ int mad_i24(int a, int b, int acc) {
  int r;
  asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(acc));
  return r;
}

// |a - b| for unsigned a, b (one v_sad_u32)
__device__ __forceinline__ uint32_t absdiff(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_sad_u32 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// flip |= bit and acc += e in the lanes of the lane mask m only (m a subset of
// the active lanes; the others keep both values): exec is narrowed to m around
// one OR and one add, where selects would cost two more operations.
__device__ __forceinline__ void accept_where(uint64_t m, uint32_t bit, uint32_t& flip, int e, int& acc) {
  uint64_t saved;
  asm volatile(
      "s_and_saveexec_b64 %0, %3\n\t"
      "v_or_b32 %1, %4, %1\n\t"
      "v_add_u32 %2, %5, %2\n\t"
      "s_mov_b64 exec, %0"
      : "=&s"(saved), "+v"(flip), "+v"(acc)
      : "s"(m), "s"(bit), "v"(e));
}

// Index of the lowest set bit, all ones for 0 (one v_ffbl_b32).
__device__ __forceinline__ uint32_t lowest_bit(uint32_t x) {
  uint32_t r;
  asm("v_ffbl_b32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// Sum over the set bits b of bb of +-J for the bond in slot d of site
// 32 w + b (J in the coupling table's integer units): -J where replica a is
// anti-aligned across the bond (bit b of anti set).  Four bits per round, their
// coupling loads in flight together; a round's slot without a bit left reads a
// fixed entry, and those reads are taken out at the end.  The lowest-bit index
// of 0 is -1: with the table in LDS (TL) that slot reads entry base - DEG,
// which lies inside LDS even at the start of the table (whatever it holds is
// read, weighed with bit 31 of anti, and taken out the same way); a table in
// global memory clamps the index to 0 instead.  At most 32 bits of 24-bit
// values, plus the same number taken out: the sum stays within an int.
template <int JK, int DEG, int TL>
__device__ __forceinline__ int boundary_sum(uint32_t bb, uint32_t anti, int w, int d, const int32_t* cf,
                                            const int8_t* cj) {
  const int cnt = (int)__popc(bb);
  const int base = 32 * w * DEG + d;
  int s = 0, slots = 0;
  while (bb) {
    // the round's four positions and signs (-1 where anti-aligned) first, then
    // its four loads together, and only then the sums (the scheduling barrier
    // keeps the loads from being spread between the multiply-adds)
    int pos[4], sg[4], v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      pos[u] = TL ? (int)lowest_bit(bb) : max((int)lowest_bit(bb), 0);
      bb &= bb - 1u;
      // the bit-field extract takes the offset mod 32 (-1: bit 31)
      sg[u] = mad_i24((int)__builtin_amdgcn_ubfe(anti, (uint32_t)pos[u], 1u), -2, 1);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int x = base + pos[u] * DEG;
      v[u] = JK ? cf[x] : (int)cj[x];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 4; ++u) s = mad_i24(v[u], sg[u], s);
    slots += 4;
  }
  const int e0 = TL ? base - DEG : base;  // the entry an empty slot reads
  const int v0 = JK ? cf[e0] : (int)cj[e0];
  return s - (slots - cnt) * mad_i24(v0, mad_i24((int)(TL ? anti >> 31 : anti & 1u), -2, 1), 0);
}

// Spin (+1/-1) of byte b of an int8 quad word.
__device__ __forceinline__ int spin_of(uint32_t word, int b) {
  return (int)(int8_t)(uint8_t)(word >> (8 * b));
}


// ----------------------------------------------------------------------------
// The lattice as bit shifts of a site bitset (bit i of word i / 32 is site i),
// used to grow clusters a whole frontier at a time.  Term t contributes
// F[i + shift] to site i wherever its condition holds.  Periodic lattices
// (index x + L y [+ L^2 z]): per axis of stride sg and coordinate c the +1
// step (shift sg where c < L-1), its wrap (shift -(L-1) sg where c = L-1), the
// -1 step (shift -sg where c > 0) and its wrap (shift (L-1) sg where c = 0).
// Chimera (index 8 (row C + col) + u): u < 4 couples to row +-1, u >= 4 to
// col +-1, open boundaries; the in-cell K4,4 bonds are applied per byte.
// ----------------------------------------------------------------------------
__device__ __forceinline__ int lattice_terms(int topo) {
  return topo == 0 ? 8 : (topo == 1 ? 12 : 4);
}

__device__ __forceinline__ int term_shift(int topo, int L, int t) {
  if (topo == 2) {
    const int s = (t < 2) ? 8 * L : 8;
    return (t & 1) ? -s : s;
  }
  const int sg = t < 4 ? 1 : (t < 8 ? L : L * L);
  switch (t & 3) {
    case 0: return sg;
    case 1: return -(L - 1) * sg;
    case 2: return -sg;
    default: return (L - 1) * sg;
  }
}

__device__ __forceinline__ bool term_holds(int topo, int L, int t, int i) {
  if (topo == 2) {
    const int cell = i >> 3, u = i & 7, row = cell / L, col = cell - row * L;
    switch (t) {
      case 0: return u < 4 && row != L - 1;
      case 1: return u < 4 && row != 0;
      case 2: return u >= 4 && col != L - 1;
      default: return u >= 4 && col != 0;
    }
  }
  const int sg = t < 4 ? 1 : (t < 8 ? L : L * L);
  const int c = (i / sg) % L;
  switch (t & 3) {
    case 0: return c != L - 1;
    case 1: return c == L - 1;
    case 2: return c != 0;
    default: return c == 0;
  }
}

// In-cell K4,4 step for four chimera cells (one byte each): a cell's sites
// u >= 4 are reached when any of its u < 4 is in F, and the other way round.
__device__ __forceinline__ uint32_t chimera_in_cell(uint32_t f) {
  uint32_t lo = f & 0x0F0F0F0Fu, hi = (f >> 4) & 0x0F0F0F0Fu;
  lo |= lo >> 1; lo |= lo >> 2;
  hi |= hi >> 1; hi |= hi >> 2;
  return ((lo & 0x01010101u) * 0xF0u) | ((hi & 0x01010101u) * 0x0Fu);
}


// Periodic 8x8x8 lattice, one 32-bit word per lane: word w = 2 z + (y >> 2)
// holds four x-rows of 8 bits.  x steps rotate within bytes, y steps move
// bytes and borrow one byte from the other half-plane (lane w ^ 1), z steps
// are the words two lanes away within the 16-lane row (DPP row rotates wrap
// at 16 words = 8 planes).  Both directions of every axis are taken, so the
// result is the full neighbourhood of the frontier.
__device__ __forceinline__ uint32_t cube8_expand(uint32_t f) {
  const uint32_t fp = (uint32_t)__builtin_amdgcn_mov_dpp((int)f, 0xB1, 0xF, 0xF, true);  // w ^ 1
  const uint32_t zp = (uint32_t)__builtin_amdgcn_mov_dpp((int)f, 0x12E, 0xF, 0xF, true); // row_ror:14
  const uint32_t zm = (uint32_t)__builtin_amdgcn_mov_dpp((int)f, 0x122, 0xF, 0xF, true); // row_ror:2
  const uint32_t xp = ((f >> 1) & 0x7F7F7F7Fu) | ((f << 7) & 0x80808080u);
  const uint32_t xm = ((f << 1) & 0xFEFEFEFEu) | ((f >> 7) & 0x01010101u);
  const uint32_t yp = (f >> 8) | (fp << 24);
  const uint32_t ym = (f << 8) | (fp >> 24);
  return xp | xm | yp | ym | zp | zm;
}


// The six neighbour words of the 8^3 layout above, in neighbour-table order
// (+x, -x, +y, -y, +z, -z): out[d] bit b = F at the d-neighbour of site 32 w + b.
__device__ __forceinline__ void cube8_dirs(uint32_t f, uint32_t out[6]) {
  const uint32_t fp = (uint32_t)__builtin_amdgcn_mov_dpp((int)f, 0xB1, 0xF, 0xF, true);
  out[0] = ((f >> 1) & 0x7F7F7F7Fu) | ((f << 7) & 0x80808080u);
  out[1] = ((f << 1) & 0xFEFEFEFEu) | ((f >> 7) & 0x01010101u);
  out[2] = (f >> 8) | (fp << 24);
  out[3] = (f << 8) | (fp >> 24);
  out[4] = (uint32_t)__builtin_amdgcn_mov_dpp((int)f, 0x12E, 0xF, 0xF, true);  // word w + 2
  out[5] = (uint32_t)__builtin_amdgcn_mov_dpp((int)f, 0x122, 0xF, 0xF, true);  // word w - 2
}


// Chimera with one word per lane (at most 64 words): word w holds cells
// 4w..4w+3, one byte each (bits u = 0..7).  The four inter-cell terms of the
// shift program (rows +-1 for u < 4, columns +-1 for u >= 4) read the words
// C/4 apart through ds_bpermute and the neighbouring words through DPP wave
// shifts; m[] are this lane's masks of those terms (edges included), so bits
// fetched from outside the move's words never survive.
struct ChimeraStep {
  int qv, rv;        // +8C bits = qv words + rv bits
  uint32_t m[4];     // masks of: row+1, row-1, col+1, col-1
};

__device__ __forceinline__ uint32_t lane_fetch(uint32_t f, int src_lane) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane << 2, (int)f);
}

// out: bits of F at the row+1, row-1, col+1, col-1 neighbour (zero where none)
__device__ __forceinline__ void chimera_inter(uint32_t f, int lane, const ChimeraStep& cs, uint32_t out[4]) {
  const uint32_t up_lo = lane_fetch(f, lane + cs.qv);
  const uint32_t up_hi = cs.rv ? lane_fetch(f, lane + cs.qv + 1) : 0u;
  const int qd = -cs.qv - (cs.rv ? 1 : 0), rd = (32 - cs.rv) & 31;
  const uint32_t dn_lo = lane_fetch(f, lane + qd);
  const uint32_t dn_hi = cs.rv ? lane_fetch(f, lane + qd + 1) : 0u;
  const uint32_t fr = (uint32_t)__builtin_amdgcn_mov_dpp((int)f, 0x130, 0xF, 0xF, true);  // lane + 1
  const uint32_t fl = (uint32_t)__builtin_amdgcn_mov_dpp((int)f, 0x138, 0xF, 0xF, true);  // lane - 1
  out[0] = (cs.rv ? __builtin_amdgcn_alignbit(up_hi, up_lo, (uint32_t)cs.rv) : up_lo) & cs.m[0];
  out[1] = (cs.rv ? __builtin_amdgcn_alignbit(dn_hi, dn_lo, (uint32_t)rd) : dn_lo) & cs.m[1];
  out[2] = __builtin_amdgcn_alignbit(fr, f, 8u) & cs.m[2];
  out[3] = __builtin_amdgcn_alignbit(f, fl, 24u) & cs.m[3];
}

// In-cell neighbour of slot k (u < 4 couples to 4 + k, u >= 4 to k).
__device__ __forceinline__ uint32_t chimera_slot(uint32_t f, int k) {
  const uint32_t lo = (f >> (4 + k)) & 0x01010101u, hi = (f >> k) & 0x01010101u;
  return ((lo << 4) - lo) | (((hi << 4) - hi) << 4);
}


// Term t of the shift program applied to a register-resident bitset (one word
// per lane, word w at lane base + w): bits F[i + shift] fetched from the
// lanes holding words w + q and w + q + 1, masked to where the term holds.
__device__ __forceinline__ uint32_t reg_term(uint32_t f, int lane, int shift, uint32_t mask) {
  const int q = shift >> 5, r = shift & 31;
  const uint32_t lo = lane_fetch(f, lane + q);
  if (r == 0) return lo & mask;
  const uint32_t hi = lane_fetch(f, lane + q + 1);
  return __builtin_amdgcn_alignbit(hi, lo, (uint32_t)r) & mask;
}


// Two words per lane (lane l holds words 2l and 2l+1, a 64-bit value) for the
// two large periodic lattices of the workloads.
//  2D L=64: lane y holds row y (x = 0..63); x steps rotate the row, y steps are
//   the rows of lanes y +- 1 (DPP wave rotates wrap at 64 rows).
//  3D L=16: lane l holds plane z = l / 4, rows y = 4 (l % 4) .. +3 (16 bits
//   each); x steps rotate within 16-bit rows, y steps shift rows and borrow one
//   row from the next / previous lane of the quad (the quad is the whole plane,
//   so the quad rotation is the periodic wrap), z steps are the lanes 4 apart.
// Neighbour bitset of direction d (neighbour-table order +x, -x, +y, -y[, +z, -z]).
__device__ __forceinline__ void pair_dir(bool sq, uint32_t lo, uint32_t hi, int lane, int d, uint32_t& olo,
                                         uint32_t& ohi) {
  if (sq) {
    switch (d) {
      case 0: olo = __builtin_amdgcn_alignbit(hi, lo, 1u); ohi = __builtin_amdgcn_alignbit(lo, hi, 1u); break;
      case 1: olo = __builtin_amdgcn_alignbit(lo, hi, 31u); ohi = __builtin_amdgcn_alignbit(hi, lo, 31u); break;
      case 2:
        olo = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo, 0x134, 0xF, 0xF, true);
        ohi = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi, 0x134, 0xF, 0xF, true);
        break;
      default:
        olo = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo, 0x13C, 0xF, 0xF, true);
        ohi = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi, 0x13C, 0xF, 0xF, true);
        break;
    }
    return;
  }
  switch (d) {
    case 0:
      olo = ((lo >> 1) & 0x7FFF7FFFu) | ((lo << 15) & 0x80008000u);
      ohi = ((hi >> 1) & 0x7FFF7FFFu) | ((hi << 15) & 0x80008000u);
      break;
    case 1:
      olo = ((lo << 1) & 0xFFFEFFFEu) | ((lo >> 15) & 0x00010001u);
      ohi = ((hi << 1) & 0xFFFEFFFEu) | ((hi >> 15) & 0x00010001u);
      break;
    case 2: {
      const uint32_t nlo = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo, 0x39, 0xF, 0xF, true);
      olo = (lo >> 16) | (hi << 16);
      ohi = (hi >> 16) | (nlo << 16);
      break;
    }
    case 3: {
      const uint32_t phi = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi, 0x93, 0xF, 0xF, true);
      olo = (lo << 16) | (phi >> 16);
      ohi = (hi << 16) | (lo >> 16);
      break;
    }
    case 4: olo = lane_fetch(lo, (lane + 4) & 63); ohi = lane_fetch(hi, (lane + 4) & 63); break;
    default: olo = lane_fetch(lo, (lane - 4) & 63); ohi = lane_fetch(hi, (lane - 4) & 63); break;
  }
}

// Bits i..i+31 of a bitset shifted by s (result bit b = F[32 w + b + s]).  F
// points at word 0 of an array padded with one zero word on each side; the
// reads are clamped to the padding, which only matters for words where the
// term's mask is zero.
__device__ __forceinline__ uint32_t shifted_word(const uint32_t* F, int w, int s, int nw) {
  int q = w + (s >> 5);
  q = q < -1 ? -1 : (q > nw - 1 ? nw - 1 : q);
  return __builtin_amdgcn_alignbit(F[q + 1], F[q], (uint32_t)(s & 31));
}


// ----------------------------------------------------------------------------
// The LDS spin image in two views.  Site-major (Metropolis): word (g, i) at
// g Np + i holds walkers 32g..32g+31 at site i.  Walker-major (cluster
// moves): for walker w and site word j, the bits of sites 32j..32j+31 -- what
// a move's q-mask and cluster bitsets are made of.  Block (g, j) is the 32
// words g Np + 32j .. g Np + 32j + 31 in both views, so the switch is an
// in-place 32 x 32 bit transpose per block; in the walker-major view walker
// 32g + r of block j sits at position r ^ (j & 31), so that the lanes of a
// move, which read consecutive words of one walker, hit distinct LDS banks.
// ----------------------------------------------------------------------------
__device__ __forceinline__ int wt_index(int w, int j, int Np) { return (w >> 5) * Np + 32 * j + ((w ^ j) & 31); }

// Row r ^ s of the half-wave (32 lanes) for s = 16, 8, 4, 2, 1.
template <int S>
__device__ __forceinline__ uint32_t partner_row(uint32_t x) {
  if constexpr (S == 16) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x401F);  // xor 16 in 32 lanes
  if constexpr (S == 8) return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, true);  // row_ror:8
  if constexpr (S == 4) {
    // lanes with bit 2 clear (banks 0, 2 of a row) read lane + 4, the others lane - 4
    const int up = __builtin_amdgcn_update_dpp(0, (int)x, 0x104, 0xF, 0x5, false);   // row_shl:4
    return (uint32_t)__builtin_amdgcn_update_dpp(up, (int)x, 0x114, 0xF, 0xA, false);  // row_shr:4
  }
  if constexpr (S == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, true);  // quad [2,3,0,1]
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, true);                     // quad [1,0,3,2]
}

// One stage of the 32 x 32 bit transpose (lane r holds row r of the block):
// the off-diagonal s x s sub-blocks of every 2s x 2s block trade places with
// the partner row r ^ s -- a row with bit s clear takes the partner's low
// column halves into its high ones, the other row the reverse.
template <int S>
__device__ __forceinline__ uint32_t transpose_stage(uint32_t x, int r) {
  constexpr uint32_t lo = S == 16 ? 0x0000FFFFu : (S == 8 ? 0x00FF00FFu : (S == 4 ? 0x0F0F0F0Fu : (S == 2 ? 0x33333333u : 0x55555555u)));
  const uint32_t p = partner_row<S>(x);
  const bool low_row = (r & S) == 0;
  const uint32_t m = low_row ? ~lo : lo;
  const uint32_t y = __builtin_amdgcn_alignbit(p, p, low_row ? 32u - S : (uint32_t)S);  // p << S or p >> S (rotated)
  return (y & m) | (x & ~m);
}

__device__ __forceinline__ uint32_t transpose32(uint32_t x, int r) {
  x = transpose_stage<16>(x, r);
  x = transpose_stage<8>(x, r);
  x = transpose_stage<4>(x, r);
  x = transpose_stage<2>(x, r);
  return transpose_stage<1>(x, r);
}

// Switches the whole image between the views (to_walkers: site-major ->
// walker-major), every wave taking two blocks at a time (one per half-wave).
// All lanes run every stage (the cross-lane reads need them); lanes past the
// last block only skip their loads and stores.
__device__ __forceinline__ void transpose_image(uint32_t* sp, int G, int nw, bool to_walkers) {
  const int lane = lane_id(), half = lane >> 5, r = lane & 31;
  const int nblk = G * nw, Np = 32 * nw, nwaves = (int)(blockDim.x >> 6);
  for (int base = 2 * wave_id(); base < nblk; base += 2 * nwaves) {
    const int blk = base + half;
    const bool live = blk < nblk;
    const int g = live ? blk / nw : 0, j = live ? blk - g * nw : 0;
    const int site_pos = g * Np + 32 * j + r, walker_pos = g * Np + 32 * j + ((r ^ j) & 31);
    const uint32_t x = live ? sp[to_walkers ? site_pos : walker_pos] : 0u;
    const uint32_t t = transpose32(x, r);
    if (live) sp[to_walkers ? walker_pos : site_pos] = t;
  }
}

// Sum over the lpm lanes of each lane group (16, 32 or 64: one, two or four
// DPP rows), returned to every lane of the group.
__device__ __forceinline__ int group_sum(int v, int lpm) {
  v = dpp_row_sum(v);
  if (lpm == 16) return v;
  const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
  const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
  if (lpm == 32) return lane_id() < 32 ? r0 + r1 : r2 + r3;
  return (r0 + r1) + (r2 + r3);
}

// Exclusive prefix sum within each lane group (rows of 16 lanes: the row
// scans; groups of 32: row 1 and row 3 add the last value of the row before;
// 64: the whole wave).
__device__ __forceinline__ int group_exclusive_scan(int v, int lpm) {
  int x = v;
  x += __builtin_amdgcn_mov_dpp(x, 0x111, 0xF, 0xF, true);  // row_shr:1
  x += __builtin_amdgcn_mov_dpp(x, 0x112, 0xF, 0xF, true);  // row_shr:2
  x += __builtin_amdgcn_mov_dpp(x, 0x114, 0xF, 0xF, true);  // row_shr:4
  x += __builtin_amdgcn_mov_dpp(x, 0x118, 0xF, 0xF, true);  // row_shr:8
  if (lpm >= 32) x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
  if (lpm == 64) x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
  return x - v;
}

// The two-word layouts' cluster growth and boundary walk, out of line: they
// run once per move batch, and inlined they push the fused kernel past its
// register budget.  LDS regions are passed as byte offsets into the dynamic
// LDS array (so the accesses stay LDS accesses).
extern __shared__ __align__(16) unsigned char lds[];

__device__ __noinline__ void pair_grow(bool sq64, uint32_t mc_off, int lane) {
  uint32_t* gmc = (uint32_t*)(lds + mc_off);
  const uint32_t m0 = gmc[4 * lane], m1 = gmc[4 * lane + 2];
  uint32_t c0 = gmc[4 * lane + 1], c1 = gmc[4 * lane + 3];
  uint32_t f0 = c0, f1 = c1;
  while (true) {
    uint32_t g0 = 0, g1 = 0;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      if (sq64 && d >= 4) break;
      uint32_t o0, o1;
      pair_dir(sq64, f0, f1, lane, d, o0, o1);
      g0 |= o0;
      g1 |= o1;
    }
    const uint32_t n0 = g0 & m0 & ~c0, n1 = g1 & m1 & ~c1;
    c0 |= n0;
    c1 |= n1;
    f0 = n0;
    f1 = n1;
    if (!__ballot((n0 | n1) != 0u)) break;
  }
  gmc[4 * lane + 1] = c0;
  gmc[4 * lane + 3] = c1;
}

// Boundary bonds (slot by slot) of one cluster in the two-word layouts;
// returns the sum of J s_a,i s_a,j over the bonds that leave it.
template <int JK, int DEG>
__device__ __noinline__ typename EnergyT<JK>::T pair_boundary(bool sq64, uint32_t mc_off, uint32_t aw_off,
                                                             uint32_t coup_off, const void* coup_global,
                                                             int lane, int& csize) {
  using E_t = typename EnergyT<JK>::T;
  const uint32_t* gmc = (const uint32_t*)(lds + mc_off);
  const uint32_t* gaw = (const uint32_t*)(lds + aw_off);
  const int32_t* cf = coup_global ? (const int32_t*)coup_global : (const int32_t*)(lds + coup_off);
  const int8_t* cj = coup_global ? (const int8_t*)coup_global : (const int8_t*)(lds + coup_off);
  const uint32_t cw0 = gmc[4 * lane + 1], cw1 = gmc[4 * lane + 3];
  const uint32_t aw0 = gaw[2 * lane], aw1 = gaw[2 * lane + 1];
  csize = __popc(cw0) + __popc(cw1);
  E_t dEa = 0;
#pragma unroll
  for (int d = 0; d < DEG; ++d) {
    uint32_t c_lo, c_hi, a_lo, a_hi;
    pair_dir(sq64, cw0, cw1, lane, d, c_lo, c_hi);
    pair_dir(sq64, aw0, aw1, lane, d, a_lo, a_hi);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint32_t bb = (h ? cw1 : cw0) & ~(h ? c_hi : c_lo);
      const uint32_t anti = (h ? aw1 : aw0) ^ (h ? a_hi : a_lo);
      while (bb) {
        const int bpos = __builtin_ctz(bb);
        bb &= bb - 1u;
        const int x = (64 * lane + 32 * h + bpos) * DEG + d;
        if (JK) {
          const double J = (double)cf[x];
          dEa += ((anti >> bpos) & 1u) ? -J : J;
        } else {
          const int J = cj[x];
          dEa += ((anti >> bpos) & 1u) ? -J : J;
        }
      }
    }
  }
  return dEa;
}

// ----------------------------------------------------------------------------
// Observables after a step (only with the measure flag; out of line so that it
// costs the fused kernel no registers).  For the two replicas (chains 2p,
// 2p+1) at each temperature: the energies, the link-overlap sum over bonds of
// q_i q_j (N_b q_l) and (sum_i q_i)^2, added to the time bin floor(log2 t) of
// the step's end t.  One wave per pair: ballots give the q-mask words, each
// lane counts the bonds of its sites whose ends differ (D; sum q_i q_j =
// N_b - 2 D).  The stored replica b may be reversed (gauge bit): that flips
// every q_i and leaves all three quantities unchanged.  LDS regions come as
// byte offsets into the dynamic LDS array.
// ----------------------------------------------------------------------------
template <int JK, int DEG>
__device__ __noinline__ void measure_step(uint32_t t_end, int N, int K, int R, int topo, int L, uint32_t sp_off,
                                          uint32_t at_off, uint32_t energy_off, uint32_t meas_off,
                                          uint32_t nbr_off, const uint16_t* nbr_global, int64_t* obs) {
  using E_t = typename EnergyT<JK>::T;
  t_end = (uint32_t)uniform((int)t_end);
  N = uniform(N); K = uniform(K); R = uniform(R); topo = uniform(topo); L = uniform(L);
  const uint32_t* sp = (const uint32_t*)(lds + uniform((int)sp_off));
  const int* at = (const int*)(lds + uniform((int)at_off));
  const E_t* energy = (const E_t*)(lds + uniform((int)energy_off));
  const uint16_t* nbr = nbr_global ? nbr_global : (const uint16_t*)(lds + uniform((int)nbr_off));
  const int lane = lane_id(), wave = wave_id(), nwaves = (int)(blockDim.x >> 6);
  const int half = R >> 1, nw = site_words(N);
  const int bin = 31 - __builtin_clz(t_end);
  const int nbonds = topo == 2 ? 16 * L * L + 8 * L * (L - 1) : N * (DEG / 2);
  uint32_t* qw = (uint32_t*)(lds + uniform((int)meas_off)) + wave * nw;
  for (int x = wave; x < K * half; x += nwaves) {
    const int k = x / half, p = x - k * half;
    const int a = at[k * R + 2 * p], b = at[k * R + 2 * p + 1];
    const int Np = 32 * nw;  // row length of the LDS spin image
    const uint32_t* rowa = sp + (a >> 5) * Np;
    const uint32_t* rowb = sp + (b >> 5) * Np;
    const int pa = a & 31, pb = b & 31;
    int n = 0;
    for (int s2 = 0; s2 * 64 < N; ++s2) {
      const int i = s2 * 64 + lane;
      const uint32_t qb = i < N ? (bit_of(rowa[i], pa) ^ bit_of(rowb[i], pb)) : 0u;
      const unsigned long long bal = __ballot(qb);
      n += __popcll(bal);
      if (lane == 0) {
        qw[2 * s2] = (uint32_t)bal;
        if (2 * s2 + 1 < nw) qw[2 * s2 + 1] = (uint32_t)(bal >> 32);
      }
    }
    n = uniform(n);
    wave_sync();
    int diff = 0;
    for (int i = lane; i < N; i += 64) {
      const uint32_t qi = (qw[i >> 5] >> (i & 31)) & 1u;
#pragma unroll
      for (int d = 0; d < DEG; ++d) {
        const int j = nbr_global ? nbr[i * DEG + d] : nbr[i * DEG + d] >> 2;  // LDS copy: byte offsets
        // each bond once: lattices from the +axis slots; chimera in-cell bonds
        // from u < 4, inter-cell bonds from the "next" slot if present
        const bool bond = topo == 2 ? (((i & 7) < 4 && d < 4) || (d == 5 && j != i)) : (d & 1) == 0;
        if (bond) diff += (int)(qi ^ ((qw[j >> 5] >> (j & 31)) & 1u));
      }
    }
    const int D = wave_sum(diff);
    if (lane == 0) {
      int64_t* o = obs + (((size_t)bin * K + k) * half + p) * kObsFields;
      // float couplings in units of 2^-20 (energies are multiples of 2^-jexp,
      // jexp <= 20: exact), so long bins stay within int64
      const int64_t ea = JK ? (int64_t)((double)energy[a] * 0x1p20) : (int64_t)energy[a];
      const int64_t eb = JK ? (int64_t)((double)energy[b] * 0x1p20) : (int64_t)energy[b];
      const int64_t q = (int64_t)N - 2 * n;
      o[0] += ea + eb;
      o[1] += (int64_t)nbonds - 2 * D;
      o[2] += q * q;
      o[3] += n < N - n ? n : N - n;  // potential cluster sites after step 2a
    }
    wave_sync();
  }
  if (threadIdx.x == 0) obs[(size_t)kObsBins * K * half * kObsFields + bin] += 1;
}

// ----------------------------------------------------------------------------
// The exact pass of a Metropolis colour (float couplings): for each queued
// task (site i, the quad pair qt, the estimate's flip bits) every walker
// whose float call was too close is decided again in double as
// u 2^-32 < exp(-beta dE); where that differs from the estimate, the spin is
// flipped back or forth, and the energy and the accepted-flip count are
// corrected.  The task's other inputs are recomputed as the sweep made them
// (the neighbours have the other colour, so they have not moved; the site's
// own bits are restored from the estimate's flips).  One lane per queued
// task; empties the wave's queue.  Out of line, so that the sweep loop keeps
// no registers for it.
// ----------------------------------------------------------------------------
// The PT swap rule between the walker carried up to rung k (energy ex) and
// the walker at rung k + 1 (energy ey), with the draw u of (k, chain): float
// couplings u 2^-32 < exp(-(beta_k - beta_k+1) D) in double after the float
// pre-filter that settles all but a thin band (as for Metropolis); integer
// couplings the threshold table of the gap D = ey - ex.
template <int JK>
__device__ __forceinline__ bool pt_swap(uint32_t u, typename EnergyT<JK>::T ex, typename EnergyT<JK>::T ey, int k,
                                        const double* beta, const float* dbl2e, const uint32_t* ptthr, int ptlen) {
  if constexpr (JK) {
    const double D = (double)ey - (double)ex;
    return accept_float(u, D, beta[k] - beta[k + 1], dbl2e[k]);
  } else {
    const int D = (int)ey - (int)ex;
    return D <= 0 || (D <= ptlen && u < ptthr[k * ptlen + (D - 1)]);
  }
}

// PT decisions of a step, up front (at most kPtTable temperatures): every
// pair (k, c), c <= k, of every chain r -- the walker that sat at rung c,
// carried up to rung k, against the walker at rung k + 1 -- decided with the
// swap rule; bit c of word (k, r) of the table is set on a swap.  Energies do
// not change during PT, so these are exactly the decisions a chain's scan
// can meet.  Out of line and with scalar arguments, like exact_pass, so that
// it does not weigh on the sweep loop's registers.
template <int JK>
__device__ __noinline__ void pt_decide(uint32_t at_off, uint32_t energy_off, uint32_t ptu_off, uint32_t ptacc_off,
                                       uint32_t beta_off, uint32_t dbl2e_off, const uint32_t* ptthr, int ptlen,
                                       int K, int R) {
  using E_t = typename EnergyT<JK>::T;
  const int* at = (const int*)(lds + uniform((int)at_off));
  const E_t* energy = (const E_t*)(lds + uniform((int)energy_off));
  const uint32_t* ptu = (const uint32_t*)(lds + uniform((int)ptu_off));
  uint32_t* ptacc = (uint32_t*)(lds + uniform((int)ptacc_off));
  const double* beta = (const double*)(lds + uniform((int)beta_off));
  const float* dbl2e = (const float*)(lds + uniform((int)dbl2e_off));
  const int T = K * (K - 1) / 2;
  for (int d = (int)threadIdx.x; d < R * T; d += (int)blockDim.x) {
    const int r = d / T, idx = d - r * T;
    int k = (int)((__builtin_sqrtf(8.0f * (float)idx + 1.0f) - 1.0f) * 0.5f);
    if ((k + 1) * (k + 2) / 2 <= idx) ++k;
    if (k * (k + 1) / 2 > idx) --k;
    const int c = idx - k * (k + 1) / 2;
    const E_t ex = energy[at[c * R + r]], ey = energy[at[(k + 1) * R + r]];
    if (pt_swap<JK>(ptu[k * R + r], ex, ey, k, beta, dbl2e, ptthr, ptlen)) atomicOr(&ptacc[k * R + r], 1u << c);
  }
}

// Full labelling of a wave's moves for the label readout (rare: only when
// labels are recorded), one move at a time with the whole wave: union-find
// over the q = -1 subgraph, roots hooked towards the smaller index, path
// compression.  Out of line, so that the cluster-move loop does not carry its
// registers.
template <int DEG, int TL>
__device__ __noinline__ void record_labels(uint32_t slots_off, uint32_t parent_off, uint32_t nbr_off,
                                           const uint16_t* nbr_global, int* labels, int* seeds, int wave, int P,
                                           int sw, int nw, int N, int nmoves) {
  wave = uniform(wave); P = uniform(P); sw = uniform(sw); nw = uniform(nw); N = uniform(N);
  nmoves = uniform(nmoves);
  const int lane = lane_id();
  const uint16_t* nbr = TL ? (const uint16_t*)(lds + uniform((int)nbr_off)) : nbr_global;
  for (int g = 0; g < P; ++g) {
    const int slot = wave * P + g;
    uint32_t* mc = (uint32_t*)(lds + uniform((int)slots_off)) + slot * sw + 2 * (nw + 2);
    const int* info = (const int*)(mc + 3 * nw);
    const int mvr = info[kInMv];
    if (mvr < 0) continue;
    int* parent = (int*)(lds + uniform((int)parent_off)) + slot * N;
    int* lab = labels + (size_t)mvr * N;
    const int nown = N > lane ? (N - lane + 63) >> 6 : 0;
    auto inmask = [&](int j) { return (mc[2 * (j >> 5)] >> (j & 31)) & 1u; };
    for (int s2 = 0; s2 < nown; ++s2) {
      const int i = s2 * 64 + lane;
      if (inmask(i)) parent[i] = i;
    }
    wave_sync();
    for (int s2 = 0; s2 < nown; ++s2) {
      const int i = s2 * 64 + lane;
      if (!inmask(i)) continue;
#pragma unroll
      for (int d = 0; d < DEG; ++d) {
        const int jn = TL ? nbr[i * DEG + d] >> 2 : nbr[i * DEG + d];  // LDS copy: byte offsets
        if (jn > i && inmask(jn)) uf_union(parent, i, jn);
      }
    }
    wave_sync();
    for (int s2 = 0; s2 < nown; ++s2) {
      const int i = s2 * 64 + lane;
      if (inmask(i))
        __hip_atomic_store(&parent[i], uf_find(parent, i), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
    wave_sync();
    for (int s2 = 0; s2 < nown; ++s2) {
      const int i = s2 * 64 + lane;
      lab[i] = inmask(i) ? uf_load(parent, i) : -1;
    }
    if (lane == 0) {
      seeds[mvr] = info[kInSeed];
      seeds[nmoves + mvr] = info[kInN];
    }
    wave_sync();
  }
}

template <int DEG, int QPT>
__device__ __noinline__ void exact_pass(uint32_t q_off, uint32_t sp_off, int Np, uint32_t nbr_off,
                                        const uint16_t* nbr_global, uint32_t coup_off, const int32_t* coup_global,
                                        uint32_t tau_off, uint32_t beta_off, uint32_t bl2e_off, uint32_t energy_off,
                                        uint32_t stats_off, int W, int Wq, int jexp, uint32_t t, uint32_t seed,
                                        uint32_t key) {
  constexpr int WPT = 4 * QPT;
  uint32_t* q = (uint32_t*)(lds + uniform((int)q_off));
  uint32_t* sp = (uint32_t*)(lds + uniform((int)sp_off));
  const uint16_t* nbr = nbr_global ? nbr_global : (const uint16_t*)(lds + uniform((int)nbr_off));
  const int32_t* cf = coup_global ? coup_global : (const int32_t*)(lds + uniform((int)coup_off));
  const int* tau = (const int*)(lds + uniform((int)tau_off));
  const double* beta = (const double*)(lds + uniform((int)beta_off));
  const float* bl2e = (const float*)(lds + uniform((int)bl2e_off));
  double* energy = (double*)(lds + uniform((int)energy_off));
  unsigned long long* stats = (unsigned long long*)(lds + uniform((int)stats_off));
  Np = uniform(Np); W = uniform(W); Wq = uniform(Wq); jexp = uniform(jexp);
  t = (uint32_t)uniform((int)t); seed = (uint32_t)uniform((int)seed); key = (uint32_t)uniform((int)key);
  const int lane = lane_id();
  const int n = uniform((int)__hip_atomic_load(&q[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT));
  const double jq2 = ldexp(1.0, 1 - jexp);
  for (int x0 = 0; x0 < n; x0 += 64) {
    const int x = x0 + lane;
    if (x >= n) continue;
    const uint32_t w0 = q[2 + 2 * x], guess = q[3 + 2 * x];
    const int i = (int)(w0 & 0xFFFFu), qt = (int)(w0 >> 16);
    const int q0 = QPT * qt, g = q0 >> 3, sh = 4 * (q0 & 7);
    uint32_t* row = sp + g * Np;
    const uint32_t own = row[i] ^ (guess << sh);
    uint32_t xw[DEG];
    int Ji[DEG], Jsum = 0;
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
      xw[d] = row[nbr_global ? nbr[i * DEG + d] : nbr[i * DEG + d] >> 2] ^ own;  // LDS copy: byte offsets
      Ji[d] = cf[i * DEG + d];
      Jsum += Ji[d];
    }
    Words4 u[QPT];
#pragma unroll
    for (int h = 0; h < QPT; ++h)
      if (h == 0 || q0 + h < Wq) u[h] = philox4x32_10((uint32_t)i, t, (uint32_t)(q0 + h), kStreamMetro, seed, key);
      else u[h] = u[0];
    uint32_t corr = 0;
    int dcnt = 0;
#pragma unroll
    for (int b = 0; b < WPT; ++b) {
      const int w = WPT * qt + b;
      if (w >= W) continue;
      int mn = 0;
#pragma unroll
      for (int d = 0; d < DEG; ++d) mn = mad_i24(__builtin_amdgcn_sbfe((int)xw[d], (unsigned)(sh + b), 1u), Ji[d], mn);
      const int e = Jsum + 2 * mn;
      const uint32_t uu = u[b >> 2].w[b & 3];
      const int k = tau[w];
      const float lqb = bl2e[k];
      const float P = __builtin_amdgcn_exp2f(__builtin_fmaf(-(float)e, lqb, 32.0f));
      if (absdiff(__float_as_uint((float)uu), __float_as_uint(P)) >= kCloseUlps) continue;
      const bool ex = e <= 0 || accept_exact(uu, (double)e * jq2, beta[k]);
      if (ex != (((guess >> b) & 1u) != 0u)) {
        corr |= 1u << b;
        atomicAdd(&energy[w], ldexp((double)(ex ? e : -e), 1 - jexp));
        dcnt += ex ? 1 : -1;
      }
    }
    if (corr) atomicXor(&row[i], corr << sh);
    if (dcnt) atomicAdd(&stats[kStatMetroAcc], (unsigned long long)(long long)dcnt);
  }
  wave_sync();
  if (lane == 0) q[0] = 0;
  wave_sync();
}

// ----------------------------------------------------------------------------
// The fused sweep-block kernel.  JK: 0 = int8 couplings, 1 = float couplings.
// DEG: neighbour slots (4 for square2d, 6 otherwise).  TL: tables in LDS.
// LAY: the cluster-move layout (kLayAny: chosen per unit).  One workgroup runs
// one unit; its spins live bit-packed in LDS for the whole block of sweeps.
// ----------------------------------------------------------------------------
template <int JK, int DEG, int TL, int LAY>
__global__ void __launch_bounds__(1024) sweep_block_kernel(const UnitDesc* __restrict__ units,
                                                          uint32_t n_sweeps, int icm_slots) {
  using E_t = typename EnergyT<JK>::T;
  extern __shared__ __align__(16) unsigned char lds[];
  const UnitDesc U = units[blockIdx.x];
  // the 8^3 build knows its unit size: 512 sites, 256 of each colour
  const int N = LAY == kLayCube8 ? 512 : U.N, Nc = LAY == kLayCube8 ? 256 : U.Nc;
  const int W = U.W, Wq = U.Wq, K = U.K, R = U.R, Kc = U.Kc, HM = U.HM;
  const int Wp = 4 * Wq, G = bit_words(Wq);
  const LdsLayout lay = lds_layout(N, DEG, Wq, K, R, HM, JK, icm_slots, TL,
                                   ((U.flags & kFlagRecord) ? 1 : 0) | ((U.flags & kFlagMeasure) ? 2 : 0), Kc,
                                   JK ? 0 : U.jpl, (int)(blockDim.x >> 6));

  uint32_t* sp = (uint32_t*)(lds + lay.sp);
  // TL: tables in LDS (neighbours as byte offsets 4 j); otherwise read-only
  // global memory (cached in L1/L2, neighbours as site indices j)
  const uint16_t* nbr = TL ? (const uint16_t*)(lds + lay.nbr) : U.nbr;
  const uint16_t* clist = TL ? (const uint16_t*)(lds + lay.clist) : U.clist;
  const int8_t* cj = TL ? (const int8_t*)(lds + lay.coup) : (const int8_t*)U.coup;
  // float couplings as integers in units of 2^-jexp (exact 24-bit values)
  const int32_t* cf = TL ? (const int32_t*)(lds + lay.coup) : (const int32_t*)U.coup;
  int* tau = (int*)(lds + lay.tau);
  int* at = (int*)(lds + lay.at);
  int* gauge = (int*)(lds + lay.gauge);
  E_t* energy = (E_t*)(lds + lay.energy);
  uint32_t* thr = (uint32_t*)(lds + lay.thr);
  double* beta = (double*)(lds + lay.beta);
  float* bl2e = (float*)(lds + lay.bl2e);
  float* dbl2e = (float*)(lds + lay.dbl2e);
  uint32_t* ptu = (uint32_t*)(lds + lay.ptu);
  uint32_t* icmu = (uint32_t*)(lds + lay.icmu);
  unsigned long long* stats = (unsigned long long*)(lds + lay.stats);

  const int tid = threadIdx.x, nthr = blockDim.x;
  // ---- load the unit into LDS; int8 quad words -> bit-packed words ----
  const int Np = 32 * site_words(N);  // LDS row length (sites past N stay zero)
  for (int x = tid; x < G * Np; x += nthr) {
    const int g = x / Np, i = x - g * Np;
    uint32_t bits = 0;
    for (int qq = 0; qq < 8; ++qq) {
      const int q = 8 * g + qq;
      if (q >= Wq || i >= N) break;
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
    // the LDS copy holds byte offsets (4 j) within a row of the spin image, so
    // the Metropolis task forms a neighbour word's address in one add (units
    // have at most kMaxSites = 4096 sites: 4 j fits 16 bits)
    for (int x = tid; x < N * DEG; x += nthr) nbr_w[x] = (uint16_t)(U.nbr[x] << 2);
    for (int x = tid; x < N; x += nthr) clist_w[x] = U.clist[x];
    if (JK) {
      int32_t* cf_w = (int32_t*)(lds + lay.coup);
      for (int x = tid; x < N * DEG; x += nthr) cf_w[x] = ((const int32_t*)U.coup)[x];
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
    if (JK) energy[x] = (E_t)((double)U.energy[x] * 0x1p-40);
    else energy[x] = (E_t)U.energy[x];
  }
  for (int x = tid; x < K * R; x += nthr) at[x] = U.at[x];
  for (int x = tid; x < K; x += nthr) {
    beta[x] = U.beta[x];
    // float couplings: beta log2 e times 2^(1 - jexp), the factor of e (the
    // field in units of 2^-jexp) in the acceptance exponent; exact (a power of 2)
    bl2e[x] = JK ? ldexpf(U.bl2e[x], 1 - U.jexp) : U.bl2e[x];
    // PT pre-filter factor: the gap of neighbouring betas times log2 e, rounded once
    dbl2e[x] = x + 1 < K ? (float)((U.beta[x] - U.beta[x + 1]) * 1.4426950408889634) : 0.0f;
  }
  for (int x = tid; x < kNumStats; x += nthr) stats[x] = 0;
  if (JK)
    for (int x = tid; x < (int)(nthr >> 6); x += nthr) ((uint32_t*)(lds + lay.exq))[x * (2 + 2 * kExactQ)] = 0;
  if (Kc > 0) {
    // shift program of the lattice and zeroed frontier padding of every slot
    const int nw = site_words(N), nterm = lattice_terms(U.topo);
    int* tshift = (int*)(lds + lay.terms);
    uint32_t* tmask = (uint32_t*)(lds + lay.terms) + kMaxTerms;
    for (int x = tid; x < nterm; x += nthr) tshift[x] = term_shift(U.topo, U.L, x);
    for (int x = tid; x < nterm * nw; x += nthr) {
      const int t = x / nw, w = x - t * nw;
      uint32_t bits = 0;
      for (int b = 0; b < 32; ++b) {
        const int i = 32 * w + b;
        if (i < N && term_holds(U.topo, U.L, t, i)) bits |= 1u << b;
      }
      tmask[x] = bits;
    }
    if (!JK && U.jpl > 0) {
      // bit planes of the couplings: plane k of (word w, slot d) holds bit k
      // (two's complement, jpl bits) of J over the sites 32 w .. 32 w + 31
      const int jpl = U.jpl;
      uint32_t* pl = (uint32_t*)(lds + lay.jplanes);
      const int8_t* gj = (const int8_t*)U.coup;
      for (int x = tid; x < nw * DEG; x += nthr) {
        const int w = x / DEG, d = x - w * DEG;
        uint32_t planes[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int b = 0; b < 32; ++b) {
          const int i = 32 * w + b;
          const uint32_t j = i < N ? (uint32_t)(uint8_t)gj[i * DEG + d] : 0u;
#pragma unroll
          for (int k = 0; k < 8; ++k) planes[k] |= ((j >> k) & 1u) << b;
        }
        for (int k = 0; k < jpl; ++k) pl[x * jpl + k] = planes[k];
      }
    }
    const int ns = slots_reserved(N, icm_slots), sw = slot_words(N);
    uint32_t* sl0 = (uint32_t*)(lds + lay.slots);
    for (int x = tid; x < ns; x += nthr) {
      uint32_t* f = sl0 + x * sw;
      f[0] = 0; f[nw + 1] = 0; f[nw + 2] = 0; f[2 * nw + 3] = 0;
    }
  }
  __syncthreads();

  const uint32_t t0 = (uint32_t)uniform((int)*U.sweep);
  const uint32_t flags = U.flags, seed = U.seed, key = U.key;
  const int lane = lane_id(), wave = wave_id(), nwaves = nthr >> 6;
  uint32_t metro_cnt = 0;  // accepted flips of this lane, flushed once per sweep

  for (uint32_t s = 0; s < n_sweeps; ++s) {
    const uint32_t t = t0 + s;
    // The random numbers of PT and ICM do not depend on the state: draw them
    // now, in parallel; the barriers of the sweep order them before their use.
    if (flags & kFlagPt)
      for (int x = tid; x < (K - 1) * R; x += nthr) {
        const int k = x / R, r = x - k * R;
        ptu[x] = philox4x32_10((uint32_t)k, t, (uint32_t)r, kStreamPt, seed, key).w[0];
        if (K >= kPtTableMin && K <= kPtTable) ((uint32_t*)(lds + lay.ptacc))[x] = 0u;  // this step's swap words
      }
    for (int x = tid; x < Kc * (R >> 1); x += nthr)
      icmu[x] = philox4x32_10((uint32_t)x, t, 0u, kStreamIcm, seed, key).w[0];
    if (flags & kFlagSkipMetro) __syncthreads();
    // ---------------- step 1: Metropolis sweep, colour 0 then colour 1 ----------
    if (!(flags & kFlagSkipMetro)) {
      // A task is one site of one colour for the walkers of QPT = 2 Philox
      // quads (8 walkers in one byte of a bit-word): the neighbour words and
      // couplings are read once for all of them, and the two Philox blocks
      // share their first round's per-lane product.
      constexpr int QPT = 2, WPT = 4 * QPT;
      const int Wqt = (Wq + QPT - 1) / QPT;
      for (int c = 0; c < 2; ++c) {
        const int nchunk = (Nc + 63) >> 6;
        const bool narrow = nchunk * DEG * WPT < 256;
        const int ntasks = Wqt * nchunk;
        // workgroups have 1, 2, 4, 8 or 16 waves: in the 8^3 build the split is
        // a shift (the other builds measured faster with the division)
        const int lgw = 31 - __builtin_clz(nwaves);
        const int tb = LAY == kLayCube8 ? (ntasks * wave) >> lgw : (int)(((long long)ntasks * wave) / nwaves);
        const int te = LAY == kLayCube8 ? (ntasks * (wave + 1)) >> lgw
                                        : (int)(((long long)ntasks * (wave + 1)) / nwaves);
        int cur_q = -1;
        int qn = 0;  // tasks this wave has queued for the exact pass (uniform)
        int acc[WPT];  // per lane: sum of e over its accepted flips (dE = 2 e in field units)
        // per walker of the current task's quads (uniform): float couplings
        // the acceptance exponent's scale, integer couplings the threshold row;
        // vmask: the walkers that exist (the last quad may be padding)
        float lq[WPT];
        int rowb[WPT];
        uint32_t vmask = 0;
#pragma unroll
        for (int b = 0; b < WPT; ++b) { acc[b] = 0; rowb[b] = 0; lq[b] = 0.0f; }
        int qt = tb / nchunk, chunk = tb - qt * nchunk;
        uint32_t* exq = (uint32_t*)(lds + lay.exq) + wave * (2 + 2 * kExactQ);
        for (int task = tb; task < te; ++task, (++chunk == nchunk ? (chunk = 0, ++qt) : 0)) {
          // past 3/8 of its share a wave outranks the waves (of any workgroup
          // on the CU) still in their first part, so colours end together
          if (task == tb + (((te - tb) * 3) >> 3)) __builtin_amdgcn_s_setprio(1);
          // the queue holds room for every lane of the next task
          if constexpr (JK) {
            if (qn > kExactQ - 64) {
              exact_pass<DEG, QPT>(lay.exq + 4u * (uint32_t)wave * (2 + 2 * kExactQ), lay.sp, Np, lay.nbr,
                                TL ? nullptr : U.nbr, lay.coup, TL ? nullptr : (const int32_t*)U.coup, lay.tau,
                                lay.beta, lay.bl2e, lay.energy, lay.stats, W, Wq, U.jexp, t, seed, key);
              qn = 0;
            }
          }
          if (qt != cur_q) {
            if (cur_q >= 0) {
              flush_energy<JK, WPT>(acc, energy + WPT * cur_q, U.jexp, narrow);
#pragma unroll
              for (int b = 0; b < WPT; ++b) acc[b] = 0;
            }
            cur_q = qt;
            if constexpr (JK) {
              // lane b (mod WPT) looks up walker WPT qt + b's scale; the wave
              // then takes the values as uniforms.  Walkers from W on are padding.
              const int wb = WPT * qt + (lane & (WPT - 1));
              const int nreal = W - WPT * qt;
              vmask = nreal >= WPT ? (1u << WPT) - 1u : (1u << nreal) - 1u;
              const float lql = wb < W ? bl2e[tau[wb]] : 0.0f;
#pragma unroll
              for (int b = 0; b < WPT; ++b) lq[b] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lql), b));
            } else {
              vmask = 0;
#pragma unroll
              for (int b = 0; b < WPT; ++b) {
                const int tb2 = uniform(WPT * qt + b < W ? tau[WPT * qt + b] : K);
                if (tb2 < K) {
                  vmask |= 1u << b;
                  rowb[b] = tb2 * HM;
                }
              }
            }
          }
          const int j = chunk * 64 + lane;
          bool queued = false;
          if (j < Nc) {
            const int q0 = QPT * qt;
            const int g = q0 >> 3, sh = 4 * (q0 & 7);
            uint32_t* row = sp + g * Np;
            const int i = clist[c * Nc + j];
            // bit sh + b of a word is walker 4 q0 + b (one bit-field extract each)
            const uint32_t own = row[i];
            uint32_t nw[DEG];
#pragma unroll
            for (int d = 0; d < DEG; ++d)
              nw[d] = TL ? *(const uint32_t*)((const unsigned char*)row + nbr[i * DEG + d]) : row[nbr[i * DEG + d]];
            Words4 u[QPT];
            const uint64_t m0 = philox_m0((uint32_t)i);
#pragma unroll
            for (int h = 0; h < QPT; ++h)
              if (h == 0 || q0 + h < Wq) u[h] = philox4x32_10_lane(m0, t, (uint32_t)(q0 + h), kStreamMetro, seed, key);
              else u[h] = u[0];
            // e = s_i h = sum_d J_d s_i s_d = sum J - 2 sum_d J_d x_d, x_d = 1 where
            // the spin and its d-neighbour differ (own word xor neighbour word,
            // once for all walkers of the task): the bit extracted sign-extended
            // (0 or -1) times J_d, 24-bit integers (float couplings in units of
            // 2^-jexp), dE = 2 e
            int Ji[DEG];
            int Jsum = 0;
            uint32_t xw[DEG];
#pragma unroll
            for (int d = 0; d < DEG; ++d) {
              xw[d] = nw[d] ^ own;
              if constexpr (JK) {
                Ji[d] = cf[i * DEG + d];
                Jsum += Ji[d];
              }
            }
            uint32_t flip = 0;
            if constexpr (JK) {
              // every walker decided by the float estimate P of 2^32 exp(-beta dE)
              // (accept iff float(u) < P), no branch; `close` keeps the nearest
              // call of the task in float bit patterns (units in the last
              // place).  Where the decision is open (1 <= P <= 2^32) the
              // exponent argument 32 - e lq lies in [0, 32] and carries at most
              // three roundings of 2^-24 relative (e and lq to float, the fma),
              // so P is within 96 ln2 2^-24 < 2^-17.8 (plus exp2's last place)
              // of the exact value: under 80 units in the last place with
              // float(u)'s own rounding.  kCloseUlps = 512 of them leave a
              // margin of six; any call that close is made again exactly, in
              // double, as the oracle does: the task is queued (rare) and
              // exact_pass redoes those calls before the colour ends
              // (same-colour sites do not interact, so a decision may wait).
              uint32_t close = 0xFFFFFFFFu;
#pragma unroll
              for (int b = 0; b < WPT; ++b) {
                int mn = 0;
#pragma unroll
                for (int d = 0; d < DEG; ++d)
                  mn = mad_i24(__builtin_amdgcn_sbfe((int)xw[d], (unsigned)(sh + b), 1u), Ji[d], mn);
                const int e = Jsum + 2 * mn;  // dE = e 2^(1 - jexp)
                const float P = __builtin_amdgcn_exp2f(__builtin_fmaf(-(float)e, lq[b], 32.0f));
                const float uf = (float)u[b >> 2].w[b & 3];
                // the lanes that accept, as a lane mask straight from the compare
                const uint64_t ok = __builtin_amdgcn_ballot_w64(uf < P) & (0ull - (uint64_t)((vmask >> b) & 1u));
                close = min(close, absdiff(__float_as_uint(uf), __float_as_uint(P)));
                accept_where(ok, 1u << (sh + b), flip, e, acc[b]);
              }
              queued = close < kCloseUlps;
              if (queued) {
                // queue the task for the exact pass at the end of the colour
                const uint32_t pos = atomicAdd(&exq[0], 1u);
                exq[2 + 2 * pos] = (uint32_t)i | ((uint32_t)qt << 16);
                exq[3 + 2 * pos] = flip >> sh;
              }
            } else {
              // int8 couplings: the site's couplings packed one per byte (slots
              // 0-3, then 4-5), and per neighbour slot d the task's four walker
              // bits of x_d in byte d; walker b's sum over d of J_d x_d is then
              // two four-byte dot products (v_dot4c_i32_i8) of its bit bytes
              // with the coupling bytes
              uint32_t Jp, Jp2 = 0u, T = 0u, T2 = 0u;
              if constexpr (DEG == 4) {
                Jp = *(const uint32_t*)(cj + i * 4);
              } else {
                const uint16_t* c16 = (const uint16_t*)(cj + i * DEG);
                Jp = (uint32_t)c16[0] | ((uint32_t)c16[1] << 16);
                Jp2 = (uint32_t)c16[2];
              }
#pragma unroll
              for (int d = 0; d < DEG; ++d) {
                const uint32_t nib = (xw[d] >> sh) & ((1u << WPT) - 1u);
                if (d < 4) T |= nib << (8 * d);
                else T2 |= nib << (8 * (d - 4));
              }
              Jsum = __builtin_amdgcn_sdot4((int)0x01010101, (int)Jp, __builtin_amdgcn_sdot4((int)0x01010101, (int)Jp2, 0, false), false);
#pragma unroll
              for (int b = 0; b < WPT; ++b) {
                const uint32_t y = (T >> b) & 0x01010101u, y2 = (T2 >> b) & 0x01010101u;
                const int sx = __builtin_amdgcn_sdot4((int)y2, (int)Jp2, __builtin_amdgcn_sdot4((int)y, (int)Jp, 0, false), false);
                const int e = Jsum - 2 * sx;  // dE = 2e
                // e <= 0 is always accepted; else u below the threshold of (T, e)
                const uint32_t th = thr[rowb[b] + (e > 0 ? e : 0)];
                const uint64_t ok = (__builtin_amdgcn_ballot_w64(e <= 0) |
                                     __builtin_amdgcn_ballot_w64(u[b >> 2].w[b & 3] < th)) &
                                    (0ull - (uint64_t)((vmask >> b) & 1u));
                accept_where(ok, 1u << (sh + b), flip, e, acc[b]);
              }
            }
            if (flip) atomicXor(&row[i], flip);  // the bits at their places sh + b
            metro_cnt += __popc(flip);
          }
          if constexpr (JK) qn += (int)__popcll(__builtin_amdgcn_ballot_w64(queued));
        }
        if (cur_q >= 0) flush_energy<JK, WPT>(acc, energy + WPT * cur_q, U.jexp, narrow);
        if constexpr (JK) {
          if (qn > 0)
            exact_pass<DEG, QPT>(lay.exq + 4u * (uint32_t)wave * (2 + 2 * kExactQ), lay.sp, Np, lay.nbr,
                                TL ? nullptr : U.nbr, lay.coup, TL ? nullptr : (const int32_t*)U.coup, lay.tau,
                                lay.beta, lay.bl2e, lay.energy, lay.stats, W, Wq, U.jexp, t, seed, key);
        }
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
      }
      {
        const int tot = wave_sum((int)metro_cnt);
        if (lane == 0 && tot) atomicAdd(&stats[kStatMetroAcc], (unsigned long long)tot);
        metro_cnt = 0;
      }
    }

    // ---------------- steps 2a + 2b: isoenergetic cluster moves ----------------
    // A move's sites are a bitset of nw words.  The spin image switches to its
    // walker-major view first (in-place bit transposes), where walker w's word
    // j holds its spins at sites 32j..32j+31.  Each ICM wave carries P moves
    // in lane groups of lpm lanes (lane li of a group owns words li, li + lpm),
    // and the groups set up their moves side by side: the q-mask word is
    // a-word ^ b-word (replicas differ, the pair's gauge parity applied), then
    // 2a, the seed (idx-th q = -1 site in ascending order, from a group prefix
    // of word popcounts).  Growth: every level expands the frontier of all P
    // clusters at once through the lattice's shift program, restricted to
    // q-mask sites not yet in the cluster, until no group's frontier is left.
    // The bonds that leave the cluster give the energy change (every q = -1
    // neighbour of the cluster is in it, so they are the bonds whose sign
    // changes in replica a), and the cluster words are xor-ed into both
    // walkers' words.  Every walker belongs to one move, so no two lanes touch
    // the same word.  Then the image switches back.
    if (Kc > 0) {
      const int half = R >> 1;
      const int nmoves = Kc * half;
      const int nw = site_words(N);
      const int lpm = icm_lanes_per_move(N), P = 64 / lpm;
      const int iwaves = (icm_slots / P) < 1 ? 1 : ((icm_slots / P) < nwaves ? (icm_slots / P) : nwaves);
      const int sw = slot_words(N);
      const int nterm = lattice_terms(U.topo);
      const int* tshift = (const int*)(lds + lay.terms);
      const uint32_t* tmask = (const uint32_t*)(lds + lay.terms) + kMaxTerms;
      // a build for one layout knows it at compile time and drops the others
      const bool chim = LAY == kLayChimReg || (LAY == kLayAny && U.topo == 2);
      const bool cube8 = LAY == kLayCube8 ||
                         (LAY == kLayAny && DEG == 6 && U.topo == 1 && U.L == 8);  // lpm = 16: one word per lane
      const bool chimreg = LAY == kLayChimReg || (LAY == kLayAny && DEG == 6 && chim && nw <= 64);  // one word per lane
      const bool latreg = LAY == kLayLatReg || (LAY == kLayAny && !chim && !cube8 && nw <= 64);  // periodic lattice, one word per lane
      // (a kLayPair build: chim, cube8, chimreg and latreg are all false)
      const bool sq64 = (LAY == kLayPair && DEG == 4) || (LAY == kLayAny && DEG == 4 && U.topo == 0 && U.L == 64);  // two words per lane
      const bool cube16 = (LAY == kLayPair && DEG == 6) || (LAY == kLayAny && DEG == 6 && U.topo == 1 && U.L == 16);
      const bool pair = sq64 || cube16;
      const bool record = (flags & kFlagRecord) && s + 1 == n_sweeps;
      // the cluster moves are short dependent chains (growth levels, set-up
      // scans): they issue ahead of Metropolis waves sharing the CU
      __builtin_amdgcn_s_setprio(2);
      transpose_image(sp, G, nw, true);
      __syncthreads();
      if (wave < iwaves) {
        const int grp = lane >> (31 - __builtin_clz(lpm)), li = lane & (lpm - 1);  // lpm: 16, 32 or 64
        uint32_t* gsl = (uint32_t*)(lds + lay.slots) + (wave * P + grp) * sw;  // my group's slot
        uint32_t* gmc = gsl + 2 * (nw + 2);
        uint32_t* gaw = gmc + 2 * nw;
        int* ginfo = (int*)(gaw + nw);
        // a wave takes P consecutive moves (neighbouring temperatures, so
        // clusters of like size): its growth and boundary loops run as long as
        // its largest cluster needs, so like sizes waste the fewest rounds
        for (int mbase = wave * P; mbase < nmoves; mbase += iwaves * P) {
          // ---- set-up: every group its own move ----
          const int mv = mbase + grp;
          const bool live = mv < nmoves;
          int a = 0, b = 0;
          uint32_t gx = 0u, um = 0u;
          if (live) {
            // (half is almost always 1 or 2: a shift instead of a division)
            const int k = half == 1 ? mv : (half == 2 ? mv >> 1 : mv / half), p2 = mv - k * half;
            a = at[k * R + 2 * p2];
            b = at[k * R + 2 * p2 + 1];
            gx = (uint32_t)(gauge[a] ^ gauge[b]);
            um = icmu[mv];
          }
          // q_i = -1 <=> the true replicas differ at i; sites past N are zero
          // in both words and are masked out of the parity term
          uint32_t mw[2] = {0u, 0u}, av[2] = {0u, 0u};
          int n = 0;
#pragma unroll
          for (int k2 = 0; k2 < 2; ++k2) {
            const int w = li + lpm * k2;
            if (live && w < nw) {
              const int rem_bits = N - 32 * w;
              const uint32_t valid = rem_bits >= 32 ? ~0u : (1u << rem_bits) - 1u;
              av[k2] = sp[wt_index(a, w, Np)];
              mw[k2] = av[k2] ^ sp[wt_index(b, w, Np)] ^ (gx ? valid : 0u);
              n += __popc(mw[k2]);
            }
          }
          n = group_sum(n, lpm);
          const bool twoa = live && (flags & kFlag2a) && 2 * n > N;
          // step 2a: reverse the second replica (the q-mask complements); the
          // cluster and frontier start empty
#pragma unroll
          for (int k2 = 0; k2 < 2; ++k2) {
            const int w = li + lpm * k2;
            if (w < nw) {
              if (twoa) {
                const int rem_bits = N - 32 * w;
                const uint32_t valid = rem_bits >= 32 ? ~0u : (1u << rem_bits) - 1u;
                mw[k2] = ~mw[k2] & valid;
              }
              gmc[2 * w] = mw[k2];
              gmc[2 * w + 1] = 0;
              gaw[w] = av[k2];
              gsl[1 + w] = 0;
            }
          }
          if (twoa) n = N - n;
          if (li == 0) {
            if (twoa) gauge[b] ^= 1;
            ginfo[kInMv] = live ? mv : -1;
            ginfo[kInA] = a;
            ginfo[kInB] = b;
            ginfo[kInN] = live ? n : 0;
            ginfo[kInSeed] = -1;
            if (live) {
              atomicAdd(&stats[kStatIcmMoves], 1ull);
              if (twoa) atomicAdd(&stats[kStat2a], 1ull);
              if (n > 0) atomicAdd(&stats[kStatIcmNontrivial], 1ull);
            }
          }
          // step 2b: the idx-th q = -1 site in ascending order seeds the
          // cluster, found from a group prefix of the words' popcounts; the
          // lane holding that word marks it (frontier, cluster, the seed)
          {
            int rem = (live && n > 0) ? (int)(((unsigned long long)um * (unsigned long long)n) >> 32) : -1;
#pragma unroll
            for (int k2 = 0; k2 < 2; ++k2) {
              if (lpm * k2 >= nw) break;
              const int w = li + lpm * k2;
              const uint32_t word = w < nw ? mw[k2] : 0u;
              const int c = __popc(word);
              const int excl = group_exclusive_scan(c, lpm);
              const int tot = group_sum(c, lpm);
              if (rem >= 0 && rem < tot) {
                if (rem >= excl && rem < excl + c) {
                  // position of the (rem - excl)-th set bit of the word, by halving
                  int kk = rem - excl, pos = 0;
                  uint32_t x = word;
#pragma unroll
                  for (int h = 16; h >= 1; h >>= 1) {
                    const int ch = __popc(x & ((1u << h) - 1u));
                    const bool up = kk >= ch;
                    kk = up ? kk - ch : kk;
                    x = up ? x >> h : x;
                    pos = up ? pos + h : pos;
                  }
                  const int seedsite = 32 * w + pos;
                  gsl[1 + w] = 1u << pos;
                  gmc[2 * w + 1] = 1u << pos;
                  ginfo[kInSeed] = seedsite;
                }
                rem = -1;
              } else if (rem >= 0) {
                rem -= tot;
              }
            }
          }
          wave_sync();
          if (record)
            record_labels<DEG, TL>(lay.slots, lay.parent, lay.nbr, TL ? nullptr : U.nbr, U.labels, U.seeds, wave, P, sw, nw, N, nmoves);
          // ---- the P clusters grow together, a whole frontier per level ----
          if (cube8) {
            // one word per lane, frontier, mask and cluster kept in registers
            const uint32_t m = gmc[2 * li];
            uint32_t c = gmc[2 * li + 1];
            uint32_t f = c;  // the seed, or nothing
            while (true) {
              const uint32_t fn = cube8_expand(f) & m & ~c;
              c |= fn;
              f = fn;
              if (!__ballot(fn != 0u)) break;
            }
            gmc[2 * li + 1] = c;
            wave_sync();
          }
          if (chimreg) {
            ChimeraStep cs;
            cs.qv = (8 * U.L) >> 5;
            cs.rv = (8 * U.L) & 31;
#pragma unroll
            for (int t = 0; t < 4; ++t) cs.m[t] = li < nw ? tmask[t * nw + li] : 0u;
            const uint32_t m = li < nw ? gmc[2 * li] : 0u;
            uint32_t c = li < nw ? gmc[2 * li + 1] : 0u;
            uint32_t f = c;
            while (true) {
              uint32_t g4[4];
              chimera_inter(f, lane, cs, g4);
              const uint32_t fn = (chimera_in_cell(f) | g4[0] | g4[1] | g4[2] | g4[3]) & m & ~c;
              c |= fn;
              f = fn;
              if (!__ballot(fn != 0u)) break;
            }
            if (li < nw) gmc[2 * li + 1] = c;
            wave_sync();
          }
          if (latreg) {
            uint32_t tm[kMaxTerms];
#pragma unroll
            for (int t = 0; t < kMaxTerms; ++t) tm[t] = (t < nterm && li < nw) ? tmask[t * nw + li] : 0u;
            const uint32_t m = li < nw ? gmc[2 * li] : 0u;
            uint32_t c = li < nw ? gmc[2 * li + 1] : 0u;
            uint32_t f = c;
            while (true) {
              uint32_t gw = 0;
#pragma unroll
              for (int t = 0; t < kMaxTerms; ++t)
                if (t < nterm) gw |= reg_term(f, lane, uniform(tshift[t]), tm[t]);
              const uint32_t fn = gw & m & ~c;
              c |= fn;
              f = fn;
              if (!__ballot(fn != 0u)) break;
            }
            if (li < nw) gmc[2 * li + 1] = c;
            wave_sync();
          }
          if (pair) {
            pair_grow(sq64, (uint32_t)((unsigned char*)gmc - lds), lane);
            wave_sync();
          }
          int cur = 0;
          while (!cube8 && !chimreg && !latreg && !pair) {
            const uint32_t* fc = gsl + 1 + cur * (nw + 2);
            uint32_t* fnx = gsl + 1 + (cur ^ 1) * (nw + 2);
            bool grew = false;
            for (int w = li; w < nw; w += lpm) {
              uint32_t gw = chim ? chimera_in_cell(fc[w]) : 0u;
              for (int t = 0; t < nterm; ++t)
                gw |= shifted_word(fc, w, tshift[t], nw) & tmask[t * nw + w];
              const uint32_t m = gmc[2 * w], c = gmc[2 * w + 1];
              const uint32_t fn = gw & m & ~c;
              fnx[w] = fn;
              if (fn) {
                gmc[2 * w + 1] = c | fn;
                grew = true;
              }
            }
            wave_sync();
            cur ^= 1;
            if (!__ballot(grew)) break;
          }
          // ---- bonds leaving the cluster, then the flips ----
          E_t dEa = 0;
          int ib = 0;  // one word per lane: the lane's boundary sum fits an int
          int csize = 0;
          {
            const int jpl = JK ? 0 : U.jpl;
            const uint32_t* jplw = (const uint32_t*)(lds + lay.jplanes);
            const int jw = min(li, nw - 1);  // lanes past the last word have no bits
            // integer couplings in the register layouts below (at most 64 words)
            // always come with their bit planes: jpl > 0 whenever moves run
            if (cube8) {
              // boundary bonds per direction d: i in the cluster, its d-neighbour
              // not (then outside the q-mask); anti-aligned in replica a where
              // the spin words differ
              const uint32_t cw = gmc[2 * li + 1], awd = gaw[li];
              uint32_t cd[6], ad[6];
              cube8_dirs(cw, cd);
              cube8_dirs(awd, ad);
              csize = __popc(cw);
              uint32_t bb[6], an[6];
#pragma unroll
              for (int d = 0; d < 6; ++d) {
                bb[d] = cw & ~cd[d];
                an[d] = awd ^ ad[d];
              }
#pragma unroll
              for (int d = 0; d < 6; ++d)
                ib += JK ? boundary_sum<1, DEG, TL>(bb[d], an[d], jw, d, cf, cj)
                   : boundary_sum_planes(bb[d], an[d], jplw + (jw * DEG + d) * jpl, jpl);
            }
            if (chimreg) {
              // slots 0-3 in-cell, 4 = row-1 / col-1, 5 = row+1 / col+1
              ChimeraStep cs;
              cs.qv = (8 * U.L) >> 5;
              cs.rv = (8 * U.L) & 31;
#pragma unroll
              for (int t = 0; t < 4; ++t) cs.m[t] = li < nw ? tmask[t * nw + li] : 0u;
              const uint32_t cw = li < nw ? gmc[2 * li + 1] : 0u, awd = li < nw ? gaw[li] : 0u;
              uint32_t ci[4], ai[4];
              chimera_inter(cw, lane, cs, ci);
              chimera_inter(awd, lane, cs, ai);
              csize = __popc(cw);
              uint32_t bbs[6], ans[6];
#pragma unroll
              for (int d = 0; d < 6; ++d) {
                uint32_t nb, na;
                if (d < 4) {
                  nb = chimera_slot(cw, d);
                  na = chimera_slot(awd, d);
                } else if (d == 4) {
                  nb = ci[1] | ci[3];
                  na = ai[1] | ai[3];
                } else {
                  nb = ci[0] | ci[2];
                  na = ai[0] | ai[2];
                }
                const uint32_t exist = d < 4 ? ~0u : (d == 4 ? (cs.m[1] | cs.m[3]) : (cs.m[0] | cs.m[2]));
                bbs[d] = cw & ~nb & exist;
                ans[d] = awd ^ na;
              }
#pragma unroll
              for (int d = 0; d < 6; ++d)
                ib += JK ? boundary_sum<1, DEG, TL>(bbs[d], ans[d], jw, d, cf, cj)
                   : boundary_sum_planes(bbs[d], ans[d], jplw + (jw * DEG + d) * jpl, jpl);
            }
            if (latreg) {
              // slot 2a = +axis a (terms 4a, 4a+1), slot 2a+1 = -axis a (terms 4a+2, 4a+3)
              const uint32_t cw = li < nw ? gmc[2 * li + 1] : 0u, awd = li < nw ? gaw[li] : 0u;
              csize = __popc(cw);
              uint32_t bbs[DEG], ans[DEG];
#pragma unroll
              for (int d = 0; d < DEG; ++d) {
                const int t0 = 2 * d;
                const int s0 = uniform(tshift[t0]), s1 = uniform(tshift[t0 + 1]);
                const uint32_t m0 = li < nw ? tmask[t0 * nw + li] : 0u;
                const uint32_t m1 = li < nw ? tmask[(t0 + 1) * nw + li] : 0u;
                const uint32_t nb = reg_term(cw, lane, s0, m0) | reg_term(cw, lane, s1, m1);
                const uint32_t na = reg_term(awd, lane, s0, m0) | reg_term(awd, lane, s1, m1);
                bbs[d] = cw & ~nb;
                ans[d] = awd ^ na;
              }
#pragma unroll
              for (int d = 0; d < DEG; ++d)
                ib += JK ? boundary_sum<1, DEG, TL>(bbs[d], ans[d], jw, d, cf, cj)
                   : boundary_sum_planes(bbs[d], ans[d], jplw + (jw * DEG + d) * jpl, jpl);
            }
            if (pair) {
              int cs2 = 0;
              dEa = pair_boundary<JK, DEG>(sq64, (uint32_t)((unsigned char*)gmc - lds),
                                           (uint32_t)((const unsigned char*)gaw - lds),
                                           TL ? (uint32_t)((const unsigned char*)cf - lds) : 0u,
                                           TL ? nullptr : U.coup, lane, cs2);
              csize = cs2;
            }
            if (!cube8 && !chimreg && !latreg && !pair) {
              // cluster and replica-a words into the (now free) padded frontier
              // buffers, then boundary bonds slot by slot through the shift program
              uint32_t* pcw = gsl + 1;
              uint32_t* paw = gsl + 1 + (nw + 2);
              for (int w = li; w < nw; w += lpm) {
                pcw[w] = gmc[2 * w + 1];
                paw[w] = gaw[w];
              }
              wave_sync();
              for (int w = li; w < nw; w += lpm) {
                const uint32_t cw = pcw[w], awd = paw[w];
                csize += __popc(cw);
#pragma unroll
                for (int d = 0; d < DEG; ++d) {
                  uint32_t nb, na, exist = ~0u;
                  if (chim && d < 4) {
                    nb = chimera_slot(cw, d);
                    na = chimera_slot(awd, d);
                  } else {
                    // lattice slot 2a / 2a+1: terms 2d, 2d+1; chimera slot 4: rows-1
                    // and cols-1 (terms 1, 3), slot 5: rows+1 and cols+1 (terms 0, 2)
                    const int ta = chim ? (d == 4 ? 1 : 0) : 2 * d;
                    const int tb = chim ? (d == 4 ? 3 : 2) : 2 * d + 1;
                    const int sa = uniform(tshift[ta]), sb = uniform(tshift[tb]);
                    const uint32_t ma = tmask[ta * nw + w], mb = tmask[tb * nw + w];
                    nb = (shifted_word(pcw, w, sa, nw) & ma) | (shifted_word(pcw, w, sb, nw) & mb);
                    na = (shifted_word(paw, w, sa, nw) & ma) | (shifted_word(paw, w, sb, nw) & mb);
                    if (chim) exist = ma | mb;
                  }
                  uint32_t bb = cw & ~nb & exist;
                  const uint32_t anti = awd ^ na;
                  while (bb) {
                    const int bpos = __builtin_ctz(bb);
                    bb &= bb - 1u;
                    const int x = (32 * w + bpos) * DEG + d;
                    if (JK) {
                      const double J = (double)cf[x];
                      dEa += ((anti >> bpos) & 1u) ? -J : J;
                    } else {
                      const int J = cj[x];
                      dEa += ((anti >> bpos) & 1u) ? -J : J;
                    }
                  }
                }
              }
            }
          }
          // the flips: the cluster words into both walkers' words (walker-major view)
          {
            const int ga = ginfo[kInA], gb = ginfo[kInB];
            if (ginfo[kInMv] >= 0 && ginfo[kInN] > 0)
              for (int w = li; w < nw; w += lpm) {
                const uint32_t cwf = gmc[2 * w + 1];
                if (cwf) {
                  sp[wt_index(ga, w, Np)] ^= cwf;
                  sp[wt_index(gb, w, Np)] ^= cwf;
                }
              }
          }
          dEa += (E_t)ib;
          // per-group sums: DPP row sums are 16-lane sums, groups are 1, 2 or 4 rows
          {
            E_t rows[4];
            if (JK) {
              double dv = (double)dEa;
              dv += dpp_d<0xB1>(dv); dv += dpp_d<0x4E>(dv); dv += dpp_d<0x141>(dv); dv += dpp_d<0x140>(dv);
#pragma unroll
              for (int r2 = 0; r2 < 4; ++r2) rows[r2] = (E_t)readlane_d(dv, 16 * r2);
            } else {
              int iv = dpp_row_sum((int)dEa);
#pragma unroll
              for (int r2 = 0; r2 < 4; ++r2) rows[r2] = (E_t)__builtin_amdgcn_readlane(iv, 16 * r2);
            }
            const int sites = wave_sum(csize);
            if (lane < P) {
              // lane g updates the two walkers of move g (distinct walkers)
              const int g = lane, rpg = 4 / P;  // DPP rows per group
              const int* inf = (const int*)((uint32_t*)(lds + lay.slots) + (wave * P + g) * sw +
                                            2 * (nw + 2) + 3 * nw);
              E_t sum = 0;
#pragma unroll
              for (int r2 = 0; r2 < 4; ++r2)
                if (r2 / rpg == g) sum += rows[r2];
              if (inf[kInMv] >= 0 && inf[kInN] != 0) {
                // float couplings: sums in units of 2^-jexp (exact scaling)
                if (JK) sum = (E_t)ldexp((double)sum, -U.jexp);
                energy[inf[kInA]] += (E_t)2 * sum;
                energy[inf[kInB]] -= (E_t)2 * sum;
              }
            }
            if (lane == 0 && sites) atomicAdd(&stats[kStatIcmSites], (unsigned long long)sites);
          }
          wave_sync();
        }
      }
      __syncthreads();
      transpose_image(sp, G, nw, false);
      __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();

    // ---------------- step 3: parallel tempering ---------------------------------
    if (flags & kFlagPt) {
      if (K >= kPtTableMin && K <= kPtTable) {
        // Every decision a chain's scan can meet is known up front: at rung k
        // the carried walker is one that sat at some rung c <= k before the
        // step, and energies do not change during PT.  All threads decide the
        // K (K - 1) / 2 pairs (k, c) of every chain; bit c of word (k, r) is
        // set on a swap.  Lane r of wave 0 then scans chain r testing bits.
        uint32_t* ptacc = (uint32_t*)(lds + lay.ptacc);
        pt_decide<JK>((uint32_t)((unsigned char*)at - lds), (uint32_t)((unsigned char*)energy - lds), lay.ptu,
                      lay.ptacc, lay.beta, lay.dbl2e, U.ptthr, U.ptlen, K, R);
        __syncthreads();
        if (wave == 0) {
          const int r = phase_lane();
          int acc_pt = 0;
          __builtin_amdgcn_s_setprio(3);
          if (r < R) {
            // rung k keeps the walker from k + 1 on a swap (the carried one
            // climbs on), else the carried one (and the walker from k + 1,
            // which sat at rung c = k + 1, is carried)
            int x = at[r], c = 0;
            int yn = at[R + r];
            uint32_t bn = ptacc[r];
            for (int k = 0; k + 1 < K; ++k) {
              const int y = yn;
              const uint32_t bits = bn;
              if (k + 2 < K) {
                yn = at[(k + 2) * R + r];
                bn = ptacc[(k + 1) * R + r];
              }
              const bool swap = (bits >> c) & 1u;
              const int stay = swap ? y : x;
              at[k * R + r] = stay;
              tau[stay] = k;
              if (!swap) {
                x = y;
                c = k + 1;
              }
              acc_pt += swap ? 1 : 0;
            }
            at[(K - 1) * R + r] = x;
            tau[x] = K - 1;
          }
          const int tot = wave_sum(acc_pt);
          if (lane == 0) {
            stats[kStatPtAttempts] += (unsigned long long)(K - 1) * R;
            stats[kStatPtAccepts] += (unsigned long long)tot;
          }
          __builtin_amdgcn_s_setprio(0);
        }
      } else {
        // Long ladders: lane r scans chain r up the ladder.  Rung k only ever
        // meets the walker carried up from rung k - 1 (or the one that sat at
        // k) and the walker still sitting at k + 1, so the carried walker and
        // its energy stay in registers, rung k is final once decided, and the
        // next rung's walker, energy and draw are read ahead.
        if (wave == 0) {
          const int r = phase_lane();
          int acc_pt = 0;
          __builtin_amdgcn_s_setprio(3);  // one serial chain: first in line on its SIMD
          if (r < R && K > 1) {
            // two rungs of read-ahead: the walker at k + 3 and the energy of the
            // walker at k + 2 are fetched while rung k is decided
            int x = at[r];
            E_t ex = energy[x];
            int yn = at[R + r];
            E_t eyn = energy[yn];
            uint32_t un = ptu[r];
            int ynn = K > 2 ? at[2 * R + r] : 0;
            for (int k = 0; k + 1 < K; ++k) {
              const int y = yn;
              const E_t ey = eyn;
              const uint32_t u = un;
              if (k + 2 < K) {
                yn = ynn;
                eyn = energy[ynn];
                un = ptu[(k + 1) * R + r];
                if (k + 3 < K) ynn = at[(k + 3) * R + r];
              }
              const bool accept = pt_swap<JK>(u, ex, ey, k, beta, dbl2e, U.ptthr, U.ptlen);
              // rung k keeps y on a swap (x climbs on), else x (and y is carried)
              const int stay = accept ? y : x;
              at[k * R + r] = stay;
              tau[stay] = k;
              if (!accept) {
                x = y;
                ex = ey;
              }
              acc_pt += accept ? 1 : 0;
            }
            at[(K - 1) * R + r] = x;
            tau[x] = K - 1;
          }
          const int tot = wave_sum(acc_pt);
          if (lane == 0) {
            stats[kStatPtAttempts] += (unsigned long long)(K - 1) * R;
            stats[kStatPtAccepts] += (unsigned long long)tot;
          }
          __builtin_amdgcn_s_setprio(0);
        }
      }
      __syncthreads();
    }

    // ---------------- observables (out of line, only when measured) ---------------
    if (flags & kFlagMeasure) {
      measure_step<JK, DEG>(t + 1u, N, K, R, U.topo, U.L, (uint32_t)((unsigned char*)sp - lds),
                            (uint32_t)((unsigned char*)at - lds), (uint32_t)((unsigned char*)energy - lds),
                            lay.meas, TL ? (uint32_t)((const unsigned char*)nbr - lds) : 0u,
                            TL ? nullptr : U.nbr, U.obs);
      __syncthreads();
    }
  }

  // ---- store the unit back (bit-packed -> int8 quad words) ----
  __syncthreads();
  for (int x = tid; x < Wq * N; x += nthr) {
    const int q = x / N, i = x - q * N;
    const uint32_t nib = (sp[(q >> 3) * Np + i] >> (4 * (q & 7))) & 0xFu;
    uint32_t w = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) w |= (((nib >> b) & 1u) ? 0xFFu : 0x01u) << (8 * b);
    U.spins[x] = w;
  }
  for (int x = tid; x < Wp; x += nthr) {
    U.tau[x] = tau[x];
    U.gauge[x] = (uint8_t)gauge[x];
    if (JK) U.energy[x] = (int64_t)((double)energy[x] * 0x1p40);
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
// slot sum is halved (exact: integer, or float couplings on their 2^-jexp grid summed
// as int64 after scaling).  grid: (Wp), block 256.
template <int JK>
__global__ void energy_kernel(const uint32_t* spins, const uint16_t* nbr, const void* coup, int N,
                              int deg, int jexp, int64_t* energy) {
  const int w = blockIdx.x, q = w >> 2, b = w & 3;
  __shared__ long long part[256];
  long long acc = 0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const int si = spin_of(spins[(size_t)q * N + i], b);
    for (int d = 0; d < deg; ++d) {
      const int j = nbr[i * deg + d];
      const int sj = spin_of(spins[(size_t)q * N + j], b);
      long long Jraw;
      if (JK) Jraw = (long long)((const int32_t*)coup)[i * deg + d] << (40 - jexp);
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


// ----------------------------------------------------------------------------
// Overlaps of the replica pairs (paper, "Benchmark model and observables":
// the spin overlap q = (1/N) sum_i q_i and the link overlap of Eq. 1,
// q_l = (1/N_b) sum over bonds of q_i q_j, with q_i = s_i^(a) s_i^(b) for the
// two replicas of a pair).  For each temperature k and pair p (chains 2p,
// 2p+1): out_q = sum_i q_i, out_ql = sum over bonds of q_i q_j.  Stored spins
// of a reversed walker (gauge bit) are the negation of its true spins; q_i
// takes the gauge parity of the two walkers, q_i q_j does not depend on it.
// Each bond is counted once: lattices from the slots of the +axis steps
// (even slots), chimera in-cell bonds from the u < 4 side (slots 0-3) and
// inter-cell bonds from the next row / column (slot 5, absent where it
// points back at the site).  grid: (K * R/2), block 256 (four waves).
// ----------------------------------------------------------------------------
template <int DEG>
__global__ void __launch_bounds__(256) overlap_kernel(const uint32_t* __restrict__ spins,
                                                      const uint16_t* __restrict__ nbr,
                                                      const int32_t* __restrict__ at,
                                                      const uint8_t* __restrict__ gauge, int N, int R,
                                                      int topo, int n_bonds, int32_t* out_q,
                                                      int32_t* out_ql) {
  __shared__ int part[2][4];
  const int half = R >> 1, x = blockIdx.x, k = x / half, p = x - k * half;
  const int a = at[k * R + 2 * p], b = at[k * R + 2 * p + 1];
  const uint32_t* wa = spins + (size_t)(a >> 2) * N;
  const uint32_t* wb = spins + (size_t)(b >> 2) * N;
  const int sa = 8 * (a & 3), sb = 8 * (b & 3);
  // q_i as a bit: 1 where the stored spins differ (byte 0xFF = down, 0x01 = up)
  auto qbit = [&](int i) { return ((wa[i] >> sa) ^ (wb[i] >> sb)) & 0x80u; };
  int nd = 0, dl = 0;  // differing sites; bonds whose ends differ in q
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const uint32_t qi = qbit(i);
    nd += qi ? 1 : 0;
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
      const int j = nbr[i * DEG + d];
      const bool bond = topo == 2 ? (((i & 7) < 4 && d < 4) || (d == 5 && j != i)) : (d & 1) == 0;
      if (bond) dl += (qi != qbit(j)) ? 1 : 0;
    }
  }
  nd = wave_sum(nd);
  dl = wave_sum(dl);
  if (lane_id() == 0) {
    part[0][threadIdx.x >> 6] = nd;
    part[1][threadIdx.x >> 6] = dl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int n = part[0][0] + part[0][1] + part[0][2] + part[0][3];
    const int D = part[1][0] + part[1][1] + part[1][2] + part[1][3];
    const int sign = (gauge[a] ^ gauge[b]) ? -1 : 1;
    out_q[x] = sign * (N - 2 * n);
    out_ql[x] = n_bonds - 2 * D;  // sum over bonds of q_i q_j
  }
}

}  // namespace icm

// ----------------------------------------------------------------------------
// launch wrappers used by the host runtime
// ----------------------------------------------------------------------------
extern "C" {

int icmk_launch_sweep(const icm::UnitDesc* d_units, int n_units, int jkind, int deg, int tables, int layout,
                      uint32_t n_sweeps, int threads, int icm_slots, size_t lds_bytes,
                      hipStream_t stream) {
  if (n_units <= 0) return 0;
  dim3 grid(n_units), block(threads);
#define ICM_LAUNCH(JK, DEG, TL, LAY)                                                            \
  hipLaunchKernelGGL((icm::sweep_block_kernel<JK, DEG, TL, LAY>), grid, block, lds_bytes, stream, \
                     d_units, n_sweeps, icm_slots)
  // the one-word layout builds exist with tables in LDS (what those units
  // use); the two-word one with the tables in either place
  const int lay = (tables || layout == icm::kLayPair) ? layout : icm::kLayAny;
  const int sel = (jkind ? 4 : 0) + (deg == 6 ? 2 : 0) + (tables ? 1 : 0);
  if (lay == icm::kLayCube8 && deg == 6) {
    if (jkind) ICM_LAUNCH(1, 6, 1, icm::kLayCube8);
    else ICM_LAUNCH(0, 6, 1, icm::kLayCube8);
  } else if (lay == icm::kLayChimReg && deg == 6) {
    if (jkind) ICM_LAUNCH(1, 6, 1, icm::kLayChimReg);
    else ICM_LAUNCH(0, 6, 1, icm::kLayChimReg);
  } else if (lay == icm::kLayPair && (deg == 4 || deg == 6)) {
    const int ps = (jkind ? 4 : 0) + (deg == 6 ? 2 : 0) + (tables ? 1 : 0);
    switch (ps) {
      case 0: ICM_LAUNCH(0, 4, 0, icm::kLayPair); break;
      case 1: ICM_LAUNCH(0, 4, 1, icm::kLayPair); break;
      case 2: ICM_LAUNCH(0, 6, 0, icm::kLayPair); break;
      case 3: ICM_LAUNCH(0, 6, 1, icm::kLayPair); break;
      case 4: ICM_LAUNCH(1, 4, 0, icm::kLayPair); break;
      case 5: ICM_LAUNCH(1, 4, 1, icm::kLayPair); break;
      case 6: ICM_LAUNCH(1, 6, 0, icm::kLayPair); break;
      default: ICM_LAUNCH(1, 6, 1, icm::kLayPair); break;
    }
  } else if (lay == icm::kLayLatReg && (deg == 4 || deg == 6)) {
    if (jkind && deg == 6) ICM_LAUNCH(1, 6, 1, icm::kLayLatReg);
    else if (jkind) ICM_LAUNCH(1, 4, 1, icm::kLayLatReg);
    else if (deg == 6) ICM_LAUNCH(0, 6, 1, icm::kLayLatReg);
    else ICM_LAUNCH(0, 4, 1, icm::kLayLatReg);
  } else {
    switch (sel) {
      case 0: ICM_LAUNCH(0, 4, 0, icm::kLayAny); break;
      case 1: ICM_LAUNCH(0, 4, 1, icm::kLayAny); break;
      case 2: ICM_LAUNCH(0, 6, 0, icm::kLayAny); break;
      case 3: ICM_LAUNCH(0, 6, 1, icm::kLayAny); break;
      case 4: ICM_LAUNCH(1, 4, 0, icm::kLayAny); break;
      case 5: ICM_LAUNCH(1, 4, 1, icm::kLayAny); break;
      case 6: ICM_LAUNCH(1, 6, 0, icm::kLayAny); break;
      case 7: ICM_LAUNCH(1, 6, 1, icm::kLayAny); break;
      default: return (int)hipErrorInvalidValue;
    }
  }
#undef ICM_LAUNCH
  if (deg != 4 && deg != 6) return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

int icmk_set_lds_limit(size_t bytes) {
  hipError_t e = hipSuccess;
  using namespace icm;
  const void* fns[24] = {
      (const void*)sweep_block_kernel<0, 4, 0, kLayAny>, (const void*)sweep_block_kernel<0, 4, 1, kLayAny>,
      (const void*)sweep_block_kernel<0, 6, 0, kLayAny>, (const void*)sweep_block_kernel<0, 6, 1, kLayAny>,
      (const void*)sweep_block_kernel<1, 4, 0, kLayAny>, (const void*)sweep_block_kernel<1, 4, 1, kLayAny>,
      (const void*)sweep_block_kernel<1, 6, 0, kLayAny>, (const void*)sweep_block_kernel<1, 6, 1, kLayAny>,
      (const void*)sweep_block_kernel<0, 6, 1, kLayCube8>, (const void*)sweep_block_kernel<1, 6, 1, kLayCube8>,
      (const void*)sweep_block_kernel<0, 6, 1, kLayChimReg>, (const void*)sweep_block_kernel<1, 6, 1, kLayChimReg>,
      (const void*)sweep_block_kernel<0, 4, 1, kLayLatReg>, (const void*)sweep_block_kernel<1, 4, 1, kLayLatReg>,
      (const void*)sweep_block_kernel<0, 6, 1, kLayLatReg>, (const void*)sweep_block_kernel<1, 6, 1, kLayLatReg>,
      (const void*)sweep_block_kernel<0, 4, 0, kLayPair>, (const void*)sweep_block_kernel<0, 4, 1, kLayPair>,
      (const void*)sweep_block_kernel<0, 6, 0, kLayPair>, (const void*)sweep_block_kernel<0, 6, 1, kLayPair>,
      (const void*)sweep_block_kernel<1, 4, 0, kLayPair>, (const void*)sweep_block_kernel<1, 4, 1, kLayPair>,
      (const void*)sweep_block_kernel<1, 6, 0, kLayPair>, (const void*)sweep_block_kernel<1, 6, 1, kLayPair>};
  for (int x = 0; x < 24; ++x) {
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


int icmk_launch_overlaps(const uint32_t* spins, const uint16_t* nbr, const int32_t* at, const uint8_t* gauge,
                         int N, int deg, int K, int R, int topo, int n_bonds, int32_t* out_q,
                         int32_t* out_ql, hipStream_t stream) {
  const int n = K * (R / 2);
  if (n <= 0) return 0;
  if (deg == 6)
    hipLaunchKernelGGL(icm::overlap_kernel<6>, dim3(n), dim3(256), 0, stream, spins, nbr, at, gauge, N, R, topo,
                       n_bonds, out_q, out_ql);
  else if (deg == 4)
    hipLaunchKernelGGL(icm::overlap_kernel<4>, dim3(n), dim3(256), 0, stream, spins, nbr, at, gauge, N, R, topo,
                       n_bonds, out_q, out_ql);
  else
    return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

int icmk_launch_energy(const uint32_t* spins, const uint16_t* nbr, const void* coup, int N, int deg,
                       int Wp, int jkind, int jexp, int64_t* energy, hipStream_t stream) {
  if (jkind)
    hipLaunchKernelGGL(icm::energy_kernel<1>, dim3(Wp), dim3(256), 0, stream, spins, nbr, coup, N,
                       deg, jexp, energy);
  else
    hipLaunchKernelGGL(icm::energy_kernel<0>, dim3(Wp), dim3(256), 0, stream, spins, nbr, coup, N,
                       deg, jexp, energy);
  return (int)hipGetLastError();
}

}  // extern "C"
