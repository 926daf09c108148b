// Internal layout shared by the host runtime (icm_runtime.cpp) and the HIP
// kernels (icm_kernels.hip).  Not part of the public ABI.
#pragma once
#include <stdint.h>

#ifndef __HIPCC__
#define ICM_HD inline
#else
#define ICM_HD __host__ __device__ inline
#endif

namespace icm {

constexpr int kMaxDeg = 6;        // neighbour slots per site (2D uses 4)
constexpr int kMaxPercSites = 16384;  // site percolation: parent + size arrays in LDS
constexpr int kMaxSites = 4096;   // an ICM lane holds at most two 32-site words of a move
constexpr int kMaxTemps = 256;
constexpr int kMaxReplicas = 64;

// Per-instance statistics block in device memory (u64 counters).
enum StatSlot {
  kStatSweeps = 0,
  kStatMetroAcc,
  kStatIcmMoves,
  kStatIcmNontrivial,
  kStatIcmSites,
  kStat2a,
  kStatPtAttempts,
  kStatPtAccepts,
  kNumStats
};

// One work unit (a whole instance) as the fused kernel sees it.  All pointers
// are device addresses inside the caller's arena.
struct UnitDesc {
  uint32_t* spins;          // [Wq][N] words; byte b of word (q, i) = walker 4q+b at site i
  const uint16_t* nbr;      // [N][deg] neighbour sites (missing chimera slots: i itself)
  const uint16_t* clist;    // [2][Nc] sites of colour 0, then colour 1
  const void* coup;         // [N][deg] int8 j, or int32 J 2^jexp (float couplings rounded to the
                            // grid 2^-jexp, 24-bit signed), slot-aligned with nbr
  const uint32_t* thr;      // int kinds: [K][HM] Metropolis thresholds, index e = s*h
  const double* beta;       // [K] 1/T_k
  const float* bl2e;        // [K] float(beta_k * log2(e)) for the fast acceptance filter
  const uint32_t* ptthr;    // int kinds: [K-1][ptlen] PT thresholds for gap D = 1..ptlen
  int32_t* tau;             // [Wp] temperature of walker (K for padding walkers)
  int32_t* at;              // [K][R] walker at temperature k in chain r
  uint8_t* gauge;           // [Wp] 1 = stored spins are the reversal of the true ones
  int64_t* energy;          // [Wp] raw energies (1/j_scale, or 2^-40 for float couplings)
  unsigned long long* stats;// [kNumStats]
  int32_t* labels;          // [Kc][R/2][N] (RECORD_LABELS only)
  int32_t* seeds;           // [Kc][R/2] seed site, then [Kc][R/2] n_minus
  int64_t* obs;             // MEASURE only: [32][K][R/2][4] observable sums, then [32] counts
  uint32_t* sweep;          // sweep counter t
  int32_t N, Nc, deg, W, Wq, K, R, Kc, HM, ptlen, jkind, jscale;
  uint32_t flags, seed, key;
  int32_t topo, L;          // lattice kind (ICM_TOPO_*) and side / cells per side
  int32_t jexp;             // float couplings: grid exponent (J = coup 2^-jexp)
  int32_t jpl;              // int8 couplings with cluster moves held in registers: bit planes of J
                            // (two's complement width of the couplings), else 0
};

constexpr uint32_t kFlag2a = 1, kFlagPt = 2, kFlagRecord = 4, kFlagSkipMetro = 8, kFlagMeasure = 16;
constexpr int kObsBins = 32, kObsFields = 4;

ICM_HD uint32_t align16(uint32_t x) { return (x + 15u) & ~15u; }

// Byte offsets of the regions of the fused kernel's LDS image of one unit.
// Spins are bit-packed in LDS: word (g, i) holds walkers 32g..32g+31 at site i,
// bit set = spin down, in rows of 32 site_words(N) words per group g (the
// sites past N are zero), so that the image transposes in place into its
// walker-major view by 32 x 32 blocks.
struct LdsLayout {
  uint32_t sp, nbr, clist, coup, tau, at, gauge, energy, thr, beta, bl2e, dbl2e, ptu, ptacc, icmu, terms, jplanes,
      slots, parent, meas, exq, stats, total;
};

// Neighbour relation of the lattice as bit shifts of a site bitset (for the
// cluster search): term t adds F[i + shift_t] to site i where bit i of mask_t
// is set.  2D: 8 terms, 3D: 12 (per axis: +1 step, its periodic wrap, -1 step,
// its wrap); chimera: 4 inter-cell terms, the in-cell K4,4 handled apart.
constexpr int kMaxTerms = 12;

ICM_HD int site_words(int N) { return (N + 31) / 32; }

// Lanes that share one ICM move (a power of two >= its bitset words, 16..64).
ICM_HD int icm_lanes_per_move(int N) {
  const int nw = site_words(N);
  return nw <= 16 ? 16 : (nw <= 32 ? 32 : 64);
}

// Per ICM move slot: two frontier buffers with a zero word on each side,
// the q-mask and cluster words interleaved, replica a's spin words, the move.
enum SlotInfo { kInMv = 0, kInA, kInB, kInN, kInSeed, kInInts = 8 };
ICM_HD int slot_words(int N) { return 2 * (site_words(N) + 2) + 3 * site_words(N) + kInInts; }
ICM_HD int slots_reserved(int N, int slots) {
  const int p = 64 / icm_lanes_per_move(N);
  return slots > p ? slots : p;
}

ICM_HD int bit_words(int Wq) { return (4 * Wq + 31) / 32; }

// Bit planes kept for int8 couplings j in [jmin, jmax]: the two's complement
// width, when cluster moves run with their bitsets in registers (at most 64
// words, one per lane); 0 otherwise.
ICM_HD int coupling_planes(int jkind, int Kc, int N, int jmin, int jmax) {
  if (jkind != 0 || Kc <= 0 || site_words(N) > 64) return 0;
  int p = 1;
  while (jmin < -(1 << (p - 1)) || jmax > (1 << (p - 1)) - 1) ++p;
  return p;
}

// Float couplings: Metropolis decisions the float estimate cannot make are
// queued per wave (site | quad-pair index << 16, the estimate's flip bits) and
// made exactly at the end of the colour; a wave's queue holds kExactQ tasks
// and is emptied early when a task could fill it.
constexpr int kExactQ = 96;
// a float Metropolis call this close (units in the last place of float(u)
// against the float estimate) is made again exactly
constexpr uint32_t kCloseUlps = 512;

// Cluster-move layouts a sweep kernel can be built for: kLayAny picks the
// layout per unit at run time; kLayCube8 (periodic 8^3 lattice, one bitset
// word per lane), kLayChimReg (chimera of at most 64 words, one word per lane),
// kLayLatReg (any other periodic lattice of at most 64 words, one word per
// lane, grown through the shift program) and kLayPair (2D L=64 and 3D L=16,
// two words per lane) carry only that layout's code, which frees the
// registers the other layouts' code would hold.  A launch takes a specialised
// build when every unit in it has that layout.
enum : int { kLayAny = 0, kLayCube8 = 1, kLayChimReg = 2, kLayLatReg = 3, kLayPair = 4 };
ICM_HD int unit_layout(int topo, int L, int deg, int N) {
  if (deg == 6 && topo == 1 && L == 8) return kLayCube8;
  if (deg == 6 && topo == 2 && site_words(N) <= 64) return kLayChimReg;
  if (topo != 2 && site_words(N) <= 64) return kLayLatReg;
  if ((deg == 4 && topo == 0 && L == 64) || (deg == 6 && topo == 1 && L == 16)) return kLayPair;
  return kLayAny;
}

// PT ladders of kPtTableMin to kPtTable temperatures decide every swap a
// chain's scan could meet up front, in parallel: word (k, r) bit c = whether
// the walker that sat at rung c, carried up to rung k, swaps with the walker at
// rung k + 1.  The scan itself then only tests bits.  Shorter ladders scan
// directly (the K (K - 1) / 2 decisions and the extra barrier do not pay for
// themselves there: measured slower at 20 temperatures, faster at 24 and 30).
constexpr int kPtTable = 33, kPtTableMin = 22;
ICM_HD int exact_queue_words(int jkind, int waves) { return jkind ? waves * (2 + 2 * kExactQ) : 0; }

// tables = 1: neighbour table, colour lists and couplings are copied into LDS;
// tables = 0: they are read from global memory (for units too large otherwise).
// jpl: bit planes of the int8 couplings kept for the cluster moves' boundary
// sums (word [(w deg + d) jpl + k] = bit k of J over the 32 sites of word w,
// slot d), 0 for none.
ICM_HD LdsLayout lds_layout(int N, int deg, int Wq, int K, int R, int HM, int jkind, int slots,
                            int tables, int extras, int Kc, int jpl, int waves) {
  // extras: bit 0 = ICM labels recorded, bit 1 = observables measured
  const int record = extras & 1, measure = extras & 2;
  LdsLayout L{};
  uint32_t o = 0;
  const int Wp = 4 * Wq;
  const uint32_t tn = tables ? (uint32_t)N : 0u;
  const uint32_t ns = Kc > 0 ? (uint32_t)slots_reserved(N, slots) : 0u;
  L.sp = o;      o = align16(o + 4u * bit_words(Wq) * 32u * site_words(N));  // rows padded to whole words
  L.nbr = o;     o = align16(o + 2u * tn * deg);
  L.clist = o;   o = align16(o + 2u * tn);
  L.coup = o;    o = align16(o + (jkind ? 4u : 1u) * tn * deg);
  L.tau = o;     o = align16(o + 4u * Wp);
  L.at = o;      o = align16(o + 4u * K * R);
  L.gauge = o;   o = align16(o + 4u * Wp);
  L.energy = o;  o = align16(o + 8u * Wp);
  L.thr = o;     o = align16(o + (jkind ? 0u : 4u * K * HM));
  L.beta = o;    o = align16(o + 8u * K);
  L.bl2e = o;    o = align16(o + 4u * K);
  L.dbl2e = o;   o = align16(o + 4u * K);   // float((beta_k - beta_k+1) log2 e), PT filter
  L.ptu = o;     o = align16(o + 4u * (K > 1 ? K - 1 : 1) * R);
  L.ptacc = o;   o = align16(o + (K >= kPtTableMin && K <= kPtTable ? 4u * (K - 1) * R : 0u));
  L.icmu = o;    o = align16(o + 4u * (Kc > 0 ? Kc * (R / 2) : 1));
  L.terms = o;   o = align16(o + (Kc > 0 ? 4u * kMaxTerms * (1 + site_words(N)) : 0u));
  L.jplanes = o; o = align16(o + 4u * (uint32_t)jpl * deg * site_words(N));
  L.slots = o;   o = align16(o + 4u * slot_words(N) * ns);
  L.parent = o;  o = align16(o + (record ? 4u * N * ns : 0u));
  L.meas = o;    o = align16(o + (measure ? 4u * site_words(N) * 16u : 0u));  // q-mask words per wave
  L.exq = o;     o = align16(o + 4u * (uint32_t)exact_queue_words(jkind, waves));
  L.stats = o;   o = align16(o + 8u * kNumStats);
  L.total = o;
  return L;
}

}  // namespace icm
