/*
 * CPU ORACLE for parallel tempering + isoenergetic cluster moves (ICM) on Ising
 * spin glasses (Zhu, Ochoa, Katzgraber, "Efficient Cluster Algorithm for Spin
 * Glasses in Any Space Dimension", arXiv:1501.05630).
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.  Only tests/,
 * __graft_entry__.smoke() and bench.py's cpu_baseline leg may load it.  It
 * shares no code, header, table or constant generator with the HIP library
 * (paper_1501_05630_amd/csrc); both sides are written from the paper and from
 * the published definition of Philox4x32-10 (Salmon et al., SC'11).
 *
 * The oracle is deliberately plain: walker-major int8 spins, explicit
 * adjacency lists, one attempt at a time, BFS for clusters, exact integer
 * energies.  Every convention it follows is listed in the comments of
 * oracle.cpp next to the paper passage it implements.
 *
 * Walkers: w = h*R + r  (h = home temperature index, r = chain).  Readout is in
 * temperature order [k][r] through the current temperature labels.
 */
#ifndef ICM_ORACLE_H
#define ICM_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_SQUARE2D = 0, ORC_CUBIC3D = 1, ORC_CHIMERA = 2, ORC_EXPLICIT = 3 };
enum { ORC_J_INT8 = 0, ORC_J_F32 = 1 };
/* ORC_FLAG_SKIP_METRO: diagnostic mode, a step is ICM (+PT) only.
   ORC_FLAG_MEASURE: after every step, accumulate the observables of the
   "Benchmark model and observables" paragraph per temperature and replica
   pair into logarithmic time bins (orc_get_observables). */
enum { ORC_FLAG_2A = 1, ORC_FLAG_PT = 2, ORC_FLAG_SKIP_METRO = 8, ORC_FLAG_MEASURE = 16 };
enum { ORC_OBS_BINS = 32, ORC_OBS_FIELDS = 4 };

typedef struct {
  int32_t topology;    /* ORC_SQUARE2D / ORC_CUBIC3D / ORC_CHIMERA / ORC_EXPLICIT */
  int32_t L;           /* lattice side, or chimera cells per side */
  /* ORC_EXPLICIT only: n_sites, n_edges edges (i,j) pairs, per-edge couplings,
     per-site colour (a proper 2-colouring).  Parallel edges are allowed. */
  int32_t n_sites;
  int32_t n_edges;
  const int32_t* edges;
  const int32_t* colours;
  int32_t jkind;       /* ORC_J_INT8 (J = j / j_scale) or ORC_J_F32 */
  int32_t j_scale;
  const void* couplings; /* int8 or float; canonical layout (see oracle.cpp) */
  int32_t n_temps;
  const double* temps; /* strictly ascending, > 0 */
  int32_t n_replicas;  /* even, >= 2 */
  int32_t icm_ntemps;  /* ICM on the coldest icm_ntemps temperatures */
  uint32_t flags;      /* ORC_FLAG_2A | ORC_FLAG_PT */
  uint32_t seed;       /* Philox key word 0 */
  uint32_t instance_key; /* Philox key word 1 */
} orc_params;

typedef struct {
  uint64_t metro_accepts;
  uint64_t icm_moves;
  uint64_t icm_nontrivial;
  uint64_t icm_cluster_sites;
  uint64_t icm_2a_flips;
  uint64_t pt_attempts;
  uint64_t pt_accepts;
} orc_stats;

typedef struct orc_sim orc_sim;

/* Philox4x32-10: out = bijection(ctr) under key. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Returns 0 on success, <0 on invalid parameters. */
int orc_create(const orc_params* p, orc_sim** out);
void orc_destroy(orc_sim* s);

int32_t orc_n_sites(const orc_sim* s);
int32_t orc_n_bonds(const orc_sim* s);
/* Neighbour list of site i (with multiplicity); returns the degree. */
int32_t orc_neighbours(const orc_sim* s, int32_t i, int32_t* out, int32_t cap);
int32_t orc_colour(const orc_sim* s, int32_t i);

/* Hot start: every walker draws its spins from Philox (INIT stream); the
   sweep counter is set to 0. */
void orc_init_hot(orc_sim* s);
/* spins [K][R][N] in temperature order; walker (k,r) gets temperature k. */
void orc_set_states(orc_sim* s, const int8_t* spins, uint32_t sweep0);
/* Runs n simulation steps (sweep, ICM, PT). */
void orc_run(orc_sim* s, uint32_t n_sweeps);
/* Same, recording the energies [K][R] (temperature order) after every step
   into trace [n_sweeps][K][R]. */
void orc_run_trace(orc_sim* s, uint32_t n_sweeps, int64_t* trace);

void orc_get_states(const orc_sim* s, int8_t* out /* [K][R][N] */);
void orc_get_energies(const orc_sim* s, int64_t* raw /* [K][R] */);
/* walker index currently holding temperature k in chain r, [K][R]. */
void orc_get_walkers(const orc_sim* s, int32_t* out);
uint32_t orc_get_sweep(const orc_sim* s);
void orc_get_stats(const orc_sim* s, orc_stats* out);
/* Labels of the last ICM move at temperature k, pair p (during the last sweep
   run): label = minimum site index of the q=-1 component, -1 off the mask.
   n_minus is the post-2a count; seed is -1 when n_minus == 0. Returns 0, or -1
   if (k,p) has no ICM. */
int orc_get_labels(const orc_sim* s, int32_t k, int32_t p, int32_t* labels,
                   int32_t* seed, int32_t* n_minus);

/* Energy (raw units: 1/j_scale for INT8; 2^-40 for F32, whose couplings are
   kept exactly as multiples of 2^-40) of one spin configuration [N]. */
int64_t orc_energy(const orc_sim* s, const int8_t* spins);
/* The coupling of each bond as the oracle stores it, raw units, [n_bonds],
   with the endpoints in bonds_ij [n_bonds][2]. */
void orc_bonds(const orc_sim* s, int32_t* bonds_ij, int64_t* j_raw);
/* Observable sums [ORC_OBS_BINS][K][R/2][ORC_OBS_FIELDS] and sample counts
   [ORC_OBS_BINS], accumulated since the last orc_init_hot / orc_set_states.  A step that ends at sweep count t (t = 1, 2, ...) lands in
   bin floor(log2 t).  Fields per pair of chains (2p, 2p+1) at temperature k:
   0: E_a + E_b (units of 1/j_scale for integer couplings; for float
   couplings the bin's exact sum rounded to a multiple of 2^-20, exact when
   every energy is one), 1: sum over bonds of q_i q_j = N_b - 2 D
   (D = bonds whose ends have different site overlaps q_i = s_a,i s_b,i),
   2: (sum_i q_i)^2, 3: min(n, N - n) for n sites with q_i = -1 (the potential
   cluster sites after step 2a). */
void orc_get_observables(const orc_sim* s, int64_t* sums, int64_t* counts);

/* Replaces the K temperatures (finite, > 0, strictly ascending); everything
   else carries on.  Returns 0, or -1 on invalid temperatures. */
int orc_set_temperatures(orc_sim* s, const double* temps);

/* Site percolation on this simulation's graph: for samples n = sample0 ..
   sample0 + n_samples - 1, site i is occupied iff word i mod 4 of
   Philox4x32-10 with counter (n, i / 4, 0, 4) and key (seed, instance_key)
   is below floor(p 2^32); out[n - sample0] = size of the largest connected
   cluster of occupied sites. */
void orc_percolation_smax(const orc_sim* s, double p, uint32_t sample0, uint32_t n_samples, int32_t* out);

/* Steps 2a and 2b alone for the pair of chains (2p, 2p+1) at temperature k,
   with u as the seed's random word (the word a step would draw), on the
   current state: the move a simulation step makes, for tests that enumerate
   every seed.  Returns 0, or -1 if (k, p) has no ICM. */
int orc_icm_step(orc_sim* s, int32_t k, int32_t p, uint32_t u);

/* Metropolis acceptance as a 2^-32 fraction for a raw energy change dE
   at temperature index k: returns the number of u in [0, 2^32) accepted. */
uint64_t orc_metro_accept_count(const orc_sim* s, int32_t k, int64_t dE_raw);

#ifdef __cplusplus
}
#endif
#endif
