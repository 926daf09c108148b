/*
 * libicm — parallel tempering with isoenergetic cluster moves (ICM) for Ising
 * spin glasses on one MI355X (gfx950).
 *
 * Method: Zhu, Ochoa, Katzgraber, "Efficient Cluster Algorithm for Spin
 * Glasses in Any Space Dimension" (arXiv:1501.05630).  One simulation step is
 * the paper's "Isoenergetic cluster algorithm" list: (1) a Metropolis sweep in
 * every replica, (2a) the spin-reversal flip when more than N/2 sites have
 * q_i = -1, (2b) one Houdayer cluster move (cluster = connected q = -1 domain of
 * a random q = -1 site, flipped in both replicas; "Reminder: Houdayer cluster
 * algorithm" paragraph) at the coldest temperatures, (3) parallel tempering.
 *
 * Conventions fixed by this library where the paper is silent:
 *   - H = -sum over bonds (each once) J_ij s_i s_j.
 *   - square2d (L even) and cubic3d (L even) are periodic, site
 *     i = x + L*y (+ L*L*z); chimera is C x C cells of K_{4,4} with open
 *     boundaries, site i = 8*(row*C + col) + u (u<4 couple vertically, u>=4
 *     horizontally).  Coupling layouts: [N][2], [N][3], [C*C][24] (see
 *     icm_instance_desc::couplings).
 *   - walkers w = h*R + r (h = starting temperature index, r = chain); PT swaps
 *     move temperature labels between walkers of one chain; ICM pairs chains
 *     (2p, 2p+1) at the same temperature.
 *   - the Metropolis sweep updates every colour-0 site, then every colour-1 site
 *     of a proper 2-colouring (lattices: (x+y[+z]) mod 2; chimera:
 *     (row+col+[u>=4]) mod 2).
 *   - random numbers: Philox4x32-10 (Salmon et al., SC'11), key (seed,
 *     instance_key), counters: Metropolis (i, t, w>>2, 0) word w&3; hot start
 *     (i, 0, w>>2, 1) word w&3, spin -1 iff bit 31 is set; ICM
 *     (k*(R/2)+p, t, 0, 2) word 0; PT (k, t, r, 3) word 0.  t is the sweep index.
 *   - integer couplings (J = j / j_scale): Metropolis accepts dE > 0 iff
 *     u < min(floor(2^32 exp(-(beta*dE)/j_scale)), 2^32-1); the PT rule uses the
 *     same form with (beta_k - beta_k+1) and the energy gap.  Energies are exact
 *     integers in units of 1/j_scale.
 *   - float couplings: the model paragraph takes Gaussian J and fixes no
 *     precision.  The library rounds every float J of an instance to the grid
 *     2^-e, e the largest exponent <= 20 for which every |J| 2^e rounds to at
 *     most 2^23 - 1 (e = 20 whenever all |J| < 8), so that each coupling is a
 *     signed 24-bit integer and local fields, energy changes and energies are
 *     exact integer sums.  Each J moves by at most 2^-(e+1): 2^-21 when all
 *     |J| < 8.  The chain simulated is the one of the rounded couplings; for
 *     couplings already on the grid nothing is rounded.  dE > 0 is accepted
 *     iff u * 2^-32 < exp(-(beta*dE)) evaluated in double (beta in double);
 *     PT likewise with (beta_k - beta_k+1) and the energy gap.  Energies are
 *     reported in units of 2^-40 (multiples of 2^(40-e) of that unit).
 *
 * Memory: the caller hands the library one device buffer (the arena, e.g. a
 * torch uint8 tensor) at icm_create; every device allocation of the library is
 * carved from it and the library never calls hipMalloc.  The arena must stay
 * alive until icm_destroy.  Host pointers passed to any call are read or
 * written before the call returns and are not retained.
 *
 * Errors: every call returns ICM_OK (0) or a negative ICM_E_* code; nothing
 * throws or aborts across this boundary.  A HIP failure returns ICM_E_DEVICE
 * and poisons the context (every later call returns ICM_E_DEVICE).
 * icm_last_error() gives a human-readable reason for the last failure.
 *
 * Threading: one context per host thread, except icm_submit / icm_poll /
 * icm_take_result, which may be called from any thread while the serving loop
 * runs.  While it runs, the loop owns the context: every other call returns
 * ICM_E_BUSY (and does not set icm_last_error, which the loop may be writing).
 */
#ifndef ICM_H
#define ICM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ICM_OK 0
#define ICM_E_INVALID -1   /* bad argument or descriptor */
#define ICM_E_NOMEM -2     /* the arena has no room */
#define ICM_E_DEVICE -3    /* HIP error; the context is poisoned */
#define ICM_E_NOTFOUND -4  /* unknown handle or ticket */
#define ICM_E_BUSY -5      /* serving loop owns the instances / result not ready */
#define ICM_E_BUFSIZE -6   /* caller buffer too small */

#define ICM_TOPO_SQUARE2D 0
#define ICM_TOPO_CUBIC3D 1
#define ICM_TOPO_CHIMERA 2

#define ICM_J_INT8 0 /* couplings int8 j, J = j / j_scale */
#define ICM_J_F32 1  /* couplings float, rounded to a 2^-e grid, e <= 20 (see above) */

#define ICM_FLAG_2A 1            /* step 2a (spin-reversal flip of the 2nd replica) */
#define ICM_FLAG_PT 2            /* step 3 (parallel tempering) */
#define ICM_FLAG_RECORD_LABELS 4 /* keep the labels of the last ICM move (parity/debug) */
#define ICM_FLAG_SKIP_METRO 8    /* diagnostic: a step is ICM (+PT) only */
#define ICM_FLAG_MEASURE 16      /* accumulate the observables after every step
                                    (icm_read_observables) */
#define ICM_OBS_BINS 32
#define ICM_OBS_FIELDS 4

typedef struct icm_ctx icm_ctx;

/* One disorder instance: graph, couplings, temperature ladder, replicas.
   Model paragraph of the paper (H, Gaussian disorder) and the Table I
   parameters (N_T temperatures, ICM on the lowest N_c of them). */
typedef struct {
  int32_t topology;      /* ICM_TOPO_* */
  int32_t L;             /* lattice side (even, >= 2) or chimera cells per side (>= 1) */
  int32_t jkind;         /* ICM_J_INT8 or ICM_J_F32 */
  int32_t j_scale;       /* ICM_J_INT8: 1..127 (J = j / j_scale); ignored for F32 */
  const void* couplings; /* host; square2d [N][2] (+x,+y bonds of site i), cubic3d
                            [N][3] (+x,+y,+z), chimera [C*C][24]: in-cell bond (u,v),
                            u<4<=v, at u*4+v-4; bond to the cell below at 16+u (u<4);
                            bond to the cell on the right at 20+u-4 (u>=4); slots that
                            would leave the grid must be 0.  F32 values need |J| <= 64. */
  int32_t n_temps;       /* K >= 1 */
  const double* temps;   /* host [K], strictly ascending, > 0; k = 0 is the coldest */
  int32_t n_replicas;    /* R: even, 2 <= R <= 64 */
  int32_t icm_ntemps;    /* K_c: ICM at the coldest K_c temperatures (0 = off) */
  uint32_t flags;        /* ICM_FLAG_* */
  uint32_t instance_key; /* Philox key word 1 (the seed is key word 0) */
} icm_instance_desc;

typedef struct {
  uint64_t sweeps;            /* sweeps run since the state was set */
  uint64_t metro_accepts;     /* accepted single-spin flips */
  uint64_t icm_moves;         /* cluster moves attempted (including n_minus == 0) */
  uint64_t icm_nontrivial;    /* moves that flipped a non-empty cluster */
  uint64_t icm_cluster_sites; /* sum of cluster sizes */
  uint64_t icm_2a_flips;      /* step-2a spin-reversal flips */
  uint64_t pt_attempts;       /* PT swap attempts */
  uint64_t pt_accepts;        /* accepted PT swaps */
} icm_stats;

/* Launch configuration of icm_run (a 0 field in icm_set_run_config keeps the
   current value). */
typedef struct {
  int32_t threads;          /* threads per workgroup for every size class: 64, 128,
                               256, 512 or 1024; -1 (and the initial value 0): per
                               class, 256 for units of up to 512 sites, 512 up to 1024,
                               1024 above.  A run launches once per size class (sites
                               <= 512, <= 1024, <= 2048, more), one workgroup per unit:
                               small workgroups let more small units share a CU */
  int32_t sweeps_per_launch;/* sweeps fused into one kernel launch */
  int32_t use_graph;        /* 1: replay launches from a captured hipGraph */
  int32_t icm_slots;        /* ICM moves in flight per workgroup, 1..64 (LDS scratch):
                               a wavefront carries 64 / l moves, l = lanes per move
                               (16, 32 or 64 for units of up to 512, 1024, 4096 sites) */
  int32_t table_placement;  /* 0: automatic, 1: neighbour/coupling tables in LDS,
                               2: tables read from global memory */
  int32_t class_threads[4]; /* per size class (sites <= 512, <= 1024, <= 2048, more):
                               threads per workgroup for that class's launches, 64 to
                               1024 as for `threads`, overriding it; 0 keeps the
                               current entry, -1 clears it (the class follows
                               `threads` again).  Initially all clear. */
} icm_run_config;

/* Creates a context on `device`, issuing all work on `hip_stream` (a
   hipStream_t, NULL = the null stream).  `arena` is a caller-owned device
   buffer of arena_bytes (>= 1 MiB, 256-byte aligned) that must outlive the
   context; `seed` is Philox key word 0 for every instance of the context.
   The container of the paper's simulations: many disorder instances, each
   with its temperatures and replicas (Table I: N_sa instances per size).
   Errors: ICM_E_INVALID (null out, arena too small or misaligned),
   ICM_E_DEVICE (no such device). */
int icm_create(icm_ctx** out, int device, void* hip_stream, void* arena, size_t arena_bytes,
               uint32_t seed);
/* Stops serving if it runs, waits for the stream, frees everything the
   context holds (not the arena, which the caller owns). */
int icm_destroy(icm_ctx* ctx);

/* One disorder instance of the model paragraph (graph, couplings J_ij) with
   its temperature ladder, replicas and cluster-move temperatures (Table I:
   N_T temperatures, cluster moves at the lowest N_c).  Copies the descriptor
   (couplings, temperatures) into the arena and returns a handle; no caller
   pointer is kept.  The state is all spins up until icm_init_states /
   icm_set_states.  Errors: ICM_E_INVALID (bad descriptor), ICM_E_NOMEM
   (arena full), ICM_E_BUSY (serving), ICM_E_DEVICE. */
int icm_add_instance(icm_ctx* ctx, const icm_instance_desc* d, int32_t* out_handle);
/* Frees the instance's arena blocks.  ICM_E_NOTFOUND, ICM_E_BUSY. */
int icm_remove_instance(icm_ctx* ctx, int32_t handle);
/* Arena bytes an instance with this descriptor needs (0 if invalid). */
size_t icm_instance_bytes(const icm_instance_desc* d);

/* Initial state (the paper does not give one): a hot start, every walker's
   spins drawn from Philox (stream INIT above); temperature labels w -> h,
   gauge cleared, sweep counter = 0, statistics and observables cleared.
   ICM_E_NOTFOUND, ICM_E_BUSY, ICM_E_DEVICE. */
int icm_init_states(icm_ctx* ctx, int32_t handle);
/* Sets spins [K][R][N] (host, any nonzero int8; < 0 means down) in
   temperature order, resets temperature labels, gauge, statistics and
   observables; sweep counter = sweep0.  The state is copied before return.
   ICM_E_INVALID (null spins), ICM_E_NOTFOUND, ICM_E_NOMEM (staging),
   ICM_E_BUSY, ICM_E_DEVICE. */
int icm_set_states(icm_ctx* ctx, int32_t handle, const int8_t* spins, uint32_t sweep0);

/* Runs n_sweeps simulation steps -- the paper's isoenergetic cluster
   algorithm list: step 1 (a Metropolis sweep of every replica), steps 2a and
   2b (at the K_c coldest temperatures, for every pair of chains), step 3 (a
   PT sweep over neighbouring temperatures) -- on every listed instance, with
   batched launches of the fused kernel (one per size class and sweep block;
   replayed from a captured graph when use_graph is set and a run spans
   several launches).  Asynchronous on the context stream; the results do not
   depend on the batch, the launch shape or the block size.
   Errors: ICM_E_INVALID (bad list, a handle twice, a unit larger than the
   device's LDS), ICM_E_NOTFOUND, ICM_E_NOMEM (work table), ICM_E_BUSY,
   ICM_E_DEVICE. */
int icm_run(icm_ctx* ctx, const int32_t* handles, int32_t n, uint32_t n_sweeps);
/* The same simulation steps with plain per-instance launches (one instance
   per launch, no graph): the baseline the batched form is measured against.
   Same errors as icm_run. */
int icm_run_per_instance(icm_ctx* ctx, const int32_t* handles, int32_t n, uint32_t n_sweeps);
/* Waits for the context stream.  ICM_E_BUSY, ICM_E_DEVICE. */
int icm_sync(icm_ctx* ctx);
/* Launch shape of later runs (fields 0 keep the current value).
   ICM_E_INVALID for values outside the ranges above, ICM_E_BUSY. */
int icm_set_run_config(icm_ctx* ctx, const icm_run_config* cfg);
int icm_get_run_config(icm_ctx* ctx, icm_run_config* cfg);

/* Energies H = -sum over bonds J_ij s_i s_j (model paragraph) of every
   walker, [K][R] in temperature order: raw (int64: units of 1/j_scale, or
   2^-40 for F32) and/or real (double); either pointer may be NULL.  cap is the
   number of elements the buffers hold (ICM_E_BUFSIZE if fewer than K R).
   Synchronizes the context stream.  ICM_E_NOTFOUND, ICM_E_BUSY,
   ICM_E_DEVICE. */
int icm_read_energies(icm_ctx* ctx, int32_t handle, int64_t* raw, double* real, size_t cap);
/* Spin configurations (the replicas of the paper's method), [K][R][N] int8
   +1/-1, in temperature order and canonical site order, step 2a's reversals
   undone (the true spins).  Synchronizes the context stream.
   ICM_E_BUFSIZE (cap < K R N), ICM_E_NOTFOUND, ICM_E_BUSY, ICM_E_DEVICE. */
int icm_read_states(icm_ctx* ctx, int32_t handle, int8_t* out, size_t cap);
/* The two overlaps of the model paragraph for the replicas of each pair
   (chains 2p, 2p+1) at temperature k, q_i = s_i^(2p) s_i^(2p+1): the spin
   overlap sum_i q_i (q = that / N) and the link overlap's numerator, the sum
   over bonds (each once) of q_i q_j (Eq. 1: q_l = that / N_b); [K][R/2]
   int32 each, formed on the device.  Either pointer may be NULL; cap is the
   number of elements each holds.  ICM_E_BUFSIZE, ICM_E_NOTFOUND, ICM_E_NOMEM
   (a scratch of 8 K R/2 bytes in the arena), ICM_E_BUSY, ICM_E_DEVICE. */
int icm_read_overlaps(icm_ctx* ctx, int32_t handle, int32_t* q_sum, int32_t* ql_sum, size_t cap);
/* Labels [N] of the last cluster move (steps 2a, 2b) of the last step run at
   temperature k, pair p: the connected q = -1 domains after step 2a, each
   site labelled with the smallest site index of its domain, -1 off the mask;
   requires ICM_FLAG_RECORD_LABELS.  seed = the seed site (-1 if no q = -1
   site), n_minus = the number of q = -1 sites after 2a.  ICM_E_INVALID (no
   labels recorded, no cluster moves at (k, pair)), ICM_E_BUFSIZE,
   ICM_E_NOTFOUND, ICM_E_BUSY, ICM_E_DEVICE. */
int icm_read_labels(icm_ctx* ctx, int32_t handle, int32_t k, int32_t pair, int32_t* labels,
                    int32_t* seed, int32_t* n_minus, size_t cap);
/* Counters of the steps since the state was set (icm_stats above): accepted
   Metropolis flips (step 1), cluster moves, their sizes and the 2a reversals
   (steps 2a, 2b), PT attempts and accepted swaps (step 3).  ICM_E_INVALID
   (null out), ICM_E_NOTFOUND, ICM_E_BUSY, ICM_E_DEVICE. */
int icm_read_stats(icm_ctx* ctx, int32_t handle, icm_stats* out);
/* Observables of the paper's "Benchmark model and observables" paragraph (the
   energy, the link overlap q_l of Eq. 1 and the spin overlap) and of its
   discussion of cluster sizes (the fraction p of potential cluster sites,
   plotted against T for the three topologies), for the two
   replicas of each ICM pair (chains 2p, 2p+1) at each temperature k, summed
   over the steps since the last icm_init_states / icm_set_states in
   logarithmic time bins: a step that ends at sweep count t (t = 1, 2, ...)
   lands in bin floor(log2 t).  Requires ICM_FLAG_MEASURE.
   sums [ICM_OBS_BINS][K][R/2][ICM_OBS_FIELDS], int64:
     0: E_a + E_b, in units of 1/j_scale for integer couplings and of 2^-20
        for float couplings (exact: their energies are multiples of the
        coupling grid; coarser than the 2^-40 of icm_read_energies so that a
        bin of up to ~2^29 steps at 4096 sites stays within int64),
     1: sum over bonds of q_i q_j = N_b q_l (q_i = s_a,i s_b,i),
     2: (sum_i q_i)^2,
     3: min(n, N - n), n = sites with q_i = -1: the potential cluster sites
        after step 2a (p = this over N);
   counts [ICM_OBS_BINS]: steps per bin.  E(q_l) = -(J^2/T)(N_b/N)(1 - q_l)
   and Delta = <E(q_l)> - <H/N> (Eq. 2) follow from the bin means.
   cap = capacity of sums in elements; ICM_E_BUFSIZE if too small. */
int icm_read_observables(icm_ctx* ctx, int32_t handle, int64_t* sums, int64_t* counts, size_t cap);
/* Walker index at (k, r), [K][R]: the permutation of replicas over
   temperatures that step 3 (parallel tempering) maintains.  ICM_E_BUFSIZE,
   ICM_E_NOTFOUND, ICM_E_BUSY, ICM_E_DEVICE. */
int icm_read_walkers(icm_ctx* ctx, int32_t handle, int32_t* out, size_t cap);
/* The instance's sweep counter t (the counter of the random streams); 0 for
   an unknown handle or while serving. */
uint32_t icm_sweep_index(icm_ctx* ctx, int32_t handle);

/* Replaces the K temperatures of an instance (same K; finite, > 0, strictly
   ascending), for annealing schedules: the paper proposes adding the cluster
   moves at every temperature step of simulated annealing (introduction), and
   hopping through a degenerate ground-state manifold with cluster moves at
   very low temperature (discussion of Fig. 1).  The walkers keep their spins,
   temperature labels, energies and sweep counter; walker (k, r) continues at
   the new T_k.  Ordered after earlier work on the context stream; returns
   when the new tables are on the device.  Integer couplings with PT: the
   PT acceptance table keeps the length it was created with, so a pair of
   temperatures closer than any pair at creation is ICM_E_INVALID.
   Errors: ICM_E_INVALID, ICM_E_NOTFOUND, ICM_E_BUSY while serving,
   ICM_E_DEVICE. */
int icm_set_temperatures(icm_ctx* ctx, int32_t handle, const double* temps);

/* Site percolation on a topology, the study behind the paper's chimera
   percolation threshold (Supplemental Material: the relative size of the
   largest cluster as order parameter, its Binder ratio
   g = (3 - <s_max^4> / <s_max^2>^2) / 2 over random site configurations).
   Sample s (s = 0 .. n_samples-1) occupies site i independently with
   probability p: word i mod 4 of Philox4x32-10 with counter
   (sample0 + s, i / 4, 0, 4) and key (context seed, key) is below
   floor(p 2^32).  smax[s] = the number of sites in the largest connected
   cluster of occupied sites (0 if none).  topology / L as in
   icm_instance_desc, up to 16384 sites (the kernel keeps 8 N + 64 bytes in
   LDS, which must also fit the device's limit per workgroup); p in [0, 1].  smax: DEVICE pointer, int32
   [n_samples], owned by the caller; written asynchronously on the context
   stream (icm_sync, or any later call that synchronizes, completes it).
   Errors: ICM_E_INVALID (topology, size beyond those limits, p, null smax,
   sample range beyond 2^32), ICM_E_BUSY while serving, ICM_E_NOMEM (neighbour table does not fit
   the arena), ICM_E_DEVICE. */
int icm_percolation_smax(icm_ctx* ctx, int32_t topology, int32_t L, double p, uint32_t sample0,
                         uint32_t n_samples, uint32_t key, int32_t* smax);

/* Serving: thermalization requests -- an instance (descriptor) and a number
   of simulation steps from a hot start, the paper's unit of work per
   disorder instance (Table I: 2^b sweeps per instance) -- arriving while
   others run.  icm_serve_start starts a host thread that admits queued
   requests at sweep-block boundaries (sweeps_per_block steps) while the
   arena has room for them, keeps their state on the device, runs the
   resident requests of each kernel variant and size class together, block
   by block, on a stream per group, and retires each when it is done.  A
   request's results are the same as when it runs alone.  Errors:
   ICM_E_INVALID (sweeps_per_block <= 0), ICM_E_BUSY (already serving),
   ICM_E_DEVICE. */
int icm_serve_start(icm_ctx* ctx, int32_t sweeps_per_block);
/* Stops admitting, returns queued requests unrun (ICM_E_BUSY in their
   result), lets the resident ones finish, joins the thread.  ICM_E_DEVICE if
   the loop failed on the device. */
int icm_serve_stop(icm_ctx* ctx);
/* Queues a request (the descriptor and couplings are copied).  Thread-safe.
   ICM_E_INVALID (bad descriptor, n_sweeps = 0), ICM_E_BUSY (not serving). */
int icm_submit(icm_ctx* ctx, const icm_instance_desc* d, uint32_t n_sweeps, uint64_t* ticket);
/* done = 1 when the result is ready; latency_us = submit-to-retire time.
   Thread-safe.  ICM_E_NOTFOUND for an unknown or taken ticket. */
int icm_poll(icm_ctx* ctx, uint64_t ticket, int32_t* done, double* latency_us);
/* Energies [K][R] raw and states [K][R][N] (either may be NULL) of a
   finished request, in the units and order of icm_read_energies /
   icm_read_states; frees the ticket.  Thread-safe.  ICM_E_BUSY (not done),
   ICM_E_BUFSIZE, ICM_E_NOTFOUND, or the request's own error (ICM_E_NOMEM if
   it can never fit the arena, ICM_E_DEVICE). */
int icm_take_result(icm_ctx* ctx, uint64_t ticket, int64_t* energies, int8_t* states,
                    size_t cap_energies, size_t cap_states);

/* Static text for an ICM_* code. */
const char* icm_strerror(int code);
/* Reason of the context's last failure (valid until the next call on it). */
const char* icm_last_error(icm_ctx* ctx);
/* Bytes of arena in use / total (the HBM budget serving admits against).
   ICM_E_INVALID, ICM_E_BUSY. */
int icm_arena_usage(icm_ctx* ctx, size_t* used, size_t* total);

#ifdef __cplusplus
}
#endif
#endif
