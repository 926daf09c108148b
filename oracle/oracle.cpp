// CPU oracle for PT + isoenergetic cluster moves.  TEST INFRASTRUCTURE ONLY:
// the product library must never load it.  See oracle.h for who may call it.
//
// What it computes, step by step, is the simulation step of the ICM paper
// (arXiv:1501.05630, "Isoenergetic cluster algorithm" list, steps 1, 2a, 2b, 3),
// with the Houdayer cluster construction of the "Reminder: Houdayer cluster
// algorithm" paragraph.  Each convention the paper leaves open is stated next
// to the code that applies it.
//
// Everything is plain on purpose: walker-major spins, adjacency lists, one
// attempt at a time, BFS for the clusters, energies recomputed from scratch.

#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10, from Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3" (SC'11): ten rounds of the Philox S-box on a 4x32-bit
// counter, the 2x32-bit key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
const uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;
const uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;

void philox(const uint32_t in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c[4] = {in[0], in[1], in[2], in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += kWeyl0; k1 += kWeyl1; }
    uint64_t p0 = (uint64_t)kMul0 * c[0];
    uint64_t p1 = (uint64_t)kMul1 * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}

// Random-stream purposes (counter word 3).
enum { kMetro = 0, kInit = 1, kIcm = 2, kPt = 3, kPerc = 4 };

struct Bond { int32_t i, j; int64_t raw; };

}  // namespace

struct orc_sim {
  orc_params p;
  int32_t N = 0, K = 0, R = 0, W = 0, Kc = 0;
  std::vector<Bond> bonds;                 // each bond once
  std::vector<std::vector<int32_t>> nbr;   // neighbour site per incident bond
  std::vector<std::vector<int64_t>> nbrJ;  // coupling (raw) per incident bond
  std::vector<int32_t> colour;
  std::vector<double> beta;                // 1 / T_k
  std::vector<int8_t> spin;                // [W][N], walker-major
  std::vector<int32_t> temp_of;            // walker -> temperature index
  std::vector<int32_t> walker_at;          // [K][R] -> walker
  std::vector<int64_t> energy;             // [W] raw units
  uint32_t sweep = 0;
  orc_stats stats{};
  std::vector<std::vector<int32_t>> last_labels;  // [Kc*R/2][N]
  std::vector<int64_t> obs;                // [32][K][R/2][4] observable sums
  std::vector<int64_t> obs_count;          // [32] samples per time bin
  std::vector<int32_t> last_seed, last_nminus;
  // float couplings: the energy field of the observables, summed exactly in
  // units of 2^-40 per [32][K][R/2] (a long bin can pass int64)
  std::vector<__int128> obs_e;
};

namespace {

// Float couplings are read exactly: the paper's model takes Gaussian J with no
// stated precision, and the caller hands over float32 values, so the oracle
// keeps each one as an integer multiple of 2^-40 (raw = J 2^40).  Every float32
// with |J| >= 2^-17 is such a multiple (its last mantissa bit is worth at least
// 2^-40); smaller ones move by at most 2^-41.  Local fields, energy changes and
// energies are then exact integer sums in units of 2^-40 (|J| <= 64 keeps every
// energy of up to 2^16 bonds within int64).
int64_t n_couplings(const orc_params& p) {
  if (p.topology == ORC_SQUARE2D) return (int64_t)p.L * p.L * 2;
  if (p.topology == ORC_CUBIC3D) return (int64_t)p.L * p.L * p.L * 3;
  if (p.topology == ORC_CHIMERA) return (int64_t)p.L * p.L * 24;
  return p.n_edges;
}

int64_t coupling_raw(const orc_params& p, int64_t idx) {
  if (p.jkind == ORC_J_INT8) return ((const int8_t*)p.couplings)[idx];
  return (int64_t)std::nearbyint(std::ldexp((double)((const float*)p.couplings)[idx], 40));
}

bool coupling_valid(const orc_params& p, int64_t idx) {
  if (p.jkind == ORC_J_INT8) return true;
  float J = ((const float*)p.couplings)[idx];
  return std::isfinite(J) && std::fabs(J) <= 64.0f;
}

void add_bond(orc_sim* s, int32_t i, int32_t j, int64_t raw) {
  s->bonds.push_back({i, j, raw});
  s->nbr[i].push_back(j); s->nbrJ[i].push_back(raw);
  s->nbr[j].push_back(i); s->nbrJ[j].push_back(raw);
}

// Builds the graph.  Square and cubic lattices are periodic; site
// i = x + L*y (+ L*L*z).  Couplings [N][d] hold the bond from i to its +x, +y
// (+z) neighbour.  Chimera: C x C cells of K_{4,4}, site i = 8*(row*C+col)+u;
// u<4 couple to the u<4 site of the cells above/below, u>=4 to the u>=4 site
// of the cells left/right; open boundaries.  Couplings [C*C][24]: 16 in-cell
// bonds (u, v) at u*4+(v-4), then 4 bonds to the cell below (16+u, u<4), then
// 4 bonds to the cell on the right (20+u-4, u>=4); entries that would leave
// the grid must be zero.
int build_graph(orc_sim* s) {
  const orc_params& p = s->p;
  int L = p.L;
  if (p.topology == ORC_SQUARE2D || p.topology == ORC_CUBIC3D) {
    if (L < 2 || (L & 1)) return -1;
    int dim = p.topology == ORC_SQUARE2D ? 2 : 3;
    s->N = dim == 2 ? L * L : L * L * L;
    s->nbr.assign(s->N, {}); s->nbrJ.assign(s->N, {}); s->colour.assign(s->N, 0);
    for (int i = 0; i < s->N; ++i) {
      int x = i % L, y = (i / L) % L, z = dim == 3 ? i / (L * L) : 0;
      s->colour[i] = (x + y + z) & 1;
      int fwd[3] = {((x + 1) % L) + L * y + L * L * z, x + L * ((y + 1) % L) + L * L * z,
                    x + L * y + L * L * ((z + 1) % L)};
      for (int d = 0; d < dim; ++d) {
        if (!coupling_valid(p, (int64_t)i * dim + d)) return -1;
        add_bond(s, i, fwd[d], coupling_raw(p, (int64_t)i * dim + d));
      }
    }
    return 0;
  }
  if (p.topology == ORC_CHIMERA) {
    int C = L;
    if (C < 1) return -1;
    s->N = 8 * C * C;
    s->nbr.assign(s->N, {}); s->nbrJ.assign(s->N, {}); s->colour.assign(s->N, 0);
    for (int row = 0; row < C; ++row)
      for (int col = 0; col < C; ++col) {
        int cell = row * C + col, base = 8 * cell;
        for (int u = 0; u < 8; ++u) s->colour[base + u] = (row + col + (u >= 4 ? 1 : 0)) & 1;
        for (int e = 0; e < 24; ++e)
          if (!coupling_valid(p, (int64_t)cell * 24 + e)) return -1;
        for (int u = 0; u < 4; ++u)
          for (int v = 4; v < 8; ++v)
            add_bond(s, base + u, base + v, coupling_raw(p, (int64_t)cell * 24 + u * 4 + (v - 4)));
        for (int u = 0; u < 4; ++u) {
          int64_t raw = coupling_raw(p, (int64_t)cell * 24 + 16 + u);
          if (row + 1 < C) add_bond(s, base + u, 8 * ((row + 1) * C + col) + u, raw);
          else if (raw != 0) return -1;
        }
        for (int u = 4; u < 8; ++u) {
          int64_t raw = coupling_raw(p, (int64_t)cell * 24 + 20 + (u - 4));
          if (col + 1 < C) add_bond(s, base + u, 8 * (row * C + col + 1) + u, raw);
          else if (raw != 0) return -1;
        }
      }
    return 0;
  }
  if (p.topology == ORC_EXPLICIT) {
    if (p.n_sites < 1 || p.n_edges < 0 || !p.colours) return -1;
    s->N = p.n_sites;
    s->nbr.assign(s->N, {}); s->nbrJ.assign(s->N, {});
    s->colour.assign(p.colours, p.colours + s->N);
    for (int e = 0; e < p.n_edges; ++e) {
      int i = p.edges[2 * e], j = p.edges[2 * e + 1];
      if (i < 0 || j < 0 || i >= s->N || j >= s->N || i == j) return -1;
      if (s->colour[i] == s->colour[j]) return -1;  // checkerboard needs a proper 2-colouring
      if (!coupling_valid(p, e)) return -1;
      add_bond(s, i, j, coupling_raw(p, e));
    }
    return 0;
  }
  return -1;
}

// H = - sum over bonds (each once) of J_ij s_i s_j  (model paragraph; the
// paper writes the sum over ordered pairs without the sign, we count each bond
// once with the usual minus sign so that E(q_l) of Eq. (1) holds with N_b bonds).
int64_t energy_of(const orc_sim* s, const int8_t* sp) {
  int64_t E = 0;
  for (const Bond& b : s->bonds) E -= b.raw * sp[b.i] * sp[b.j];
  return E;
}

uint32_t draw(const orc_sim* s, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t purpose, int word) {
  uint32_t ctr[4] = {c0, c1, c2, purpose}, key[2] = {s->p.seed, s->p.instance_key}, out[4];
  philox(ctr, key, out);
  return out[word];
}

uint32_t clamp_threshold(double x) {
  // floor(2^32 * p), capped at 2^32 - 1 (p can round to 1.0 as beta -> 0).
  double t = std::floor(std::ldexp(x, 32));
  return t >= 4294967295.0 ? 4294967295u : (uint32_t)t;
}

// Metropolis rule min(1, exp(-beta dE)); dE <= 0 is always accepted.
bool metro_accept(const orc_sim* s, int k, int64_t dE, uint32_t u) {
  if (dE <= 0) return true;
  double beta = s->beta[k];
  if (s->p.jkind == ORC_J_INT8) {
    uint32_t thr = clamp_threshold(std::exp(-(beta * (double)dE) / (double)s->p.j_scale));
    return u < thr;
  }
  double p = std::exp(-(beta * std::ldexp((double)dE, -40)));
  return std::ldexp((double)u, -32) < p;
}

// Step 1: one Metropolis sweep (N single-spin updates) in every replica.  The
// sweep visits all sites of colour 0, then all sites of colour 1; sites of one
// colour do not interact, so the order inside a colour does not matter.
void metropolis_sweep(orc_sim* s, uint32_t t) {
  for (int c = 0; c < 2; ++c)
    for (int w = 0; w < s->W; ++w) {
      int8_t* sp = &s->spin[(size_t)w * s->N];
      int k = s->temp_of[w];
      for (int i = 0; i < s->N; ++i) {
        if (s->colour[i] != c) continue;
        int64_t h = 0;
        for (size_t e = 0; e < s->nbr[i].size(); ++e) h += s->nbrJ[i][e] * sp[s->nbr[i][e]];
        int64_t dE = 2 * (int64_t)sp[i] * h;
        uint32_t u = draw(s, (uint32_t)i, t, (uint32_t)(w >> 2), kMetro, w & 3);
        if (metro_accept(s, k, dE, u)) {
          sp[i] = (int8_t)-sp[i];
          s->stats.metro_accepts++;
        }
      }
    }
  for (int w = 0; w < s->W; ++w) s->energy[w] = energy_of(s, &s->spin[(size_t)w * s->N]);
}

// Connected components of the subgraph induced by mask, by breadth-first
// search started from each unlabelled mask site in ascending order, so every
// component is labelled by its smallest site index.
void label_components(const orc_sim* s, const std::vector<char>& mask, std::vector<int32_t>& label) {
  label.assign(s->N, -1);
  std::deque<int32_t> q;
  for (int i = 0; i < s->N; ++i) {
    if (!mask[i] || label[i] >= 0) continue;
    label[i] = i;
    q.push_back(i);
    while (!q.empty()) {
      int v = q.front(); q.pop_front();
      for (int j : s->nbr[v])
        if (mask[j] && label[j] < 0) { label[j] = i; q.push_back(j); }
    }
  }
}

// Steps 2a and 2b for the pair of chains (2p, 2p+1) at temperature k, the
// seed drawn from the word u.
void icm_move_with(orc_sim* s, int k, int p, uint32_t u) {
  int a = s->walker_at[k * s->R + 2 * p], b = s->walker_at[k * s->R + 2 * p + 1];
  int8_t* sa = &s->spin[(size_t)a * s->N];
  int8_t* sb = &s->spin[(size_t)b * s->N];
  // Site overlap q_i = s_i^(1) s_i^(2); the cluster domain is q_i = -1.
  std::vector<char> mask(s->N);
  int n = 0;
  for (int i = 0; i < s->N; ++i) { mask[i] = sa[i] != sb[i]; n += mask[i]; }
  // 2a: more than N/2 sites with q = -1 -> flip every spin of one replica (the
  // second walker of the pair), which maps q -> -q and keeps both energies.
  if ((s->p.flags & ORC_FLAG_2A) && 2 * n > s->N) {
    for (int i = 0; i < s->N; ++i) { sb[i] = (int8_t)-sb[i]; mask[i] = !mask[i]; }
    n = s->N - n;
    s->stats.icm_2a_flips++;
  }
  s->stats.icm_moves++;
  int slot = k * (s->R / 2) + p;
  s->last_nminus[slot] = n;
  std::vector<int32_t>& label = s->last_labels[slot];
  if (n == 0) { label.assign(s->N, -1); s->last_seed[slot] = -1; return; }
  // 2b: a uniformly chosen q = -1 site seeds the cluster: idx = floor(u n / 2^32)
  // picks the idx-th mask site in ascending site order.
  int idx = (int)(((uint64_t)u * (uint64_t)n) >> 32);
  int seed = -1;
  for (int i = 0, seen = 0; i < s->N; ++i)
    if (mask[i]) { if (seen == idx) { seed = i; break; } ++seen; }
  // The cluster is the connected q = -1 domain of the seed, added with
  // probability 1; its spins are flipped in both replicas.
  label_components(s, mask, label);
  s->last_seed[slot] = seed;
  int64_t size = 0;
  for (int i = 0; i < s->N; ++i)
    if (label[i] == label[seed]) { sa[i] = (int8_t)-sa[i]; sb[i] = (int8_t)-sb[i]; ++size; }
  s->energy[a] = energy_of(s, sa);
  s->energy[b] = energy_of(s, sb);
  s->stats.icm_nontrivial++;
  s->stats.icm_cluster_sites += (uint64_t)size;
}

void icm_move(orc_sim* s, int k, int p, uint32_t t) {
  const uint32_t slot = (uint32_t)(k * (s->R / 2) + p);
  icm_move_with(s, k, p, draw(s, slot, t, 0u, kIcm, 0));
}

// Step 3: parallel tempering between neighbouring temperatures,
// min(1, exp[(beta_k - beta_{k+1}) (E_k - E_{k+1})]); every neighbouring pair is
// attempted once per step, coldest pair first, in each chain.
void pt_step(orc_sim* s, uint32_t t) {
  for (int r = 0; r < s->R; ++r)
    for (int k = 0; k + 1 < s->K; ++k) {
      int x = s->walker_at[k * s->R + r], y = s->walker_at[(k + 1) * s->R + r];
      int64_t D = s->energy[y] - s->energy[x];
      bool accept = D <= 0;
      s->stats.pt_attempts++;
      if (!accept) {
        uint32_t u = draw(s, (uint32_t)k, t, (uint32_t)r, kPt, 0);
        double dbeta = s->beta[k] - s->beta[k + 1];
        if (s->p.jkind == ORC_J_INT8) {
          uint32_t thr = clamp_threshold(std::exp(-(dbeta * (double)D) / (double)s->p.j_scale));
          accept = u < thr;
        } else {
          double p = std::exp(-(dbeta * std::ldexp((double)D, -40)));
          accept = std::ldexp((double)u, -32) < p;
        }
      }
      if (accept) {
        s->walker_at[k * s->R + r] = y;
        s->walker_at[(k + 1) * s->R + r] = x;
        s->temp_of[x] = k + 1;
        s->temp_of[y] = k;
        s->stats.pt_accepts++;
      }
    }
}

}  // namespace

extern "C" {

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  philox(ctr, key, out);
}

int orc_create(const orc_params* p, orc_sim** out) {
  *out = nullptr;
  if (!p || p->n_temps < 1 || p->n_replicas < 2 || (p->n_replicas & 1)) return -1;
  if (p->icm_ntemps < 0 || p->icm_ntemps > p->n_temps) return -1;
  if (p->jkind != ORC_J_INT8 && p->jkind != ORC_J_F32) return -1;
  if (p->jkind == ORC_J_INT8 && (p->j_scale < 1 || p->j_scale > 127)) return -1;
  for (int k = 0; k < p->n_temps; ++k) {
    if (!(p->temps[k] > 0.0) || !std::isfinite(p->temps[k])) return -1;
    if (k > 0 && !(p->temps[k] > p->temps[k - 1])) return -1;
  }
  orc_sim* s = new orc_sim();
  s->p = *p;
  if (p->jkind == ORC_J_F32 && p->topology != ORC_EXPLICIT) {
    const int64_t n = n_couplings(*p);
    for (int64_t x = 0; x < n; ++x) {
      const float J = ((const float*)p->couplings)[x];
      if (!std::isfinite(J) || std::fabs(J) > 64.0f) { delete s; return -1; }
    }
  }
  if (build_graph(s) != 0) { delete s; return -1; }
  s->K = p->n_temps; s->R = p->n_replicas; s->W = s->K * s->R; s->Kc = p->icm_ntemps;
  s->beta.resize(s->K);
  for (int k = 0; k < s->K; ++k) s->beta[k] = 1.0 / p->temps[k];
  s->spin.assign((size_t)s->W * s->N, 1);
  s->temp_of.resize(s->W); s->walker_at.resize(s->W);
  for (int w = 0; w < s->W; ++w) { s->temp_of[w] = w / s->R; s->walker_at[w] = w; }
  s->energy.assign(s->W, 0);
  int slots = s->Kc * (s->R / 2);
  s->last_labels.assign(slots, std::vector<int32_t>(s->N, -1));
  s->last_seed.assign(slots, -1); s->last_nminus.assign(slots, 0);
  s->p.couplings = nullptr; s->p.temps = nullptr; s->p.edges = nullptr; s->p.colours = nullptr;
  for (int w = 0; w < s->W; ++w) s->energy[w] = energy_of(s, &s->spin[(size_t)w * s->N]);
  *out = s;
  return 0;
}

void orc_destroy(orc_sim* s) { delete s; }

int32_t orc_n_sites(const orc_sim* s) { return s->N; }
int32_t orc_n_bonds(const orc_sim* s) { return (int32_t)s->bonds.size(); }
int32_t orc_colour(const orc_sim* s, int32_t i) { return s->colour[i]; }

int32_t orc_neighbours(const orc_sim* s, int32_t i, int32_t* out, int32_t cap) {
  int32_t d = (int32_t)s->nbr[i].size();
  for (int32_t e = 0; e < d && e < cap; ++e) out[e] = s->nbr[i][e];
  return d;
}

void orc_init_hot(orc_sim* s) {
  // Hot start: s = +1 when bit 31 of the walker's INIT word is 0, else -1.
  for (int w = 0; w < s->W; ++w) {
    for (int i = 0; i < s->N; ++i) {
      uint32_t u = draw(s, (uint32_t)i, 0u, (uint32_t)(w >> 2), kInit, w & 3);
      s->spin[(size_t)w * s->N + i] = (u >> 31) ? -1 : 1;
    }
    s->temp_of[w] = w / s->R;
    s->walker_at[w] = w;
    s->energy[w] = energy_of(s, &s->spin[(size_t)w * s->N]);
  }
  s->sweep = 0;
  s->obs.clear();
  s->obs_e.clear();
  s->obs_count.clear();
}

void orc_set_states(orc_sim* s, const int8_t* spins, uint32_t sweep0) {
  for (int w = 0; w < s->W; ++w) {
    for (int i = 0; i < s->N; ++i) s->spin[(size_t)w * s->N + i] = spins[(size_t)w * s->N + i] < 0 ? -1 : 1;
    s->temp_of[w] = w / s->R;
    s->walker_at[w] = w;
    s->energy[w] = energy_of(s, &s->spin[(size_t)w * s->N]);
  }
  s->sweep = sweep0;
  s->obs.clear();
  s->obs_e.clear();
  s->obs_count.clear();
}

// Observables of the "Benchmark model and observables" paragraph, for the two
// replicas (chains 2p, 2p+1) at each temperature after a step: the energies,
// the link overlap's numerator sum_bonds s_a,i s_a,j s_b,i s_b,j (q_l times
// N_b), the squared spin overlap and the number of potential cluster sites
// (sites of negative overlap after step 2a's reversal, i.e. min(n, N - n) for
// n sites where the replicas differ: the fraction p the paper plots against T
// is this count over N), summed per logarithmic time bin.  E(q_l) of Eq. 1 and
// Delta of Eq. 2 follow from these sums and the bin counts.
void measure(orc_sim* s, uint32_t t_after) {
  const size_t pairs = (size_t)s->K * (s->R / 2);
  if (s->obs.empty()) {
    s->obs.assign((size_t)ORC_OBS_BINS * pairs * ORC_OBS_FIELDS, 0);
    s->obs_e.assign((size_t)ORC_OBS_BINS * pairs, 0);
    s->obs_count.assign(ORC_OBS_BINS, 0);
  }
  int bin = 0;
  while ((t_after >> (bin + 1)) != 0) ++bin;
  s->obs_count[bin] += 1;
  std::vector<int> q(s->N);
  for (int k = 0; k < s->K; ++k)
    for (int p = 0; p < s->R / 2; ++p) {
      const int a = s->walker_at[k * s->R + 2 * p], b = s->walker_at[k * s->R + 2 * p + 1];
      int64_t qsum = 0;
      for (int i = 0; i < s->N; ++i) {
        q[i] = s->spin[(size_t)a * s->N + i] * s->spin[(size_t)b * s->N + i];
        qsum += q[i];
      }
      int64_t link = 0;
      for (const Bond& e : s->bonds) link += q[e.i] * q[e.j];
      const size_t slot = ((size_t)bin * s->K + k) * (s->R / 2) + p;
      int64_t* o = &s->obs[slot * ORC_OBS_FIELDS];
      const int64_t e2 = s->energy[a] + s->energy[b];
      if (s->p.jkind == ORC_J_F32) s->obs_e[slot] += e2;  // units of 2^-40, reported in 2^-20
      else o[0] += e2;
      o[1] += link;
      o[2] += qsum * qsum;
      const int64_t nminus = ((int64_t)s->N - qsum) / 2;
      o[3] += std::min(nminus, (int64_t)s->N - nminus);
    }
}

void orc_run(orc_sim* s, uint32_t n_sweeps) {
  for (uint32_t n = 0; n < n_sweeps; ++n) {
    uint32_t t = s->sweep;
    if (!(s->p.flags & ORC_FLAG_SKIP_METRO)) metropolis_sweep(s, t);  // step 1
    for (int k = 0; k < s->Kc; ++k)                    // steps 2a, 2b (T <~ J)
      for (int p = 0; p < s->R / 2; ++p) icm_move(s, k, p, t);
    if (s->p.flags & ORC_FLAG_PT) pt_step(s, t);       // step 3
    s->sweep = t + 1;
    if (s->p.flags & ORC_FLAG_MEASURE) measure(s, t + 1);
  }
}

void orc_run_trace(orc_sim* s, uint32_t n_sweeps, int64_t* trace) {
  for (uint32_t n = 0; n < n_sweeps; ++n) {
    orc_run(s, 1);
    orc_get_energies(s, trace + (size_t)n * s->K * s->R);
  }
}

void orc_get_states(const orc_sim* s, int8_t* out) {
  for (int k = 0; k < s->K; ++k)
    for (int r = 0; r < s->R; ++r) {
      int w = s->walker_at[k * s->R + r];
      std::memcpy(out + ((size_t)k * s->R + r) * s->N, &s->spin[(size_t)w * s->N], s->N);
    }
}

void orc_get_energies(const orc_sim* s, int64_t* raw) {
  for (int k = 0; k < s->K; ++k)
    for (int r = 0; r < s->R; ++r) raw[k * s->R + r] = s->energy[s->walker_at[k * s->R + r]];
}

void orc_get_walkers(const orc_sim* s, int32_t* out) {
  for (int i = 0; i < s->W; ++i) out[i] = s->walker_at[i];
}

uint32_t orc_get_sweep(const orc_sim* s) { return s->sweep; }

void orc_get_stats(const orc_sim* s, orc_stats* out) { *out = s->stats; }

int orc_get_labels(const orc_sim* s, int32_t k, int32_t p, int32_t* labels, int32_t* seed,
                   int32_t* n_minus) {
  if (k < 0 || k >= s->Kc || p < 0 || p >= s->R / 2) return -1;
  int slot = k * (s->R / 2) + p;
  std::memcpy(labels, s->last_labels[slot].data(), sizeof(int32_t) * s->N);
  *seed = s->last_seed[slot];
  *n_minus = s->last_nminus[slot];
  return 0;
}

int64_t orc_energy(const orc_sim* s, const int8_t* spins) { return energy_of(s, spins); }

void orc_bonds(const orc_sim* s, int32_t* ij, int64_t* raw) {
  for (size_t b = 0; b < s->bonds.size(); ++b) {
    ij[2 * b] = s->bonds[b].i; ij[2 * b + 1] = s->bonds[b].j; raw[b] = s->bonds[b].raw;
  }
}

void orc_get_observables(const orc_sim* s, int64_t* sums, int64_t* counts) {
  const size_t pairs = (size_t)s->K * (s->R / 2);
  const size_t n = (size_t)ORC_OBS_BINS * pairs * ORC_OBS_FIELDS;
  for (size_t x = 0; x < n; ++x) sums[x] = s->obs.empty() ? 0 : s->obs[x];
  if (s->p.jkind == ORC_J_F32 && !s->obs.empty())
    for (size_t slot = 0; slot < (size_t)ORC_OBS_BINS * pairs; ++slot) {
      // the bin's exact sum in units of 2^-40, rounded half up to a multiple of
      // 2^-20 (exact whenever every energy is a multiple of 2^-20)
      const __int128 v = s->obs_e[slot] + ((__int128)1 << 19);
      sums[slot * ORC_OBS_FIELDS] = (int64_t)(v >> 20);
    }
  for (int b = 0; b < ORC_OBS_BINS; ++b) counts[b] = s->obs_count.empty() ? 0 : s->obs_count[b];
}

// New temperatures for the same K slots (simulated annealing with cluster
// moves at every temperature step, introduction): only the inverse
// temperatures change; spins, labels, energies and the sweep counter stay.
int orc_set_temperatures(orc_sim* s, const double* temps) {
  for (int k = 0; k < s->K; ++k) {
    if (!(temps[k] > 0.0) || !std::isfinite(temps[k])) return -1;
    if (k > 0 && !(temps[k] > temps[k - 1])) return -1;
  }
  for (int k = 0; k < s->K; ++k) s->beta[k] = 1.0 / temps[k];
  return 0;
}

// Site percolation on the simulation's graph (Supplemental Material: the
// largest cluster of randomly occupied sites, whose Binder ratio locates the
// chimera percolation threshold).  Every site is occupied independently with
// probability p: the Philox word for site i of sample n is compared with
// floor(p 2^32); the occupied sites are split into connected components by
// breadth-first search, and the largest component's size is reported.
void orc_percolation_smax(const orc_sim* s, double p, uint32_t sample0, uint32_t n_samples, int32_t* out) {
  const uint64_t thr = (uint64_t)std::floor(p * 4294967296.0);
  const uint32_t key[2] = {s->p.seed, s->p.instance_key};
  std::vector<char> occupied(s->N);
  std::vector<int32_t> label;
  std::vector<int32_t> size(s->N);
  for (uint32_t n = 0; n < n_samples; ++n) {
    for (int i = 0; i < s->N; ++i) {
      const uint32_t ctr[4] = {sample0 + n, (uint32_t)(i / 4), 0u, (uint32_t)kPerc};
      uint32_t r[4];
      philox(ctr, key, r);
      occupied[i] = (uint64_t)r[i % 4] < thr;
    }
    label_components(s, occupied, label);
    std::fill(size.begin(), size.end(), 0);
    int32_t best = 0;
    for (int i = 0; i < s->N; ++i)
      if (label[i] >= 0) best = std::max(best, ++size[label[i]]);
    out[n] = best;
  }
}

int orc_icm_step(orc_sim* s, int32_t k, int32_t p, uint32_t u) {
  if (k < 0 || k >= s->Kc || p < 0 || p >= s->R / 2) return -1;
  icm_move_with(s, k, p, u);
  return 0;
}

uint64_t orc_metro_accept_count(const orc_sim* s, int32_t k, int64_t dE) {
  if (dE <= 0) return 1ull << 32;
  double beta = s->beta[k];
  if (s->p.jkind == ORC_J_INT8)
    return clamp_threshold(std::exp(-(beta * (double)dE) / (double)s->p.j_scale));
  double p = std::exp(-(beta * std::ldexp((double)dE, -40)));
  double x = std::ldexp(p, 32);  // accepted u satisfy u < x
  double c = std::ceil(x);
  return (uint64_t)c;
}

}  // extern "C"
