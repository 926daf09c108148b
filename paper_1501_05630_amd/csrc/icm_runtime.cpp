// Host runtime of libicm: context, arena sub-allocator, topology tables,
// acceptance tables, instance lifecycle, batched launches, readout and the
// serving loop.  Everything crosses the boundary through include/icm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/icm.h"
#include "icm_internal.h"

extern "C" {
int icmk_launch_sweep(const icm::UnitDesc* d_units, int n_units, int jkind, int deg, int tables, int layout,
                      uint32_t n_sweeps, int threads, int icm_slots, size_t lds_bytes,
                      hipStream_t stream);
int icmk_set_lds_limit(size_t bytes);
int icmk_set_percolation_lds_limit(size_t bytes);
int icmk_launch_init(uint32_t* spins, int N, int Wq, int W, uint32_t seed, uint32_t key,
                     hipStream_t stream);
int icmk_launch_scatter(uint32_t* spins, const int8_t* src, int N, int Wq, int W,
                        hipStream_t stream);
int icmk_launch_energy(const uint32_t* spins, const uint16_t* nbr, const void* coup, int N, int deg,
                       int Wp, int jkind, int jexp, int64_t* energy, hipStream_t stream);
int icmk_launch_overlaps(const uint32_t* spins, const uint16_t* nbr, const int32_t* at, const uint8_t* gauge,
                         int N, int deg, int K, int R, int topo, int n_bonds, int32_t* out_q,
                         int32_t* out_ql, hipStream_t stream);
size_t icmk_percolation_lds(int N);
int icmk_launch_percolation(const uint16_t* nbr, int N, int deg, unsigned long long thr, uint32_t sample0,
                            uint32_t n_samples, uint32_t seed, uint32_t key, int32_t* smax, int n_cus,
                            size_t lds_cu, hipStream_t stream);
}

namespace {

using icm::UnitDesc;

// ----------------------------------------------------------------------------
// Arena: first-fit sub-allocation of the caller's device buffer.
// ----------------------------------------------------------------------------
class Arena {
 public:
  void reset(char* base, size_t bytes) {
    base_ = base;
    size_ = bytes;
    free_.clear();
    free_[0] = bytes;
    used_ = 0;
  }
  char* alloc(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        size_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        live_[off] = bytes;
        used_ += bytes;
        return base_ + off;
      }
    }
    return nullptr;
  }
  void release(void* p) {
    if (!p) return;
    size_t off = (char*)p - base_;
    auto it = live_.find(off);
    if (it == live_.end()) return;
    size_t bytes = it->second;
    live_.erase(it);
    used_ -= bytes;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + bytes == nx->first) {
      bytes += nx->second;
      free_.erase(nx);
    }
    auto pv = free_.lower_bound(off);
    if (pv != free_.begin()) {
      --pv;
      if (pv->first + pv->second == off) {
        pv->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  char* base_ = nullptr;
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_, live_;
};

// ----------------------------------------------------------------------------
// Topology: neighbour slots, colour lists and the forward bond list.
// ----------------------------------------------------------------------------
struct Topology {
  int topo = 0, L = 0, N = 0, deg = 0;
  std::vector<uint16_t> nbr;                 // [N][deg]
  std::vector<uint16_t> clist;               // [2][N/2]
  std::vector<std::pair<int, int>> bonds;    // each bond once (for overlaps)
  // For coupling layout: for site i and slot d, the index into the canonical
  // coupling array, or -1 for a missing chimera neighbour.
  std::vector<int32_t> cidx;                 // [N][deg]
  uint16_t* d_nbr = nullptr;
  uint16_t* d_clist = nullptr;
  int refs = 0;
};

bool build_topology(int topo, int L, Topology& T, int max_sites = icm::kMaxSites) {
  T.topo = topo;
  T.L = L;
  if (topo == ICM_TOPO_SQUARE2D || topo == ICM_TOPO_CUBIC3D) {
    if (L < 2 || (L & 1)) return false;
    const int dim = topo == ICM_TOPO_SQUARE2D ? 2 : 3;
    T.N = dim == 2 ? L * L : L * L * L;
    T.deg = 2 * dim;
    if (T.N > max_sites) return false;
    T.nbr.assign((size_t)T.N * T.deg, 0);
    T.cidx.assign((size_t)T.N * T.deg, -1);
    std::vector<int> col(T.N);
    for (int i = 0; i < T.N; ++i) {
      const int x = i % L, y = (i / L) % L, z = dim == 3 ? i / (L * L) : 0;
      col[i] = (x + y + z) & 1;
      const int c[3] = {x, y, z};
      for (int a = 0; a < dim; ++a) {
        int cp[3] = {c[0], c[1], c[2]}, cm[3] = {c[0], c[1], c[2]};
        cp[a] = (c[a] + 1) % L;
        cm[a] = (c[a] + L - 1) % L;
        const int ip = cp[0] + L * cp[1] + L * L * cp[2];
        const int im = cm[0] + L * cm[1] + L * L * cm[2];
        T.nbr[(size_t)i * T.deg + 2 * a] = (uint16_t)ip;
        T.nbr[(size_t)i * T.deg + 2 * a + 1] = (uint16_t)im;
        T.cidx[(size_t)i * T.deg + 2 * a] = i * dim + a;        // bond i -> i+a
        T.cidx[(size_t)i * T.deg + 2 * a + 1] = im * dim + a;   // bond (i-a) -> i
        T.bonds.push_back({i, ip});
      }
    }
    for (int c = 0; c < 2; ++c)
      for (int i = 0; i < T.N; ++i)
        if (col[i] == c) T.clist.push_back((uint16_t)i);
    return (int)T.clist.size() == T.N;
  }
  if (topo == ICM_TOPO_CHIMERA) {
    const int C = L;
    if (C < 1) return false;
    T.N = 8 * C * C;
    T.deg = 6;
    if (T.N > max_sites) return false;
    T.nbr.assign((size_t)T.N * 6, 0);
    T.cidx.assign((size_t)T.N * 6, -1);
    std::vector<int> col(T.N);
    for (int row = 0; row < C; ++row)
      for (int cc = 0; cc < C; ++cc) {
        const int cell = row * C + cc, base = 8 * cell;
        for (int u = 0; u < 8; ++u) {
          const int i = base + u;
          col[i] = (row + cc + (u >= 4 ? 1 : 0)) & 1;
          size_t o = (size_t)i * 6;
          // four in-cell partners
          for (int v = 0; v < 4; ++v) {
            const int partner = u < 4 ? 4 + v : v;
            T.nbr[o + v] = (uint16_t)(base + partner);
            T.cidx[o + v] = cell * 24 + (u < 4 ? u * 4 + v : v * 4 + (u - 4));
          }
          // two inter-cell partners: u<4 vertical (row-1, row+1), u>=4 horizontal
          int prev = -1, next = -1, cprev = -1, cnext = -1;
          if (u < 4) {
            if (row > 0) { prev = 8 * ((row - 1) * C + cc) + u; cprev = ((row - 1) * C + cc) * 24 + 16 + u; }
            if (row + 1 < C) { next = 8 * ((row + 1) * C + cc) + u; cnext = cell * 24 + 16 + u; }
          } else {
            if (cc > 0) { prev = 8 * (row * C + cc - 1) + u; cprev = (row * C + cc - 1) * 24 + 20 + (u - 4); }
            if (cc + 1 < C) { next = 8 * (row * C + cc + 1) + u; cnext = cell * 24 + 20 + (u - 4); }
          }
          T.nbr[o + 4] = (uint16_t)(prev >= 0 ? prev : i);
          T.cidx[o + 4] = cprev;
          T.nbr[o + 5] = (uint16_t)(next >= 0 ? next : i);
          T.cidx[o + 5] = cnext;
          if (u < 4)
            for (int v = 4; v < 8; ++v) T.bonds.push_back({i, base + v});
          if (next >= 0) T.bonds.push_back({i, next});
        }
      }
    for (int c = 0; c < 2; ++c)
      for (int i = 0; i < T.N; ++i)
        if (col[i] == c) T.clist.push_back((uint16_t)i);
    return (int)T.clist.size() == T.N;
  }
  return false;
}

int coupling_count(int topo, int L) {
  if (topo == ICM_TOPO_SQUARE2D) return L * L * 2;
  if (topo == ICM_TOPO_CUBIC3D) return L * L * L * 3;
  if (topo == ICM_TOPO_CHIMERA) return L * L * 24;
  return 0;
}

// ----------------------------------------------------------------------------
// Acceptance tables (integer couplings).  For a raw energy change dE (units of
// 1/j_scale) the number of accepted u in [0, 2^32) is
// min(floor(2^32 exp(-(beta dE)/j_scale)), 2^32 - 1).
// ----------------------------------------------------------------------------
uint32_t threshold_of(double x) {
  const double v = std::floor(std::ldexp(std::exp(x), 32));
  return v >= 4294967295.0 ? 4294967295u : (uint32_t)v;
}

struct Instance {
  int32_t handle = -1;
  Topology* topo = nullptr;
  int N = 0, deg = 0, K = 0, R = 0, W = 0, Wq = 0, Wp = 0, Kc = 0, HM = 0, ptlen = 0;
  int jkind = 0, jscale = 1;
  int jexp = 0;                      // float couplings: grid exponent
  int jpl = 0;                       // int8 couplings: bit planes for the cluster moves
  uint32_t flags = 0, key = 0;
  std::vector<double> temps;
  uint32_t sweep_host = 0;
  size_t obs_words = 0;              // observable sums + counts (MEASURE)
  std::vector<int64_t> obs_zero;     // host source for clearing them
  // device regions
  std::vector<void*> blocks;  // everything this instance owns in the arena
  UnitDesc unit{};
  size_t lds_bytes_at(int slots, int tables, int threads) const {
    return icm::lds_layout(N, deg, Wq, K, R, HM, jkind, slots, tables,
                           ((flags & ICM_FLAG_RECORD_LABELS) ? 1 : 0) | ((flags & ICM_FLAG_MEASURE) ? 2 : 0),
                           Kc, jpl, threads / 64).total;
  }
};

struct Request;

}  // namespace

struct icm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t capture_stream = nullptr;  // private stream for graph capture
  // extra streams (default priority) that run the launches of different
  // kernel variants / size classes of one icm_run concurrently
  hipStream_t side[3] = {nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> events;
  uint32_t seed = 0;
  Arena arena;
  std::atomic<bool> poisoned{false};
  std::string last_error;
  std::map<std::pair<int, int>, std::unique_ptr<Topology>> topologies;
  std::map<int32_t, std::unique_ptr<Instance>> instances;
  int32_t next_handle = 1;
  size_t lds_limit = 65536;
  int n_cus = 256;
  size_t lds_cu = 0;                 // LDS bytes per compute unit
  icm_run_config cfg{0, 256, 0, 32, 0, {0, 0, 0, 0}};
  // unit tables cached per (handle list)
  std::map<std::vector<int32_t>, UnitDesc*> unit_tables;
  // captured graphs per (handle list, sweeps per launch, launches)
  struct GraphKey {
    std::vector<int32_t> handles;
    uint32_t spl, launches;
    int threads, slots;
    bool operator<(const GraphKey& o) const {
      return std::tie(handles, spl, launches, threads, slots) <
             std::tie(o.handles, o.spl, o.launches, o.threads, o.slots);
    }
  };
  std::map<GraphKey, hipGraphExec_t> graphs;
  // serving
  std::mutex mu;
  std::condition_variable cv;
  std::thread server;
  std::atomic<bool> serving{false};
  int serve_block = 256;
  uint64_t next_ticket = 1;
  std::map<uint64_t, std::shared_ptr<Request>> requests;
  std::deque<std::shared_ptr<Request>> queue;
};

namespace {

struct Request {
  uint64_t ticket = 0;
  icm_instance_desc desc{};
  std::vector<uint8_t> couplings;
  std::vector<double> temps;
  uint32_t n_sweeps = 0, done_sweeps = 0;
  int32_t handle = -1;
  bool done = false;
  int error = ICM_OK;
  std::chrono::steady_clock::time_point t_submit, t_done;
  std::vector<int64_t> energies;
  std::vector<int8_t> states;
};

int fail(icm_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->last_error = buf;
    if (code == ICM_E_DEVICE) c->poisoned = true;
  }
  return code;
}

#define HIP_OK(ctx, expr)                                                              \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(ctx, ICM_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

#define KERNEL_OK(ctx, expr)                                                                   \
  do {                                                                                         \
    int _e = (expr);                                                                           \
    if (_e != 0)                                                                               \
      return fail(ctx, ICM_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString((hipError_t)_e)); \
  } while (0)

int check_ctx(icm_ctx* c) {
  if (!c) return ICM_E_INVALID;
  if (c->poisoned) return ICM_E_DEVICE;
  return ICM_OK;
}

// Entry points other than the serving calls: while the serving loop runs it
// owns the instances, the arena and the run configuration, so they return
// ICM_E_BUSY (without touching last_error, which the loop may be writing).
int guard(icm_ctx* c) {
  const int rc = check_ctx(c);
  if (rc) return rc;
  return c->serving ? ICM_E_BUSY : ICM_OK;
}

int validate_desc(const icm_instance_desc* d, std::string& why) {
  if (!d) { why = "null descriptor"; return ICM_E_INVALID; }
  if (d->topology < 0 || d->topology > 2) { why = "unknown topology"; return ICM_E_INVALID; }
  if (d->topology != ICM_TOPO_CHIMERA && (d->L < 2 || (d->L & 1))) { why = "L must be even and >= 2"; return ICM_E_INVALID; }
  if (d->topology == ICM_TOPO_CHIMERA && d->L < 1) { why = "chimera needs C >= 1"; return ICM_E_INVALID; }
  if (d->L > 4096) { why = "L too large"; return ICM_E_INVALID; }
  long long N = d->topology == ICM_TOPO_SQUARE2D ? (long long)d->L * d->L
              : d->topology == ICM_TOPO_CUBIC3D ? (long long)d->L * d->L * d->L
                                                 : 8LL * d->L * d->L;
  if (N > icm::kMaxSites) { why = "more sites than the resident kernel supports"; return ICM_E_INVALID; }
  if (d->jkind != ICM_J_INT8 && d->jkind != ICM_J_F32) { why = "unknown coupling kind"; return ICM_E_INVALID; }
  if (d->jkind == ICM_J_INT8 && (d->j_scale < 1 || d->j_scale > 127)) { why = "j_scale must be 1..127"; return ICM_E_INVALID; }
  if (!d->couplings) { why = "null couplings"; return ICM_E_INVALID; }
  if (d->n_temps < 1 || d->n_temps > icm::kMaxTemps || !d->temps) { why = "bad temperature count"; return ICM_E_INVALID; }
  for (int k = 0; k < d->n_temps; ++k) {
    if (!(d->temps[k] > 0.0) || !std::isfinite(d->temps[k])) { why = "temperatures must be finite and > 0"; return ICM_E_INVALID; }
    if (k > 0 && !(d->temps[k] > d->temps[k - 1])) { why = "temperatures must be strictly ascending"; return ICM_E_INVALID; }
  }
  if (d->n_replicas < 2 || (d->n_replicas & 1) || d->n_replicas > icm::kMaxReplicas) { why = "n_replicas must be even, 2..64"; return ICM_E_INVALID; }
  if (d->icm_ntemps < 0 || d->icm_ntemps > d->n_temps) { why = "icm_ntemps out of range"; return ICM_E_INVALID; }
  if (d->flags & ~31u) { why = "unknown flags"; return ICM_E_INVALID; }
  const int nc = coupling_count(d->topology, d->L);
  if (d->jkind == ICM_J_F32) {
    const float* J = (const float*)d->couplings;
    for (int x = 0; x < nc; ++x)
      if (!std::isfinite(J[x]) || std::fabs(J[x]) > 64.0f) { why = "float couplings must be finite with |J| <= 64"; return ICM_E_INVALID; }
  }
  if (d->topology == ICM_TOPO_CHIMERA) {
    const int C = d->L;
    for (int row = 0; row < C; ++row)
      for (int cc = 0; cc < C; ++cc)
        for (int e = 16; e < 24; ++e) {
          const bool off = (e < 20 && row == C - 1) || (e >= 20 && cc == C - 1);
          if (!off) continue;
          const size_t x = (size_t)(row * C + cc) * 24 + e;
          const bool nz = d->jkind == ICM_J_F32 ? ((const float*)d->couplings)[x] != 0.0f
                                                : ((const int8_t*)d->couplings)[x] != 0;
          if (nz) { why = "chimera coupling slot leaves the grid but is nonzero"; return ICM_E_INVALID; }
        }
  }
  return ICM_OK;
}

// Float couplings are rounded to the grid 2^-e, e the largest exponent <= 20
// for which every |J| 2^e rounds to at most 2^23 - 1 (e = 20 whenever all
// |J| < 8): each coupling is then a signed 24-bit integer in units of 2^-e,
// so local fields and energy changes are exact integer sums.
int grid_exponent(const float* J, size_t n) {
  double m = 0.0;
  for (size_t x = 0; x < n; ++x) m = std::max(m, std::fabs((double)J[x]));
  int e = 20;
  while (e > -32 && std::nearbyint(std::ldexp(m, e)) > 8388607.0) --e;
  return e;
}

int32_t grid_coupling(float J, int e) { return (int32_t)std::nearbyint(std::ldexp((double)J, e)); }

Topology* get_topology(icm_ctx* c, int topo, int L, int& rc, int max_sites = icm::kMaxSites) {
  rc = ICM_OK;
  auto key = std::make_pair(topo, L);
  auto it = c->topologies.find(key);
  if (it != c->topologies.end()) return it->second.get();
  auto T = std::make_unique<Topology>();
  if (!build_topology(topo, L, *T, max_sites)) { rc = ICM_E_INVALID; return nullptr; }
  T->d_nbr = (uint16_t*)c->arena.alloc(T->nbr.size() * 2);
  T->d_clist = (uint16_t*)c->arena.alloc(T->clist.size() * 2);
  if (!T->d_nbr || !T->d_clist) {
    c->arena.release(T->d_nbr);
    c->arena.release(T->d_clist);
    rc = ICM_E_NOMEM;
    return nullptr;
  }
  if (hipMemcpyAsync(T->d_nbr, T->nbr.data(), T->nbr.size() * 2, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(T->d_clist, T->clist.data(), T->clist.size() * 2, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    rc = ICM_E_DEVICE;
    return nullptr;
  }
  Topology* raw = T.get();
  c->topologies[key] = std::move(T);
  return raw;
}

struct Sizes {
  size_t spins, coup, thr, ptthr, beta, bl2e, tau, at, gauge, energy, stats, labels, seeds, sweep, obs;
  int HM, ptlen;
};

// Threshold tables and sizes for a validated descriptor.
int plan_instance(const icm_instance_desc* d, const Topology& T, Sizes& S,
                  std::vector<uint32_t>* thr, std::vector<uint32_t>* ptthr, std::string& why) {
  const int N = T.N, K = d->n_temps, R = d->n_replicas, W = K * R, Wq = (W + 3) / 4;
  S.HM = 1;
  S.ptlen = 0;
  if (d->jkind == ICM_J_INT8) {
    const int8_t* J = (const int8_t*)d->couplings;
    int hmax = 0;
    for (int i = 0; i < N; ++i) {
      int h = 0;
      for (int s = 0; s < T.deg; ++s) {
        const int ci = T.cidx[(size_t)i * T.deg + s];
        if (ci >= 0) h += std::abs((int)J[ci]);
      }
      hmax = std::max(hmax, h);
    }
    S.HM = hmax + 1;
    if (thr) {
      thr->assign((size_t)K * S.HM, 0);
      for (int k = 0; k < K; ++k) {
        const double beta = 1.0 / d->temps[k];
        (*thr)[(size_t)k * S.HM] = 4294967295u;
        for (int e = 1; e < S.HM; ++e)
          (*thr)[(size_t)k * S.HM + e] = threshold_of(-(beta * (double)(2 * e)) / (double)d->j_scale);
      }
    }
    if (K > 1 && (d->flags & ICM_FLAG_PT)) {
      // table length: the first gap with a zero threshold, for every k
      const int cap = 1 << 16;
      int len = 0;
      for (int k = 0; k + 1 < K; ++k) {
        const double dbeta = 1.0 / d->temps[k] - 1.0 / d->temps[k + 1];
        int D = 1;
        while (D <= cap && threshold_of(-(dbeta * (double)D) / (double)d->j_scale) != 0) ++D;
        if (D > cap) { why = "temperatures too close for the integer PT table"; return ICM_E_INVALID; }
        len = std::max(len, D);
      }
      S.ptlen = len;
      if (ptthr) {
        ptthr->assign((size_t)(K - 1) * len, 0);
        for (int k = 0; k + 1 < K; ++k) {
          const double dbeta = 1.0 / d->temps[k] - 1.0 / d->temps[k + 1];
          for (int D = 1; D <= len; ++D)
            (*ptthr)[(size_t)k * len + D - 1] = threshold_of(-(dbeta * (double)D) / (double)d->j_scale);
        }
      }
    }
  }
  S.spins = (size_t)Wq * N * 4;
  S.coup = (size_t)N * T.deg * (d->jkind == ICM_J_F32 ? 4 : 1);
  S.thr = d->jkind == ICM_J_INT8 ? (size_t)K * S.HM * 4 : 0;
  S.ptthr = (size_t)std::max(0, K - 1) * S.ptlen * 4;
  S.beta = (size_t)K * 8;
  S.bl2e = (size_t)K * 4;
  S.tau = (size_t)Wq * 4 * 4;
  S.at = (size_t)K * R * 4;
  S.gauge = (size_t)Wq * 4;
  S.energy = (size_t)Wq * 4 * 8;
  S.stats = icm::kNumStats * 8;
  const int slots = d->icm_ntemps * (R / 2);
  S.labels = (d->flags & ICM_FLAG_RECORD_LABELS) ? (size_t)slots * N * 4 : 0;
  S.seeds = (d->flags & ICM_FLAG_RECORD_LABELS) ? (size_t)slots * 2 * 4 : 0;
  S.sweep = 4;
  S.obs = (d->flags & ICM_FLAG_MEASURE)
              ? ((size_t)icm::kObsBins * K * (R / 2) * icm::kObsFields + icm::kObsBins) * 8
              : 0;
  (void)W;
  return ICM_OK;
}

size_t total_bytes(const Sizes& S) {
  size_t t = 0;
  for (size_t b : {S.spins, S.coup, S.thr, S.ptthr, S.beta, S.bl2e, S.tau, S.at, S.gauge, S.energy,
                   S.stats, S.labels, S.seeds, S.sweep, S.obs})
    t += (std::max(b, size_t(1)) + 255) & ~size_t(255);
  return t;
}

void release_instance(icm_ctx* c, Instance* in) {
  for (void* p : in->blocks) c->arena.release(p);
  in->blocks.clear();
  if (in->topo) in->topo->refs--;
}

int reset_walkers(icm_ctx* c, Instance* in, uint32_t sweep0) {
  std::vector<int32_t> tau(in->Wp), at((size_t)in->K * in->R);
  for (int w = 0; w < in->Wp; ++w) tau[w] = w < in->W ? w / in->R : in->K;
  for (int x = 0; x < in->K * in->R; ++x) at[x] = x;
  std::vector<uint8_t> gauge(in->Wp, 0);
  std::vector<unsigned long long> stats(icm::kNumStats, 0);
  HIP_OK(c, hipMemcpyAsync(in->unit.tau, tau.data(), tau.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync(in->unit.at, at.data(), at.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync(in->unit.gauge, gauge.data(), gauge.size(), hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync(in->unit.stats, stats.data(), stats.size() * 8, hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync(in->unit.sweep, &sweep0, 4, hipMemcpyHostToDevice, c->stream));
  if (in->flags & ICM_FLAG_MEASURE) {
    in->obs_zero.assign(in->obs_words, 0);
    HIP_OK(c, hipMemcpyAsync(in->unit.obs, in->obs_zero.data(), in->obs_words * 8, hipMemcpyHostToDevice,
                             c->stream));
  }
  HIP_OK(c, hipStreamSynchronize(c->stream));
  in->sweep_host = sweep0;
  return ICM_OK;
}

int add_instance_impl(icm_ctx* c, const icm_instance_desc* d, int32_t* out) {
  std::string why;
  int rc = validate_desc(d, why);
  if (rc) return fail(c, rc, "invalid descriptor: %s", why.c_str());
  Topology* T = get_topology(c, d->topology, d->L, rc);
  if (!T) return fail(c, rc, rc == ICM_E_NOMEM ? "arena full (topology tables)" : "cannot build topology");
  Sizes S{};
  std::vector<uint32_t> thr, ptthr;
  rc = plan_instance(d, *T, S, &thr, &ptthr, why);
  if (rc) return fail(c, rc, "%s", why.c_str());
  auto in = std::make_unique<Instance>();
  in->topo = T;
  in->N = T->N;
  in->deg = T->deg;
  in->K = d->n_temps;
  in->R = d->n_replicas;
  in->W = in->K * in->R;
  in->Wq = (in->W + 3) / 4;
  in->Wp = 4 * in->Wq;
  in->Kc = d->icm_ntemps;
  in->HM = S.HM;
  in->ptlen = S.ptlen;
  in->jkind = d->jkind;
  in->jscale = d->jkind == ICM_J_INT8 ? d->j_scale : 1;
  in->jexp = d->jkind == ICM_J_F32
                  ? grid_exponent((const float*)d->couplings, (size_t)coupling_count(d->topology, d->L))
                  : 0;
  if (d->jkind == ICM_J_INT8) {
    int jmin = 0, jmax = 0;
    const int8_t* j8 = (const int8_t*)d->couplings;
    for (size_t x = 0; x < (size_t)coupling_count(d->topology, d->L); ++x) {
      jmin = std::min(jmin, (int)j8[x]);
      jmax = std::max(jmax, (int)j8[x]);
    }
    in->jpl = icm::coupling_planes(0, in->Kc, in->N, jmin, jmax);
  }
  in->flags = d->flags;
  in->key = d->instance_key;
  in->temps.assign(d->temps, d->temps + d->n_temps);
  auto grab = [&](size_t bytes) -> void* {
    void* p = c->arena.alloc(std::max(bytes, size_t(1)));
    if (p) in->blocks.push_back(p);
    return p;
  };
  UnitDesc& U = in->unit;
  U.spins = (uint32_t*)grab(S.spins);
  U.coup = grab(S.coup);
  U.thr = (const uint32_t*)grab(S.thr);
  U.ptthr = (const uint32_t*)grab(S.ptthr);
  U.beta = (const double*)grab(S.beta);
  U.bl2e = (const float*)grab(S.bl2e);
  U.tau = (int32_t*)grab(S.tau);
  U.at = (int32_t*)grab(S.at);
  U.gauge = (uint8_t*)grab(S.gauge);
  U.energy = (int64_t*)grab(S.energy);
  U.stats = (unsigned long long*)grab(S.stats);
  U.labels = (int32_t*)grab(S.labels);
  U.seeds = (int32_t*)grab(S.seeds);
  U.sweep = (uint32_t*)grab(S.sweep);
  U.obs = (int64_t*)grab(S.obs);
  in->obs_words = S.obs / 8;
  if (in->blocks.size() != 15) {
    T->refs++;
    release_instance(c, in.get());
    return fail(c, ICM_E_NOMEM, "arena full: instance needs %zu bytes", total_bytes(S));
  }
  T->refs++;
  U.nbr = T->d_nbr;
  U.clist = T->d_clist;
  U.N = in->N;
  U.Nc = in->N / 2;
  U.deg = in->deg;
  U.W = in->W;
  U.Wq = in->Wq;
  U.K = in->K;
  U.R = in->R;
  U.Kc = in->Kc;
  U.HM = in->HM;
  U.ptlen = in->ptlen;
  U.jkind = in->jkind;
  U.jscale = in->jscale;
  U.flags = in->flags;
  U.topo = T->topo;
  U.jexp = in->jexp;
  U.jpl = in->jpl;
  U.L = T->L;
  U.seed = c->seed;
  U.key = in->key;

  // device couplings [N][deg], slot-aligned with the neighbour table
  const int N = in->N, deg = in->deg;
  std::vector<uint8_t> coup(S.coup, 0);
  for (int i = 0; i < N; ++i)
    for (int s = 0; s < deg; ++s) {
      const int ci = T->cidx[(size_t)i * deg + s];
      if (d->jkind == ICM_J_F32) {
        const int32_t v = ci >= 0 ? grid_coupling(((const float*)d->couplings)[ci], in->jexp) : 0;
        std::memcpy(&coup[((size_t)i * deg + s) * 4], &v, 4);
      } else {
        coup[(size_t)i * deg + s] = (uint8_t)(ci >= 0 ? ((const int8_t*)d->couplings)[ci] : 0);
      }
    }
  std::vector<double> beta(in->K);
  std::vector<float> bl2e(in->K);
  for (int k = 0; k < in->K; ++k) {
    beta[k] = 1.0 / d->temps[k];
    bl2e[k] = (float)(beta[k] / std::log(2.0));
  }
  std::vector<int64_t> e0(in->Wp, 0);
  HIP_OK(c, hipMemcpyAsync((void*)U.coup, coup.data(), coup.size(), hipMemcpyHostToDevice, c->stream));
  if (S.thr) HIP_OK(c, hipMemcpyAsync((void*)U.thr, thr.data(), S.thr, hipMemcpyHostToDevice, c->stream));
  if (S.ptthr) HIP_OK(c, hipMemcpyAsync((void*)U.ptthr, ptthr.data(), S.ptthr, hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync((void*)U.beta, beta.data(), S.beta, hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync((void*)U.bl2e, bl2e.data(), S.bl2e, hipMemcpyHostToDevice, c->stream));
  // all spins up: every word 0x01010101
  HIP_OK(c, hipMemsetD32Async((hipDeviceptr_t)U.spins, 0x01010101, S.spins / 4, c->stream));
  int r2 = reset_walkers(c, in.get(), 0);
  if (r2) return r2;
  KERNEL_OK(c, icmk_launch_energy(U.spins, U.nbr, U.coup, N, deg, in->Wp, in->jkind, in->jexp, U.energy,
                                  c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  const int32_t h = c->next_handle++;
  in->handle = h;
  c->instances[h] = std::move(in);
  *out = h;
  return ICM_OK;
}

Instance* find(icm_ctx* c, int32_t h) {
  auto it = c->instances.find(h);
  return it == c->instances.end() ? nullptr : it->second.get();
}

void drop_cached_tables(icm_ctx* c, int32_t h) {
  for (auto it = c->unit_tables.begin(); it != c->unit_tables.end();) {
    if (std::find(it->first.begin(), it->first.end(), h) != it->first.end()) {
      c->arena.release(it->second);
      it = c->unit_tables.erase(it);
    } else {
      ++it;
    }
  }
  for (auto it = c->graphs.begin(); it != c->graphs.end();) {
    if (std::find(it->first.handles.begin(), it->first.handles.end(), h) != it->first.handles.end()) {
      (void)hipGraphExecDestroy(it->second);
      it = c->graphs.erase(it);
    } else {
      ++it;
    }
  }
}

// Groups of instances that share a kernel instantiation (coupling kind, degree).
struct Group {
  int jkind, deg, cls, layout;  // layout: icm::unit_layout of its units (kLayAny: mixed, as in serving)
  std::vector<int32_t> handles;
};

// Size classes of units (sites): up to 512, 1024, 2048, more.  Units of one
// class share a launch (its LDS size is the largest member's).  Threads per
// workgroup of a class: its class_threads entry if set, else the configured
// count, else (threads = 0, automatic) 256 up to 512 sites, 512 up to 1024,
// 1024 above.
int size_class(int N) { return N <= 512 ? 0 : (N <= 1024 ? 1 : (N <= 2048 ? 2 : 3)); }

int class_threads(const icm_run_config& cfg, int cls) {
  if (cfg.class_threads[cls] > 0) return cfg.class_threads[cls];
  if (cfg.threads > 0) return cfg.threads;
  return cls == 0 ? 256 : (cls == 1 ? 512 : 1024);
}

// Units of one size class and coupling kind share a launch, split by their
// cluster-move layout (8^3, chimera of up to 64 words, other one-word
// lattices, two-word lattices, anything else), so that each layout runs in
// the kernel build made for it.
std::vector<Group> group_handles(icm_ctx* c, const int32_t* handles, int n) {
  std::vector<Group> g;
  for (int x = 0; x < n; ++x) {
    Instance* in = find(c, handles[x]);
    const int cls = size_class(in->N);
    const int lay = icm::unit_layout(in->unit.topo, in->unit.L, in->unit.deg, in->unit.N);
    auto it = std::find_if(g.begin(), g.end(), [&](const Group& q) {
      return q.jkind == in->jkind && q.deg == in->deg && q.cls == cls && q.layout == lay;
    });
    if (it == g.end()) g.push_back({in->jkind, in->deg, cls, lay, {handles[x]}});
    else it->handles.push_back(handles[x]);
  }
  return g;
}

// Picks the ICM slot count and where the tables live so that the largest unit
// of the group fits the LDS limit: tables in LDS with as many slots as asked,
// else fewer slots, else tables in global memory.
int effective_slots(icm_ctx* c, const std::vector<int32_t>& hs, int threads, int want, size_t& lds,
                    int& tables) {
  // no more slots than the waves can carry: 64 / lanes-per-move moves each
  int per_wave = 4;
  for (int32_t h : hs) per_wave = std::min(per_wave, 64 / icm::icm_lanes_per_move(find(c, h)->N));
  const int top = std::max(1, std::min(want, per_wave * (threads / 64)));
  const int first = c->cfg.table_placement == 2 ? 0 : 1;
  const int last = c->cfg.table_placement == 1 ? 1 : 0;
  for (tables = first; tables >= last; --tables) {
    for (int slots = top; slots >= 1; --slots) {
      lds = 0;
      for (int32_t h : hs) lds = std::max(lds, find(c, h)->lds_bytes_at(slots, tables, threads));
      if (lds <= c->lds_limit) return slots;
      if (tables && slots <= std::min(top, 4)) break;  // prefer global tables over < 4 slots
    }
  }
  tables = 0;
  return 1;
}

int unit_table(icm_ctx* c, const std::vector<int32_t>& hs, UnitDesc** out) {
  auto it = c->unit_tables.find(hs);
  if (it != c->unit_tables.end()) { *out = it->second; return ICM_OK; }
  UnitDesc* d = (UnitDesc*)c->arena.alloc(sizeof(UnitDesc) * hs.size());
  if (!d) return fail(c, ICM_E_NOMEM, "arena full (unit table)");
  std::vector<UnitDesc> host;
  for (int32_t h : hs) host.push_back(find(c, h)->unit);
  HIP_OK(c, hipMemcpyAsync(d, host.data(), sizeof(UnitDesc) * hs.size(), hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  c->unit_tables[hs] = d;
  *out = d;
  return ICM_OK;
}

// The cluster-move layout all of the units share (a kernel built for it alone
// runs them), else kLayAny.
int group_layout(icm_ctx* c, const std::vector<int32_t>& hs) {
  int lay = -1;
  for (int32_t h : hs) {
    const UnitDesc& u = find(c, h)->unit;
    const int l = icm::unit_layout(u.topo, u.L, u.deg, u.N);
    if (lay >= 0 && l != lay) return icm::kLayAny;
    lay = l;
  }
  return lay < 0 ? icm::kLayAny : lay;
}

int launch_group(icm_ctx* c, const Group& g, uint32_t n_sweeps, bool per_instance, hipStream_t strm) {
  const int threads = class_threads(c->cfg, g.cls);
  const int layout = group_layout(c, g.handles);
  size_t lds = 0;
  int tables = 1;
  const int slots = effective_slots(c, g.handles, threads, c->cfg.icm_slots, lds, tables);
  if (lds > c->lds_limit)
    return fail(c, ICM_E_INVALID, "instance needs %zu bytes of LDS, the device allows %zu", lds, c->lds_limit);
  const uint32_t spl = c->cfg.sweeps_per_launch > 0 ? (uint32_t)c->cfg.sweeps_per_launch : n_sweeps;
  if (per_instance) {
    for (int32_t h : g.handles) {
      UnitDesc* d = nullptr;
      std::vector<int32_t> one{h};
      int rc = unit_table(c, one, &d);
      if (rc) return rc;
      for (uint32_t done = 0; done < n_sweeps; done += spl) {
        const uint32_t n = std::min(spl, n_sweeps - done);
        KERNEL_OK(c, icmk_launch_sweep(d, 1, g.jkind, g.deg, tables, group_layout(c, one), n, threads, slots,
                                       lds, strm));
      }
    }
    return ICM_OK;
  }
  UnitDesc* d = nullptr;
  int rc = unit_table(c, g.handles, &d);
  if (rc) return rc;
  const uint32_t full = n_sweeps / spl, rest = n_sweeps % spl;
  if (c->cfg.use_graph && full > 1) {
    icm_ctx::GraphKey key{g.handles, spl, full, threads, slots + 64 * tables};
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
      // Capture on a private stream (the context stream may be the legacy null
      // stream, which cannot be captured); the graph is replayed on strm.
      if (!c->capture_stream)
        HIP_OK(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
      HIP_OK(c, hipStreamSynchronize(c->stream));
      hipGraph_t graph;
      HIP_OK(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
      for (uint32_t x = 0; x < full; ++x) {
        int e = icmk_launch_sweep(d, (int)g.handles.size(), g.jkind, g.deg, tables, layout, spl, threads,
                                  slots, lds, c->capture_stream);
        if (e) {
          hipGraph_t dummy;
          (void)hipStreamEndCapture(c->capture_stream, &dummy);
          return fail(c, ICM_E_DEVICE, "launch during capture failed");
        }
      }
      HIP_OK(c, hipStreamEndCapture(c->capture_stream, &graph));
      hipGraphExec_t exec;
      HIP_OK(c, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      HIP_OK(c, hipGraphDestroy(graph));
      it = c->graphs.emplace(key, exec).first;
    }
    HIP_OK(c, hipGraphLaunch(it->second, strm));
  } else {
    for (uint32_t x = 0; x < full; ++x)
      KERNEL_OK(c, icmk_launch_sweep(d, (int)g.handles.size(), g.jkind, g.deg, tables, layout, spl, threads, slots,
                                     lds, strm));
  }
  if (rest)
    KERNEL_OK(c, icmk_launch_sweep(d, (int)g.handles.size(), g.jkind, g.deg, tables, layout, rest, threads, slots,
                                   lds, strm));
  return ICM_OK;
}

int run_impl(icm_ctx* c, const int32_t* handles, int32_t n, uint32_t n_sweeps, bool per_instance) {
  if (n < 0 || (n > 0 && !handles)) return fail(c, ICM_E_INVALID, "bad handle list");
  for (int x = 0; x < n; ++x) {
    if (!find(c, handles[x])) return fail(c, ICM_E_NOTFOUND, "unknown handle %d", handles[x]);
    for (int y = 0; y < x; ++y)
      if (handles[y] == handles[x]) return fail(c, ICM_E_INVALID, "handle %d listed twice", handles[x]);
  }
  if (n == 0 || n_sweeps == 0) return ICM_OK;
  const std::vector<Group> groups = group_handles(c, handles, n);
  if (per_instance || groups.size() == 1) {
    for (const Group& g : groups) {
      int rc = launch_group(c, g, n_sweeps, per_instance, c->stream);
      if (rc) return rc;
    }
  } else {
    // The groups run concurrently on up to three side streams (fork after the
    // work queued so far, join the context stream to all of them): a class of
    // small, latency-bound units then shares the device with the large ones
    // instead of holding it alone, which measured faster on the uneven 3D
    // batch than running classes that fill the device one after another.
    const size_t nside = std::min<size_t>(groups.size(), 3);
    while (c->events.size() < nside + 1) {
      hipEvent_t e;
      HIP_OK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
      c->events.push_back(e);
    }
    for (size_t x = 0; x < nside; ++x)
      if (!c->side[x]) HIP_OK(c, hipStreamCreateWithFlags(&c->side[x], hipStreamNonBlocking));
    // device work tables first: building one synchronises the context stream,
    // which must not wait for a group already launched
    for (const Group& g : groups) {
      UnitDesc* d = nullptr;
      int rc = unit_table(c, g.handles, &d);
      if (rc) return rc;
    }
    HIP_OK(c, hipEventRecord(c->events[0], c->stream));
    for (size_t x = 0; x < nside; ++x) HIP_OK(c, hipStreamWaitEvent(c->side[x], c->events[0], 0));
    for (size_t x = 0; x < groups.size(); ++x) {
      int rc = launch_group(c, groups[x], n_sweeps, false, c->side[x % 3]);
      if (rc) return rc;
    }
    for (size_t x = 0; x < nside; ++x) {
      HIP_OK(c, hipEventRecord(c->events[x + 1], c->side[x]));
      HIP_OK(c, hipStreamWaitEvent(c->stream, c->events[x + 1], 0));
    }
  }
  for (int x = 0; x < n; ++x) find(c, handles[x])->sweep_host += n_sweeps;
  return ICM_OK;
}

struct HostState {
  std::vector<uint32_t> spins;
  std::vector<int32_t> at;
  std::vector<uint8_t> gauge;
  std::vector<int64_t> energy;
};

int fetch_state(icm_ctx* c, Instance* in, HostState& hs, bool spins) {
  hs.at.resize((size_t)in->K * in->R);
  hs.gauge.resize(in->Wp);
  hs.energy.resize(in->Wp);
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (spins) {
    hs.spins.resize((size_t)in->Wq * in->N);
    HIP_OK(c, hipMemcpy(hs.spins.data(), in->unit.spins, hs.spins.size() * 4, hipMemcpyDeviceToHost));
  }
  HIP_OK(c, hipMemcpy(hs.at.data(), in->unit.at, hs.at.size() * 4, hipMemcpyDeviceToHost));
  HIP_OK(c, hipMemcpy(hs.gauge.data(), in->unit.gauge, hs.gauge.size(), hipMemcpyDeviceToHost));
  HIP_OK(c, hipMemcpy(hs.energy.data(), in->unit.energy, hs.energy.size() * 8, hipMemcpyDeviceToHost));
  return ICM_OK;
}

void states_from(const Instance* in, const HostState& hs, int8_t* out) {
  const int N = in->N;
  for (int k = 0; k < in->K; ++k)
    for (int r = 0; r < in->R; ++r) {
      const int w = hs.at[(size_t)k * in->R + r];
      const int q = w >> 2, b = w & 3;
      const int sign = hs.gauge[w] ? -1 : 1;
      int8_t* dst = out + ((size_t)k * in->R + r) * N;
      for (int i = 0; i < N; ++i)
        dst[i] = (int8_t)(sign * (int)(int8_t)(uint8_t)(hs.spins[(size_t)q * N + i] >> (8 * b)));
    }
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char* icm_strerror(int code) {
  switch (code) {
    case ICM_OK: return "ok";
    case ICM_E_INVALID: return "invalid argument";
    case ICM_E_NOMEM: return "arena exhausted";
    case ICM_E_DEVICE: return "device error";
    case ICM_E_NOTFOUND: return "not found";
    case ICM_E_BUSY: return "busy";
    case ICM_E_BUFSIZE: return "buffer too small";
    default: return "unknown error";
  }
}

const char* icm_last_error(icm_ctx* c) { return c ? c->last_error.c_str() : "null context"; }

int icm_create(icm_ctx** out, int device, void* stream, void* arena, size_t arena_bytes, uint32_t seed) {
  if (!out) return ICM_E_INVALID;
  *out = nullptr;
  if (!arena || arena_bytes < (1u << 20) || ((uintptr_t)arena & 255)) return ICM_E_INVALID;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return ICM_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return ICM_E_DEVICE;
  auto c = std::make_unique<icm_ctx>();
  c->device = device;
  c->stream = (hipStream_t)stream;
  c->seed = seed;
  c->arena.reset((char*)arena, arena_bytes);
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
    c->lds_limit = (size_t)lds;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    c->n_cus = cus;
  int lds_cu = 0;
  c->lds_cu = c->lds_limit;
  if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) == hipSuccess &&
      lds_cu > 0)
    c->lds_cu = std::max(c->lds_limit, (size_t)lds_cu);
  (void)icmk_set_lds_limit(c->lds_limit);
  (void)icmk_set_percolation_lds_limit(c->lds_limit);
  (void)hipGetLastError();
  *out = c.release();
  return ICM_OK;
}

int icm_destroy(icm_ctx* c) {
  if (!c) return ICM_E_INVALID;
  icm_serve_stop(c);
  (void)hipStreamSynchronize(c->stream);
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  for (hipStream_t& x : c->side)
    if (x) (void)hipStreamDestroy(x);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  delete c;
  return ICM_OK;
}

size_t icm_instance_bytes(const icm_instance_desc* d) {
  std::string why;
  if (validate_desc(d, why)) return 0;
  Topology T;
  if (!build_topology(d->topology, d->L, T)) return 0;
  Sizes S{};
  if (plan_instance(d, T, S, nullptr, nullptr, why)) return 0;
  return total_bytes(S);
}

int icm_add_instance(icm_ctx* c, const icm_instance_desc* d, int32_t* out) {
  int rc = guard(c);
  if (rc) return rc;
  if (!out) return fail(c, ICM_E_INVALID, "null output handle");
  return add_instance_impl(c, d, out);
}

int icm_remove_instance(icm_ctx* c, int32_t h) {
  int rc = guard(c);
  if (rc) return rc;
  Instance* in = find(c, h);
  if (!in) return fail(c, ICM_E_NOTFOUND, "unknown handle %d", h);
  HIP_OK(c, hipStreamSynchronize(c->stream));
  drop_cached_tables(c, h);
  release_instance(c, in);
  c->instances.erase(h);
  return ICM_OK;
}

static int init_states_impl(icm_ctx* c, int32_t h) {
  int rc = ICM_OK;
  Instance* in = find(c, h);
  if (!in) return fail(c, ICM_E_NOTFOUND, "unknown handle %d", h);
  KERNEL_OK(c, icmk_launch_init(in->unit.spins, in->N, in->Wq, in->W, c->seed, in->key, c->stream));
  rc = reset_walkers(c, in, 0);
  if (rc) return rc;
  KERNEL_OK(c, icmk_launch_energy(in->unit.spins, in->unit.nbr, in->unit.coup, in->N, in->deg, in->Wp,
                                  in->jkind, in->jexp, in->unit.energy, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return ICM_OK;
}

int icm_init_states(icm_ctx* c, int32_t h) {
  int rc = guard(c);
  if (rc) return rc;
  return init_states_impl(c, h);
}

int icm_set_temperatures(icm_ctx* c, int32_t h, const double* temps) {
  int rc = guard(c);
  if (rc) return rc;
  Instance* in = find(c, h);
  if (!in) return fail(c, ICM_E_NOTFOUND, "unknown handle %d", h);
  if (!temps) return fail(c, ICM_E_INVALID, "null temperatures");
  const int K = in->K;
  for (int k = 0; k < K; ++k) {
    if (!(temps[k] > 0.0) || !std::isfinite(temps[k]))
      return fail(c, ICM_E_INVALID, "temperatures must be finite and > 0");
    if (k > 0 && !(temps[k] > temps[k - 1]))
      return fail(c, ICM_E_INVALID, "temperatures must be strictly ascending");
  }
  UnitDesc& U = in->unit;
  std::vector<uint32_t> thr, ptthr;
  if (in->jkind == ICM_J_INT8) {
    // the same tables as at creation, over the instance's local-field bound
    thr.assign((size_t)K * in->HM, 0);
    for (int k = 0; k < K; ++k) {
      const double beta = 1.0 / temps[k];
      thr[(size_t)k * in->HM] = 4294967295u;
      for (int e = 1; e < in->HM; ++e)
        thr[(size_t)k * in->HM + e] = threshold_of(-(beta * (double)(2 * e)) / (double)in->jscale);
    }
    if (in->ptlen > 0) {
      // the PT table keeps its length: every gap past it must have a zero threshold
      ptthr.assign((size_t)(K - 1) * in->ptlen, 0);
      for (int k = 0; k + 1 < K; ++k) {
        const double dbeta = 1.0 / temps[k] - 1.0 / temps[k + 1];
        if (threshold_of(-(dbeta * (double)(in->ptlen + 1)) / (double)in->jscale) != 0)
          return fail(c, ICM_E_INVALID, "temperatures %d, %d too close for the instance's PT table", k, k + 1);
        for (int D = 1; D <= in->ptlen; ++D)
          ptthr[(size_t)k * in->ptlen + D - 1] = threshold_of(-(dbeta * (double)D) / (double)in->jscale);
      }
    }
  }
  std::vector<double> beta(K);
  std::vector<float> bl2e(K);
  for (int k = 0; k < K; ++k) {
    beta[k] = 1.0 / temps[k];
    bl2e[k] = (float)(beta[k] / std::log(2.0));
  }
  if (!thr.empty())
    HIP_OK(c, hipMemcpyAsync((void*)U.thr, thr.data(), thr.size() * 4, hipMemcpyHostToDevice, c->stream));
  if (!ptthr.empty())
    HIP_OK(c, hipMemcpyAsync((void*)U.ptthr, ptthr.data(), ptthr.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync((void*)U.beta, beta.data(), (size_t)K * 8, hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync((void*)U.bl2e, bl2e.data(), (size_t)K * 4, hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  in->temps.assign(temps, temps + K);
  return ICM_OK;
}

int icm_percolation_smax(icm_ctx* c, int32_t topology, int32_t L, double p, uint32_t sample0,
                         uint32_t n_samples, uint32_t key, int32_t* smax) {
  int rc = guard(c);
  if (rc) return rc;
  if (!(p >= 0.0 && p <= 1.0)) return fail(c, ICM_E_INVALID, "occupation probability outside [0, 1]");
  if (n_samples > 0 && !smax) return fail(c, ICM_E_INVALID, "null output");
  if ((uint64_t)sample0 + n_samples > (1ull << 32))
    return fail(c, ICM_E_INVALID, "sample indices beyond 2^32");
  Topology* T = get_topology(c, topology, L, rc, icm::kMaxPercSites);
  if (!T) return fail(c, rc, "invalid topology or size");
  if (T->N > icm::kMaxPercSites || icmk_percolation_lds(T->N) > c->lds_limit)
    return fail(c, ICM_E_INVALID, "%d sites exceed the percolation kernel's LDS", T->N);
  // floor(p 2^32) is exact in double: p scaled by a power of two
  const unsigned long long thr = (unsigned long long)std::floor(p * 4294967296.0);
  KERNEL_OK(c, icmk_launch_percolation(T->d_nbr, T->N, T->deg, thr, sample0, n_samples, c->seed, key, smax,
                                       c->n_cus, c->lds_cu, c->stream));
  return ICM_OK;
}

int icm_set_states(icm_ctx* c, int32_t h, const int8_t* spins, uint32_t sweep0) {
  int rc = guard(c);
  if (rc) return rc;
  Instance* in = find(c, h);
  if (!in) return fail(c, ICM_E_NOTFOUND, "unknown handle %d", h);
  if (!spins) return fail(c, ICM_E_INVALID, "null spins");
  const size_t bytes = (size_t)in->W * in->N;
  int8_t* tmp = (int8_t*)c->arena.alloc(bytes);
  if (!tmp) return fail(c, ICM_E_NOMEM, "arena full (state staging)");
  int r = ICM_OK;
  if (hipMemcpyAsync(tmp, spins, bytes, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      icmk_launch_scatter(in->unit.spins, tmp, in->N, in->Wq, in->W, c->stream) != 0 ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    r = fail(c, ICM_E_DEVICE, "state upload failed");
  c->arena.release(tmp);
  if (r) return r;
  rc = reset_walkers(c, in, sweep0);
  if (rc) return rc;
  KERNEL_OK(c, icmk_launch_energy(in->unit.spins, in->unit.nbr, in->unit.coup, in->N, in->deg, in->Wp,
                                  in->jkind, in->jexp, in->unit.energy, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return ICM_OK;
}

int icm_run(icm_ctx* c, const int32_t* handles, int32_t n, uint32_t n_sweeps) {
  int rc = guard(c);
  if (rc) return rc;
  return run_impl(c, handles, n, n_sweeps, false);
}

int icm_run_per_instance(icm_ctx* c, const int32_t* handles, int32_t n, uint32_t n_sweeps) {
  int rc = guard(c);
  if (rc) return rc;
  return run_impl(c, handles, n, n_sweeps, true);
}

int icm_sync(icm_ctx* c) {
  int rc = guard(c);
  if (rc) return rc;
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return ICM_OK;
}

int icm_set_run_config(icm_ctx* c, const icm_run_config* cfg) {
  int rc = guard(c);
  if (rc) return rc;
  if (!cfg) return fail(c, ICM_E_INVALID, "null config");
  icm_run_config n = c->cfg;
  auto valid_threads = [](int t) { return t == 64 || t == 128 || t == 256 || t == 512 || t == 1024 || t == -1; };
  if (cfg->threads) {
    if (!valid_threads(cfg->threads))
      return fail(c, ICM_E_INVALID, "threads must be 64, 128, 256, 512, 1024, or -1 for the per-class default");
    n.threads = cfg->threads < 0 ? 0 : cfg->threads;
  }
  for (int k = 0; k < 4; ++k) {
    if (!cfg->class_threads[k]) continue;
    if (!valid_threads(cfg->class_threads[k]))
      return fail(c, ICM_E_INVALID, "class_threads[%d] must be 64, 128, 256, 512, 1024, or -1 to clear", k);
    n.class_threads[k] = cfg->class_threads[k] < 0 ? 0 : cfg->class_threads[k];
  }
  if (cfg->sweeps_per_launch < 0) return fail(c, ICM_E_INVALID, "negative sweeps_per_launch");
  if (cfg->sweeps_per_launch) n.sweeps_per_launch = cfg->sweeps_per_launch;
  n.use_graph = cfg->use_graph ? 1 : 0;
  if (cfg->icm_slots < 0 || cfg->icm_slots > 64) return fail(c, ICM_E_INVALID, "icm_slots must be 0..64");
  if (cfg->icm_slots) n.icm_slots = cfg->icm_slots;
  if (cfg->table_placement < 0 || cfg->table_placement > 2)
    return fail(c, ICM_E_INVALID, "table_placement must be 0, 1 or 2");
  n.table_placement = cfg->table_placement;
  c->cfg = n;
  return ICM_OK;
}

int icm_get_run_config(icm_ctx* c, icm_run_config* cfg) {
  if (!c || !cfg) return ICM_E_INVALID;
  if (c->serving) return ICM_E_BUSY;
  *cfg = c->cfg;
  return ICM_OK;
}

static int read_energies_impl(icm_ctx* c, int32_t h, int64_t* raw, double* real, size_t cap) {
  int rc = ICM_OK;
  Instance* in = find(c, h);
  if (!in) return fail(c, ICM_E_NOTFOUND, "unknown handle %d", h);
  if (cap < (size_t)in->K * in->R) return fail(c, ICM_E_BUFSIZE, "need %d elements", in->K * in->R);
  HostState hs;
  rc = fetch_state(c, in, hs, false);
  if (rc) return rc;
  const double unit = in->jkind == ICM_J_F32 ? std::ldexp(1.0, -40) : 1.0 / in->jscale;
  for (int x = 0; x < in->K * in->R; ++x) {
    const int64_t e = hs.energy[hs.at[x]];
    if (raw) raw[x] = e;
    if (real) real[x] = (double)e * unit;
  }
  return ICM_OK;
}

int icm_read_energies(icm_ctx* c, int32_t h, int64_t* raw, double* real, size_t cap) {
  int rc = guard(c);
  if (rc) return rc;
  return read_energies_impl(c, h, raw, real, cap);
}

static int read_states_impl(icm_ctx* c, int32_t h, int8_t* out, size_t cap) {
  int rc = ICM_OK;
  Instance* in = find(c, h);
  if (!in) return fail(c, ICM_E_NOTFOUND, "unknown handle %d", h);
  if (!out || cap < (size_t)in->W * in->N) return fail(c, ICM_E_BUFSIZE, "need %d bytes", in->W * in->N);
  HostState hs;
  rc = fetch_state(c, in, hs, true);
  if (rc) return rc;
  states_from(in, hs, out);
  return ICM_OK;
}

int icm_read_states(icm_ctx* c, int32_t h, int8_t* out, size_t cap) {
  int rc = guard(c);
  if (rc) return rc;
  return read_states_impl(c, h, out, cap);
}

int icm_read_walkers(icm_ctx* c, int32_t h, int32_t* out, size_t cap) {
  int rc = guard(c);
  if (rc) return rc;
  Instance* in = find(c, h);
  if (!in) return fail(c, ICM_E_NOTFOUND, "unknown handle %d", h);
  if (!out || cap < (size_t)in->K * in->R) return fail(c, ICM_E_BUFSIZE, "need %d elements", in->K * in->R);
  HostState hs;
  rc = fetch_state(c, in, hs, false);
  if (rc) return rc;
  std::memcpy(out, hs.at.data(), hs.at.size() * 4);
  return ICM_OK;
}

int icm_read_overlaps(icm_ctx* c, int32_t h, int32_t* q_sum, int32_t* ql_sum, size_t cap) {
  int rc = guard(c);
  if (rc) return rc;
  Instance* in = find(c, h);
  if (!in) return fail(c, ICM_E_NOTFOUND, "unknown handle %d", h);
  const int half = in->R / 2, n = in->K * half;
  if (cap < (size_t)n) return fail(c, ICM_E_BUFSIZE, "need %d elements", n);
  int32_t* d = (int32_t*)c->arena.alloc((size_t)2 * n * 4);
  if (!d) return fail(c, ICM_E_NOMEM, "arena full (overlap readout)");
  std::vector<int32_t> host((size_t)2 * n);
  const int e = icmk_launch_overlaps(in->unit.spins, in->unit.nbr, in->unit.at, in->unit.gauge, in->N, in->deg,
                                     in->K, in->R, in->topo->topo, (int)in->topo->bonds.size(), d, d + n,
                                     c->stream);
  int r = ICM_OK;
  if (e != 0 || hipMemcpyAsync(host.data(), d, host.size() * 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    r = fail(c, ICM_E_DEVICE, "overlap readout failed");
  c->arena.release(d);
  if (r) return r;
  if (q_sum) std::memcpy(q_sum, host.data(), (size_t)n * 4);
  if (ql_sum) std::memcpy(ql_sum, host.data() + n, (size_t)n * 4);
  return ICM_OK;
}

int icm_read_labels(icm_ctx* c, int32_t h, int32_t k, int32_t pair, int32_t* labels, int32_t* seed,
                    int32_t* n_minus, size_t cap) {
  int rc = guard(c);
  if (rc) return rc;
  Instance* in = find(c, h);
  if (!in) return fail(c, ICM_E_NOTFOUND, "unknown handle %d", h);
  if (!(in->flags & ICM_FLAG_RECORD_LABELS)) return fail(c, ICM_E_INVALID, "instance does not record labels");
  const int half = in->R / 2;
  if (k < 0 || k >= in->Kc || pair < 0 || pair >= half) return fail(c, ICM_E_INVALID, "no ICM at (k, pair)");
  if (!labels || cap < (size_t)in->N) return fail(c, ICM_E_BUFSIZE, "need %d elements", in->N);
  const int mv = k * half + pair, nmoves = in->Kc * half;
  HIP_OK(c, hipStreamSynchronize(c->stream));
  HIP_OK(c, hipMemcpy(labels, in->unit.labels + (size_t)mv * in->N, (size_t)in->N * 4, hipMemcpyDeviceToHost));
  int32_t sv[2];
  HIP_OK(c, hipMemcpy(&sv[0], in->unit.seeds + mv, 4, hipMemcpyDeviceToHost));
  HIP_OK(c, hipMemcpy(&sv[1], in->unit.seeds + nmoves + mv, 4, hipMemcpyDeviceToHost));
  if (seed) *seed = sv[0];
  if (n_minus) *n_minus = sv[1];
  return ICM_OK;
}

int icm_read_observables(icm_ctx* c, int32_t h, int64_t* sums, int64_t* counts, size_t cap) {
  int rc = guard(c);
  if (rc) return rc;
  Instance* in = find(c, h);
  if (!in) return fail(c, ICM_E_NOTFOUND, "unknown handle %d", h);
  if (!(in->flags & ICM_FLAG_MEASURE)) return fail(c, ICM_E_INVALID, "instance does not measure observables");
  const size_t n = in->obs_words - icm::kObsBins;
  if (cap < n) return fail(c, ICM_E_BUFSIZE, "observables need %zu elements", n);
  std::vector<int64_t> all(in->obs_words);
  HIP_OK(c, hipStreamSynchronize(c->stream));
  HIP_OK(c, hipMemcpy(all.data(), in->unit.obs, in->obs_words * 8, hipMemcpyDeviceToHost));
  if (sums) std::memcpy(sums, all.data(), n * 8);
  if (counts) std::memcpy(counts, all.data() + n, icm::kObsBins * 8);
  return ICM_OK;
}

int icm_read_stats(icm_ctx* c, int32_t h, icm_stats* out) {
  int rc = guard(c);
  if (rc) return rc;
  Instance* in = find(c, h);
  if (!in) return fail(c, ICM_E_NOTFOUND, "unknown handle %d", h);
  if (!out) return fail(c, ICM_E_INVALID, "null output");
  unsigned long long s[icm::kNumStats];
  HIP_OK(c, hipStreamSynchronize(c->stream));
  HIP_OK(c, hipMemcpy(s, in->unit.stats, sizeof s, hipMemcpyDeviceToHost));
  out->sweeps = s[icm::kStatSweeps];
  out->metro_accepts = s[icm::kStatMetroAcc];
  out->icm_moves = s[icm::kStatIcmMoves];
  out->icm_nontrivial = s[icm::kStatIcmNontrivial];
  out->icm_cluster_sites = s[icm::kStatIcmSites];
  out->icm_2a_flips = s[icm::kStat2a];
  out->pt_attempts = s[icm::kStatPtAttempts];
  out->pt_accepts = s[icm::kStatPtAccepts];
  return ICM_OK;
}

uint32_t icm_sweep_index(icm_ctx* c, int32_t h) {
  if (!c || c->serving) return 0;
  Instance* in = find(c, h);
  return in ? in->sweep_host : 0;
}

int icm_arena_usage(icm_ctx* c, size_t* used, size_t* total) {
  if (!c) return ICM_E_INVALID;
  if (c->serving) return ICM_E_BUSY;
  if (used) *used = c->arena.used();
  if (total) *total = c->arena.size();
  return ICM_OK;
}

}  // extern "C"

// ============================================================================
// Serving loop: continuous batching at sweep-block boundaries.
// ============================================================================
namespace {

size_t desc_coupling_bytes(const icm_instance_desc* d) {
  return (size_t)coupling_count(d->topology, d->L) * (d->jkind == ICM_J_F32 ? 4 : 1);
}

// Resident requests that share a kernel variant and size class advance
// together, one sweep block at a time, on a serving stream of their own: a
// group launches its next block as soon as its previous one is done, so small
// requests are not held back by the block time of large ones.
struct ServeGroup {
  int jkind = 0, deg = 0, cls = 0;
  std::vector<std::shared_ptr<Request>> members;   // resident, not finished
  std::vector<std::shared_ptr<Request>> inflight;  // those in the running block
  uint32_t block = 0;
  bool running = false;
  hipStream_t strm = nullptr;
  hipEvent_t done = nullptr;
};

void retire(icm_ctx* c, const std::shared_ptr<Request>& r) {
  Instance* in = find(c, r->handle);
  std::vector<int64_t> e((size_t)in->K * in->R);
  std::vector<int8_t> st((size_t)in->W * in->N);
  read_energies_impl(c, r->handle, e.data(), nullptr, e.size());
  read_states_impl(c, r->handle, st.data(), st.size());
  drop_cached_tables(c, r->handle);
  release_instance(c, in);
  c->instances.erase(r->handle);
  std::lock_guard<std::mutex> lk(c->mu);
  r->energies = std::move(e);
  r->states = std::move(st);
  r->done = true;
  r->t_done = std::chrono::steady_clock::now();
}

void fail_all(icm_ctx* c, std::vector<ServeGroup>& groups) {
  c->poisoned = true;
  std::lock_guard<std::mutex> lk(c->mu);
  for (auto& g : groups)
    for (auto& r : g.members) {
      r->error = ICM_E_DEVICE;
      r->done = true;
      r->t_done = std::chrono::steady_clock::now();
    }
  for (auto& r : c->queue) {
    r->error = ICM_E_DEVICE;
    r->done = true;
    r->t_done = std::chrono::steady_clock::now();
  }
  c->queue.clear();
}

void serve_loop(icm_ctx* c) {
  constexpr int kServeStreams = 4;
  hipStream_t streams[kServeStreams] = {};
  std::vector<ServeGroup> groups;
  bool ok = true;
  for (auto& x : streams) ok = ok && hipStreamCreateWithFlags(&x, hipStreamNonBlocking) == hipSuccess;
  auto group_of = [&](Instance* in) -> ServeGroup* {
    const int cls = size_class(in->N);
    for (auto& g : groups)
      if (g.jkind == in->jkind && g.deg == in->deg && g.cls == cls) return &g;
    ServeGroup g;
    g.jkind = in->jkind;
    g.deg = in->deg;
    g.cls = cls;
    g.strm = streams[groups.size() % kServeStreams];
    if (hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess) return nullptr;
    groups.push_back(std::move(g));
    return &groups.back();
  };
  auto resident = [&] {
    for (auto& g : groups)
      if (!g.members.empty()) return true;
    return false;
  };
  while (ok) {
    bool progressed = false, stopping = false;
    std::vector<std::shared_ptr<Request>> admitted;
    {
      std::lock_guard<std::mutex> lk(c->mu);
      stopping = !c->serving;
      if (stopping) {
        // stopping: whatever is still queued is returned unrun
        for (auto& r : c->queue) {
          r->error = ICM_E_BUSY;
          r->done = true;
          r->t_done = std::chrono::steady_clock::now();
        }
        c->queue.clear();
      }
      // admission: as many queued requests as the arena holds, in arrival order
      while (!c->queue.empty() && !c->poisoned) {
        std::shared_ptr<Request> r = c->queue.front();
        int32_t h = -1;
        int rc = add_instance_impl(c, &r->desc, &h);
        if (rc == ICM_E_NOMEM && (resident() || !admitted.empty())) break;  // wait for a retirement
        c->queue.pop_front();
        if (rc == ICM_OK) rc = init_states_impl(c, h);
        if (rc != ICM_OK) {  // invalid, or larger than the whole arena
          r->error = rc;
          r->done = true;
          r->t_done = std::chrono::steady_clock::now();
          continue;
        }
        r->handle = h;
        admitted.push_back(r);
      }
    }
    if (!admitted.empty()) {
      progressed = true;
      // the hot starts ran on the context stream: done before any group uses them
      if (hipStreamSynchronize(c->stream) != hipSuccess) { fail_all(c, groups); break; }
      for (auto& r : admitted) {
        ServeGroup* g = group_of(find(c, r->handle));
        if (!g) { ok = false; break; }
        g->members.push_back(r);
      }
      if (!ok) { fail_all(c, groups); break; }
    }
    // completions
    for (auto& g : groups) {
      if (!g.running) continue;
      const hipError_t q = hipEventQuery(g.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) { ok = false; break; }
      g.running = false;
      progressed = true;
      for (auto& r : g.inflight) {
        r->done_sweeps += g.block;
        if (r->done_sweeps < r->n_sweeps) continue;
        g.members.erase(std::find(g.members.begin(), g.members.end(), r));
        retire(c, r);
      }
      g.inflight.clear();
    }
    if (!ok) { fail_all(c, groups); break; }
    // launches: every idle group with resident requests starts its next block
    for (auto& g : groups) {
      if (g.running || g.members.empty()) continue;
      uint32_t b = (uint32_t)c->serve_block;
      Group lg{g.jkind, g.deg, g.cls, icm::kLayAny, {}};
      for (auto& r : g.members) {
        b = std::min(b, r->n_sweeps - r->done_sweeps);
        lg.handles.push_back(r->handle);
      }
      if (launch_group(c, lg, b, false, g.strm) != ICM_OK || hipEventRecord(g.done, g.strm) != hipSuccess) {
        ok = false;
        break;
      }
      for (auto& r : g.members) find(c, r->handle)->sweep_host += b;
      g.inflight = g.members;
      g.block = b;
      g.running = true;
      progressed = true;
    }
    if (!ok) { fail_all(c, groups); break; }
    if (stopping) {
      bool busy = false;
      for (auto& g : groups) busy = busy || g.running || !g.members.empty();
      if (!busy) break;
    }
    if (!progressed) {
      std::unique_lock<std::mutex> lk(c->mu);
      c->cv.wait_for(lk, std::chrono::microseconds(200),
                     [&] { return (!c->queue.empty() && !c->poisoned) || !c->serving; });
    }
  }
  for (auto& x : streams)
    if (x) (void)hipStreamSynchronize(x);
  for (auto& g : groups) (void)hipEventDestroy(g.done);
  for (auto& x : streams)
    if (x) (void)hipStreamDestroy(x);
}

}  // namespace

extern "C" {

int icm_serve_start(icm_ctx* c, int32_t sweeps_per_block) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (c->serving) return ICM_E_BUSY;
  if (sweeps_per_block <= 0) return fail(c, ICM_E_INVALID, "sweeps_per_block must be > 0");
  c->serve_block = sweeps_per_block;
  c->serving = true;
  c->server = std::thread(serve_loop, c);
  return ICM_OK;
}

int icm_serve_stop(icm_ctx* c) {
  if (!c) return ICM_E_INVALID;
  if (!c->server.joinable()) return ICM_OK;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->serving = false;
  }
  c->cv.notify_all();
  c->server.join();
  return c->poisoned ? ICM_E_DEVICE : ICM_OK;
}

int icm_submit(icm_ctx* c, const icm_instance_desc* d, uint32_t n_sweeps, uint64_t* ticket) {
  if (!c || !ticket) return ICM_E_INVALID;
  std::string why;
  if (validate_desc(d, why)) return ICM_E_INVALID;
  if (n_sweeps == 0) return ICM_E_INVALID;
  auto r = std::make_shared<Request>();
  r->desc = *d;
  r->couplings.assign((const uint8_t*)d->couplings, (const uint8_t*)d->couplings + desc_coupling_bytes(d));
  r->temps.assign(d->temps, d->temps + d->n_temps);
  r->desc.couplings = r->couplings.data();
  r->desc.temps = r->temps.data();
  r->n_sweeps = n_sweeps;
  r->t_submit = std::chrono::steady_clock::now();
  {
    std::lock_guard<std::mutex> lk(c->mu);
    if (!c->serving) return ICM_E_BUSY;
    r->ticket = c->next_ticket++;
    c->requests[r->ticket] = r;
    c->queue.push_back(r);
    *ticket = r->ticket;
  }
  c->cv.notify_all();
  return ICM_OK;
}

int icm_poll(icm_ctx* c, uint64_t ticket, int32_t* done, double* latency_us) {
  if (!c || !done) return ICM_E_INVALID;
  std::lock_guard<std::mutex> lk(c->mu);
  auto it = c->requests.find(ticket);
  if (it == c->requests.end()) return ICM_E_NOTFOUND;
  *done = it->second->done ? 1 : 0;
  if (latency_us && it->second->done)
    *latency_us = std::chrono::duration<double, std::micro>(it->second->t_done - it->second->t_submit).count();
  return ICM_OK;
}

int icm_take_result(icm_ctx* c, uint64_t ticket, int64_t* energies, int8_t* states, size_t cap_e,
                    size_t cap_s) {
  if (!c) return ICM_E_INVALID;
  std::lock_guard<std::mutex> lk(c->mu);
  auto it = c->requests.find(ticket);
  if (it == c->requests.end()) return ICM_E_NOTFOUND;
  Request& r = *it->second;
  if (!r.done) return ICM_E_BUSY;
  if (r.error != ICM_OK || r.energies.empty()) {  // the request failed
    const int e = r.error != ICM_OK ? r.error : ICM_E_DEVICE;
    c->requests.erase(it);
    return e;
  }
  if ((energies && cap_e < r.energies.size()) || (states && cap_s < r.states.size())) return ICM_E_BUFSIZE;
  if (energies) std::memcpy(energies, r.energies.data(), r.energies.size() * 8);
  if (states) std::memcpy(states, r.states.data(), r.states.size());
  c->requests.erase(it);
  return ICM_OK;
}

}  // extern "C"
