// C ABI of the solver (declared in include/fdfd.h): argument checking, plan
// construction (analysis, level schedule, task lists, device arenas) and the
// calls that enqueue the kernels of fdfd_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "analysis.h"
#include "plan.hpp"

namespace fdfd {

const char* const kKernelClassNames[KC_COUNT] = {"setup",     "front_small", "large_tiles", "fwd_sweep",
                                                 "bwd_sweep", "residual",    "gradient"};

hipEvent_t profile_event(Plan& P) {
  if (!P.event_pool.empty()) {
    hipEvent_t e = P.event_pool.back();
    P.event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Caller has synchronised the stream the events were recorded on.
void profile_collect(Plan& P) {
  for (const PendingTiming& t : P.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.e0, t.e1) == hipSuccess) {
      KernelTotals& k = P.totals[t.cls];
      k.launches += 1;
      k.ms += ms;
      k.bytes += t.bytes;
      k.flops += t.flops;
    }
    P.event_pool.push_back(t.e0);
    P.event_pool.push_back(t.e1);
  }
  P.pending.clear();
}

}  // namespace fdfd

struct fdfd_plan_s {
  fdfd::Plan p;
};

// Work vectors of fdfd_solve_noalloc: one file-scope device array, which every
// GPU the library runs on holds (at its own address) until the process ends.
// Host code must not use the array's name as a device address: its address
// on each device comes from hipGetSymbolAddress (scratch_address below).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

using fdfd::Plan;

thread_local std::string g_error;

struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) changed = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

fdfd_status fail(Plan* P, fdfd_status s, const std::string& msg) {
  if (P) P->last_error = msg;
  g_error = msg;
  return s;
}

fdfd_status hip_fail(Plan* P, hipError_t e, const char* what) {
  return fail(P, FDFD_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Device address of the scratch array on device dev (which must be current),
// resolved once per device and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Carves one solve's work vectors (nsys x nrhs columns) from base, each
// region 256-byte aligned; returns the bytes used (base may be null to size).
size_t carve_solve_work(const Plan& P, int nrhs, unsigned char* base, fdfd::SolveWork* w) {
  const size_t cols = (size_t)P.desc.nsys * nrhs, cs = P.csize, N = (size_t)P.an.N;
  const size_t sum_u = std::max<size_t>(1, (size_t)P.an.upd_ptr.back());
  const size_t parts = std::max<size_t>(1, (size_t)P.part_total);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) & ~size_t(255);
    return base ? base + at : nullptr;
  };
  unsigned char* y = take(cols * N * cs);
  unsigned char* wv = take(cols * sum_u * cs);
  unsigned char* zv = take(cols * N * cs);
  unsigned char* pv = take(cols * parts * cs);
  unsigned char* res = take(cols * N * 16);
  unsigned char* partial = take(cols * (size_t)P.res_blocks * 16);
  if (w) {
    w->y = y;
    w->wv = wv;
    w->zv = zv;
    w->pv = pv;
    w->res = reinterpret_cast<double2*>(res);
    w->partial = reinterpret_cast<double*>(partial);
  }
  return off;
}

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::atoi(v);
}

template <typename T>
fdfd_status upload(Plan& P, T** dst, const std::vector<T>& src) {
  const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) return fail(&P, FDFD_ERR_NOMEM, "hipMalloc of an analysis table failed");
  P.allocations.push_back(d);
  P.device_bytes += (int64_t)bytes;
  if (!src.empty()) {
    e = hipMemcpy(d, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(&P, e, "uploading an analysis table");
  }
  *dst = static_cast<T*>(d);
  return FDFD_OK;
}

fdfd_status alloc(Plan& P, void** dst, size_t bytes) {
  bytes = std::max<size_t>(bytes, 256);
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) return fail(&P, FDFD_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  P.allocations.push_back(d);
  P.device_bytes += (int64_t)bytes;
  *dst = d;
  return FDFD_OK;
}

void free_all(Plan& P) {
  for (hipEvent_t& e : P.phase_ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  for (auto& g : P.graphs) (void)hipGraphExecDestroy(g.exec);
  P.graphs.clear();
  if (P.cap_stream) (void)hipStreamDestroy(P.cap_stream);
  P.cap_stream = nullptr;
  for (const auto& t : P.pending) {
    (void)hipEventDestroy(t.e0);
    (void)hipEventDestroy(t.e1);
  }
  P.pending.clear();
  for (hipEvent_t e : P.event_pool) (void)hipEventDestroy(e);
  P.event_pool.clear();
  for (void* d : P.allocations) (void)hipFree(d);
  P.allocations.clear();
  if (P.status_host) (void)hipHostFree(P.status_host);
  P.status_host = nullptr;
}

// Level schedule: the bottom levels whose panels fit the LDS budget run in the
// one-workgroup-per-front kernel; every level above them runs in the tile task
// graph, whose task list (topological: level, assembly, then block steps) is
// built here.  Tiles of a front's pivot columns (J < nbk) are assembled, then
// updated right-looking (UPD): one pivot block at a time in the rows of pivot
// blocks, so the pivot-block chain can proceed, and syrk_group blocks at a
// time in the update rows; the tiles of its Schur complement (I >= J >= nbk)
// are produced by SYRK tasks, each of which accumulates the products of a
// group of syrk_group pivot blocks and read-modify-writes its tile once per
// group (the first group also gathers the children's contributions, which is
// the assembly of those tiles).
void build_schedule(Plan& P, size_t small_cap, std::vector<int32_t>& tasks, std::vector<int32_t>& tile_base,
                    std::vector<int32_t>& is_tiled) {
  const fdfd::Analysis& A = P.an;
  const size_t cs = P.csize;
  const int T = 64;
  P.levels.clear();
  for (int l = 0; l < A.nlevels; ++l) {
    fdfd::LevelPlan L;
    L.first = A.level_ptr[l];
    L.count = A.level_ptr[l + 1] - A.level_ptr[l];
    L.max_m = L.max_p = L.max_u = 0;
    size_t need = 0;
    for (int k = L.first; k < L.first + L.count; ++k) {
      const int f = A.level_fronts[k];
      L.max_m = std::max(L.max_m, A.m(f));
      L.max_p = std::max(L.max_p, A.npiv[f]);
      L.max_u = std::max(L.max_u, A.nupd[f]);
      // panel, d, 1/d, then the dense routines' scratch (the LDL^T's 2 x 64
      // pivot-column buffer, and the stencils staged before it: 5p values and
      // 4p indices from d on); then the children's gather rows (two rows of m ints)
      const size_t scratch = std::max<size_t>(128, 5 * (size_t)A.npiv[f]);
      const size_t rows = (8 * (size_t)A.m(f) + 15) & ~size_t(15);
      need = std::max(need, ((size_t)A.m(f) * A.npiv[f] + 2 * (size_t)A.npiv[f] + scratch) * cs + rows);
      L.lbytes += P.front_lbytes[f];
    }
    // the one-workgroup kernel keeps at most 64 pivot columns (16 per wave)
    L.small = need <= small_cap && L.max_p <= 64;
    L.small_lds = need;
    P.levels.push_back(L);
  }
  P.small_prefix = 0;
  while (P.small_prefix < (int)P.levels.size() && P.levels[P.small_prefix].small) ++P.small_prefix;
  // the bottom levels whose fronts all have at most 64 rows and 40 pivots,
  // or at most 128 rows (two per lane) and 16 pivots, are factored one
  // wavefront per front, a launch per level, when the level's slices fit the
  // LDS (four per workgroup with one row per lane, one with two);
  // FDFD_WAVE_FRONTS caps the number of such levels (0 keeps every level in
  // the one-workgroup kernel)
  P.wave_front_levels.clear();
  {
    const int cap = env_int("FDFD_WAVE_FRONTS", 1 << 20);
    // fronts a two-row level needs (FDFD_WAVE_MIN_FRONTS); counted per
    // system, so that a batch of systems is factored exactly as each alone
    const int64_t two_row_min = env_int("FDFD_WAVE_MIN_FRONTS", 16 * P.n_cu);
    const size_t lds_dyn = P.lds_limit > 512 ? P.lds_limit - 512 : 65536;
    for (int l = 0; l < P.small_prefix && (int)P.wave_front_levels.size() < cap; ++l) {
      int mmax = 0, pmax = 0, umax = 0;
      for (int k = P.levels[l].first; k < P.levels[l].first + P.levels[l].count; ++k) {
        const int f = A.level_fronts[k];
        mmax = std::max(mmax, A.m(f));
        pmax = std::max(pmax, A.npiv[f]);
        umax = std::max(umax, A.nupd[f]);
      }
      const int nr = mmax > 64 ? 2 : 1;
      // per wave: four couplings per row (value and pivot column), later the
      // update rows of L (u x p) in the same bytes; p pivots, a 64-entry
      // column buffer, two rows of 64 nr gather indices
      const size_t ub = (std::max((size_t)umax * pmax * cs, 4 * (size_t)mmax * (cs + sizeof(int32_t))) + 15) / 16 * 16;
      const size_t ldsw = (ub + ((size_t)pmax + 64) * cs + 128 * (size_t)nr * sizeof(int32_t) + 15) / 16 * 16;
      const int wpg = nr == 2 ? 1 : 4;
      if (mmax > 128 || pmax > (nr == 2 ? 16 : 40) || (size_t)wpg * ldsw > lds_dyn) break;
      // a two-row level runs one wave per front: only with enough fronts to
      // fill the chip (otherwise a workgroup per front goes faster)
      if (nr == 2 && (int64_t)P.levels[l].count < two_row_min) break;
      P.wave_front_levels.push_back({(int)ldsw, pmax, nr});
    }
  }
  tasks.clear();
  tile_base.assign(A.nfronts, 0);
  is_tiled.assign(A.nfronts, 0);
  P.ntiles = 0;
  P.tiled_flops = 0;
  const int G = std::max(1, P.syrk_group);
  auto push = [&](int type, int f, int k, int I, int J) {
    tasks.push_back(type);
    tasks.push_back(f);
    tasks.push_back(k);
    tasks.push_back(I);
    tasks.push_back(J);
  };
  for (int l = P.small_prefix; l < (int)P.levels.size(); ++l) {
    const fdfd::LevelPlan& L = P.levels[l];
    int kmax = 0;
    for (int q = L.first; q < L.first + L.count; ++q) {
      const int f = A.level_fronts[q];
      const int nbk = (A.npiv[f] + T - 1) / T, nut = (A.nupd[f] + T - 1) / T, R = nbk + nut;
      is_tiled[f] = 1;
      tile_base[f] = P.ntiles;
      P.ntiles += R * (R + 1) / 2;
      P.tiled_flops += P.front_flops[f];
      kmax = std::max(kmax, nbk);
      for (int I = 0; I < R; ++I)
        for (int J = 0; J <= I && J < nbk; ++J) push(0, f, 0, I, J);
    }
    // Step k: DIAG(0) (k = 0 only); FUSED(k+1) = TRSM(k+1,k) + UPD(k+1,k+1,k) +
    // DIAG(k+1) while block k+1 is a pivot block; the other TRSM(I,k); the other
    // UPD(I,J,k).  Every task waits only for tasks listed before it.
    for (int k = 0; k < kmax; ++k) {
      if (k == 0)
        for (int q = L.first; q < L.first + L.count; ++q) push(1, A.level_fronts[q], 0, 0, 0);
      for (int q = L.first; q < L.first + L.count; ++q) {
        const int f = A.level_fronts[q];
        const int nbk = (A.npiv[f] + T - 1) / T;
        if (k + 1 < nbk) push(5, f, k + 1, k + 1, k + 1);
      }
      for (int q = L.first; q < L.first + L.count; ++q) {
        const int f = A.level_fronts[q];
        const int nbk = (A.npiv[f] + T - 1) / T, R = nbk + (A.nupd[f] + T - 1) / T;
        if (nbk <= k) continue;
        for (int I = k + 1; I < R; ++I)
          if (!(I == k + 1 && k + 1 < nbk)) push(2, f, k, I, k);
      }
      for (int q = L.first; q < L.first + L.count; ++q) {
        const int f = A.level_fronts[q];
        const int nbk = (A.npiv[f] + T - 1) / T, R = nbk + (A.nupd[f] + T - 1) / T;
        if (nbk <= k) continue;
        const int k1 = k + 1;
        for (int J = k1; J < nbk; ++J) {
          // rows of pivot blocks: one block at a time (the chain waits on them)
          for (int I = J; I < nbk; ++I)
            if (!(I == k1 && J == k1)) push(3, f, k | (k1 << 16), I, J);
          // update rows: a group of blocks at a time, the last group ending at J
          if (k1 == J || k1 % G == 0) {
            const int k0 = ((k1 - 1) / G) * G;
            for (int I = nbk; I < R; ++I) push(3, f, k0 | (k1 << 16), I, J);
          }
        }
      }
      // SYRK over the pivot blocks [k0, k + 1) once the group is complete
      for (int q = L.first; q < L.first + L.count; ++q) {
        const int f = A.level_fronts[q];
        const int nbk = (A.npiv[f] + T - 1) / T, R = nbk + (A.nupd[f] + T - 1) / T;
        if (nbk <= k || R == nbk) continue;
        const int k1 = k + 1;
        if (k1 % G != 0 && k1 != nbk) continue;
        const int k0 = ((k1 - 1) / G) * G;
        for (int J = nbk; J < R; ++J)
          for (int I = J; I < R; ++I) push(6, f, k0 | (k1 << 16), I, J);
      }
    }
    // INV(k) after the level's steps: the rest of each pivot block's inverse,
    // once step k's TRSM tasks are done (the last block with no TRSM inverts in DIAG)
    for (int q = L.first; q < L.first + L.count; ++q) {
      const int f = A.level_fronts[q];
      const int nbk = (A.npiv[f] + T - 1) / T, R = nbk + (A.nupd[f] + T - 1) / T;
      for (int k = 0; k < nbk && k < R - 1; ++k) push(4, f, k, k, k);
    }
  }
  P.ntile_tasks = (int32_t)(tasks.size() / 5);
}

// The bottom levels' sweep items (P.wave_levels set): every front of height
// <= H belongs to the subtree of its highest ancestor of height <= H, which
// one wavefront sweeps whole, children before parents (no wait between them);
// the fronts above H up to the wave levels' top are items of their own, level
// by level.  No subtree item depends on another.  H (FDFD_SWEEP_GROUP
// overrides it) is the highest level up to 3 that still has 16 fronts per CU.
void build_wave_items(Plan& P) {
  const fdfd::Analysis& A = P.an;
  const int lw = P.wave_levels;
  int hdef = 0;
  for (int l = 1; l <= 3 && l < lw; ++l)
    if ((int64_t)P.levels[l].count * P.desc.nsys >= 16 * (int64_t)P.n_cu) hdef = l;
  P.sweep_group = lw > 0 ? std::max(0, std::min(env_int("FDFD_SWEEP_GROUP", hdef), lw - 1)) : 0;
  const int H = P.sweep_group;
  std::vector<int32_t>& seq = P.wave_seq_host;
  std::vector<int32_t>& iptr = P.wave_item_ptr_host;
  seq.clear();
  iptr.assign(1, 0);
  std::vector<int32_t> stack;
  for (int l = 0; l < lw && l <= H; ++l)
    for (int k = P.levels[l].first; k < P.levels[l].first + P.levels[l].count; ++k) {
      const int g = A.level_fronts[k];
      const int par = A.parent[g];
      if (A.height[g] > H || (par >= 0 && A.height[par] <= H)) continue;  // not a subtree root
      // post-order of g's subtree: reversed pre-order with children pushed in order
      const size_t at = seq.size();
      stack.assign(1, g);
      while (!stack.empty()) {
        const int f = stack.back();
        stack.pop_back();
        seq.push_back(f);
        for (int c = A.child_ptr[f]; c < A.child_ptr[f + 1]; ++c) stack.push_back(A.child_list[c]);
      }
      std::reverse(seq.begin() + (std::ptrdiff_t)at, seq.end());
      iptr.push_back((int32_t)seq.size());
    }
  for (int l = H + 1; l < lw; ++l)
    for (int k = P.levels[l].first; k < P.levels[l].first + P.levels[l].count; ++k) {
      seq.push_back(A.level_fronts[k]);
      iptr.push_back((int32_t)seq.size());
    }
  P.wave_items = (int32_t)iptr.size() - 1;
}

// Graph replay of launch chains (FDFD_GRAPH).  A chain is recorded on the
// plan's own capture stream (the caller's may be the null stream, which cannot
// be captured), instantiated once per argument set and launched on the
// caller's stream.  While the caller records a graph of its own, the chain is
// launched directly into that recording.
constexpr size_t kMaxGraphs = 16;

template <typename Launch>
fdfd_status run_chain(Plan& P, std::vector<uint64_t> key, hipStream_t st, const char* what, Launch launch) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const bool outer = hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
  if (!(P.desc.flags & FDFD_GRAPH) || outer) {
    const hipError_t e = launch(st);
    return e == hipSuccess ? FDFD_OK : hip_fail(&P, e, what);
  }
  size_t i = 0;
  while (i < P.graphs.size() && P.graphs[i].key != key) ++i;
  if (i == P.graphs.size()) {
    if (P.graphs.size() >= kMaxGraphs) {
      // the oldest graph may still run on the last stream
      (void)hipStreamSynchronize(P.last_stream);
      (void)hipStreamSynchronize(st);
      (void)hipGraphExecDestroy(P.graphs.front().exec);
      P.graphs.erase(P.graphs.begin());
    }
    hipError_t e = hipStreamBeginCapture(P.cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(&P, e, "hipStreamBeginCapture");
    const hipError_t el = launch(P.cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(P.cap_stream, &g);
    if (el != hipSuccess || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(&P, el != hipSuccess ? el : e, what);
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiateWithFlags(&ex, g, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(&P, e, "hipGraphInstantiate");
    P.graphs.push_back(Plan::GraphEntry{std::move(key), ex});
    ++P.graph_records;
    i = P.graphs.size() - 1;
  } else if (i + 1 != P.graphs.size()) {
    Plan::GraphEntry g = std::move(P.graphs[i]);
    P.graphs.erase(P.graphs.begin() + i);
    P.graphs.push_back(std::move(g));
    i = P.graphs.size() - 1;
  }
  const hipError_t e = hipGraphLaunch(P.graphs[i].exec, st);
  return e == hipSuccess ? FDFD_OK : hip_fail(&P, e, "hipGraphLaunch");
}

inline uint64_t bits(const void* p) { return (uint64_t)(uintptr_t)p; }
inline uint64_t bits(double v) {
  uint64_t u;
  std::memcpy(&u, &v, sizeof(u));
  return u;
}

fdfd_status check_desc(const fdfd_desc* d) {
  if (!d) return fail(nullptr, FDFD_ERR_ARG, "desc is NULL");
  if (d->nx < 2 || d->ny < 2) return fail(nullptr, FDFD_ERR_ARG, "nx and ny must be >= 2");
  if (d->npml_x < 0 || d->npml_y < 0 || 2 * d->npml_x >= d->nx || 2 * d->npml_y >= d->ny)
    return fail(nullptr, FDFD_ERR_ARG, "need 0 <= 2*npml < n on both axes");
  if (d->nsys < 1 || d->nsys > 64) return fail(nullptr, FDFD_ERR_ARG, "nsys must be in [1, 64]");
  if (d->max_rhs < 1 || d->max_rhs > 64) return fail(nullptr, FDFD_ERR_ARG, "max_rhs must be in [1, 64]");
  if (d->prec != FDFD_C128 && d->prec != FDFD_C64_IR) return fail(nullptr, FDFD_ERR_ARG, "unknown precision");
  if (d->leaf < 0) return fail(nullptr, FDFD_ERR_ARG, "leaf must be >= 0");
  if (d->small_lds < -1) return fail(nullptr, FDFD_ERR_ARG, "small_lds must be >= -1");
  if (d->reserved != 0 || d->reserved2 != 0) return fail(nullptr, FDFD_ERR_ARG, "reserved fields must be 0");
  if (d->syrk_group < -1 || d->split_kb < -1 || d->block_split < -1)
    return fail(nullptr, FDFD_ERR_ARG, "schedule knobs must be >= -1");
  if (d->mem_cap_bytes < 0) return fail(nullptr, FDFD_ERR_ARG, "mem_cap_bytes must be >= 0");
  if (d->flags & ~(FDFD_ANALYZE_HOST_ONLY | FDFD_PROFILE | FDFD_GRAPH | FDFD_POL_TE))
    return fail(nullptr, FDFD_ERR_ARG, "unknown desc flags");
  if ((d->flags & FDFD_GRAPH) && ((d->flags & FDFD_PROFILE) || std::getenv("FDFD_TRACE")))
    return fail(nullptr, FDFD_ERR_ARG, "FDFD_GRAPH cannot be combined with FDFD_PROFILE or FDFD_TRACE");
  if ((int64_t)d->nx * d->ny > ((int64_t)1 << 28)) return fail(nullptr, FDFD_ERR_ARG, "grid too large");
  return FDFD_OK;
}

}  // namespace

extern "C" {

const char* fdfd_status_str(fdfd_status s) {
  switch (s) {
    case FDFD_OK: return "ok";
    case FDFD_ERR_ARG: return "invalid argument";
    case FDFD_ERR_STATE: return "call out of order";
    case FDFD_ERR_NOMEM: return "out of device memory";
    case FDFD_ERR_HIP: return "HIP runtime error";
    case FDFD_ERR_NUMERIC: return "numerical failure";
    case FDFD_WARN_PIVOT: return "pivots perturbed";
  }
  return "unknown status";
}

const char* fdfd_last_error(fdfd_plan plan) {
  if (!plan) return g_error.c_str();
  return plan->p.last_error.c_str();
}

fdfd_status fdfd_analyze(const fdfd_desc* desc, fdfd_plan* out) {
  if (!out) return fail(nullptr, FDFD_ERR_ARG, "out is NULL");
  *out = nullptr;
  const auto t_start = std::chrono::steady_clock::now();
  auto ms_since = [](std::chrono::steady_clock::time_point t) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
  };
  fdfd_status s = check_desc(desc);
  if (s != FDFD_OK) return s;
  fdfd_plan_s* h = new (std::nothrow) fdfd_plan_s();
  if (!h) return fail(nullptr, FDFD_ERR_NOMEM, "host allocation failed");
  Plan& P = h->p;
  P.desc = *desc;
  P.host_only = (desc->flags & FDFD_ANALYZE_HOST_ONLY) != 0;
  P.is_c64 = desc->prec == FDFD_C64_IR;
  P.csize = P.is_c64 ? 8 : 16;
  // static pivoting threshold: sqrt of the factor precision's unit roundoff
  // unless FDFD_PIVOT_TAU overrides it
  P.pivot_tau = P.is_c64 ? 2.44140625e-4 : 1.0536712127723509e-8;
  if (const char* t = std::getenv("FDFD_PIVOT_TAU")) {
    const double v = std::atof(t);
    if (v > 0.0 && v < 1.0) P.pivot_tau = v;
  }
  const int leaf = desc->leaf > 0 ? desc->leaf : env_int("FDFD_LEAF", 36);
  const std::string err = fdfd::analyze_grid(desc->nx, desc->ny, leaf, P.an);
  if (!err.empty()) {
    delete h;
    return fail(nullptr, FDFD_ERR_ARG, err);
  }
  P.front_flops.resize(P.an.nfronts);
  P.front_lbytes.resize(P.an.nfronts);
  P.factor_lbytes = 0;
  for (int f = 0; f < P.an.nfronts; ++f) {
    const double p = P.an.npiv[f], u = P.an.nupd[f];
    P.front_flops[f] = 8.0 * (p * p * p + 3.0 * p * p * u + 3.0 * p * u * u) / 6.0;
    P.front_lbytes[f] = (p * (p + 1) / 2 + u * p) * (double)P.csize;
    P.factor_lbytes += P.front_lbytes[f];
  }
  P.analyze_ms = ms_since(t_start);
  const auto t_setup = std::chrono::steady_clock::now();
  P.profile = (desc->flags & FDFD_PROFILE) != 0;
  // FDFD_SYRK_GROUP: pivot blocks per Schur-complement task (0 = all of them)
  P.syrk_group = desc->syrk_group != 0 ? desc->syrk_group : env_int("FDFD_SYRK_GROUP", fdfd::kSyrkGroup);
  if (P.syrk_group <= 0) P.syrk_group = 1 << 20;
  if (P.host_only) {
    // the schedule a device plan with the default LDS budgets would run
    P.csize = P.is_c64 ? 8 : 16;
    const size_t cap = desc->small_lds > 0 ? (size_t)desc->small_lds : desc->small_lds < 0 ? 0 : 65536;
    std::vector<int32_t> tasks, tile_base, is_tiled;
    build_schedule(P, cap, tasks, tile_base, is_tiled);
    P.tile_tasks_host = tasks;
    P.wave_levels = P.small_prefix;
    build_wave_items(P);
    P.setup_ms = ms_since(t_setup);
    *out = h;
    return FDFD_OK;
  }

  int dev = desc->device;
  if (dev < 0 && hipGetDevice(&dev) != hipSuccess) {
    delete h;
    return fail(nullptr, FDFD_ERR_HIP, "no HIP device");
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || dev >= ndev) {
    delete h;
    return fail(nullptr, FDFD_ERR_HIP, "HIP device not available");
  }
  P.device = dev;
  DeviceGuard guard(dev);
  {
    // the allocation-free solve's work array: its address on this device
    void* sp = nullptr;
    const hipError_t e = scratch_address(dev, &sp);
    if (e != hipSuccess) {
      delete h;
      return fail(nullptr, FDFD_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
  }
  int lds_limit = 65536;
  (void)hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  int ncu = 0;
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  P.n_cu = ncu > 0 ? ncu : 256;
  P.lds_limit = (size_t)lds_limit;
  const size_t cs = P.csize;
  // the tile kernels need the diagonal task's 64 x 64 block in LDS
  if (fdfd::tile_lds_entries() * cs > (size_t)lds_limit - 512) {
    delete h;
    return fail(nullptr, FDFD_ERR_HIP, "device LDS too small for 64-wide front blocks");
  }
  size_t small_cap = desc->small_lds > 0    ? (size_t)desc->small_lds
                     : desc->small_lds < 0  ? 0
                                            : (size_t)env_int("FDFD_SMALL_LDS", 65536);
  // a few hundred bytes stay free for the kernels' static LDS
  const size_t lds_dyn = (size_t)lds_limit - 512;
  small_cap = std::min(small_cap, lds_dyn);
  P.small_lds = small_cap == 0 ? -1 : (int)small_cap;


  std::vector<int32_t> tasks, tile_base, is_tiled;
  build_schedule(P, small_cap, tasks, tile_base, is_tiled);
  // the fronts factored one workgroup per front (plain L, D) are swept one
  // wavefront per front
  P.wave_levels = P.small_prefix;
  P.wave_ld = 0;
  for (int l = 0; l < P.wave_levels; ++l) P.wave_ld = std::max(P.wave_ld, P.levels[l].max_m);
  build_wave_items(P);
  // forward sweep items of the levels above: per level, the fronts' pivot
  // parts, then the update-row chunks of the fronts whose L21 is split.  The pivot part
  // of a front with many pivot blocks is itself split, one item per 64-row
  // pivot block (part -1 - j for block j), whose triangular solves stream the
  // other blocks' results as they are published; such a front always has
  // its update rows in chunks.
  std::vector<int32_t> fwd_items, bwd_items, nch(P.an.nfronts, 0), chunk_base(P.an.nfronts, 0);
  std::vector<int32_t> blk_base(P.an.nfronts, -1);
  std::vector<int64_t> part_base(P.an.nfronts, 0);
  {
    int nc_total = 0, nb_total = 0;
    // FDFD_SPLIT_KB: the L21 size (KiB) from which a front is split;
    // FDFD_BLOCK_SPLIT: pivot blocks from which the pivot part is split (0 = never)
    const int split_kb =
        desc->split_kb != 0 ? desc->split_kb : env_int("FDFD_SPLIT_KB", (int)(fdfd::kSplitBytes >> 10));
    const int64_t split_bytes = split_kb < 0 ? INT64_MAX : (int64_t)split_kb << 10;
    const int block_split = desc->block_split != 0 ? (desc->block_split < 0 ? 0 : desc->block_split)
                                                   : env_int("FDFD_BLOCK_SPLIT", fdfd::kBlockSplit);
    P.split_kb = split_kb < 0 ? -1 : split_kb;
    P.block_split = block_split > 0 ? block_split : -1;
    // per level, every front's pivot part first, then all the update-row
    // chunks (a chunk waits for its front's pivot part; listing the level's
    // pivot parts together lets them all start at once)
    for (int l = P.wave_levels; l < (int)P.levels.size(); ++l) {
      const int k_lo = P.levels[l].first, k_hi = k_lo + P.levels[l].count;
      for (int k = k_lo; k < k_hi; ++k) {
        const int f = P.an.level_fronts[k];
        const int64_t p = P.an.npiv[f], u = P.an.nupd[f];
        const int nbk = (int)((p + fdfd::kChunkRows - 1) / fdfd::kChunkRows);
        const bool bsplit = block_split > 0 && nbk >= block_split;
        const bool split = u > 0 && (bsplit || u * p * (int64_t)cs >= split_bytes);
        const int nc = split ? (int)((u + fdfd::kChunkRows - 1) / fdfd::kChunkRows) : 0;
        nch[f] = nc;
        chunk_base[f] = nc_total;
        nc_total += nc;
        if (bsplit) {
          blk_base[f] = nb_total;
          nb_total += nbk;
          for (int j = 0; j < nbk; ++j) {
            fwd_items.push_back(f);
            fwd_items.push_back(-1 - j);
          }
        } else {
          fwd_items.push_back(f);
          fwd_items.push_back(-1);
        }
      }
      for (int k = k_lo; k < k_hi; ++k) {
        const int f = P.an.level_fronts[k];
        for (int j = 0; j < nch[f]; ++j) {
          fwd_items.push_back(f);
          fwd_items.push_back(j);
        }
      }
    }
    P.n_fwd_items = (int32_t)(fwd_items.size() / 2);
    P.nchunk = nc_total;
    P.nblk = nb_total;
    // backward: root first, a front's chunks (partial column sums of its
    // update rows) right before its pivot part, a split pivot part's blocks
    // last to first (a pivot part releases the level below, so each front's
    // items stay together)
    int64_t pt = 0;
    for (int l = (int)P.levels.size() - 1; l >= P.wave_levels; --l) {
      const int k_lo = P.levels[l].first, k_hi = k_lo + P.levels[l].count;
      for (int k = k_hi - 1; k >= k_lo; --k) {
        const int f = P.an.level_fronts[k];
        for (int j = 0; j < nch[f]; ++j) {
          bwd_items.push_back(f);
          bwd_items.push_back(j);
        }
        if (blk_base[f] >= 0) {
          const int nbk = (P.an.npiv[f] + fdfd::kChunkRows - 1) / fdfd::kChunkRows;
          for (int j = nbk - 1; j >= 0; --j) {
            bwd_items.push_back(f);
            bwd_items.push_back(-1 - j);
          }
        } else {
          bwd_items.push_back(f);
          bwd_items.push_back(-1);
        }
        part_base[f] = pt;
        pt += (int64_t)nch[f] * P.an.npiv[f];
      }
    }
    P.part_total = pt;
    P.n_bwd_items = (int32_t)(bwd_items.size() / 2);
  }
  // the sweeps take the right-hand sides in groups that fit the LDS (and at
  // most FDFD_SWEEP_RHS at a time); one column of the largest front has to
  P.rhs_cap = std::max(1, env_int("FDFD_SWEEP_RHS", 64));
  // the tile tasks address a child's whole update block (and a pivot block's
  // 64 columns of a front) through one buffer resource of fewer than 2 GiB:
  // fronts up to 11585 rows in complex128, 16383 in complex64
  if ((int64_t)P.an.max_front * P.an.max_front * (int64_t)P.csize >= ((int64_t)1 << 31)) {
    delete h;
    return fail(nullptr, FDFD_ERR_ARG, "front too large for the tile kernels");
  }
  if (fdfd::solve_lds_bytes(P, 1) > lds_dyn) {
    delete h;
    return fail(nullptr, FDFD_ERR_ARG, "front too large for the solve kernels");
  }

  // memory plan
  const int64_t N = P.an.N, nsys = desc->nsys, R = desc->max_rhs;
  const int64_t sum_u = P.an.upd_ptr.back();
  // one cell per residual thread up to 2^22 cells (one workgroup then sums
  // the per-workgroup partials)
  P.res_blocks = (int32_t)std::min<int64_t>(16384, std::max<int64_t>(1, (N + 255) / 256));
  const int64_t need = nsys * P.an.fac_total * (int64_t)cs + nsys * P.an.upd_total * (int64_t)cs +
                       nsys * (int64_t)P.ntiles * 4 + nsys * ((int64_t)P.an.nfronts + P.nchunk + P.nblk) * 4 +
                       nsys * (2 * desc->nx + 2 * desc->ny + 2) * 16 + nsys * 8 + nsys * N * 8 +
                       2 * nsys * R * N * (int64_t)cs + nsys * R * (sum_u + P.part_total) * (int64_t)cs +
                       2 * nsys * R * N * 16 +
                       nsys * R * P.res_blocks * 16 + (int64_t)sizeof(fdfd::DevStatus);
  if (desc->mem_cap_bytes > 0 && need > desc->mem_cap_bytes) {
    delete h;
    return fail(nullptr, FDFD_ERR_NOMEM,
                "plan needs " + std::to_string(need) + " device bytes, above mem_cap_bytes");
  }

  fdfd_status st = FDFD_OK;
#define TRY(x)                   \
  do {                           \
    st = (x);                    \
    if (st != FDFD_OK) goto bad; \
  } while (0)
  {
    const fdfd::Analysis& A = P.an;
    TRY(upload(P, &P.t.pbeg, A.pbeg));
    TRY(upload(P, &P.t.npiv, A.npiv));
    TRY(upload(P, &P.t.nupd, A.nupd));
    TRY(upload(P, &P.t.child_ptr, A.child_ptr));
    TRY(upload(P, &P.t.child_list, A.child_list));
    TRY(upload(P, &P.t.upd_ptr, A.upd_ptr));
    TRY(upload(P, &P.t.upd_idx, A.upd_idx));
    TRY(upload(P, &P.t.gmap, A.gmap));
    TRY(upload(P, &P.t.nbr_row, A.nbr_row));
    TRY(upload(P, &P.t.perm, A.perm));
    TRY(upload(P, &P.t.iperm, A.iperm));
    TRY(upload(P, &P.t.level_fronts, A.level_fronts));
    TRY(upload(P, &P.t.wave_seq, P.wave_seq_host));
    TRY(upload(P, &P.t.wave_item_ptr, P.wave_item_ptr_host));
    TRY(upload(P, &P.t.tile_tasks, tasks));
    P.tile_tasks_host = tasks;
    TRY(upload(P, &P.t.tile_base, tile_base));
    TRY(upload(P, &P.t.is_tiled, is_tiled));
    TRY(upload(P, &P.t.fwd_items, fwd_items));
    TRY(upload(P, &P.t.bwd_items, bwd_items));
    TRY(upload(P, &P.t.part_base, part_base));
    TRY(upload(P, &P.t.nch, nch));
    TRY(upload(P, &P.t.chunk_base, chunk_base));
    TRY(upload(P, &P.t.blk_base, blk_base));
    TRY(upload(P, &P.t.parent, A.parent));
    TRY(upload(P, &P.t.height, A.height));
    TRY(upload(P, &P.t.fac_off, A.fac_off));
    TRY(upload(P, &P.t.upd_off, A.upd_off));
    TRY(upload(P, &P.t.gmap_ptr, A.gmap_ptr));
    TRY(alloc(P, &P.fac, nsys * A.fac_total * cs));
    TRY(alloc(P, &P.upd, nsys * A.upd_total * cs));
    TRY(alloc(P, (void**)&P.tile_state, nsys * (int64_t)std::max(1, P.ntiles) * 4));
    TRY(alloc(P, (void**)&P.tile_done, nsys * (int64_t)A.nfronts * 4));
    TRY(alloc(P, (void**)&P.pml, nsys * (2 * desc->nx + 2 * desc->ny + 2) * 16));
    TRY(alloc(P, (void**)&P.omega, nsys * 8));
    TRY(alloc(P, (void**)&P.eps, nsys * N * 8));
    TRY(alloc(P, &P.y, nsys * R * N * cs));
    TRY(alloc(P, &P.wv, nsys * R * std::max<int64_t>(1, sum_u) * cs));
    TRY(alloc(P, &P.zv, nsys * R * N * cs));
    TRY(alloc(P, &P.pv, nsys * R * std::max<int64_t>(1, P.part_total) * cs));
    TRY(alloc(P, (void**)&P.xw, nsys * R * N * 16));
    TRY(alloc(P, (void**)&P.res, nsys * R * N * 16));
    TRY(alloc(P, (void**)&P.partial, nsys * R * P.res_blocks * 16));
    TRY(alloc(P, (void**)&P.status, sizeof(fdfd::DevStatus)));
    TRY(alloc(P, (void**)&P.counters, fdfd::kCounterBytes));
    TRY(alloc(P, (void**)&P.done, nsys * ((int64_t)A.nfronts + P.nchunk + P.nblk) * 4));
    hipError_t e = hipMemset(P.counters, 0, fdfd::kCounterBytes);
    if (e == hipSuccess) e = hipMemset(P.done, 0, nsys * ((int64_t)A.nfronts + P.nchunk + P.nblk) * 4);
    if (e == hipSuccess) e = hipMemset(P.status, 0, sizeof(fdfd::DevStatus));
    if (e != hipSuccess) {
      st = hip_fail(&P, e, "hipMemset");
      goto bad;
    }
    if (const char* tp = std::getenv("FDFD_TRACE")) {
      // task traces for performance analysis: written to this file by fdfd_query
      P.trace_path = tp;
      const int nsm = (P.small_prefix > 0 ? P.levels[P.small_prefix - 1].first + P.levels[P.small_prefix - 1].count
                                          : 0) * (int)nsys;
      const int caps[4] = {nsm, P.ntile_tasks * (int)nsys, A.nfronts * (int)nsys, A.nfronts * (int)nsys};
      for (int k = 0; k < 4; ++k) {
        P.trace_cap[k] = caps[k];
        if (caps[k] > 0) TRY(alloc(P, (void**)&P.trace_buf[k], (size_t)caps[k] * 4 * sizeof(long long)));
      }
    }
    if (desc->flags & FDFD_GRAPH) {
      e = hipStreamCreateWithFlags(&P.cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) {
        st = hip_fail(&P, e, "hipStreamCreate");
        goto bad;
      }
    }
    for (hipEvent_t& ev : P.phase_ev) {
      if (e == hipSuccess) e = hipEventCreate(&ev);
    }
    if (e != hipSuccess) {
      st = hip_fail(&P, e, "hipEventCreate");
      goto bad;
    }
    e = hipHostMalloc((void**)&P.status_host, sizeof(fdfd::DevStatus), hipHostMallocDefault);
    if (e != hipSuccess) {
      st = fail(&P, FDFD_ERR_NOMEM, "pinned host allocation failed");
      goto bad;
    }
    e = fdfd::configure_kernels(P, lds_limit);
    if (e != hipSuccess) {
      st = hip_fail(&P, e, "hipFuncSetAttribute");
      goto bad;
    }
    e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      st = hip_fail(&P, e, "analysis upload");
      goto bad;
    }
  }
#undef TRY
  P.solve_lds_max = fdfd::solve_lds_bytes(P, fdfd::solve_rhs_group(P, desc->max_rhs));
  P.rhs_group = fdfd::solve_rhs_group(P, desc->max_rhs);
  P.setup_ms = ms_since(t_setup);
  *out = h;
  return FDFD_OK;
bad:
  g_error = P.last_error;
  free_all(P);
  delete h;
  return st;
}

fdfd_status fdfd_refactor(fdfd_plan plan, const double* eps_dev, int64_t eps_sys_stride,
                          const double* omega_host, void* hip_stream) {
  if (!plan) return fail(nullptr, FDFD_ERR_ARG, "plan is NULL");
  Plan& P = plan->p;
  if (P.host_only) return fail(&P, FDFD_ERR_STATE, "host-only plan cannot factor");
  if (!eps_dev || !omega_host) return fail(&P, FDFD_ERR_ARG, "eps_dev and omega_host must be non-NULL");
  if (eps_sys_stride < 0 || (eps_sys_stride > 0 && eps_sys_stride < P.an.N))
    return fail(&P, FDFD_ERR_ARG, "eps_sys_stride must be 0 or >= nx*ny");
  std::vector<double> om(omega_host, omega_host + P.desc.nsys);
  for (double w : om)
    if (!(w > 0.0) || !std::isfinite(w)) return fail(&P, FDFD_ERR_ARG, "omega must be positive and finite");
  DeviceGuard guard(P.device);
  P.omega_host = om;
  hipStream_t st = (hipStream_t)hip_stream;
  std::vector<uint64_t> key = {0, bits(eps_dev), (uint64_t)eps_sys_stride};
  for (double w : om) key.push_back(bits(w));
  (void)hipEventRecord(P.phase_ev[0], st);
  const fdfd_status r = run_chain(P, std::move(key), st, "refactor launch", [&](hipStream_t s) {
    return fdfd::launch_refactor(P, eps_dev, eps_sys_stride, s);
  });
  if (r != FDFD_OK) return r;
  (void)hipEventRecord(P.phase_ev[1], st);
  P.phase_rec[0] = true;
  P.last_stream = st;
  P.factored = true;
  return FDFD_OK;
}

fdfd_status fdfd_solve(fdfd_plan plan, const void* b_dev, void* x_dev, int32_t nrhs, int32_t max_ir,
                       double ir_tol, void* hip_stream) {
  if (!plan) return fail(nullptr, FDFD_ERR_ARG, "plan is NULL");
  Plan& P = plan->p;
  if (P.host_only) return fail(&P, FDFD_ERR_STATE, "host-only plan cannot solve");
  if (!P.factored) return fail(&P, FDFD_ERR_STATE, "solve before refactor");
  if (!b_dev || !x_dev) return fail(&P, FDFD_ERR_ARG, "b_dev and x_dev must be non-NULL");
  if (nrhs < 1 || nrhs > P.desc.max_rhs) return fail(&P, FDFD_ERR_ARG, "nrhs must be in [1, max_rhs]");
  if (max_ir < 0 || max_ir > 100) return fail(&P, FDFD_ERR_ARG, "max_ir must be in [0, 100]");
  if (!(ir_tol > 0.0)) ir_tol = 1e-12;
  DeviceGuard guard(P.device);
  hipStream_t st = (hipStream_t)hip_stream;
  (void)hipEventRecord(P.phase_ev[2], st);
  const fdfd_status r = run_chain(
      P, {1, bits(b_dev), bits(x_dev), (uint64_t)nrhs, (uint64_t)max_ir, bits(ir_tol)}, st, "solve launch",
      [&](hipStream_t s) {
        return fdfd::launch_solve(P, 0, (const double2*)b_dev, (double2*)x_dev, nrhs, max_ir, ir_tol, s);
      });
  if (r != FDFD_OK) return r;
  (void)hipEventRecord(P.phase_ev[3], st);
  P.phase_rec[1] = true;
  P.last_stream = st;
  return FDFD_OK;
}

fdfd_status fdfd_solve_noalloc(fdfd_plan plan, const void* b_dev, void* x_dev, int32_t nrhs, int32_t max_ir,
                               double ir_tol, void* hip_stream) {
  if (!plan) return fail(nullptr, FDFD_ERR_ARG, "plan is NULL");
  Plan& P = plan->p;
  if (P.host_only) return fail(&P, FDFD_ERR_STATE, "host-only plan cannot solve");
  if (!P.factored) return fail(&P, FDFD_ERR_STATE, "solve before refactor");
  if (P.profile) return fail(&P, FDFD_ERR_STATE, "fdfd_solve_noalloc does not run on FDFD_PROFILE plans");
  if (!b_dev || !x_dev) return fail(&P, FDFD_ERR_ARG, "b_dev and x_dev must be non-NULL");
  if (nrhs < 1 || nrhs > P.desc.max_rhs) return fail(&P, FDFD_ERR_ARG, "nrhs must be in [1, max_rhs]");
  if (max_ir < 0 || max_ir > 100) return fail(&P, FDFD_ERR_ARG, "max_ir must be in [0, 100]");
  if (!(ir_tol > 0.0)) ir_tol = 1e-12;
  const size_t need = carve_solve_work(P, nrhs, nullptr, nullptr);
  if (need > kScratchBytes)
    return fail(&P, FDFD_ERR_ARG,
                "fdfd_solve_noalloc needs " + std::to_string(need) + " bytes of work space for this plan and nrhs; "
                "the limit is " + std::to_string(kScratchBytes) + " (use fdfd_solve)");
  DeviceGuard guard(P.device);
  void* base = nullptr;
  hipError_t e = scratch_address(P.device, &base);
  if (e != hipSuccess) return hip_fail(&P, e, "hipGetSymbolAddress(scratch)");
  fdfd::SolveWork w;
  carve_solve_work(P, nrhs, static_cast<unsigned char*>(base), &w);
  hipStream_t st = (hipStream_t)hip_stream;
  e = fdfd::launch_solve(P, 0, (const double2*)b_dev, (double2*)x_dev, nrhs, max_ir, ir_tol, st, &w);
  if (e != hipSuccess) return hip_fail(&P, e, "solve launch");
  P.last_stream = st;
  return FDFD_OK;
}

fdfd_status fdfd_adjoint_grad(fdfd_plan plan, const void* x_dev, const void* g_dev, int32_t nrhs,
                              int32_t max_ir, double ir_tol, void* lambda_dev, double* grad_dev,
                              int32_t flags, void* hip_stream) {
  if (!plan) return fail(nullptr, FDFD_ERR_ARG, "plan is NULL");
  Plan& P = plan->p;
  if (P.host_only) return fail(&P, FDFD_ERR_STATE, "host-only plan cannot solve");
  if (!P.factored) return fail(&P, FDFD_ERR_STATE, "adjoint before refactor");
  if (!x_dev || !g_dev || !grad_dev) return fail(&P, FDFD_ERR_ARG, "x_dev, g_dev and grad_dev must be non-NULL");
  if (nrhs < 1 || nrhs > P.desc.max_rhs) return fail(&P, FDFD_ERR_ARG, "nrhs must be in [1, max_rhs]");
  if (max_ir < 0 || max_ir > 100) return fail(&P, FDFD_ERR_ARG, "max_ir must be in [0, 100]");
  if (flags & ~(FDFD_GRAD_ACCUMULATE | FDFD_GRAD_SUM_SYSTEMS)) return fail(&P, FDFD_ERR_ARG, "unknown flags");
  if (!(ir_tol > 0.0)) ir_tol = 1e-12;
  DeviceGuard guard(P.device);
  hipStream_t st = (hipStream_t)hip_stream;
  (void)hipEventRecord(P.phase_ev[4], st);
  const fdfd_status r = run_chain(
      P,
      {2, bits(x_dev), bits(g_dev), (uint64_t)nrhs, (uint64_t)max_ir, bits(ir_tol), bits(lambda_dev),
       bits(grad_dev), (uint64_t)flags},
      st, "adjoint launch", [&](hipStream_t s) {
        hipError_t e = fdfd::launch_solve(P, 1, (const double2*)g_dev, nullptr, nrhs, max_ir, ir_tol, s);
        if (e == hipSuccess)
          e = fdfd::launch_gradient(P, (const double2*)x_dev, P.xw, nrhs, (double2*)lambda_dev, grad_dev, flags,
                                    s);
        return e;
      });
  if (r != FDFD_OK) return r;
  (void)hipEventRecord(P.phase_ev[5], st);
  P.phase_rec[2] = true;
  P.last_stream = st;
  return FDFD_OK;
}

fdfd_status fdfd_query(fdfd_plan plan, fdfd_info* info) {
  if (!plan || !info) return fail(nullptr, FDFD_ERR_ARG, "plan and info must be non-NULL");
  Plan& P = plan->p;
  std::memset(info, 0, sizeof(*info));
  const fdfd::Analysis& A = P.an;
  info->n = A.N;
  info->nfronts = A.nfronts;
  info->nlevels = A.nlevels;
  info->nnz_factor = A.nnz_l;
  info->factor_bytes = A.fac_total * (int64_t)P.csize;
  info->update_bytes = A.upd_total * (int64_t)P.csize;
  info->device_bytes = P.device_bytes;
  info->refactor_flops = A.flops_factor;
  info->schur_flops = A.flops_schur;
  info->max_front = A.max_front;
  info->max_pivots = A.max_piv;
  info->leaf = A.leaf;
  info->small_levels = P.small_prefix;
  info->min_pivot_ratio = -1.0;
  info->rel_residual_solve = -1.0;
  info->rel_residual_adjoint = -1.0;
  info->refactor_ms = info->solve_ms = info->adjoint_ms = -1.0;
  info->rhs_group = P.rhs_group;
  info->syrk_group = P.syrk_group >= (1 << 20) ? -1 : P.syrk_group;
  info->split_kb = P.split_kb;
  info->block_split = P.block_split;
  info->small_lds = P.small_lds;
  info->analyze_ms = P.analyze_ms;
  info->setup_ms = P.setup_ms;
  if (P.host_only) return FDFD_OK;
  DeviceGuard guard(P.device);
  hipError_t e = hipMemcpyAsync(P.status_host, P.status, sizeof(fdfd::DevStatus), hipMemcpyDeviceToHost,
                                P.last_stream);
  if (e == hipSuccess) e = hipStreamSynchronize(P.last_stream);
  if (e != hipSuccess) return hip_fail(&P, e, "status read-back");
  const fdfd::DevStatus& S = *P.status_host;
  double* phase_ms[3] = {&info->refactor_ms, &info->solve_ms, &info->adjoint_ms};
  for (int k = 0; k < 3; ++k) {
    float ms = 0.f;
    if (P.phase_rec[k] && hipEventSynchronize(P.phase_ev[2 * k + 1]) == hipSuccess &&
        hipEventElapsedTime(&ms, P.phase_ev[2 * k], P.phase_ev[2 * k + 1]) == hipSuccess)
      *phase_ms[k] = ms;
  }
  info->n_perturbed = S.n_perturbed;
  double mr;
  std::memcpy(&mr, &S.min_ratio_bits, sizeof(double));
  info->min_pivot_ratio = P.factored ? mr : -1.0;
  info->ir_steps_solve = S.ir_steps_solve;
  info->ir_steps_adjoint = S.ir_steps_adj;
  info->rel_residual_solve = S.rel_solve;
  info->rel_residual_adjoint = S.rel_adj;
  info->device_flags = (S.nonfinite ? 1 : 0) | (S.ir_failed_solve ? 2 : 0) | (S.ir_failed_adj ? 4 : 0) |
                       (S.spin_timeout ? 8 : 0);
  if (!P.trace_path.empty()) {
    FILE* fp = std::fopen(P.trace_path.c_str(), "w");
    if (fp) {
      for (int k = 0; k < 4; ++k) {
        if (!P.trace_buf[k] || P.trace_n[k] == 0) continue;
        std::vector<long long> tr((size_t)P.trace_n[k] * 4);
        if (hipMemcpy(tr.data(), P.trace_buf[k], tr.size() * sizeof(long long), hipMemcpyDeviceToHost) != hipSuccess)
          continue;
        const int ns = P.desc.nsys;
        for (int t = 0; t < P.trace_n[k]; ++t) {
          // item: tile task record (type front k I J) for the tile graph, else the front
          int it[5] = {-1, -1, -1, -1, -1};
          if (k == 1) {
            for (int q = 0; q < 5; ++q) it[q] = P.tile_tasks_host[5 * (t / ns) + q];
          } else if (k >= 2 && P.wave_items > 0) {
            // a bottom-level sweep item: its subtree root (or single front)
            const int pos = t / ns, item = k == 2 ? pos : P.wave_items - 1 - pos;
            it[1] = P.wave_seq_host[P.wave_item_ptr_host[item + 1] - 1];
          } else {
            const int pos = t / ns;
            // the small-front launch starts above the levels k_wave_fronts took
            const int nwl = (int)P.wave_front_levels.size();
            const int skip = k == 0 && nwl > 0 ? P.levels[nwl - 1].first + P.levels[nwl - 1].count : 0;
            it[1] = A.level_fronts[k == 3 ? A.nfronts - 1 - pos : skip + pos];
          }
          std::fprintf(fp, "%d %d %lld %lld %lld %lld %d %d %d %d %d\n", k, t, tr[4 * t], tr[4 * t + 1],
                       tr[4 * t + 2], tr[4 * t + 3], it[0], it[1], it[2], it[3], it[4]);
        }
      }
      std::fclose(fp);
    }
  }
  if (S.nonfinite) return fail(&P, FDFD_ERR_NUMERIC, "non-finite value in the factor or residual");
  if (S.spin_timeout) return fail(&P, FDFD_ERR_NUMERIC, "a device dependency wait timed out");
  if (S.ir_failed_solve || S.ir_failed_adj)
    return fail(&P, FDFD_ERR_NUMERIC, "iterative refinement did not reach its tolerance");
  if (S.n_perturbed > 0) return FDFD_WARN_PIVOT;
  return FDFD_OK;
}

fdfd_status fdfd_kernel_stats(fdfd_plan plan, fdfd_kernel_stat* out, int32_t max_entries, int32_t* n_out) {
  if (!plan || !n_out || (!out && max_entries > 0) || max_entries < 0)
    return fail(nullptr, FDFD_ERR_ARG, "plan and n_out must be non-NULL");
  Plan& P = plan->p;
  *n_out = 0;
  if (!P.profile || P.host_only) return fail(&P, FDFD_ERR_STATE, "plan was not analysed with FDFD_PROFILE");
  DeviceGuard guard(P.device);
  hipError_t e = hipStreamSynchronize(P.last_stream);
  if (e != hipSuccess) return hip_fail(&P, e, "stream synchronise");
  fdfd::profile_collect(P);
  int n = 0;
  for (int c = 0; c < fdfd::KC_COUNT && n < max_entries; ++c, ++n) {
    fdfd_kernel_stat& k = out[n];
    std::memset(&k, 0, sizeof(k));
    std::strncpy(k.name, fdfd::kKernelClassNames[c], sizeof(k.name) - 1);
    k.launches = P.totals[c].launches;
    k.total_ms = P.totals[c].ms;
    k.alg_bytes = P.totals[c].bytes;
    k.alg_flops = P.totals[c].flops;
    P.totals[c] = fdfd::KernelTotals();
  }
  *n_out = n;
  return FDFD_OK;
}

fdfd_status fdfd_get_table(fdfd_plan plan, int32_t which, int32_t* out, int64_t count) {
  if (!plan || !out) return fail(nullptr, FDFD_ERR_ARG, "plan and out must be non-NULL");
  Plan& P = plan->p;
  const fdfd::Analysis& A = P.an;
  if (which == FDFD_TABLE_PERM) {
    if (count < A.N) return fail(&P, FDFD_ERR_ARG, "buffer too small");
    std::copy(A.perm.begin(), A.perm.end(), out);
    return FDFD_OK;
  }
  if (which == FDFD_TABLE_FRONTS) {
    if (count < 4 * (int64_t)A.nfronts) return fail(&P, FDFD_ERR_ARG, "buffer too small");
    for (int f = 0; f < A.nfronts; ++f) {
      out[4 * f] = A.pbeg[f];
      out[4 * f + 1] = A.npiv[f];
      out[4 * f + 2] = A.nupd[f];
      out[4 * f + 3] = A.parent[f];
    }
    return FDFD_OK;
  }
  if (which == FDFD_TABLE_UPDATE) {
    if (count < (int64_t)A.upd_idx.size()) return fail(&P, FDFD_ERR_ARG, "buffer too small");
    std::copy(A.upd_idx.begin(), A.upd_idx.end(), out);
    return FDFD_OK;
  }
  if (which == FDFD_TABLE_TASKS) {
    if (count < 1 + (int64_t)P.tile_tasks_host.size()) return fail(&P, FDFD_ERR_ARG, "buffer too small");
    out[0] = (int32_t)(P.tile_tasks_host.size() / 5);
    std::copy(P.tile_tasks_host.begin(), P.tile_tasks_host.end(), out + 1);
    return FDFD_OK;
  }
  if (which == FDFD_TABLE_SWEEP_ITEMS) {
    const std::vector<int32_t>& ip = P.wave_item_ptr_host;
    const std::vector<int32_t>& sq = P.wave_seq_host;
    const int64_t n = 2 + (int64_t)ip.size() + (int64_t)sq.size();
    if (count < n) return fail(&P, FDFD_ERR_ARG, "buffer too small");
    out[0] = (int32_t)ip.size() - 1;
    out[1] = P.sweep_group;
    std::copy(ip.begin(), ip.end(), out + 2);
    std::copy(sq.begin(), sq.end(), out + 2 + ip.size());
    return FDFD_OK;
  }
  return fail(&P, FDFD_ERR_ARG, "unknown table");
}

void fdfd_destroy(fdfd_plan plan) {
  if (!plan) return;
  Plan& P = plan->p;
  if (!P.host_only) {
    DeviceGuard guard(P.device);
    if (P.last_stream) (void)hipStreamSynchronize(P.last_stream);
    (void)hipDeviceSynchronize();
    free_all(P);
  }
  delete plan;
}

}  // extern "C"
