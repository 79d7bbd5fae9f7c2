// Internal plan layout shared by the C ABI (fdfd_api.cpp) and the kernel
// launchers (fdfd_kernels.hip).  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "analysis.h"
#include "../../include/fdfd.h"

namespace fdfd {

// Device status, one per plan.  Written by kernels, read by fdfd_query.
struct DevStatus {
  unsigned long long anorm_bits[64];     // per system max |entry| of S*A (double bits)
  unsigned long long min_ratio_bits;     // min |d_k| / anorm over the refactor (double bits)
  int n_perturbed;
  int nonfinite;                         // set when a non-finite pivot or residual appears
  int spin_timeout;                      // a dependency wait gave up (never expected)
  int ir_flag;                           // 1 = current refinement converged (early exit)
  int ir_steps;                          // steps taken by the current refinement
  int ir_failed;                         // the current refinement missed its tolerance
  double ir_rel;                         // max relative residual of the current refinement
  int ir_steps_solve, ir_steps_adj;
  double rel_solve, rel_adj;
  int ir_failed_solve, ir_failed_adj;
};

// Device copies of the analysis tables.
struct DevTables {
  int32_t *pbeg = nullptr, *npiv = nullptr, *nupd = nullptr;
  int32_t *child_ptr = nullptr, *child_list = nullptr;
  int32_t *upd_ptr = nullptr, *upd_idx = nullptr;
  int32_t *gmap = nullptr, *nbr_row = nullptr;
  int32_t *perm = nullptr, *iperm = nullptr;
  int32_t *level_fronts = nullptr;
  int32_t *wave_seq = nullptr, *wave_item_ptr = nullptr;  // bottom-level sweep items
  int32_t *parent = nullptr, *height = nullptr;
  int32_t *tile_tasks = nullptr, *tile_base = nullptr, *is_tiled = nullptr;
  int32_t *fwd_items = nullptr, *bwd_items = nullptr, *nch = nullptr, *chunk_base = nullptr, *blk_base = nullptr;
  int64_t *part_base = nullptr;
  int64_t *fac_off = nullptr, *upd_off = nullptr, *gmap_ptr = nullptr;
};

struct LevelPlan {
  int32_t first, count;        // slice of level_fronts
  bool small;                  // panel fits the one-workgroup LDS kernel
  size_t small_lds;            // dynamic LDS bytes of that kernel
  int32_t max_m, max_p, max_u;
  double lbytes = 0;           // lower-trapezoid factor bytes of the level (one system)
};

// Kernel classes for FDFD_PROFILE timing.
enum KernelClass {
  KC_SETUP = 0, KC_FRONT_SMALL, KC_LARGE_TILES, KC_FWD_SWEEP, KC_BWD_SWEEP, KC_RESIDUAL, KC_GRADIENT,
  KC_COUNT
};
extern const char* const kKernelClassNames[KC_COUNT];

struct PendingTiming {
  int cls;
  hipEvent_t e0, e1;
  double bytes, flops;
};

struct KernelTotals {
  int64_t launches = 0;
  double ms = 0.0, bytes = 0.0, flops = 0.0;
};

struct Plan {
  fdfd_desc desc{};
  Analysis an;
  bool host_only = false;
  double analyze_ms = 0.0, setup_ms = 0.0;  // host time of fdfd_analyze's two phases
  int device = 0;
  bool is_c64 = false;
  size_t csize = 16;           // bytes of one factor scalar (complex)
  double pivot_tau = 0;        // pivots below pivot_tau * ||SA||_max are perturbed
  DevTables t;
  std::vector<LevelPlan> levels;
  int32_t ntile_tasks = 0;     // tasks of the tile graph (one system)
  int32_t ntiles = 0;          // packed tiles of the tiled fronts (one system)
  double tiled_flops = 0;      // partial-LDL^T flops of the tiled fronts (one system)
  size_t solve_lds_max = 0;
  int rhs_group = 1;  // right-hand sides per sweep pass at max_rhs
  int rhs_cap = 64;   // at most this many per pass (FDFD_SWEEP_RHS)
  int split_kb = 0, block_split = 0, small_lds = 0;  // schedule knobs in effect (-1: never)
  // bottom levels factored one wavefront per front (k_wave_fronts), one
  // launch each: LDS bytes per wave and the largest pivot count of the level
  struct WaveLevel {
    int ldsw, pmax, nr;  // LDS per wave, pivot bound, rows per lane (1 or 2)
  };
  std::vector<WaveLevel> wave_front_levels;
  int32_t small_prefix = 0;    // leading levels run by the small-front launches (one per level)
  int32_t syrk_group = 8;      // pivot blocks accumulated per Schur-complement tile task
  int32_t n_cu = 256;
  size_t lds_limit = 65536;
  int32_t wave_levels = 0;      // bottom levels swept one wavefront per front
  int32_t wave_ld = 0;          // largest front (rows) among them
  int32_t wave_items = 0;       // their sweep items: a subtree (children first) or one front
  int32_t sweep_group = 0;      // height of the subtrees one sweep item takes
  std::vector<int32_t> wave_seq_host, wave_item_ptr_host;
  // Forward sweep of the tiled levels: work items (front, part) in claim
  // order, part -1 the pivot rows, part j >= 0 the j-th kChunkRows update
  // rows of a front whose L21 is split over several workgroups.
  int32_t n_fwd_items = 0;
  int32_t nchunk = 0;           // update-row chunks of all split fronts (one system)
  int32_t nblk = 0;             // pivot-block items of all block-split fronts (one system)
  int32_t n_bwd_items = 0;
  int64_t part_total = 0;       // backward: sum over split fronts of chunks x pivots

  // arenas (device)
  void* fac = nullptr;         // nsys * fac_total scalars
  void* upd = nullptr;         // nsys * upd_total scalars
  double2* pml = nullptr;      // nsys * (2nx + 2ny + 2)
  double* omega = nullptr;     // nsys
  double* eps = nullptr;       // nsys * N (copy taken at refactor)
  void* y = nullptr;           // nsys * max_rhs * N scalars (elimination order)
  void* wv = nullptr;          // nsys * max_rhs * sum(u) scalars (update vectors)
  void* zv = nullptr;          // nsys * max_rhs * N scalars: z = L11^-1 v of split fronts
  void* pv = nullptr;          // nsys * max_rhs * part_total scalars: backward chunk sums
  double2* xw = nullptr;       // nsys * max_rhs * N (adjoint work solution)
  double2* res = nullptr;      // nsys * max_rhs * N (FP64 residual)
  double* partial = nullptr;   // nsys * max_rhs * res_blocks * 2
  int32_t res_blocks = 0;
  DevStatus* status = nullptr;
  int32_t* counters = nullptr;  // [0..1] persistent-queue counters, [2] residual blocks,
                                // [kEpochSlot] epoch of the last persistent launch
  int32_t* done = nullptr;      // [nsys][nfronts] completion epochs, then [nsys][nchunk], then [nsys][nblk]
  int32_t* tile_state = nullptr;  // [nsys][ntiles] tile versions
  int32_t* tile_done = nullptr;   // [nsys][nfronts] finished update tiles
  DevStatus* status_host = nullptr;  // pinned
  int64_t device_bytes = 0;
  std::vector<void*> allocations;

  // task traces (FDFD_TRACE=<file>): 0 small fronts, 1 tile graph, 2 fwd, 3 bwd sweep
  long long* trace_buf[4] = {nullptr, nullptr, nullptr, nullptr};
  int32_t trace_cap[4] = {0, 0, 0, 0};
  int32_t trace_n[4] = {0, 0, 0, 0};
  std::string trace_path;
  std::vector<int32_t> tile_tasks_host;
  // FDFD_PROFILE
  bool profile = false;
  std::vector<hipEvent_t> event_pool;
  std::vector<PendingTiming> pending;
  KernelTotals totals[KC_COUNT];
  // per-front algorithmic figures (host)
  std::vector<double> front_flops;   // real flops of the front's partial LDL^T
  std::vector<double> front_lbytes;  // bytes of the lower-trapezoid factor
  double factor_lbytes = 0;          // sum of front_lbytes (one system)

  // FDFD_GRAPH: each call's launch chain, recorded once per argument set on
  // cap_stream and replayed on the caller's stream (least recently used last)
  struct GraphEntry {
    std::vector<uint64_t> key;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  hipStream_t cap_stream = nullptr;
  int64_t graph_records = 0;         // chains recorded so far (a measurement aid)

  // per-phase device time (fdfd_query): events around the launches of the
  // last refactor (0, 1), solve (2, 3) and adjoint (4, 5)
  hipEvent_t phase_ev[6] = {};
  bool phase_rec[3] = {false, false, false};

  hipStream_t last_stream = nullptr;
  std::vector<double> omega_host;
  bool factored = false;
  std::string last_error;
};

// The epoch of the last persistent launch sits in its own 128-byte line of
// the counters array, apart from the counters that take atomics.
constexpr int kEpochSlot = 32;
// Sweeps of the tiled levels: a front whose L21 holds at least kSplitBytes is
// swept as its pivot rows plus chunks of kChunkRows update rows, one
// workgroup each.
constexpr int kChunkRows = 64;
constexpr int64_t kSplitBytes = 128 << 10;
// A front with at least kBlockSplit pivot blocks has its pivot part swept as
// one item per pivot block (FDFD_BLOCK_SPLIT overrides it, 0 = never).
constexpr int kBlockSplit = 6;
constexpr size_t kCounterBytes = 256;
// Pivot blocks whose products one Schur-complement tile task accumulates
// before it writes the tile (FDFD_SYRK_GROUP overrides it at analysis).
constexpr int kSyrkGroup = 8;

// Work vectors of one solve call: the elimination-order vector y, the update
// vectors wv, the split fronts' hand-over buffers zv / pv, the FP64 residual,
// the residual's per-block partial norms and its last-block counter (which
// must be 0 when the call starts; the residual kernel leaves it at 0).  The
// plan's arenas by default; fdfd_solve_noalloc carves them from a static
// device array.
struct SolveWork {
  void* y = nullptr;
  void* wv = nullptr;
  void* zv = nullptr;
  void* pv = nullptr;
  double2* res = nullptr;
  double* partial = nullptr;
};

// Kernel launchers (fdfd_kernels.hip).  Each returns hipSuccess or the first
// launch error.
hipError_t launch_refactor(Plan& P, const double* eps, int64_t eps_stride, hipStream_t st);
// Solves (SA) X = RHS for every system and nrhs columns with IR.  mode 0:
// forward (rhs = S b, result into x_out, overwritten); mode 1: adjoint
// (rhs = g, lam' into P.xw, then lam = S lam' into lam_out if not null).
hipError_t launch_solve(Plan& P, int mode, const double2* rhs, double2* x_out, int32_t nrhs,
                        int32_t max_ir, double tol, hipStream_t st, const SolveWork* work = nullptr);
hipError_t launch_gradient(Plan& P, const double2* x, const double2* lam_sym, int32_t nrhs,
                           double2* lam_out, double* grad, int32_t flags, hipStream_t st);
size_t solve_lds_bytes(const Plan& P, int nrhs);
// right-hand sides one sweep pass takes at once (the solves loop over groups)
int solve_rhs_group(const Plan& P, int nrhs);

// Complex entries of LDS the tile-graph tasks need: the TRSM task's 64 x 64
// tile, 64 x 64 pivot block and 64 x 16 buffer, the largest of the task types.
inline size_t tile_lds_entries() { return 2 * 64 * 64 + 64 * 16; }
// FDFD_PROFILE helpers (fdfd_api.cpp)
hipEvent_t profile_event(Plan& P);
void profile_collect(Plan& P);
hipError_t configure_kernels(Plan& P, int lds_limit);

}  // namespace fdfd
