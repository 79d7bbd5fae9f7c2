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
  int32_t *mslot = nullptr, *parent = nullptr;
  int64_t *fac_off = nullptr, *upd_off = nullptr, *gmap_ptr = nullptr;
  int32_t *tasks = nullptr;  // task lists of the large-front path
};

// One block step of the large-front path at one level.
struct BlockStep {
  int32_t kb, nb;
  int64_t diag_off;  int32_t ndiag;    // fronts with p > kb (task buffer offsets)
  int64_t trsm_off;  int32_t ntrsm;    // (front, first row) pairs
  int64_t upd_off;   int32_t nupd;     // (front, tile row, tile col) triples
  double diag_flops = 0, trsm_flops = 0, upd_flops = 0;  // algorithmic work per system
};

struct LevelPlan {
  int32_t first, count;        // slice of level_fronts
  bool small;                  // fused one-workgroup-per-front kernel
  size_t small_lds;            // dynamic LDS bytes of the fused kernel
  int64_t asm_off; int32_t nasm;   // assembly tasks (front, c0, c1), large path
  std::vector<BlockStep> steps;
  int32_t max_m, max_p, max_u;
  double lbytes = 0;           // lower-trapezoid factor bytes of the level (one system)
  double asm_bytes = 0;        // front entries written by the large-path assembly
};

// Kernel classes for FDFD_PROFILE timing.
enum KernelClass {
  KC_SETUP = 0, KC_FRONT_SMALL, KC_ASSEMBLE_LARGE, KC_DIAG_LARGE, KC_TRSM_LARGE, KC_UPDATE_LARGE,
  KC_FWD_SWEEP, KC_BWD_SWEEP, KC_RESIDUAL, KC_GRADIENT, KC_COUNT
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
  int device = 0;
  bool is_c64 = false;
  size_t csize = 16;           // bytes of one factor scalar (complex)
  DevTables t;
  std::vector<LevelPlan> levels;
  int32_t nb_large = 64;       // block width of the large-front path
  int32_t tile_trsm = 64;      // rows per trsm task
  int32_t tile_upd = 64;       // update tile edge
  int32_t nmslot = 0;
  size_t solve_lds_max = 0;
  int32_t small_prefix = 0;    // leading levels run by one persistent small-front launch
  size_t small_lds_prefix = 0;
  int32_t n_cu = 256;
  size_t lds_limit = 65536;
  bool sweep_levels = false;    // sweeps as one launch per level instead of one persistent launch
  bool small_levels = false;    // small fronts as one launch per level

  // arenas (device)
  void* fac = nullptr;         // nsys * fac_total scalars
  void* upd = nullptr;         // nsys * upd_total scalars
  void* mscr = nullptr;        // nsys * nmslot * nb^2 scalars (trsm multipliers)
  double2* pml = nullptr;      // nsys * (2nx + 2ny + 2)
  double* omega = nullptr;     // nsys
  double* eps = nullptr;       // nsys * N (copy taken at refactor)
  void* y = nullptr;           // nsys * max_rhs * N scalars (elimination order)
  void* wv = nullptr;          // nsys * max_rhs * sum(u) scalars (update vectors)
  double2* xw = nullptr;       // nsys * max_rhs * N (adjoint work solution)
  double2* res = nullptr;      // nsys * max_rhs * N (FP64 residual)
  double* partial = nullptr;   // nsys * max_rhs * res_blocks * 2
  int32_t res_blocks = 0;
  DevStatus* status = nullptr;
  int32_t* counters = nullptr;  // [0..1] persistent-queue counters, [2] residual blocks
  int32_t* done = nullptr;      // [nsys][nfronts] completion epochs
  int32_t epoch = 0;            // last epoch handed to a persistent launch
  DevStatus* status_host = nullptr;  // pinned
  int64_t device_bytes = 0;
  std::vector<void*> allocations;

  // FDFD_PROFILE
  bool profile = false;
  std::vector<hipEvent_t> event_pool;
  std::vector<PendingTiming> pending;
  KernelTotals totals[KC_COUNT];
  // per-front algorithmic figures (host)
  std::vector<double> front_flops;   // real flops of the front's partial LDL^T
  std::vector<double> front_lbytes;  // bytes of the lower-trapezoid factor
  double factor_lbytes = 0;          // sum of front_lbytes (one system)

  hipStream_t last_stream = nullptr;
  std::vector<double> omega_host;
  bool factored = false;
  std::string last_error;
};

// Kernel launchers (fdfd_kernels.hip).  Each returns hipSuccess or the first
// launch error.
hipError_t launch_refactor(Plan& P, const double* eps, int64_t eps_stride, hipStream_t st);
// Solves (SA) X = RHS for every system and nrhs columns with IR.  mode 0:
// forward (rhs = S b, result into x_out, overwritten); mode 1: adjoint
// (rhs = g, lam' into P.xw, then lam = S lam' into lam_out if not null).
hipError_t launch_solve(Plan& P, int mode, const double2* rhs, double2* x_out, int32_t nrhs,
                        int32_t max_ir, double tol, hipStream_t st);
hipError_t launch_gradient(Plan& P, const double2* x, const double2* lam_sym, int32_t nrhs,
                           double2* lam_out, double* grad, int32_t flags, hipStream_t st);
hipError_t launch_status_reset(Plan& P, hipStream_t st);
size_t solve_lds_bytes(const Plan& P, int nrhs);
// FDFD_PROFILE helpers (fdfd_api.cpp)
hipEvent_t profile_event(Plan& P);
void profile_collect(Plan& P);
hipError_t configure_kernels(Plan& P, int lds_limit);

}  // namespace fdfd
