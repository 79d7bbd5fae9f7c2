// HIP kernels (gfx950) of the cached-analysis multifrontal solver:
//   value assembly + extend-add (gather form), dense complex-symmetric partial
//   LDL^T per front, level-scheduled forward / backward sweeps, FP64 residual
//   and refinement control, and the adjoint gradient of Eq. (3).
// Templated over the factor scalar: R = double (complex128) or float (complex64).
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "plan.hpp"

namespace fdfd {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxSys = 64;
constexpr int kBW = 64;  // diagonal-block width shared by the factor layout and the sweeps

template <typename R> struct Cx;
template <> struct Cx<float> { typedef float2 T; };
template <> struct Cx<double> { typedef double2 T; };

template <typename C> __device__ __forceinline__ C czero() { C z; z.x = 0; z.y = 0; return z; }
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { a.x += b.x; a.y += b.y; return a; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { a.x -= b.x; a.y -= b.y; return a; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
// acc - a*b
template <typename C> __device__ __forceinline__ C cfms(C acc, C a, C b) {
  acc.x = acc.x - a.x * b.x + a.y * b.y;
  acc.y = acc.y - a.x * b.y - a.y * b.x;
  return acc;
}
// 1/a: the hardware reciprocal estimate refined by two Newton steps (each
// squares the relative error), within a couple of ulp of the rounded quotient
// for the normal, finite a the pivots have; half the dependent operations of
// an IEEE division, which sits on the serial chain of every pivot step.
__device__ __forceinline__ double rcp_nr(double a) {
  double r = __builtin_amdgcn_rcp(a);
  r = fma(r, fma(-a, r, 1.0), r);
  return fma(r, fma(-a, r, 1.0), r);
}
__device__ __forceinline__ float rcp_nr(float a) {
  const float r = __builtin_amdgcn_rcpf(a);
  return fmaf(r, fmaf(-a, r, 1.0f), r);
}
template <typename C> __device__ __forceinline__ C cinv(C d) {
  const auto r = rcp_nr(d.x * d.x + d.y * d.y);
  C o;
  o.x = d.x * r;
  o.y = -d.y * r;
  return o;
}
template <typename C> __device__ __forceinline__ C from_d2(double2 v) {
  C r;
  r.x = (decltype(r.x))v.x;
  r.y = (decltype(r.y))v.y;
  return r;
}
template <typename C> __device__ __forceinline__ double2 to_d2(C v) {
  return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 ddiv(double2 a, double2 b) {
  const double s = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / s, (a.y * b.x - a.x * b.y) / s);
}
__device__ __forceinline__ double2 dadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 dsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// Everything a kernel needs about the plan, passed by value.
struct KArgs {
  const int32_t *pbeg, *npiv, *nupd, *child_ptr, *child_list, *upd_ptr, *upd_idx;
  const int32_t *gmap, *nbr_row, *perm, *iperm, *parent, *height;
  const int64_t *fac_off, *upd_off, *gmap_ptr;
  int32_t nx, ny, N, nsys;
  int64_t fac_total, upd_total, sum_u;
  const double2* pml;
  const double* eps;
  const double* omega;
  void* fac;
  void* upd;
  DevStatus* st;
  double tau;
  int32_t nfronts;
  int32_t te;  // 1: the TE (Hz) operator, 0: TM (Ez)
  int32_t below_done;  // fronts of height < below_done were factored by earlier launches (k_wave_fronts)
};

// ---------------------------------------------------------------------------
// Operator coefficients of S*A (S = diag(sx_c sy_c)) at one cell.
// ---------------------------------------------------------------------------
struct Stencil {
  double2 diag, c[4];  // couplings to x-1, x+1, y-1, y+1
};

// The permittivity on the four faces of cell (i, j) of system s (TE): the
// mean of the two cells a face separates, the cell's own on the grid edge.
// Both cells of a face evaluate the same expression, so the couplings of S*A
// stay exactly symmetric.
__device__ __forceinline__ void face_eps(const KArgs& a, int s, int n, double (&ef)[4]) {
  const int nx = a.nx, i = n % nx, j = n / nx;
  const double* E = a.eps + (int64_t)s * a.N;
  const double e = E[n];
  ef[0] = i > 0 ? 0.5 * (e + E[n - 1]) : e;
  ef[1] = i < nx - 1 ? 0.5 * (e + E[n + 1]) : e;
  ef[2] = j > 0 ? 0.5 * (e + E[n - nx]) : e;
  ef[3] = j < a.ny - 1 ? 0.5 * (e + E[n + nx]) : e;
}

// TM (Ez):  S*A = Sy_c Dxb Sx_f^-1 Dxf + Sx_c Dyb Sy_f^-1 Dyf + omega^2 eps Sx_c Sy_c
// TE (Hz):  S*A = Sy_c Dxb (eps_x Sx_f)^-1 Dxf + Sx_c Dyb (eps_y Sy_f)^-1 Dyf + omega^2 Sx_c Sy_c
__device__ __forceinline__ Stencil stencil_at(const KArgs& a, int s, int n) {
  const int nx = a.nx, ny = a.ny;
  const int i = n % nx, j = n / nx;
  const double2* tab = a.pml + (int64_t)s * (2 * nx + 2 * ny + 2);
  const double2 sxc = tab[i], sxf0 = tab[nx + i], sxf1 = tab[nx + i + 1];
  const double2 syc = tab[2 * nx + 1 + j], syf0 = tab[2 * nx + 1 + ny + j],
                syf1 = tab[2 * nx + 1 + ny + j + 1];
  Stencil S;
  S.c[0] = ddiv(syc, sxf0);
  S.c[1] = ddiv(syc, sxf1);
  S.c[2] = ddiv(sxc, syf0);
  S.c[3] = ddiv(sxc, syf1);
  const double w = a.omega[s];
  const double2 sc = dmul(sxc, syc);
  double2 d;
  if (a.te) {
    double ef[4];
    face_eps(a, s, n, ef);
#pragma unroll
    for (int k = 0; k < 4; ++k) S.c[k] = make_double2(S.c[k].x / ef[k], S.c[k].y / ef[k]);
    d = make_double2(w * w * sc.x, w * w * sc.y);
  } else {
    const double e = a.eps[(int64_t)s * a.N + n];
    d = make_double2(w * w * e * sc.x, w * w * e * sc.y);
  }
  d = dsub(d, dadd(dadd(S.c[0], S.c[1]), dadd(S.c[2], S.c[3])));
  S.diag = d;
  return S;
}

__device__ __forceinline__ double2 sym_scale(const KArgs& a, int s, int n) {
  const int nx = a.nx, ny = a.ny;
  const int i = n % nx, j = n / nx;
  const double2* tab = a.pml + (int64_t)s * (2 * nx + 2 * ny + 2);
  return dmul(tab[i], tab[2 * nx + 1 + j]);
}

// Entry (r, c), r >= c, of front f before elimination: the original entry of
// S*A (only in pivot columns) plus the children's update blocks (extend-add in
// gather form: every entry reads its contributions, fixed child order).
// Data one workgroup writes and another reads within the same launch (update
// matrices, tiles of large fronts, sweep vectors) moves through agent-coherent
// accesses: relaxed agent-scope atomics, i.e. loads and stores with the sc1
// bit, which bypass the per-XCD caches that are not coherent with each other.
// The completion flags then only need the writer's stores to have completed
// before the flag is set; no agent-scope fence (an L2 write-back or
// invalidate, serialised per XCD and costing microseconds when hundreds of
// workgroups issue them) runs per task.
template <typename C> __device__ __forceinline__ C ld_ag(const C* p) {
  typedef unsigned long long u64;
  u64* q = reinterpret_cast<u64*>(const_cast<C*>(p));
  u64 w[sizeof(C) / 8];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(C) / 8); ++i) w[i] = __hip_atomic_load(q + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  C v;
  __builtin_memcpy(&v, w, sizeof(C));
  return v;
}

template <typename C> __device__ __forceinline__ void st_ag(C* p, C v) {
  typedef unsigned long long u64;
  u64* q = reinterpret_cast<u64*>(p);
  u64 w[sizeof(C) / 8];
  __builtin_memcpy(w, &v, sizeof(C));
#pragma unroll
  for (int i = 0; i < (int)(sizeof(C) / 8); ++i) __hip_atomic_store(q + i, w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Agent-coherent loads through a buffer resource: the same sc1 loads as
// ld_ag, but one 16-byte (complex128) or 8-byte (complex64) load per entry,
// and a load whose byte offset lies outside the resource reads zero, so the
// rows and columns outside a partial tile are masked by their offsets (one
// select per row) rather than by a branch around every load.  The resource
// spans fewer than 2 GiB; kOob is an offset outside every such range.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr unsigned kOob = 0x80000000u;
constexpr int kCacheSc1 = 16;  // cache-policy operand of the buffer loads: sc1

// base and bytes must be the same in every lane (the resource lives in
// scalar registers); they are read from the first lane, so that values the
// compiler cannot prove uniform (a task's front, read from LDS) do not turn
// every load into a loop over the distinct descriptors.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* base, unsigned bytes) {
  const unsigned long long b = (unsigned long long)base;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  void* p = (void*)(((unsigned long long)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(p, 0, (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}

template <typename C> __device__ __forceinline__ C ld_buf(__amdgpu_buffer_rsrc_t r, unsigned off) {
  C v;
  if constexpr (sizeof(C) == 16) {
    const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, kCacheSc1);
    __builtin_memcpy(&v, &w, 16);
  } else {
    const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kCacheSc1);
    __builtin_memcpy(&v, &w, 8);
  }
  return v;
}

template <typename C> __device__ __forceinline__ void st_buf(__amdgpu_buffer_rsrc_t r, unsigned off, C v) {
  if constexpr (sizeof(C) == 16) {
    u32x4 w;
    __builtin_memcpy(&w, &v, 16);
    __builtin_amdgcn_raw_buffer_store_b128(w, r, off, 0, kCacheSc1);
  } else {
    u32x2 w;
    __builtin_memcpy(&w, &v, 8);
    __builtin_amdgcn_raw_buffer_store_b64(w, r, off, 0, kCacheSc1);
  }
}

// Copies a column-major global block (leading dimension ld; rows < nrows,
// columns < ncols; tri = 0 all, 1 lower with diagonal, 2 strictly lower) into
// a zero-padded kBW x kBW LDS block.  Lane = row, wave w takes columns w,
// w+4, ...; all sixteen loads of a thread are in flight before the first
// store, so the block costs about one memory latency.
enum { kAll = 0, kLower = 1, kStrict = 2 };

template <typename C>
__device__ __forceinline__ void stage_block(C* S, const C* g, int64_t ld, int nrows, int ncols, int tri,
                                            const C* scale = nullptr, int64_t scale_stride = 0) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  C v[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int c = wave + 4 * t;
    const bool keep = c < ncols && lane < nrows && (tri == kAll || lane > c || (tri == kLower && lane == c));
    v[t] = keep ? ld_ag(g + (int64_t)c * ld + lane) : czero<C>();
  }
  if (scale) {  // column c times scale[c * scale_stride] (the same for the whole wave)
    C d[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int c = wave + 4 * t;
      d[t] = c < ncols ? ld_ag(scale + (int64_t)c * scale_stride) : czero<C>();
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) v[t] = cmul(v[t], d[t]);
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) S[(wave + 4 * t) * kBW + lane] = v[t];
}

// Original (symmetrised) operator entries of the pivot columns [c0, c0 + nc)
// of front f, one thread per column, staged for the assembly loops:
// sv[5 t] = diagonal, sv[5 t + 1 + d] = coupling to neighbour d (x-1, x+1,
// y-1, y+1), nb[4 t + d] = that neighbour's front row (-1 if not in the front).
template <typename C>
__device__ void stage_columns(const KArgs& a, int s, int f, int c0, int nc, C* sv, int* nb) {
  for (int t = threadIdx.x; t < nc; t += kThreads) {
    const int q = a.pbeg[f] + c0 + t;
    const Stencil S = stencil_at(a, s, a.perm[q]);
    sv[5 * t] = from_d2<C>(S.diag);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      sv[5 * t + 1 + d] = from_d2<C>(S.c[d]);
      nb[4 * t + d] = a.nbr_row[4 * (int64_t)q + d];
    }
  }
}

// Entry (r, c) of the original matrix from staged column t (= c - c0).
template <typename C>
__device__ __forceinline__ C staged_entry(const C* sv, const int* nb, int t, int r, int c) {
  C v = czero<C>();
  if (r == c) v = sv[5 * t];
#pragma unroll
  for (int d = 0; d < 4; ++d)
    if (nb[4 * t + d] == r) v = sv[5 * t + 1 + d];
  return v;
}

// Static pivot perturbation: |d| < thr becomes d (1 + thr/|d|) (thr if d = 0).
// The test uses |d|^2 against thr^2, so a square root is taken only when a
// pivot is perturbed; min2 tracks the smallest |d|^2 seen.
template <typename C>
__device__ __forceinline__ C fix_pivot(C d, double thr, double anorm, int& npert, double& min2, int& nonfin) {
  const double a2 = (double)d.x * d.x + (double)d.y * d.y;
  if (!(a2 <= DBL_MAX)) nonfin = 1;
  min2 = fmin(min2, a2);
  if (a2 < thr * thr) {
    ++npert;
    if (a2 == 0.0) {
      d.x = (decltype(d.x))thr;
      d.y = 0;
    } else {
      const double g = 1.0 + thr / sqrt(a2);
      d.x = (decltype(d.x))(d.x * g);
      d.y = (decltype(d.y))(d.y * g);
    }
  }
  return d;
}

// min2: smallest |d|^2 of the pivots examined by this thread (INFINITY if none).
// Pivot statistics of several fronts, gathered in registers and flushed with
// one set of device atomics: one atomic per front on the same status words
// serialises at the memory side when hundreds of thousands of small fronts
// finish within a few milliseconds.
struct PivotStats {
  int npert = 0, nonfin = 0;
  double ratio = INFINITY;  // min |d_k| / ||SA||_max
  __device__ __forceinline__ void add(int np, double min2, int nf, double anorm) {
    npert += np;
    nonfin |= nf;
    if (min2 < INFINITY) ratio = fmin(ratio, anorm > 0 ? sqrt(min2) / anorm : sqrt(min2));
  }
  __device__ __forceinline__ void flush(DevStatus* st) const {
    if (npert) atomicAdd(&st->n_perturbed, npert);
    if (nonfin) atomicExch(&st->nonfinite, 1);
    if (ratio < INFINITY) {
      // a positive double's bits order like its value; the minimum only
      // changes for the few fronts below it, so most flushes end at the load
      const unsigned long long b = (unsigned long long)__double_as_longlong(ratio);
      if (b < __hip_atomic_load(&st->min_ratio_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMin(&st->min_ratio_bits, b);
    }
  }
};

__device__ __forceinline__ void record_pivots(DevStatus* st, int npert, double min2, int nonfin, double anorm) {
  PivotStats ps;
  ps.add(npert, min2, nonfin, anorm);
  ps.flush(st);
}

__device__ __forceinline__ double anorm_of(const KArgs& a, int s) {
  return __longlong_as_double((long long)a.st->anorm_bits[s]);
}

// ---------------------------------------------------------------------------
// Per-refactor set-up: PML tables, eps copy, ||S*A||_max, status reset.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 stretch(double pos, int n, int npml, double w) {
  if (npml <= 0) return make_double2(1.0, 0.0);
  const double d = fmax(fmax(npml - pos, pos - (double)(n - npml)), 0.0) / npml;
  const double sigma = (32.0 / npml) * d * d * d;
  return make_double2(1.0, sigma / w);
}

struct Omegas {
  double w[kMaxSys];
};

__global__ void k_setup(KArgs a, Omegas om, int npml_x, int npml_y) {
  const int s = blockIdx.x;
  const int nx = a.nx, ny = a.ny;
  double2* tab = const_cast<double2*>(a.pml) + (int64_t)s * (2 * nx + 2 * ny + 2);
  const double w = om.w[s];
  for (int t = threadIdx.x; t < 2 * nx + 2 * ny + 2; t += blockDim.x) {
    double2 v;
    if (t < nx) v = stretch(t + 0.5, nx, npml_x, w);
    else if (t < 2 * nx + 1) v = stretch(t - nx, nx, npml_x, w);
    else if (t < 2 * nx + 1 + ny) v = stretch(t - (2 * nx + 1) + 0.5, ny, npml_y, w);
    else v = stretch(t - (2 * nx + 1 + ny), ny, npml_y, w);
    tab[t] = v;
  }
  if (threadIdx.x == 0) {
    const_cast<double*>(a.omega)[s] = w;
    a.st->anorm_bits[s] = 0ull;
    if (s == 0) {
      a.st->min_ratio_bits = (unsigned long long)__double_as_longlong(INFINITY);
      a.st->n_perturbed = 0;
      a.st->nonfinite = 0;
      a.st->spin_timeout = 0;
      // the solves before this refactor used the previous factor: their
      // refinement figures no longer describe the plan
      a.st->ir_steps_solve = 0;
      a.st->ir_steps_adj = 0;
      a.st->rel_solve = -1.0;
      a.st->rel_adj = -1.0;
      a.st->ir_failed_solve = 0;
      a.st->ir_failed_adj = 0;
    }
  }
}

__global__ void k_copy_eps(KArgs a, const double* eps_in, int64_t stride) {
  const int s = blockIdx.y;
  double* dst = const_cast<double*>(a.eps) + (int64_t)s * a.N;
  const double* src = eps_in + (int64_t)s * stride;
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
       n += (int64_t)gridDim.x * blockDim.x)
    dst[n] = src[n];
}

__global__ __launch_bounds__(kThreads) void k_anorm(KArgs a) {
  const int s = blockIdx.y;
  double mx = 0.0;
  int nonfin = 0;
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
       n += (int64_t)gridDim.x * blockDim.x) {
    const Stencil S = stencil_at(a, s, (int)n);
    double v = hypot(S.diag.x, S.diag.y);
    if (!(v <= DBL_MAX)) nonfin = 1;
    for (int d = 0; d < 4; ++d) v = fmax(v, hypot(S.c[d].x, S.c[d].y));
    mx = fmax(mx, v);
  }
  __shared__ double red[kThreads];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(&a.st->anorm_bits[s], (unsigned long long)__double_as_longlong(red[0]));
    if (nonfin) atomicExch(&a.st->nonfinite, 1);
  }
}

// ---------------------------------------------------------------------------
// Persistent, dependency-driven launches.  Work items are claimed in level
// order from an atomic counter; an item first waits (bounded spin) until the
// items it depends on have stored this launch's epoch in their done flag.
// Items are claimed in topological order, so every awaited item is held by a
// workgroup that is already running and waits only on earlier items: every
// wait ends.  The spin limit turns an unexpected stall into a status flag
// rather than a hang.  The last workgroup to leave resets the counters for the
// next launch on the stream.
// ---------------------------------------------------------------------------
constexpr int kSpinLimit = 1 << 24;

struct Queue {
  int32_t* counter;  // [0] next item, [1] workgroups that have left, [kEpochSlot] last epoch
  int32_t* done;     // [nsys][nfronts] epoch of the last completion
  DevStatus* st;
  long long* trace;  // optional: per item claim / ready / finish times and workgroup
  int32_t ntasks, wait;
};

// The launch's epoch is read from device memory (one past the previous
// launch's) rather than passed by the host, so the same launch recorded in a
// HIP graph gets a fresh epoch on every replay.  Every workgroup reads it
// before it can leave, and the last one to leave stores it back.  The value
// was written by an earlier launch on the stream, which the launch boundary
// makes visible, so a plain (cached) load suffices: an agent-scope load from
// thousands of workgroups at once would queue on one memory channel.  The
// value is made wave-uniform explicitly; left to the compiler it shifted the
// register allocation of the forward sweep into scratch spills.
__device__ __forceinline__ int launch_epoch(const Queue& q) {
  return __builtin_amdgcn_readfirstlane(q.counter[kEpochSlot]) + 1;
}

__device__ __forceinline__ void trace_mark(const Queue& q, int t, int slot) {
  if (q.trace && threadIdx.x == 0 && t < q.ntasks) q.trace[4 * (int64_t)t + slot] = (long long)wall_clock64();
}

__device__ __forceinline__ int claim(const Queue& q, int* sh) {
  __syncthreads();
  if (threadIdx.x == 0) *sh = atomicAdd(&q.counter[0], 1);
  __syncthreads();
  const int t = *sh;
  trace_mark(q, t, 0);
  if (q.trace && threadIdx.x == 0 && t < q.ntasks) q.trace[4 * (int64_t)t + 3] = blockIdx.x;
  return t;
}

__device__ __forceinline__ void leave(const Queue& q, int ep) {
  if (threadIdx.x == 0) {
    const int n = atomicAdd(&q.counter[1], 1);
    if (n == (int)(gridDim.x * gridDim.y * gridDim.z) - 1) {
      q.counter[0] = 0;
      q.counter[1] = 0;
      __hip_atomic_store(q.counter + kEpochSlot, ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Polls with relaxed agent-scope loads (they read past the non-coherent
// caches without invalidating them).  Once every awaited flag is seen the
// caller issues a workgroup-scope acquire (it keeps the data loads below the
// poll; those loads are agent-coherent themselves) and a barrier.
__device__ __forceinline__ void wait_flag(const Queue& q, int ep, const int32_t* p) {
  int it = 0;
  while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ep) {
    if (++it > kSpinLimit) {
      atomicExch(&q.st->spin_timeout, 1);
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// One thread per child (each flag read is a memory round trip).
__device__ __forceinline__ void wait_children(const Queue& q, int ep, const KArgs& a, int s, int f) {
  for (int k = a.child_ptr[f] + threadIdx.x; k < a.child_ptr[f + 1]; k += blockDim.x) {
    const int c = a.child_list[k];
    // a child factored by k_wave_fronts finished with that earlier launch
    if (a.height[c] < a.below_done) continue;
    wait_flag(q, ep, q.done + (int64_t)s * a.nfronts + c);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  __syncthreads();
}

__device__ __forceinline__ void wait_parent(const Queue& q, int ep, const KArgs& a, int s, int f) {
  if (threadIdx.x == 0 && a.parent[f] >= 0) {
    wait_flag(q, ep, q.done + (int64_t)s * a.nfronts + a.parent[f]);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
  __syncthreads();
}

// Before a completion flag is set, every wave waits until its (agent-coherent)
// stores have completed; a workgroup barrier alone does not wait for other
// waves' stores.  The compiler-level release fence keeps the stores above it.
__device__ __forceinline__ void drain_stores() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt and lgkmcnt unconstrained (gfx9 encoding)
}

// Orders one wavefront's LDS accesses across its lanes (its LDS operations
// complete in program order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void publish(const Queue& q, int ep, int64_t idx) {
  drain_stores();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(q.done + idx, ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Dense building blocks on LDS-resident, column-major panels (leading
// dimension ld).  Wave w takes columns w, w+4, ...; lane l takes rows l, l+64,
// ... so no index arithmetic needs a division.
// ---------------------------------------------------------------------------

// Matrix-core instructions used on LDS-resident operands: 16x16x4 products in
// the factor precision.  Operand lanes: A row l%16 / B column l%16 at
// k = l/16; the result row of register r differs between the f64 and f32
// instructions (row()); its column is l%16.  The tile routines below put the
// output-column operand in the A slot, so each register holds the transposed
// product: the output row varies with l%16, and a store of sixteen lanes to a
// column-major LDS block covers consecutive entries (the other way round the
// sixteen lanes would hit one bank, a whole column apart).
template <typename R> struct Mfma;
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};

// Broadcast of lane j's value to the whole wave (j uniform).
template <typename C> __device__ __forceinline__ C bcast_c(C v, int j) {
  constexpr int n = sizeof(C) / 4;
  int w[n];
  __builtin_memcpy(w, &v, sizeof(C));
#pragma unroll
  for (int i = 0; i < n; ++i) w[i] = __builtin_amdgcn_readlane(w[i], j);
  C o;
  __builtin_memcpy(&o, w, sizeof(C));
  return o;
}

template <typename C> __device__ __forceinline__ C shfl_c(C v, int lane) {
  v.x = __shfl(v.x, lane);
  v.y = __shfl(v.y, lane);
  return v;
}

template <typename C> __device__ __forceinline__ C shfl_xor_c(C v, int mask) {
  v.x = __shfl_xor(v.x, mask);
  v.y = __shfl_xor(v.y, mask);
  return v;
}

// LDL^T of the b x b (b <= 16) diagonal sub-block at (o, o) together with the
// rows below it up to row 63, by wave 0 alone: lane l holds row l of the
// sub-block's columns in registers.  Each step the lanes of the sub-block
// publish their entry of the pivot column to colbuf and every lane reads it
// back as broadcasts (one wave, so the LDS accesses stay in order without a
// barrier).  Leaves the unit-lower L (scaled) in place for rows < min(m, 64)
// and d, 1/d in dd / invd; lane 0 keeps the statistics.
template <typename C>
__device__ void ldl_sub16(C* F, int ld, int o, int b, int m, C* dd, C* invd, C* colbuf, double thr, double anorm,
                          int& npert, double& minr, int& nonfin) {
  const int l = threadIdx.x;
  const bool act = l >= o && l < m;
  C row[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) row[q] = (act && q < b && o + q <= l) ? F[(o + q) * ld + l] : czero<C>();
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if (k < b) {
      if (l >= o && l < o + 16) colbuf[l - o] = row[k];
      __builtin_amdgcn_wave_barrier();
      C cj[16];
#pragma unroll
      for (int j = k; j < 16; ++j) cj[j] = colbuf[j];
      int np = 0, nf = 0;
      double mr = INFINITY;
      const C d = fix_pivot(cj[k], thr, anorm, np, mr, nf);
      const C inv = cinv(d);
      if (l == 0) {
        npert += np;
        minr = fmin(minr, mr);
        nonfin |= nf;
        dd[o + k] = d;
        invd[o + k] = inv;
      }
      const C lk = cmul(row[k], inv);
      // Branch-free: lanes l < o + j only touch entries above the diagonal,
      // which are never published (colbuf reads start at k) nor stored.
#pragma unroll
      for (int j = k + 1; j < 16; ++j)
        if (j < b) row[j] = cfms(row[j], lk, cj[j]);
      const bool below = l > o + k;
      row[k].x = below ? lk.x : row[k].x;
      row[k].y = below ? lk.y : row[k].y;
      __builtin_amdgcn_wave_barrier();
    }
  }
  if (act) {
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (q < b && o + q < l) F[(o + q) * ld + l] = row[q];
  }
}

// The same factorisation with all four waves: lane l holds row l, wave w the
// sub-block columns w, w+4, w+8, w+12.  Each step the owner of pivot column k
// publishes it to one of two alternating LDS buffers, one barrier, and every
// wave forms l_k = a_k / d_k itself and updates its own columns (the same
// operations, in the same order per entry, as ldl_sub16).  All LDS reads of a
// step are issued together right after the barrier, before the step's writes
// (d, 1/d), and the column updates are computed unconditionally and selected
// (w is scalar), so a step costs one LDS round trip instead of one per read.
// colbuf: 2 x 64.  Called by the whole workgroup.
template <typename C>
__device__ void ldl_sub16_mw(C* F, int ld, int o, int b, int m, C* dd, C* invd, C* colbuf, double thr,
                             double anorm, int& npert, double& minr, int& nonfin) {
  const int l = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool act = l >= o && l < m;
  C col[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int q = w + 4 * t;
    col[t] = (act && q < b && o + q <= l) ? F[(o + q) * ld + l] : czero<C>();
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if (k < b) {
      C* buf = colbuf + (k & 1) * 64;
      if (w == (k & 3)) buf[l] = col[k >> 2];
      __syncthreads();
      const C piv = buf[o + k];
      const C bl = buf[l];
      C cj[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) cj[t] = buf[o + w + 4 * t];
      int np = 0, nf = 0;
      double mr = INFINITY;
      const C d = fix_pivot(piv, thr, anorm, np, mr, nf);
      const C inv = cinv(d);
      const C lk = cmul(bl, inv);
      // Lanes l < o + j only touch entries above the diagonal, which are
      // never published nor stored.
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int j = w + 4 * t;
        const C upd = cfms(col[t], lk, cj[t]);
        if (j > k && j < b) col[t] = upd;
      }
      if (w == (k & 3)) {
        const bool below = l > o + k;
        col[k >> 2].x = below ? lk.x : col[k >> 2].x;
        col[k >> 2].y = below ? lk.y : col[k >> 2].y;
      }
      if (threadIdx.x == 0) {
        npert += np;
        minr = fmin(minr, mr);
        nonfin |= nf;
        dd[o + k] = d;
        invd[o + k] = inv;
      }
    }
  }
  if (act) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int q = w + 4 * t;
      if (q < b && o + q < l) F[(o + q) * ld + l] = col[t];
    }
  }
}

// Rows r in [r0, m) of the sub-block's columns: L_r = F_r L_ss^-T D^-1 by
// forward substitution, one row per thread.
template <typename C>
__device__ void trsm_rows16(C* F, int ld, int o, int b, int r0, int m, const C* invd) {
  for (int r = r0 + (int)threadIdx.x; r < m; r += kThreads) {
    C y[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (j < b) {
        C v = F[(o + j) * ld + r];
#pragma unroll
        for (int q = 0; q < j; ++q) v = cfms(v, y[q], F[(o + q) * ld + o + j]);
        y[j] = v;
      }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (j < b) F[(o + j) * ld + r] = cmul(y[j], invd[o + j]);
  }
}

// Trailing update of the panel columns c in [c0, p), rows r >= c:
// F[r][c] -= sum_q L[r][o+q] d_q L[c][o+q].  The d-scaled columns go to Lsc
// first; then lane = row (its 16 L values in registers), wave w takes the
// columns c0+w, c0+w+4, ... and reads their scaled rows as broadcasts.
template <typename C>
__device__ void trail16(C* F, int ld, int o, int b, int c0, int p, int m, const C* dd) {
  // the d-scaled rows d_q L[c][o+q] go to rows o .. o+15 of column c, above
  // its diagonal (c >= c0 = o + 16): nothing reads the panel's upper part,
  // and the updates below touch rows >= c0 only
  for (int idx = threadIdx.x; idx < (p - c0) * 16; idx += kThreads) {
    const int c = c0 + (idx >> 4), q = idx & 15;
    F[c * ld + o + q] = q < b ? cmul(F[(o + q) * ld + c], dd[o + q]) : czero<C>();
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = c0 + lane; r < m; r += 64) {
    C lr[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) lr[q] = q < b ? F[(o + q) * ld + r] : czero<C>();
    // uniform trip count: rows r < c update entries above the diagonal,
    // which no later step reads
    for (int c = c0 + wave; c < p; c += 4) {
      const C* sc = F + c * ld + o;
      C acc = F[c * ld + r];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc = cfms(acc, lr[q], sc[q]);
      F[c * ld + r] = acc;
    }
  }
}

// Trailing update on the matrix cores for a kBW x kBW block (ld = kBW, the
// DIAG task): F[r][c] -= sum_q L[r][o+q] d_q L[c][o+q] for c0 <= c <= r < kBW,
// with c0 = o + 16.  The d-scaled rows go to Bt[q][c] (scratch, 16 x kBW);
// the lower 16 x 16 output blocks are shared out over the waves, K = 16 as
// four 4-deep k-steps of four real MFMAs.  Entries above the diagonal inside
// diagonal blocks are updated too; nothing reads them.
template <typename C>
__device__ __forceinline__ void trail_mfma(C* F, int o, int b, int c0, int p, const C* dd, C* Bt) {
  typedef decltype(F->x) R;
  typedef typename Mfma<R>::v4 v4;
  for (int idx = threadIdx.x; idx < 16 * kBW; idx += kThreads) {
    const int q = idx >> 6, c = idx & 63;
    Bt[idx] = (q < b && c >= c0 && c < p) ? cmul(F[(o + q) * kBW + c], dd[o + q]) : czero<C>();
  }
  __syncthreads();
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6, i = l & 15, kq = l >> 4;
  const int nbr = (kBW - c0) >> 4, bb0 = c0 >> 4, nblk = nbr * (nbr + 1) / 2;
  for (int bid = wave; bid < nblk; bid += 4) {
    // bid -> (bi, bj), bj <= bi, counted from bb0
    int bi = 0, rem = bid;
    while (rem > bi) {
      rem -= bi + 1;
      ++bi;
    }
    const int BI = bb0 + bi, BJ = bb0 + rem;
    v4 re = v4{0, 0, 0, 0}, im = v4{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int q = 4 * ks + kq;
      const C av = F[(o + q) * kBW + 16 * BI + i];
      const C bv = Bt[q * kBW + 16 * BJ + i];
      re = Mfma<R>::op(bv.x, av.x, re);
      im = Mfma<R>::op(bv.y, av.x, im);
      re = Mfma<R>::op(bv.y, -av.y, re);
      im = Mfma<R>::op(bv.x, av.y, im);
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      C* dst = F + (16 * BJ + Mfma<R>::row(l, rr)) * kBW + 16 * BI + i;
      C v = *dst;
      v.x -= re[rr];
      v.y -= im[rr];
      *dst = v;
    }
  }
}

// Blocked right-looking LDL^T of the first p (<= 64) columns of an m-row LDS
// panel: per 16-column sub-block, wave 0 factors the diagonal sub-block, all
// threads solve the rows below it and update the remaining panel columns.
// Leaves the unit-lower L in place and d, 1/d in dd / invd.
// scratch: the pivot column buffer (2 x 64 entries of LDS); the diagonal tile
// (DiagTile) also keeps its d-scaled rows there (16 x 64), the panel of a
// small front in its own upper part.
// DiagTile: the kBW x kBW pivot block of the DIAG task (ld = m = kBW), whose
// trailing updates run on the matrix cores.
template <bool DiagTile = false, typename C>
__device__ void ldl_blocked(C* F, int ld, int m, int p, C* dd, C* invd, C* scratch, double thr, double anorm,
                            int& npert, double& minr, int& nonfin) {
  for (int o = 0; o < p; o += 16) {
    const int b = min(16, p - o);
    ldl_sub16_mw(F, ld, o, b, m, dd, invd, scratch, thr, anorm, npert, minr, nonfin);
    __syncthreads();
    if (m > 64) {
      trsm_rows16(F, ld, o, b, 64, m, invd);
      __syncthreads();
    }
    if (o + b < p) {
      if (DiagTile) trail_mfma(F, o, b, o + b, p, dd, scratch);
      else trail16(F, ld, o, b, o + b, p, m, dd);
      __syncthreads();
    }
  }
}

// In-place inverse of the unit-lower nb x nb (nb <= 64) block at F, in two
// parts.  invert_diag16: each wave inverts one 16 x 16 diagonal sub-block
// (lane j builds column j).  invert_offdiag: the off-diagonal sub-blocks in
// ascending block columns and rows, X_ij = -X_ii sum_{j<=k<i} L_ik X_kj,
// through the 16 x 16 scratch T (reads the X_ii left by invert_diag16).
template <typename C>
__device__ __forceinline__ void invert_diag16(C* F, int ld, int nb) {
  // Lane and wave are made opaque here so that the identity column and the
  // LDS addresses below are formed in the task, not hoisted out of the
  // persistent task loop: hoisted, these lane-dependent values lived across
  // every task type and were spilled, and each step waited for their
  // reloads from scratch memory.
  int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  asm volatile("" : "+v"(lane), "+v"(wave));
  const int nsb = (nb + 15) / 16;
  if (wave < nsb) {
    const int j = lane;
    const int o = 16 * wave, b = min(16, nb - o);
    // Right-looking: once x_k is final every later row takes its term
    // -L_ik x_k, so the dependent chain is one step per column (a row-by-row
    // form chains all i terms of a row).  Per entry the subtractions and
    // their order are those of the row-by-row form; x_k = 0 for k < j, so
    // the sums give the column (and 0 above the diagonal, never stored).
    C x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      x[i].x = i == j ? 1 : 0;
      x[i].y = 0;
    }
#pragma unroll
    for (int k = 0; k < 15; ++k) {
      if (k < b) {
        C lc[16];
#pragma unroll
        for (int i = k + 1; i < 16; ++i) lc[i] = i < b ? F[(o + k) * ld + o + i] : czero<C>();
#pragma unroll
        for (int i = k + 1; i < 16; ++i) x[i] = cfms(x[i], lc[i], x[k]);
      }
      // keeps the next column's loads from being hoisted (register pressure)
      __builtin_amdgcn_sched_barrier(0);
    }
    if (j < b) {
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (i > j && i < b) F[(o + j) * ld + o + i] = x[i];
    }
  }
  __syncthreads();
}

template <typename C>
__device__ __forceinline__ void invert_offdiag(C* F, int ld, int nb, C* T) {
  const int nsb = (nb + 15) / 16;
  // r varies fastest across lanes: the reads of a row-r column are consecutive
  // entries, the reads of column c are broadcasts (with c fastest, sixteen
  // lanes would read addresses a whole column apart: 16-way bank conflicts)
  const int r = threadIdx.x & 15, c = threadIdx.x >> 4;
  for (int jb = 0; jb + 1 < nsb; ++jb) {
    for (int ib = jb + 1; ib < nsb; ++ib) {
      const int ri = 16 * ib, cj = 16 * jb, bi = min(16, nb - ri), bj = min(16, nb - cj);
      // every lane computes (clamped addresses); only r < bi, c < bj store
      const int rr = min(r, bi - 1), cc = min(c, bj - 1);
      C acc = czero<C>();
      for (int kb = jb; kb < ib; ++kb) {
        const int rk = 16 * kb, bk = min(16, nb - rk);
        const bool diag = kb == jb;
#pragma unroll 4
        for (int q = 0; q < 16; ++q) {
          if (q < bk) {  // uniform across the workgroup
            // X_{kb,jb}[q][c]: unit lower on the diagonal block
            const C st = F[(cj + cc) * ld + rk + q];
            C xv = st;
            if (diag) {
              xv.x = q > c ? st.x : (q == c ? 1 : 0);
              xv.y = q > c ? st.y : 0;
            }
            acc = cadd(acc, cmul(F[(rk + q) * ld + ri + rr], xv));
          }
        }
      }
      if (r < bi && c < bj) T[c * 16 + r] = acc;
      __syncthreads();
      if (r < bi && c < bj) {
        C v = czero<C>();
#pragma unroll 4
        for (int q = 0; q < 16; ++q) {
          const C xl = F[(ri + q) * ld + ri + r];
          C xv;
          xv.x = q < r ? xl.x : (q == r ? 1 : 0);
          xv.y = q < r ? xl.y : 0;
          if (q < bi) v = cadd(v, cmul(xv, T[c * 16 + q]));
        }
        v.x = -v.x;
        v.y = -v.y;
        F[(cj + c) * ld + ri + r] = v;
      }
      __syncthreads();
    }
  }
}

template <typename C>
__device__ __forceinline__ void invert_blocked(C* F, int ld, int nb, C* T) {
  invert_diag16(F, ld, nb);
  invert_offdiag(F, ld, nb, T);
}

// ---------------------------------------------------------------------------
// Small fronts: one workgroup per (front, system), whole panel in LDS.
// Assembly, partial LDL^T of the pivot columns, Schur update of the u x u
// block (4 x 4 register tiles) straight into the front's update slot, then the
// panel (its lower trapezoid: unit-lower L and D on the diagonal).
// LDS: F (m x p) | d (p) | 1/d (p) | scratch | the children's gather rows.
// The stencils of the pivot columns are staged in the d / 1/d / scratch area,
// which is free until the factorisation starts.
// ---------------------------------------------------------------------------
// (the 2 x 64 pivot-column buffer of the LDL^T, and the stencils staged before
// it: 5p values and 4p indices from d on)
__host__ __device__ constexpr int small_scratch_entries(int p) { return 5 * p > 128 ? 5 * p : 128; }

// The children of a front (at most two: the separator tree is binary), read
// once per front: the compiler cannot keep these table reads out of a loop
// that also stores to global memory, and each would cost a dependent memory
// round trip per batch.
template <typename C>
struct Kids {
  int n;
  const C* u0;
  const C* u1;
  int nu0, nu1;
};

template <typename C>
__device__ __forceinline__ Kids<C> kids_of(const KArgs& a, int s, int f) {
  Kids<C> k;
  const int cb = a.child_ptr[f];
  k.n = a.child_ptr[f + 1] - cb;
  const C* U = (const C*)a.upd + (int64_t)s * a.upd_total;
  const int ch0 = k.n > 0 ? a.child_list[cb] : 0, ch1 = k.n > 1 ? a.child_list[cb + 1] : 0;
  k.u0 = U + (k.n > 0 ? a.upd_off[ch0] : 0);
  k.u1 = U + (k.n > 1 ? a.upd_off[ch1] : 0);
  k.nu0 = k.n > 0 ? a.nupd[ch0] : 0;
  k.nu1 = k.n > 1 ? a.nupd[ch1] : 0;
  return k;
}

// Component-wise select, so that conditional updates of a register array
// stay branch-free (a branch around each update makes the compiler keep the
// array in scratch across the branches).
template <typename C> __device__ __forceinline__ C csel(bool c, C a, C b) {
  C r;
  r.x = c ? a.x : b.x;
  r.y = c ? a.y : b.y;
  return r;
}

// Children's contributions to NB front entries (rr[e], cc[e]) (rr[e] >= cc[e],
// rr[e] < 0 marks an unused slot), the children's gather rows staged in LDS
// (gl: one row of m ints per child).  The loads of both children are issued
// together: one memory round trip for the batch.
template <typename C, int NB>
__device__ __forceinline__ void add_children_lds(const Kids<C>& k, int m, const int* gl, const int (&rr)[NB],
                                                 const int (&cc)[NB], C (&val)[NB]) {
  // every load unconditional (entry 0 of the block where the entry is not
  // the child's; a missing child's block pointer is the arena's start) and
  // its value selected after all are issued: a load inside a branch would be
  // waited for before the branch ends, one memory round trip per entry
  C v0[NB], v1[NB];
  bool h0[NB], h1[NB];
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    const bool use = rr[e] >= 0;
    const int g0r = use && k.n > 0 ? gl[rr[e]] : -1, g0c = use && k.n > 0 ? gl[cc[e]] : -1;
    const int g1r = use && k.n > 1 ? gl[m + rr[e]] : -1, g1c = use && k.n > 1 ? gl[m + cc[e]] : -1;
    h0[e] = g0r >= 0 && g0c >= 0;
    h1[e] = g1r >= 0 && g1c >= 0;
    v0[e] = ld_ag(k.u0 + (h0[e] ? (int64_t)g0c * k.nu0 + g0r : 0));
    v1[e] = ld_ag(k.u1 + (h1[e] ? (int64_t)g1c * k.nu1 + g1r : 0));
  }
#pragma unroll
  for (int e = 0; e < NB; ++e)
    val[e] = cadd(cadd(val[e], csel(h0[e], v0[e], czero<C>())), csel(h1[e], v1[e], czero<C>()));
}

// The loads of a small front that depend on no other front: the pivot
// columns' stencils (into the staging area) and the children's gather rows.
// Issued before the wait for the children.
template <typename R>
__device__ __forceinline__ void small_front_stage(const KArgs& a, int s, int f, unsigned char* smem_raw) {
  typedef typename Cx<R>::T C;
  C* F = reinterpret_cast<C*>(smem_raw);
  const int p = a.npiv[f], m = p + a.nupd[f];
  C* dd = F + (int64_t)m * p;
  stage_columns(a, s, f, 0, p, dd, reinterpret_cast<int*>(dd + 5 * p));
  int* gl = reinterpret_cast<int*>(dd + 2 * p + small_scratch_entries(p));
  const int nch = a.child_ptr[f + 1] - a.child_ptr[f];
  const int32_t* g = a.gmap + a.gmap_ptr[f];
  for (int k = threadIdx.x; k < nch * m; k += kThreads) gl[k] = g[k];
}

// One 64 x 64 tile (ti, tj) of a small front's update block on the matrix
// cores: U = the children's contributions - L_u D L_u^T.  Every wave owns
// 16 x 16 blocks (bi, bj) of the tile (on a diagonal tile the ten on or
// below its diagonal, three or two per wave; off it one block row per wave)
// and accumulates their real and imaginary parts over the p pivot columns,
// four at a time (depth zero-padded past p).  Rows past u read a valid row
// and are zeroed.  Lane l holds entries (16 bi + (l & 15), 16 bj + row(l, r)).
template <typename R>
__device__ __forceinline__ void schur_tile_mfma(const typename Cx<R>::T* F, int m, int p, int u, int ti, int tj,
                                                const typename Cx<R>::T* dd, const Kids<typename Cx<R>::T>& kids,
                                                const int* gl, typename Cx<R>::T* U) {
  typedef typename Cx<R>::T C;
  typedef typename Mfma<R>::v4 v4;
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = l & 15, kq = l >> 4;
  int nblk, bi[4], bj[4];
  if (ti == tj) {
    nblk = wave < 2 ? 3 : 2;
    bi[0] = wave < 2 ? 3 : 2;
    bj[0] = wave == 0 ? 0 : wave == 1 ? 2 : wave == 2 ? 0 : 2;
    bi[1] = wave < 2 ? 3 : wave == 2 ? 2 : 1;
    bj[1] = wave == 0 ? 1 : wave == 1 ? 3 : 1;
    bi[2] = wave == 0 ? 0 : 1;
    bj[2] = 0;
    bi[3] = 0;
    bj[3] = 0;
  } else {
    nblk = 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      bi[t] = wave;
      bj[t] = t;
    }
  }
  v4 re[4], im[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    re[t] = v4{0, 0, 0, 0};
    im[t] = v4{0, 0, 0, 0};
  }
  const C* Fu = F + p;  // the update rows of the pivot columns
#pragma unroll 2
  for (int k0 = 0; k0 < p; k0 += 4) {
    const int q = k0 + kq;
    const bool qok = q < p;
    const int qc = qok ? q : p - 1;
    const C dq = dd[qc];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < nblk) {  // uniform per wave
        const int ra = ti + 16 * bi[t] + i, rb = tj + 16 * bj[t] + i;
        const C a0 = Fu[qc * m + min(ra, u - 1)];
        const C b0 = Fu[qc * m + min(rb, u - 1)];
        const C av = csel(qok && ra < u, a0, czero<C>());
        const C bv = csel(qok && rb < u, cmul(b0, dq), czero<C>());
        re[t] = Mfma<R>::op(bv.x, av.x, re[t]);
        im[t] = Mfma<R>::op(bv.y, av.x, im[t]);
        re[t] = Mfma<R>::op(bv.y, -av.y, re[t]);
        im[t] = Mfma<R>::op(bv.x, av.y, im[t]);
      }
    }
  }
  // the children's contributions and the store, two blocks (eight entries)
  // per batch
#pragma unroll
  for (int t0 = 0; t0 < 4; t0 += 2) {
    if (t0 < nblk) {  // uniform per wave
      int rr[8], cc[8];
      C v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int t = t0 + (e >> 2), r4 = e & 3;
        const int rw = ti + 16 * bi[t] + i, cl = tj + 16 * bj[t] + Mfma<R>::row(l, r4);
        const bool ok = t < nblk && rw < u && cl < u && rw >= cl;
        rr[e] = ok ? p + rw : -1;
        cc[e] = p + cl;
        v[e] = czero<C>();
      }
      add_children_lds<C, 8>(kids, m, gl, rr, cc, v);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int t = t0 + (e >> 2), r4 = e & 3;
        if (rr[e] >= 0) {
          C acc;
          acc.x = re[t][r4];
          acc.y = im[t][r4];
          st_ag(U + (int64_t)(cc[e] - p) * u + (rr[e] - p), csub(v[e], acc));
        }
      }
    }
  }
}

template <typename R>
__device__ void small_front(const KArgs& a, const Queue& q, int ep, int s, int f, const Kids<typename Cx<R>::T>& kids,
                            unsigned char* smem_raw, PivotStats& ps) {
  typedef typename Cx<R>::T C;
  C* F = reinterpret_cast<C*>(smem_raw);
  const int p = a.npiv[f], u = a.nupd[f], m = p + u;
  C* dd = F + (int64_t)m * p;
  C* invd = dd + p;  // followed by small_scratch_entries(p) entries of scratch
  const int* gl = reinterpret_cast<const int*>(dd + 2 * p + small_scratch_entries(p));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  {
    // the stencils staged by small_front_stage (the barrier after the wait
    // for the children orders them)
    const C* sv = dd;
    const int* nbv = reinterpret_cast<const int*>(dd + 5 * p);
    // four columns per wave (c, c+4, c+8, c+12) and two rows (lane, lane + 64)
    // per batch of eight entries
    for (int cb = wave; cb < p; cb += 16)
      for (int r0 = lane; r0 < m; r0 += 128) {
        int rr[8], cc[8];
        C v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int c = cb + 4 * (e & 3), r = r0 + 64 * (e >> 2);
          const bool ok = c < p && r < m && r >= c;
          rr[e] = ok ? r : -1;
          cc[e] = c;
          v[e] = ok ? staged_entry(sv, nbv, c, r, c) : czero<C>();
        }
        add_children_lds<C, 8>(kids, m, gl, rr, cc, v);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int c = cb + 4 * (e & 3), r = r0 + 64 * (e >> 2);
          if (c < p && r < m) F[c * m + r] = v[e];
        }
      }
    __syncthreads();
  }

  const double anorm = anorm_of(a, s);
  const double thr = a.tau * anorm;
  int npert = 0, nonfin = 0;
  double minr = INFINITY;
  ldl_blocked(F, m, m, p, dd, invd, invd + p, thr, anorm, npert, minr, nonfin);

  // Schur complement: U = F22 - L_u D L_u^T over the update rows.
  C* U = (C*)a.upd + (int64_t)s * a.upd_total + a.upd_off[f];
  for (int ti = 0; ti < u; ti += 64)
    for (int tj = 0; tj <= ti; tj += 64) schur_tile_mfma<R>(F, m, p, u, ti, tj, dd, kids, gl, U);
  // the parent needs only the update block: release it before the panel
  publish(q, ep, s * a.nfronts + f);
  // Stored panel of a small front (p <= 64): D on the diagonal and the
  // unit-lower L below it, no inverse (the sweeps of these fronts solve with
  // L11 in registers of one wavefront, a chain of p lane broadcasts, far
  // shorter than a memory round trip).  Nothing reads above the diagonal.
  C* L = (C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  for (int c = wave; c < p; c += 4)
    for (int r = c + lane; r < m; r += 64) L[(int64_t)c * m + r] = r > c ? F[c * m + r] : dd[c];
  if (threadIdx.x == 0) ps.add(npert, minr, nonfin, anorm);
}

// Pivot step K of the leaf LDL^T and every step after it, unrolled through
// template recursion so that the row stays in registers (a loop the compiler
// declines to unroll fully would index x dynamically, i.e. through scratch).
template <int K, int PMAX, int NR, typename C>
struct LeafSteps {
  __device__ __forceinline__ static void run(C (&x)[NR][PMAX], C* col, C* dd, int p, int lane, double thr,
                                             double anorm, int& npert, double& minr, int& nonfin) {
    if constexpr (K < PMAX) {
      if (K >= p) return;
      // the pivot rows are all among the first 64 (p <= 64): they publish
      // the column; a lane's second row (lane + 64 > K) only takes updates
      col[lane] = x[0][K];
      wave_sync();
      const C d = fix_pivot(col[K], thr, anorm, npert, minr, nonfin);
      const C di = cinv(d);
      const C l0 = csel(lane > K, cmul(x[0][K], di), czero<C>());
      C l1 = czero<C>();
      if constexpr (NR == 2) l1 = cmul(x[1][K], di);
#pragma unroll
      for (int j = K + 1; j < PMAX; ++j)
        if (j < p) {
          const C cj = col[j];
          x[0][j] = csel(lane >= j, csub(x[0][j], cmul(l0, cj)), x[0][j]);
          if constexpr (NR == 2) x[1][j] = csub(x[1][j], cmul(l1, cj));
        }
      x[0][K] = csel(lane > K, l0, csel(lane == K, d, x[0][K]));
      if constexpr (NR == 2) x[1][K] = l1;
      if (lane == 0) dd[K] = d;
      wave_sync();
      LeafSteps<K + 1, PMAX, NR, C>::run(x, col, dd, p, lane, thr, anorm, npert, minr, nonfin);
    }
  }
};

// Fronts of the bottom levels (at most 64 NR rows and PMAX pivots), one
// wavefront per front (one to four per workgroup), each with its own slice of
// LDS; every child was factored by an earlier launch.
//   * Lane i holds rows i (and i + 64 when NR = 2) of the pivot columns in
//     registers: a pivot row's diagonal from its own stencil, and each row's
//     entries in the earlier pivot columns from the couplings those pivot
//     lanes leave in its four LDS slots (one per direction); then both
//     children's entries of the rows are added (loads through the gather
//     rows, staged in LDS).
//   * Right-looking LDL^T with the loops unrolled against PMAX: at step k
//     every lane publishes its a_ik to a 64-entry LDS buffer (the pivot rows
//     are all among the first 64), reads the column back as broadcasts, and
//     row i > k takes a_ij -= (a_ik / d_k) a_jk for the pivot columns
//     k < j <= i.
//   * The panel (D on the diagonal, unit-lower L below, as k_front_small
//     stores it) goes to the factor arena; the update block
//     U = F22 - L_u D L_u^T is formed entry by entry over its lower triangle,
//     enumerated column by column across the lanes (so the stores of a column
//     are contiguous): the children's entries of F22 plus the products from
//     the update rows of L, published to LDS (the only panel part kept there).
// The waves run independently (one wave's LDS operations complete in program
// order), where the one-workgroup kernel spends a workgroup and a barrier per
// pivot step on each front.  Pivots are checked and perturbed as in every
// other factor path.
template <typename R, int PMAX, int NR>
__device__ __forceinline__ void wave_front(const KArgs& a, int f, int s, int ldsw, unsigned char* smem_raw,
                                           PivotStats& ps) {
  typedef typename Cx<R>::T C;
  constexpr int GW = 64 * NR;  // gather-row width: rows lane (and lane + 64)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = a.npiv[f], u = a.nupd[f], m = p + u, pb = a.pbeg[f];
  // the wave's slice: the rows' couplings (4m values, then 4m pivot
  // columns) until the rows are loaded, after the elimination the update
  // rows of L (u x p) in the same bytes; then p pivots, a 64-entry column
  // buffer and two rows of GW gather indices
  unsigned char* base = smem_raw + (size_t)wave * ldsw;
  const int ub = (max(u * p * (int)sizeof(C), 4 * m * ((int)sizeof(C) + 4)) + 15) & ~15;
  C* Fu = reinterpret_cast<C*>(base);
  C* sv = reinterpret_cast<C*>(base);
  int* sc = reinterpret_cast<int*>(base + 4 * m * sizeof(C));
  C* dd = reinterpret_cast<C*>(base + ub);
  C* col = dd + p;
  int* gl = reinterpret_cast<int*>(col + 64);
  const int cb = a.child_ptr[f], nch = a.child_ptr[f + 1] - cb;
  const int32_t* g = a.gmap + a.gmap_ptr[f];
#pragma unroll
  for (int h = 0; h < NR; ++h) {
    const int r = lane + 64 * h;
#pragma unroll
    for (int k = 0; k < 2; ++k) gl[GW * k + r] = k < nch && r < m ? g[k * m + r] : -1;
    if (r < m) {
#pragma unroll
      for (int d = 0; d < 4; ++d) sc[4 * r + d] = -1;
    }
  }
  wave_sync();
  C x[NR][PMAX];
#pragma unroll
  for (int h = 0; h < NR; ++h)
#pragma unroll
    for (int c = 0; c < PMAX; ++c) x[h][c] = czero<C>();
  if (lane < p) {
    // pivot lane c: its diagonal, and its couplings to the later rows r > c
    // go to row r's slots, one per direction (a row has one neighbour per
    // direction, so no two pivots share a slot)
    const int q = pb + lane;
    const Stencil S = stencil_at(a, s, a.perm[q]);
    const C dg = from_d2<C>(S.diag);
#pragma unroll
    for (int c = 0; c < PMAX; ++c) x[0][c] = csel(c == lane, dg, x[0][c]);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int r = a.nbr_row[4 * (int64_t)q + d];
      if (r > lane) {
        sv[4 * r + d] = from_d2<C>(S.c[d]);
        sc[4 * r + d] = lane;
      }
    }
  }
  wave_sync();
#pragma unroll
  for (int h = 0; h < NR; ++h) {
    const int r = lane + 64 * h;
    if (r < m) {
      // row r's entries in the pivot columns before it
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const int c = sc[4 * r + d];
        const C v = sv[4 * r + d];
#pragma unroll
        for (int k = 0; k < PMAX; ++k) x[h][k] = csel(k == c, v, x[h][k]);
      }
    }
  }
  // the children's entries of row lane in the pivot columns (both children's loads in flight together)
  const C* Ub = (const C*)a.upd + (int64_t)s * a.upd_total;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (k < nch) {
      const int chf = a.child_list[cb + k];
      const int uk = a.nupd[chf];
      const C* Uk = Ub + a.upd_off[chf];
      int gi[NR];
#pragma unroll
      for (int h = 0; h < NR; ++h) gi[h] = gl[GW * k + lane + 64 * h];
      // eight columns' loads per row in flight at a time (all PMAX at once
      // would hold the kernel to fewer waves per SIMD)
#pragma unroll
      for (int c0 = 0; c0 < PMAX; c0 += 8) {
        if (c0 < p) {
          C w[NR][8];
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int c = c0 + t;
            const int gc = gl[GW * k + min(c, 63)];
#pragma unroll
            for (int h = 0; h < NR; ++h) {
              const int r = lane + 64 * h;
              const bool ok = c < p && gi[h] >= 0 && gc >= 0 && r >= c && r < m;
              w[h][t] = ok ? Uk[(int64_t)gc * uk + gi[h]] : czero<C>();
            }
          }
#pragma unroll
          for (int h = 0; h < NR; ++h)
#pragma unroll
            for (int t = 0; t < 8; ++t)
              if (c0 + t < PMAX) x[h][c0 + t] = cadd(x[h][c0 + t], w[h][t]);
        }
      }
    }
  }
  const double anorm = anorm_of(a, s);
  const double thr = a.tau * anorm;
  int npert = 0, nonfin = 0;
  double minr = INFINITY;
  LeafSteps<0, PMAX, NR, C>::run(x, col, dd, p, lane, thr, anorm, npert, minr, nonfin);
  // the panel to the factor arena (row lane: D on the diagonal, L below)
  C* L = (C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
#pragma unroll
  for (int h = 0; h < NR; ++h) {
    const int r = lane + 64 * h;
#pragma unroll
    for (int c = 0; c < PMAX; ++c)
      if (c < p && r < m && r >= c) L[(int64_t)c * m + r] = x[h][c];
  }
  if (u > 0) {
    // the update rows of L back into LDS: the products read them (and d)
    // as broadcasts
#pragma unroll
    for (int h = 0; h < NR; ++h) {
      const int r = lane + 64 * h;
#pragma unroll
      for (int c = 0; c < PMAX; ++c)
        if (c < p && r >= p && r < m) Fu[c * u + r - p] = x[h][c];
    }
    wave_sync();
    C* U = (C*)a.upd + (int64_t)s * a.upd_total + a.upd_off[f];
    const int ntri = u * (u + 1) / 2;
    const C* Uk[2];
    int uk[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int chf = k < nch ? a.child_list[cb + k] : f;
      Uk[k] = Ub + a.upd_off[chf];
      uk[k] = a.nupd[chf];
    }
    // entry e of the lower triangle, column by column: column cc, row rr >= cc
    auto entry = [&](int e, int& cc, int& rr) {
      cc = 0;
      int off = 0;
      if (e < ntri) {
        // off(c) = c u - c (c - 1) / 2 is the first entry of column c
        cc = (int)((2.0 * u + 1.0 - sqrt((2.0 * u + 1.0) * (2.0 * u + 1.0) - 8.0 * e)) * 0.5);
        cc = max(0, min(cc, u - 1));
        while (cc > 0 && cc * u - cc * (cc - 1) / 2 > e) --cc;
        while (cc + 1 < u && (cc + 1) * u - (cc + 1) * cc / 2 <= e) ++cc;
        off = cc * u - cc * (cc - 1) / 2;
      }
      rr = cc + (e - off);
    };
    // the children's entries of F22 at (p + rr, p + cc): the loads are
    // unconditional (entry 0 where the row or column is not the child's; a
    // missing child's gather rows are -1 and its pointer is this front's own
    // block) and their values are selected and added only when used, so the
    // loads stay in flight across the products formed before
    auto kids_load = [&](int cc, int rr, bool ok, C (&val)[2], bool (&hit)[2]) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int gr = ok ? gl[GW * k + p + rr] : -1;
        const int gc = ok ? gl[GW * k + p + cc] : -1;
        hit[k] = gr >= 0 && gc >= 0;
        val[k] = Uk[k][hit[k] ? (int64_t)gc * uk[k] + gr : 0];
      }
    };
    auto kids_sum = [&](const C (&val)[2], const bool (&hit)[2]) {
      C v = czero<C>();
#pragma unroll
      for (int k = 0; k < 2; ++k) v = cadd(v, csel(hit[k], val[k], czero<C>()));
      return v;
    };
    // the loop once with the children's loads and once without (a leaf):
    // a uniform branch around the loads inside it would make every use
    // wait for all loads in flight
    auto rounds = [&](auto kids) {
      constexpr bool KIDS = decltype(kids)::value;
      // QD rounds of 64 entries per batch; the next batch's loads are in flight
      // while this batch's products are formed
      constexpr int QD = NR == 2 ? 3 : PMAX <= 8 ? 1 : 2;
      int cq[QD], rq[QD];
      C kv[QD][2];
      bool kh[QD][2];
#pragma unroll
      for (int q = 0; q < QD; ++q) {
        entry(64 * q + lane, cq[q], rq[q]);
        if constexpr (KIDS) kids_load(cq[q], rq[q], 64 * q + lane < ntri, kv[q], kh[q]);
      }
      for (int e0 = 0; e0 < ntri; e0 += 64 * QD) {
        int cn[QD], rn[QD];
        C kvn[QD][2];
        bool khn[QD][2];
#pragma unroll
        for (int q = 0; q < QD; ++q) {
          const int e = e0 + 64 * (QD + q) + lane;
          entry(e, cn[q], rn[q]);
          if constexpr (KIDS) kids_load(cn[q], rn[q], e < ntri, kvn[q], khn[q]);
        }
#pragma unroll
        for (int q = 0; q < QD; ++q) {
          const bool ok = e0 + 64 * q + lane < ntri;
          C v = czero<C>();
          if constexpr (KIDS) v = kids_sum(kv[q], kh[q]);
          // indices in range for every lane, so the sum needs no per-lane
          // branch (a branch per term would keep its LDS reads from overlapping)
          const int ra = ok ? rq[q] : 0, ca = ok ? cq[q] : 0;
          C acc = czero<C>();
#pragma unroll 4
          for (int k = 0; k < p; ++k) acc = cadd(acc, cmul(Fu[k * u + ra], cmul(Fu[k * u + ca], dd[k])));
          if (ok) U[(int64_t)cq[q] * u + rq[q]] = csub(v, acc);
        }
#pragma unroll
        for (int q = 0; q < QD; ++q) {
          cq[q] = cn[q];
          rq[q] = rn[q];
          if constexpr (KIDS) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
              kv[q][k] = kvn[q][k];
              kh[q][k] = khn[q][k];
            }
          }
        }
      }
    };
    if (nch > 0) rounds(std::true_type{});
    else rounds(std::false_type{});
  }
  ps.add(npert, minr, nonfin, anorm);
}

// Waves per SIMD the register budget must allow: three for up to 24 pivots
// and one row per lane (the bottom level's fronts), two otherwise.  A
// workgroup holds one to four waves (blockDim), each with its own front.
template <typename R, int PMAX, int NR>
__global__ __launch_bounds__(kThreads, PMAX <= 24 && NR == 1 ? 3 : 2) void k_wave_fronts(KArgs a,
                                                                                        const int32_t* order,
                                                                                        int nitems, int ldsw) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int item = blockIdx.x * (int)(blockDim.x >> 6) + wave;
  if (item >= nitems) return;  // the whole wave: nothing below synchronises the workgroup
  extern __shared__ __align__(16) unsigned char smem_raw[];
  PivotStats ps;
  wave_front<R, PMAX, NR>(a, order[item / a.nsys], item % a.nsys, ldsw, smem_raw, ps);
  if (lane == 0) ps.flush(a.st);
}

// Persistent launch over fronts order[0 .. ntasks/nsys): with q.wait set, a
// front first waits for its children (claimed earlier in the same launch).
// Registers for two workgroups per CU in complex128, three in complex64
// (complex128 at three spills heavily and runs slower).
template <typename R>
__global__ __launch_bounds__(kThreads, sizeof(R) == 8 ? 2 : 3) void k_front_small(KArgs a, Queue q,
                                                                                 const int32_t* order) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int sh;
  const int ep = launch_epoch(q);
  PivotStats ps;
  for (;;) {
    const int t = claim(q, &sh);
    if (t >= q.ntasks) break;
    const int f = order[t / a.nsys], s = t % a.nsys;
    // independent of the wait below: the stencils, gather rows and children
    small_front_stage<R>(a, s, f, smem_raw);
    const Kids<typename Cx<R>::T> kids = kids_of<typename Cx<R>::T>(a, s, f);
    if (q.wait) wait_children(q, ep, a, s, f);
    else __syncthreads();
    trace_mark(q, t, 1);
    small_front<R>(a, q, ep, s, f, kids, smem_raw, ps);
    trace_mark(q, t, 2);
  }
  if (threadIdx.x == 0) ps.flush(a.st);
  leave(q, ep);
}

// ---------------------------------------------------------------------------
// Large fronts: one persistent launch runs a task graph over 64 x 64 tiles.
// The rows (and columns) of a front are cut into chunks: pivot blocks of kBW
// from row 0 up to p, then update chunks of kBW from row p up to m.  Tasks:
//   ASM(I,J)     assemble tile (I,J): original entries + children's blocks
//   DIAG(k)      LDL^T of pivot block k, inverse of its unit-lower part
//   TRSM(k,I)    tile (I,k) <- F_Ik Xinv_k^T D_k^-1
//   UPD(I,J,[k0,k1))  tile (I,J) -= sum_k L_Ik D_k L_Jk^T  (k0 <= k < k1 <= J, J < nbk)
//   SYRK(I,J,[k0,k1)) the same for the Schur-complement tiles (I >= J >= nbk)
// Each tile carries a version (1 after ASM, +1 per modification); a task
// waits for the exact versions it reads and writes, and publishes the next.
// A front's update tiles count their final versions in done[], which the
// parent's ASM tasks wait for.  Tasks are listed in topological order
// (level, then block step), so every wait ends (see the queue notes above).
// ---------------------------------------------------------------------------
struct TileArgs {
  const int32_t* tasks;      // 5 ints per task: type, front, k, I, J
  int32_t* state;            // [nsys][ntiles] tile versions
  int32_t* done;             // [nsys][nfronts] final update tiles per front
  const int32_t* tile_base;  // [nfronts] first packed tile of a front
  const int32_t* is_tiled;   // [nfronts] 1 if the front is factored by this launch
  int32_t ntiles;
};

enum { T_ASM = 0, T_DIAG = 1, T_TRSM = 2, T_UPD = 3, T_INV = 4, T_FUSED = 5, T_SYRK = 6 };

struct Chunks {
  int p, u, m, nbk, nut;
  __device__ Chunks(int p_, int u_) : p(p_), u(u_), m(p_ + u_), nbk((p_ + kBW - 1) / kBW), nut((u_ + kBW - 1) / kBW) {}
  __device__ int lo(int I) const { return I < nbk ? I * kBW : p + (I - nbk) * kBW; }
  __device__ int hi(int I) const { return I < nbk ? min(p, (I + 1) * kBW) : min(m, p + (I - nbk + 1) * kBW); }
};

__device__ __forceinline__ int tile_id(int I, int J) { return I * (I + 1) / 2 + J; }

__device__ __forceinline__ void wait_value(const int32_t* p, int v, DevStatus* st) {
  int it = 0;
  while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != v) {
    if (++it > kSpinLimit) {
      atomicExch(&st->spin_timeout, 1);
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

__device__ __forceinline__ void wait_at_least(const int32_t* p, int v, DevStatus* st) {
  int it = 0;
  while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) {
    if (++it > kSpinLimit) {
      atomicExch(&st->spin_timeout, 1);
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Address of entry (r, c) of front f: the factor panel for pivot columns, the
// update block otherwise.
template <typename C>
__device__ __forceinline__ C* front_elem(const KArgs& a, int s, int f, int p, int u, int m, int r, int c) {
  if (c < p) return (C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f] + (int64_t)c * m + r;
  return (C*)a.upd + (int64_t)s * a.upd_total + a.upd_off[f] + (int64_t)(c - p) * u + (r - p);
}

// Tile (rows [r0, r0 + nr), columns [c0, c0 + nc)) of front f in memory, as
// one buffer: the panel's pivot columns or the update block (a tile lies
// wholly in one of them), columns >= nc outside it.  Entry (r0 + lane,
// c0 + wave + 4t) is at byte offset rowoff + t * colstride; rowoff is kOob
// for lanes >= nr, so their loads read zero and their stores are dropped.
struct TileMem {
  __amdgpu_buffer_rsrc_t rs;
  unsigned colstride, rowoff;
};

template <typename C>
__device__ __forceinline__ TileMem tile_mem(const KArgs& a, int s, int f, const Chunks& ch, int r0, int nr, int c0,
                                            int nc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool piv = c0 < ch.p;
  const C* base = piv ? (const C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f] + (int64_t)c0 * ch.m
                      : (const C*)a.upd + (int64_t)s * a.upd_total + a.upd_off[f] + (int64_t)(c0 - ch.p) * ch.u;
  const unsigned ld = piv ? ch.m : ch.u;
  const int row = piv ? r0 + lane : r0 - ch.p + lane;
  TileMem t;
  t.rs = buffer_of(base, (unsigned)nc * ld * (unsigned)sizeof(C));
  t.colstride = 4u * ld * (unsigned)sizeof(C);
  t.rowoff = lane < nr ? ((unsigned)wave * ld + (unsigned)row) * (unsigned)sizeof(C) : kOob;
  return t;
}

// The children's gather rows for tile (rows r0.., columns c0..) of front f,
// into LDS (the maps are static, so this may run before the task's waits):
// kid[128 k + e], e < 64, is child k's update-block row of tile row r0 + e,
// and kid[128 k + 64 + e] that of tile column c0 + e (-1: none).  A front has
// at most two children (each dissection step halves a rectangle), so the 256
// threads cover them in one pass.
__device__ __forceinline__ void stage_kid_rows(const KArgs& a, int f, int m, int r0, int nr, int c0, int nc, int* kid) {
  static_assert(kThreads == 256, "two children x 128 gather rows per thread block");
  const int nch = a.child_ptr[f + 1] - a.child_ptr[f];
  const int k = threadIdx.x >> 7, e = threadIdx.x & 127;
  if (k < nch) {
    const int32_t* g = a.gmap + a.gmap_ptr[f] + (int64_t)k * m;
    kid[threadIdx.x] = e < 64 ? (e < nr ? g[r0 + e] : -1) : (e - 64 < nc ? g[c0 + e - 64] : -1);
  }
}

// v[t] += the children's update-block entries that land on the lower-
// triangle entry (r0 + lane, c0 + wave + 4t) of the tile, child 0 then child
// 1, from the rows stage_kid_rows put in kid: both children's sixteen loads
// per thread are in flight together.
template <typename C>
__device__ __forceinline__ void add_kids_tile(const KArgs& a, int s, int f, const int* kid, int r0, int c0,
                                              C (&v)[16]) {
  const int cb = a.child_ptr[f], nch = a.child_ptr[f + 1] - cb;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = r0 + lane;
  const C* Ub = (const C*)a.upd + (int64_t)s * a.upd_total;
  C w[2][16];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (k < nch) {
      const int chf = a.child_list[cb + k];
      const unsigned nu = a.nupd[chf];
      const __amdgpu_buffer_rsrc_t rs = buffer_of(Ub + a.upd_off[chf], nu * nu * (unsigned)sizeof(C));
      const int gr = kid[128 * k + lane];
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int c = wave + 4 * t;
        const int gc = kid[128 * k + 64 + c];
        const bool ok = gr >= 0 && gc >= 0 && r >= c0 + c;
        w[k][t] = ld_buf<C>(rs, ok ? ((unsigned)gc * nu + (unsigned)gr) * (unsigned)sizeof(C) : kOob);
      }
    } else {
#pragma unroll
      for (int t = 0; t < 16; ++t) w[k][t] = czero<C>();
    }
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) v[t] = cadd(cadd(v[t], w[0][t]), w[1][t]);
}

// LDS of ASM(I,J): the staged stencils (5 kBW entries), their neighbour rows
// (4 kBW ints), then the children's gather rows (256 ints).
template <typename C> __device__ __forceinline__ int* asm_kid_rows(unsigned char* smem) {
  return reinterpret_cast<int*>(smem + 5 * kBW * sizeof(C) + 4 * kBW * sizeof(int));
}

// The first part of ASM(I,J) on a pivot column chunk: the original operator
// entries of its columns (stage_columns), which depend on no other task, so
// the kernel runs it before the task's dependency wait.  A barrier follows in
// the caller before task_asm reads them.
template <typename R>
__device__ __forceinline__ void asm_stage(const KArgs& a, int s, int f, int I, int J, unsigned char* smem) {
  typedef typename Cx<R>::T C;
  const Chunks ch(a.npiv[f], a.nupd[f]);
  const int c0 = ch.lo(J), nc = ch.hi(J) - c0;
  if (c0 < ch.p) {
    C* sv = reinterpret_cast<C*>(smem);
    stage_columns(a, s, f, c0, nc, sv, reinterpret_cast<int*>(sv + 5 * kBW));
  }
  const int r0 = ch.lo(I);
  stage_kid_rows(a, f, ch.m, r0, ch.hi(I) - r0, c0, nc, asm_kid_rows<C>(smem));
}

// ASM(I,J): the tile's original entries (pivot columns only, from the
// stencils asm_stage placed in LDS) plus the children's update-block entries
// that land on it, from the gather rows asm_stage also staged before the
// task's wait: after the wait one round of value loads (both children's at
// once) and one of stores.  Lane = row, wave w takes the columns w, w+4, ...
template <typename R>
__device__ __forceinline__ void task_asm(const KArgs& a, int s, int f, int I, int J, unsigned char* smem) {
  typedef typename Cx<R>::T C;
  const Chunks ch(a.npiv[f], a.nupd[f]);
  const int r0 = ch.lo(I), r1 = ch.hi(I), c0 = ch.lo(J), c1 = ch.hi(J);
  const int nr = r1 - r0, nc = c1 - c0;
  const bool piv = c0 < ch.p;  // pivot chunks hold original entries
  C* sv = reinterpret_cast<C*>(smem);  // the pivot columns' stencils, staged by asm_stage
  int* nbv = reinterpret_cast<int*>(sv + 5 * kBW);
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = r0 + lane;
  C v[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int tt = wave + 4 * t, c = c0 + tt;
    const bool ok = lane < nr && tt < nc && r >= c;
    v[t] = (ok && piv) ? staged_entry(sv, nbv, tt, r, c) : czero<C>();
  }
  add_kids_tile<C>(a, s, f, asm_kid_rows<C>(smem), r0, c0, v);
  // pivot columns are written whole (zeros above the diagonal), update
  // blocks in their lower triangle
  const TileMem tm = tile_mem<C>(a, s, f, ch, r0, nr, c0, nc);
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const bool ok = piv || r >= c0 + wave + 4 * t;
    st_buf<C>(tm.rs, ok ? tm.rowoff + t * tm.colstride : kOob, v[t]);
  }
}

// DIAG(k): LDL^T of the nb x nb pivot block, blocked by 16, and the inverses
// of its 16 x 16 diagonal sub-blocks in place of theirs (what the TRSM tasks
// of step k use).  When no TRSM follows (last pivot block of a front without
// update rows) the off-diagonal sub-blocks are inverted here too (kDiagFull);
// otherwise INV(k) (kInvOnly) turns them into those of L_kk^-1 once every TRSM
// of step k has read them.  The forward and backward sweeps apply the whole
// inverse.  One routine for both task types keeps a single inlined copy.
enum { kDiagPart = 0, kDiagFull = 1, kInvOnly = 2 };

// The LDS part of DIAG on a staged kBW x kBW block B (lower triangle): LDL^T,
// 16 x 16 diagonal inverses, and for kDiagFull also the off-diagonal inverse
// blocks; d in dd, 1/d in invd, T a 16 x 64 scratch.  kInvOnly: B holds the
// factor of an earlier DIAG and only the off-diagonal inverse blocks are formed.
template <typename R, typename C>
__device__ __forceinline__ void diag_core(const KArgs& a, int s, C* B, C* dd, C* invd, C* T, int nb, int mode) {
  double anorm = 0.0;
  int npert = 0, nonfin = 0;
  double minr = INFINITY;
  if (mode != kInvOnly) {
    anorm = anorm_of(a, s);
    ldl_blocked<true>(B, kBW, kBW, nb, dd, invd, T, a.tau * anorm, anorm, npert, minr, nonfin);
    invert_diag16(B, kBW, nb);
  }
  if (mode != kDiagPart) invert_offdiag(B, kBW, nb, T);
  if (mode != kInvOnly && threadIdx.x == 0) record_pivots(a.st, npert, minr, nonfin, anorm);
}

// Writes the factored kBW x kBW pivot block from LDS to the panel (inverse
// blocks below the diagonal, d on it); kInvOnly writes only the off-diagonal
// 16 x 16 inverse blocks.
template <typename C>
__device__ __forceinline__ void diag_store(C* L, int m, const C* B, const C* dd, int nb, bool inv_only) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (inv_only) {
    for (int c = wave; c < nb; c += 4)
      if (lane < nb && (lane >> 4) > (c >> 4)) st_ag(L + (int64_t)c * m + lane, B[c * kBW + lane]);
  } else {
    for (int c = wave; c < nb; c += 4)
      for (int r = c + lane; r < nb; r += 64) st_ag(L + (int64_t)c * m + r, (r > c) ? B[c * kBW + r] : dd[c]);
  }
}

template <typename R>
__device__ __forceinline__ void task_diag(const KArgs& a, int s, int f, int k, int mode, unsigned char* smem) {
  typedef typename Cx<R>::T C;
  C* B = reinterpret_cast<C*>(smem);  // kBW x kBW, column major
  C* dd = B + kBW * kBW;
  C* invd = dd + kBW;
  C* T = invd + kBW;  // 16 x 64 scratch
  const int p = a.npiv[f], m = p + a.nupd[f];
  const int k0 = k * kBW, nb = min(kBW, p - k0);
  C* L = (C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f] + (int64_t)k0 * m + k0;
  stage_block(B, L, m, nb, nb, mode == kInvOnly ? kStrict : kLower);
  __syncthreads();
  diag_core<R>(a, s, B, dd, invd, T, nb, mode);
  diag_store(L, m, B, dd, nb, mode == kInvOnly);
}

// TRSM in LDS: X <- F L_kk^-T (without D^-1) for a staged kBW x kBW tile Xs
// (in place) and pivot block Ls, by block forward substitution over the
// 16-column blocks J of the pivot block, with w_JJ = L_JJ^-1 in the diagonal
// sub-blocks:  V_J = F_J - sum_{K<J} X_K L_JK^T,  X_J = V_J w_JJ^T.  Thread t
// owns rows t%32 and t%32 + 32 and columns 2 (t/32) + {0,1} of a block.
// Vs: kBW x 16 scratch.  Ends with a barrier.
template <typename C>
__device__ __forceinline__ void trsm_core(C* Xs, const C* Ls, C* Vs, int nb) {
  const int ra = threadIdx.x & 31, cb = 2 * (threadIdx.x >> 5);
  const int nsb = (nb + 15) / 16;
  for (int J = 0; J < nsb; ++J) {
    const int j0 = 16 * J;
    C v[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) v[x][y] = Xs[(j0 + cb + y) * kBW + ra + 32 * x];
    // four steps' LDS reads in flight before their products (j0 % 16 == 0)
    for (int q0 = 0; q0 < j0; q0 += 4) {
      C x0[4], x1[4], l0[4], l1[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int q = q0 + e;
        x0[e] = Xs[q * kBW + ra];
        x1[e] = Xs[q * kBW + ra + 32];
        l0[e] = Ls[q * kBW + j0 + cb];
        l1[e] = Ls[q * kBW + j0 + cb + 1];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[0][0] = cfms(v[0][0], x0[e], l0[e]);
        v[0][1] = cfms(v[0][1], x0[e], l1[e]);
        v[1][0] = cfms(v[1][0], x1[e], l0[e]);
        v[1][1] = cfms(v[1][1], x1[e], l1[e]);
      }
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) Vs[(cb + y) * kBW + ra + 32 * x] = v[x][y];
    __syncthreads();
    C o[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) o[x][y] = czero<C>();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const C v0 = Vs[q * kBW + ra], v1 = Vs[q * kBW + ra + 32];
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const int c = cb + y;
        const C st = Ls[(j0 + q) * kBW + j0 + c];
        C w;  // w_JJ[c][q]: unit diagonal, zero above
        w.x = q < c ? st.x : (q == c ? 1 : 0);
        w.y = q < c ? st.y : 0;
        o[0][y] = cadd(o[0][y], cmul(v0, w));
        o[1][y] = cadd(o[1][y], cmul(v1, w));
      }
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) Xs[(j0 + cb + y) * kBW + ra + 32 * x] = o[x][y];
    __syncthreads();
  }
}

// TRSM(I,k): tile (I,k) <- F_Ik L_kk^-T D_k^-1.
template <typename R>
__device__ __forceinline__ void task_trsm(const KArgs& a, int s, int f, int k, int I, unsigned char* smem) {
  typedef typename Cx<R>::T C;
  C* Xs = reinterpret_cast<C*>(smem);  // kBW x kBW column major: F_Ik, then X in place
  C* Ls = Xs + kBW * kBW;              // kBW x kBW: the pivot block (L_JK, w_JJ, D)
  C* Vs = Ls + kBW * kBW;              // kBW x 16
  const Chunks ch(a.npiv[f], a.nupd[f]);
  const int m = ch.m, k0 = k * kBW, nb = min(kBW, ch.p - k0);
  const int r0 = ch.lo(I), nr = ch.hi(I) - r0;
  C* L = (C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // zero padding beyond nr rows / nb columns keeps the products finite
  stage_block(Xs, L + (int64_t)k0 * m + r0, m, nr, nb, kAll);
  stage_block(Ls, L + (int64_t)k0 * m + k0, m, nb, nb, kLower);
  __syncthreads();
  trsm_core(Xs, Ls, Vs, nb);
  for (int c = wave; c < nb; c += 4)
    if (lane < nr) st_ag(L + (int64_t)(k0 + c) * m + r0 + lane, cmul(Xs[c * kBW + lane], cinv(Ls[c * kBW + c])));
}

// Matrix-core (MFMA) product of two LDS-resident complex 64 x 64 operands:
// O[c][r] = sum_q A[q][r] B[q][c] (all column major with leading dimension
// kBW, zero padded).  Wave w owns output rows 16w..16w+15 as four 16 x 16
// blocks; per block and 4-deep k-step the complex product is four real
// 16x16x4 MFMAs (re += ar br - ai bi, im += ar bi + ai br), with B's column
// block in the instruction's A slot so that the result is the block's
// transpose (output row = l%16, output column per register from Mfma::row,
// conflict-free column-major stores).  O may alias A or B: the
// products finish (barrier) before O is written, and a barrier follows.
template <typename R, typename C>
__device__ __forceinline__ void mfma_tile_abt(const C* A, const C* B, C* O) {
  typedef typename Mfma<R>::v4 v4;
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = l & 15, kq = l >> 4;
  v4 re[4], im[4];
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) {
    re[bj] = v4{0, 0, 0, 0};
    im[bj] = v4{0, 0, 0, 0};
  }
#pragma unroll 4
  for (int k0 = 0; k0 < kBW; k0 += 4) {
    const int q = k0 + kq;
    const C av = A[q * kBW + 16 * wave + i];
    const R nai = -av.y;
    C bv[4];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) bv[bj] = B[q * kBW + 16 * bj + i];
    // eight independent accumulators per pass, so no MFMA waits on the previous one
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      re[bj] = Mfma<R>::op(bv[bj].x, av.x, re[bj]);
      im[bj] = Mfma<R>::op(bv[bj].y, av.x, im[bj]);
    }
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      re[bj] = Mfma<R>::op(bv[bj].y, nai, re[bj]);
      im[bj] = Mfma<R>::op(bv[bj].x, av.y, im[bj]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int bj = 0; bj < 4; ++bj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      C v;
      v.x = re[bj][r];
      v.y = im[bj][r];
      O[(16 * bj + Mfma<R>::row(l, r)) * kBW + 16 * wave + i] = v;
    }
  __syncthreads();
}

// Lower block triangle of the same product (the 10 of 16 output blocks with
// bj <= bi; what a diagonal tile's update needs), shared out over the waves
// three, three, two and two blocks at a time.  O may alias A or B.
template <typename R, typename C>
__device__ __forceinline__ void mfma_tile_abt_lower(const C* A, const C* B, C* O) {
  typedef typename Mfma<R>::v4 v4;
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = l & 15, kq = l >> 4;
  // (bi, bj) per wave: {(3,0),(3,1),(0,0)}, {(3,2),(3,3),(1,0)}, {(2,0),(2,1)}, {(2,2),(1,1)}
  const int nblk = wave < 2 ? 3 : 2;
  int bi[3], bj[3];
  bi[0] = wave < 2 ? 3 : 2;
  bj[0] = wave == 0 ? 0 : wave == 1 ? 2 : wave == 2 ? 0 : 2;
  bi[1] = wave < 2 ? 3 : wave == 2 ? 2 : 1;
  bj[1] = wave == 0 ? 1 : wave == 1 ? 3 : 1;
  bi[2] = wave == 0 ? 0 : 1;
  bj[2] = 0;
  v4 re[3], im[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    re[t] = v4{0, 0, 0, 0};
    im[t] = v4{0, 0, 0, 0};
  }
#pragma unroll 4
  for (int k0 = 0; k0 < kBW; k0 += 4) {
    const int q = k0 + kq;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      if (t < nblk) {  // uniform per wave
        const C av = A[q * kBW + 16 * bi[t] + i];
        const C bv = B[q * kBW + 16 * bj[t] + i];
        re[t] = Mfma<R>::op(bv.x, av.x, re[t]);
        im[t] = Mfma<R>::op(bv.y, av.x, im[t]);
        re[t] = Mfma<R>::op(bv.y, -av.y, re[t]);
        im[t] = Mfma<R>::op(bv.x, av.y, im[t]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < 3; ++t)
    if (t < nblk) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        C v;
        v.x = re[t][r];
        v.y = im[t][r];
        O[(16 * bj[t] + Mfma<R>::row(l, r)) * kBW + 16 * bi[t] + i] = v;
      }
    }
  __syncthreads();
}


// Tile update over a group of pivot blocks:
//   T_IJ -= sum_{k0 <= k < k1} L_Ik D_k L_Jk^T,
// accumulated on the matrix cores over the whole group before the tile is
// touched.  Each wave's A operand (its 16 output rows) is private to it and
// goes from memory straight into registers in the matrix-core layout, one
// block ahead; B (shared by the four waves) is scaled by the pivots as it is
// written to one of two LDS buffers, in the middle of the previous block's
// products, so a block costs one barrier and no idle matrix core between
// blocks.  The tile is then read and written once.  Used by
//   SYRK(I,J,[k0,k1))  tiles of the front's Schur complement (I >= J >= nbk);
//                      the first group gathers the children's update-block
//                      entries instead of reading the tile (its assembly);
//   UPD(I,J,[k0,k1))   tiles of the pivot columns (J < nbk), assembled by ASM:
//                      one block at a time for the rows of pivot blocks (the
//                      chain of the front waits for them), a group at a time
//                      for the update rows.
// The one-block-per-task form instead reads and writes the tile, and pays a
// task's claim, waits and store drain, once per pivot block.
// Operands of one pivot block of a tile update, loaded from memory ahead of
// their use: A (this wave's 16 output rows) straight into registers in the
// matrix-core layout, af[s] = L[r0 + 16 wave + l % 16][kb + 4 s + l / 16]; B
// (the 64 output columns, lane = row, wave w the columns w, w + 4, ...) and,
// in lanes 0..15, the pivots d of those sixteen columns.  The block's kn
// columns form one buffer, so columns beyond kn read zero.
template <typename C>
__device__ __forceinline__ void tile_block_load(const C* L, int m, int kb, int kn, int r0, int nr, int c0, int nc,
                                                C (&af)[16], C (&vb)[16], C& dq) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const __amdgpu_buffer_rsrc_t rs = buffer_of(L + (int64_t)kb * m, (unsigned)(kn * m) * (unsigned)sizeof(C));
  const unsigned cs = sizeof(C), step = 4u * (unsigned)m * cs;
  unsigned oa = 16 * wave + i < nr ? ((unsigned)(kq * m + r0 + 16 * wave + i)) * cs : kOob;
  unsigned ob = lane < nc ? ((unsigned)(wave * m + c0 + lane)) * cs : kOob;
  asm volatile("" : "+v"(oa), "+v"(ob));  // formed load by load, not hoisted into the caller's loop
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    af[t] = ld_buf<C>(rs, oa + t * step);
    vb[t] = ld_buf<C>(rs, ob + t * step);
  }
  dq = ld_buf<C>(rs, lane < 16 ? ((unsigned)((wave + 4 * lane) * (m + 1) + kb)) * cs : kOob);
}

// B of the next block into its LDS buffer, each column scaled by its pivot:
// Bs[q][c] = d_q L[c0 + c][kb + q].
template <typename C>
__device__ __forceinline__ void tile_block_stage(const C (&vb)[16], C dq, C* Bs) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < 16; ++t) Bs[(wave + 4 * t) * kBW + lane] = cmul(vb[t], bcast_c(dq, t));
}

// Steps [S0, S1) of one block's products on the matrix cores:
// O[c][r] += sum_q A[q][r] Bs[q][c] with A from registers (af) and Bs from LDS
// (the next step's LDS reads issued before this step's products); wave w
// owns output rows 16w..16w+15 as four 16 x 16 blocks (the layout of
// mfma_tile_abt).
template <int S0, int S1, typename R, typename C>
__device__ __forceinline__ void tile_block_mfma(const C (&af)[16], const C* Bs, typename Mfma<R>::v4 (&re)[4],
                                                typename Mfma<R>::v4 (&im)[4]) {
  const int l = threadIdx.x & 63, i = l & 15, kq = l >> 4;
  C bn[4];
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) bn[bj] = Bs[(4 * S0 + kq) * kBW + 16 * bj + i];
#pragma unroll
  for (int st = S0; st < S1; ++st) {
    C bv[4];
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) bv[bj] = bn[bj];
    if (st + 1 < S1) {
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) bn[bj] = Bs[(4 * (st + 1) + kq) * kBW + 16 * bj + i];
    }
    const C av = af[st];
    const R nai = -av.y;
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      re[bj] = Mfma<R>::op(bv[bj].x, av.x, re[bj]);
      im[bj] = Mfma<R>::op(bv[bj].y, av.x, im[bj]);
    }
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      re[bj] = Mfma<R>::op(bv[bj].y, nai, re[bj]);
      im[bj] = Mfma<R>::op(bv[bj].x, av.y, im[bj]);
    }
  }
}

// One block of the pipelined update: products of block k (registers afc,
// LDS Bc) in two halves; between them the next block's B goes into the other
// buffer Bn (its loads, issued before the first half, have arrived); the
// next block's operands are loaded into afn, vb, dq first.  One barrier per
// block: after it every wave is done with Bc and Bn is complete.
template <typename R, typename C>
__device__ __forceinline__ void tile_block_step(const C* L, int m, int p, int k, int k1, int r0, int nr, int c0,
                                                int nc, C (&afc)[16], C (&afn)[16], C (&vb)[16], C& dq, const C* Bc,
                                                C* Bn, typename Mfma<R>::v4 (&re)[4], typename Mfma<R>::v4 (&im)[4]) {
  const bool next = k + 1 < k1;
  if (next) tile_block_load(L, m, (k + 1) * kBW, min(kBW, p - (k + 1) * kBW), r0, nr, c0, nc, afn, vb, dq);
  tile_block_mfma<0, 8, R>(afc, Bc, re, im);
  if (next) tile_block_stage(vb, dq, Bn);
  tile_block_mfma<8, 16, R>(afc, Bc, re, im);
  __syncthreads();
}

template <typename R>
__device__ __forceinline__ void task_tile_update(const KArgs& a, int s, int f, int k0, int k1, int I, int J,
                                                 unsigned char* smem) {
  typedef typename Cx<R>::T C;
  typedef typename Mfma<R>::v4 v4;
  C* B0 = reinterpret_cast<C*>(smem);  // two B buffers; at the end the products O[c][r] in B0
  C* B1 = B0 + kBW * kBW;
  C* As = B0;
  const Chunks ch(a.npiv[f], a.nupd[f]);
  const int m = ch.m, p = ch.p, u = ch.u;
  const int r0 = ch.lo(I), nr = ch.hi(I) - r0, c0 = ch.lo(J), nc = ch.hi(J) - c0;
  const C* L = (const C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v4 re[4], im[4];
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) {
    re[bj] = v4{0, 0, 0, 0};
    im[bj] = v4{0, 0, 0, 0};
  }
  // the first group of a Schur tile assembles it from the children: their
  // gather rows go to LDS now (the loop's barriers order them before use)
  const bool first = k0 == 0 && J >= ch.nbk;
  int* kid = reinterpret_cast<int*>(B1 + kBW * kBW);
  if (first) stage_kid_rows(a, f, m, r0, nr, c0, nc, kid);
  C af0[16], af1[16], vb[16], dq;
  tile_block_load(L, m, k0 * kBW, min(kBW, p - k0 * kBW), r0, nr, c0, nc, af0, vb, dq);
  tile_block_stage(vb, dq, B0);
  __syncthreads();
  for (int k = k0; k < k1; k += 2) {
    tile_block_step<R>(L, m, p, k, k1, r0, nr, c0, nc, af0, af1, vb, dq, B0, B1, re, im);
    if (k + 1 >= k1) break;
    tile_block_step<R>(L, m, p, k + 1, k1, r0, nr, c0, nc, af1, af0, vb, dq, B1, B0, re, im);
  }
  __syncthreads();
#pragma unroll
  for (int bj = 0; bj < 4; ++bj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      C v;
      v.x = re[bj][r];
      v.y = im[bj][r];
      As[(16 * bj + Mfma<R>::row(lane, r)) * kBW + 16 * wave + (lane & 15)] = v;
    }
  __syncthreads();
  // the tile's lower triangle: read (or assembled from the children), minus
  // the products, written back
  const TileMem tm = tile_mem<C>(a, s, f, ch, r0, nr, c0, nc);
  C v[16];
  if (first) {
#pragma unroll
    for (int t = 0; t < 16; ++t) v[t] = czero<C>();
    add_kids_tile<C>(a, s, f, kid, r0, c0, v);
  } else {
#pragma unroll
    for (int t = 0; t < 16; ++t)
      v[t] = ld_buf<C>(tm.rs, r0 + lane >= c0 + wave + 4 * t ? tm.rowoff + t * tm.colstride : kOob);
  }
#pragma unroll
  for (int t = 0; t < 16; ++t)
    st_buf<C>(tm.rs, r0 + lane >= c0 + wave + 4 * t ? tm.rowoff + t * tm.colstride : kOob,
              csub(v[t], As[(wave + 4 * t) * kBW + lane]));
}

// FUSED(k): the critical chain of one pivot step in one workgroup,
// TRSM(k, k-1) -> UPD(k, k, k-1) -> DIAG(k), with the intermediate tiles kept
// in LDS.  L_{k,k-1} = X D^-1 is written out (and its version published
// before the update, so the other updates of step k-1 can use it); the update
// uses A = X D^-1 and B = X (= L_{k,k-1} D); the updated diagonal tile is
// factored without a round trip through memory.
template <typename R>
__device__ __forceinline__ void task_fused(const KArgs& a, int s, int f, int k, int mode, int32_t* st,
                                           unsigned char* smem) {
  typedef typename Cx<R>::T C;
  C* Xs = reinterpret_cast<C*>(smem);  // tile (k, k-1): F, X, L = X D^-1, then the update product
  C* Ls = Xs + kBW * kBW;              // pivot block k-1; then X (B operand); then tile (k, k)
  C* Vs = Ls + kBW * kBW;              // kBW x 16 scratch; D_{k-1}
  const Chunks ch(a.npiv[f], a.nupd[f]);
  const int m = ch.m, kp0 = (k - 1) * kBW, k0 = k * kBW, nb = min(kBW, ch.p - k0);
  C* L = (C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  stage_block(Xs, L + (int64_t)kp0 * m + k0, m, nb, kBW, kAll);
  stage_block(Ls, L + (int64_t)kp0 * m + kp0, m, kBW, kBW, kLower);
  __syncthreads();
  trsm_core(Xs, Ls, Vs, kBW);
  if (threadIdx.x < kBW) Vs[threadIdx.x] = cinv(Ls[threadIdx.x * kBW + threadIdx.x]);
  __syncthreads();
  for (int c = wave; c < kBW; c += 4) {
    const C x = Xs[c * kBW + lane];
    const C l = cmul(x, Vs[c]);
    Ls[c * kBW + lane] = x;
    Xs[c * kBW + lane] = l;
    if (lane < nb) st_ag(L + (int64_t)(kp0 + c) * m + k0 + lane, l);
  }
  drain_stores();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(st + tile_id(k, k - 1), k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // tile (k, k) (final but for this step's update) is loaded before the
  // product so that the loads overlap it
  C t[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int c = wave + 4 * q;
    const bool keep = c < nb && lane < nb && lane >= c;
    t[q] = keep ? ld_ag(L + (int64_t)(k0 + c) * m + k0 + lane) : czero<C>();
  }
  mfma_tile_abt_lower<R>(Xs, Ls, Xs);
  // tile (k, k) - product, into Ls (lower triangle), then DIAG(k) with its
  // pivots and scratch in the Xs region.  The lane index is made opaque here
  // so that the sixteen LDS addresses are formed in the task: hoisted out of
  // the persistent loop they were spilled, one scratch round trip each.
  int ln = lane;
  asm volatile("" : "+v"(ln));
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int c = wave + 4 * q;
    const bool keep = c < nb && ln < nb && ln >= c;
    t[q] = keep ? csub(t[q], Xs[c * kBW + ln]) : czero<C>();
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) Ls[(wave + 4 * q) * kBW + ln] = t[q];
  __syncthreads();
  C* dd = Xs;
  C* invd = dd + kBW;
  C* T = invd + kBW;
  diag_core<R>(a, s, Ls, dd, invd, T, nb, mode);
  diag_store(L + (int64_t)k0 * m + k0, m, Ls, dd, nb, false);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_large_tiles(KArgs a, TileArgs ta, Queue q) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int sh;
  const int ep = launch_epoch(q);
  for (;;) {
    const int t = claim(q, &sh);
    if (t >= q.ntasks) break;
    const int32_t* tk = ta.tasks + 5 * (t / a.nsys);
    const int s = t % a.nsys;
    const int type = tk[0], f = tk[1], k = tk[2], I = tk[3], J = tk[4];
    const Chunks ch(a.npiv[f], a.nupd[f]);
    int32_t* st = ta.state + (int64_t)s * ta.ntiles + ta.tile_base[f];
    if (type == T_ASM) asm_stage<R>(a, s, f, I, J, smem_raw);  // independent of the wait below
    {
      // the task's dependencies, one thread each (each read is a memory
      // round trip; one thread reading them in turn would chain them)
      const int tid = threadIdx.x;
      if (type == T_ASM) {
        const int c = a.child_ptr[f] + tid;
        if (c < a.child_ptr[f + 1]) {
          const int cf = a.child_list[c];
          if (ta.is_tiled[cf]) {
            const int nut = (a.nupd[cf] + kBW - 1) / kBW;
            wait_at_least(ta.done + (int64_t)s * a.nfronts + cf, nut * (nut + 1) / 2, a.st);
          }
        }
      } else if (type == T_DIAG) {
        if (tid == 0) wait_value(st + tile_id(k, k), k + 1, a.st);
      } else if (type == T_TRSM) {
        if (tid == 0) wait_value(st + tile_id(k, k), k + 2, a.st);
        if (tid == 1) wait_value(st + tile_id(I, k), k + 1, a.st);
      } else if (type == T_INV) {
        for (int i = k + 1 + tid; i < ch.nbk + ch.nut; i += kThreads) wait_value(st + tile_id(i, k), k + 2, a.st);
      } else if (type == T_FUSED) {
        if (tid == 0) wait_value(st + tile_id(k - 1, k - 1), k + 1, a.st);
        if (tid == 1) wait_value(st + tile_id(k, k - 1), k, a.st);
        if (tid == 2) wait_value(st + tile_id(k, k), k, a.st);
      } else if (type == T_SYRK) {
        // rows I and J of the panel final up to block k1 - 1 (their TRSM), the
        // previous group's result, and for the first group the children
        const int k0 = k & 0xffff, k1 = k >> 16;
        if (tid == 0) wait_value(st + tile_id(I, k1 - 1), k1 + 1, a.st);
        if (tid == 1) wait_value(st + tile_id(J, k1 - 1), k1 + 1, a.st);
        if (tid == 2 && k0 > 0) wait_value(st + tile_id(I, J), k0, a.st);
        if (k0 == 0 && tid >= 64) {
          const int c = a.child_ptr[f] + tid - 64;
          if (c < a.child_ptr[f + 1]) {
            const int cf = a.child_list[c];
            if (ta.is_tiled[cf]) {
              const int nut = (a.nupd[cf] + kBW - 1) / kBW;
              wait_at_least(ta.done + (int64_t)s * a.nfronts + cf, nut * (nut + 1) / 2, a.st);
            }
          }
        }
      } else {
        // UPD over the blocks [k0, k1): rows I and J final up to block k1 - 1,
        // the tile updated by every block before k0
        const int k0 = k & 0xffff, k1 = k >> 16;
        if (tid == 0) wait_value(st + tile_id(I, k1 - 1), k1 + 1, a.st);
        if (tid == 1) wait_value(st + tile_id(J, k1 - 1), k1 + 1, a.st);
        if (tid == 2) wait_value(st + tile_id(I, J), k0 + 1, a.st);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    __syncthreads();
    trace_mark(q, t, 1);
    int tile = 0, ver = 0;
    if (type == T_ASM) {
      task_asm<R>(a, s, f, I, J, smem_raw);
      tile = tile_id(I, J);
      ver = 1;
    } else if (type == T_DIAG || type == T_INV) {
      task_diag<R>(a, s, f, k, type == T_INV ? kInvOnly : k == ch.nbk + ch.nut - 1 ? kDiagFull : kDiagPart,
                   smem_raw);
      tile = type == T_INV ? -1 : tile_id(k, k);
      ver = k + 2;
    } else if (type == T_TRSM) {
      task_trsm<R>(a, s, f, k, I, smem_raw);
      tile = tile_id(I, k);
      ver = k + 2;
    } else if (type == T_FUSED) {
      task_fused<R>(a, s, f, k, k == ch.nbk + ch.nut - 1 ? kDiagFull : kDiagPart, st, smem_raw);
      tile = tile_id(k, k);
      ver = k + 2;
    } else if (type == T_SYRK) {
      task_tile_update<R>(a, s, f, k & 0xffff, k >> 16, I, J, smem_raw);
      tile = tile_id(I, J);
      ver = k >> 16;
    } else {
      task_tile_update<R>(a, s, f, k & 0xffff, k >> 16, I, J, smem_raw);
      tile = tile_id(I, J);
      ver = (k >> 16) + 1;
    }
    drain_stores();
    __syncthreads();
    if (threadIdx.x == 0 && tile >= 0) {
      __hip_atomic_store(st + tile, ver, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // a front's update tile is final after its last Schur-complement group
      if (type == T_SYRK && (k >> 16) == ch.nbk)
        __hip_atomic_fetch_add(ta.done + (int64_t)s * a.nfronts + f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    trace_mark(q, t, 2);
  }
  leave(q, ep);
}

// Clears tile versions and completion counts before the task-graph launch.
__global__ void k_tiles_reset(int32_t* state, int64_t nstate, int32_t* done, int64_t ndone) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nstate + ndone;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < nstate) state[i] = 0;
    else done[i - nstate] = 0;
  }
}

// ---------------------------------------------------------------------------
// Solves.  Multifrontal sweeps over the separator tree, one persistent launch
// per direction.  y holds the elimination-order vector ([sys][rhs][N], factor
// precision), wv each front's update vector ([sys][rhs][sum u]).  The forward
// sweep reads the right-hand side in grid order (optionally scaled by S) and
// the backward sweep writes (or adds) the solution in grid order, so no
// separate permutation passes run.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool done(const int* flag) { return flag && *(volatile const int*)flag; }

struct SweepArgs {
  const double2* src;  // forward: right-hand sides, grid order
  double2* out;        // backward: solution, grid order
  void* y;
  void* wv;
  const int* flag;     // refinement converged: skip the launch
  int64_t io_ld;       // src / out: entries from one system's columns to the next
  int32_t nrhs, scale_src, accumulate;
  DevStatus* st;       // with status_mode >= 0: record "no refinement" for that solve
  int32_t status_mode; // -1, 0 (forward solve) or 1 (adjoint solve)
  int32_t lev_lo, lev_hi;  // the launch's fronts have heights in [lev_lo, lev_hi);
                           // fronts outside finished in an earlier launch
  int32_t wave_ld;         // wave-item launches: LDS entries per wave and RHS
  // forward launch of the tiled levels: (front, part) items, update-row
  // chunks per front and their first flag slot, z of split fronts
  const int32_t* items;
  const int32_t* nch;
  const int32_t* chunk_base;
  void* zv;
  int32_t nchunk;
  // backward launch of the tiled levels: partial column sums of the chunks
  const int64_t* part_base;
  void* pv;
  int64_t part_total;
  // fronts swept as one item per pivot block: first block flag (-1: not split)
  const int32_t* blk_base;
  int32_t nblk;
};

// Completion flag of update-row chunk j of front f (after the fronts' flags).
__device__ __forceinline__ const int32_t* chunk_flag(const Queue& q, const KArgs& a, const SweepArgs& w, int s,
                                                     int f, int j) {
  return q.done + (int64_t)a.nsys * a.nfronts + (int64_t)s * w.nchunk + w.chunk_base[f] + j;
}

// Completion flag of pivot block j of a block-split front f (after the chunks' flags).
__device__ __forceinline__ const int32_t* blk_flag(const Queue& q, const KArgs& a, const SweepArgs& w, int s, int f,
                                                   int j) {
  return q.done + (int64_t)a.nsys * (a.nfronts + w.nchunk) + (int64_t)s * w.nblk + w.blk_base[f] + j;
}

// Waits of a sweep launch: only on fronts of the same launch (the others
// finished before the launch began and carry an older epoch).  Called by one
// thread, which spins; the caller orders its later loads after it.
// A child whose update rows are split in chunks (w.nch, forward launch of the
// tiled levels only) is complete when all its chunks are.  The flags are
// shared out over threads tid of nt (each flag read is a memory round trip,
// so one thread reading them in turn would chain them); the caller orders its
// later loads after the waits (fence + barrier).
__device__ __forceinline__ void sweep_wait_children(const Queue& q, int ep, const KArgs& a, const SweepArgs& w,
                                                    int s, int f, int tid, int nt) {
  int base = 0;  // position of the child's first flag among all the item's flags
  for (int k = a.child_ptr[f]; k < a.child_ptr[f + 1]; ++k) {
    const int c = a.child_list[k];
    if (a.height[c] < w.lev_lo) continue;
    const int nc = w.nch ? w.nch[c] : 0;
    const int nf = nc > 0 ? nc : 1;
    for (int j = tid - base; j < nf; j += nt)
      if (j >= 0) wait_flag(q, ep, nc > 0 ? chunk_flag(q, a, w, s, c, j) : q.done + (int64_t)s * a.nfronts + c);
    base += nf;
  }
}

__device__ __forceinline__ void sweep_wait_parent(const Queue& q, int ep, const KArgs& a, const SweepArgs& w,
                                                  int s, int f) {
  const int par = a.parent[f];
  if (par >= 0 && a.height[par] < w.lev_hi) wait_flag(q, ep, q.done + (int64_t)s * a.nfronts + par);
}

__device__ __forceinline__ void sweep_status(const SweepArgs& w) {
  if (w.status_mode >= 0 && blockIdx.x == 0 && threadIdx.x == 0) {
    // a solve without refinement: no steps, no residual, no failure
    if (w.status_mode == 0) {
      w.st->ir_steps_solve = 0;
      w.st->rel_solve = -1.0;
      w.st->ir_failed_solve = 0;
    } else {
      w.st->ir_steps_adj = 0;
      w.st->rel_adj = -1.0;
      w.st->ir_failed_adj = 0;
    }
  }
}

// Loads in flight per thread in the sweeps: the sweeps stream the factor once,
// so the time of a front is its load rounds times the memory latency; every
// loop below issues kSweepBatch independent loads before it uses the first.
constexpr int kSweepBatch = 16;

// The tiled-level sweeps run one kSweepThreads-thread workgroup per front: the
// few large fronts of those levels are processed one or two at a time, so a
// front's time is its load rounds, and more waves keep more loads in flight.
constexpr int kSweepThreads = 512;
constexpr int kSW = kSweepThreads / 64;   // waves
constexpr int kRowStep = 64 * kSW / 4;    // rows per step of the below-block update
constexpr int kNQ = kSW / 4;              // row parts of the backward column sums

// One front of the forward sweep.  V = [rhs_p; 0] + the children's update
// vectors; then for each kBW-wide pivot block: V_blk <- Xinv V_blk with the
// inverted unit-lower diagonal block stored in the panel (the waves split the
// columns, partial sums meet in LDS), and V_below -= L_below,blk V_blk,
// kRowStep rows per step (wave w: rows 64 (w / 4) + lane of the step, columns
// w % 4, w % 4 + 4, ...; sixteen loads per thread in flight).  Finally
// y_p = D^-1 V_p and the update vector is V_u.  split: only the pivot rows
// (the update rows are chunk items, fwd_chunk), and z = V_p goes to w.zv.
template <typename R>
__device__ void fwd_front(const KArgs& a, const SweepArgs& w, int s, int f, bool split, unsigned char* smem) {
  typedef typename Cx<R>::T C;
  const int p = a.npiv[f], u = a.nupd[f], m = split ? p : p + u, pb = a.pbeg[f];
  const int ldl = p + u;  // leading dimension of the panel
  const int nrhs = w.nrhs;
  C* red = reinterpret_cast<C*>(smem);  // nrhs x 4 x kRowStep (>= nrhs x kSW x kBW) partial sums
  C* V = red + 4 * kRowStep * nrhs;     // nrhs x m
  const C* L = (const C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  C* Y = (C*)w.y + (int64_t)s * nrhs * a.N;
  C* W = (C*)w.wv + (int64_t)s * nrhs * a.sum_u;
  const double2* B = w.src + (int64_t)s * w.io_ld;
  const int cb = a.child_ptr[f], nch = a.child_ptr[f + 1] - cb;
  const int32_t* g = a.gmap + a.gmap_ptr[f];  // rows of length ldl per child
  for (int idx = threadIdx.x; idx < m * nrhs; idx += kSweepThreads) {
    const int col = idx / m, r = idx - col * m;
    // the gather rows of up to two children first, then every value load
    int gr[2];
    int64_t base[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      gr[k] = k < nch ? g[k * ldl + r] : -1;
      base[k] = k < nch ? (int64_t)col * a.sum_u + a.upd_ptr[a.child_list[cb + k]] : 0;
    }
    double2 bv = make_double2(0.0, 0.0);
    if (r < p) bv = B[(int64_t)col * a.N + a.perm[pb + r]];
    C cv[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) cv[k] = gr[k] >= 0 ? ld_ag(W + base[k] + gr[k]) : czero<C>();
    if (r < p && w.scale_src) bv = dmul(bv, sym_scale(a, s, a.perm[pb + r]));
    C v = cadd(from_d2<C>(bv), cadd(cv[0], cv[1]));
    for (int k = 2; k < nch; ++k) {
      const int gk = g[k * ldl + r];
      if (gk >= 0) v = cadd(v, ld_ag(W + (int64_t)col * a.sum_u + a.upd_ptr[a.child_list[cb + k]] + gk));
    }
    V[col * m + r] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cg = wave & 3, rq = wave >> 2;
  for (int k0 = 0; k0 < p; k0 += kBW) {
    const int kn = min(kBW, p - k0), k1 = k0 + kn;
    const C* Xb = L + (int64_t)k0 * ldl + k0;
    {
      // V_blk <- Xinv V_blk: lane = row, wave w takes columns w, w + kSW, ... < lane
      constexpr int NT = kBW / kSW;
      C xv[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int j = wave + kSW * t;
        xv[t] = (lane < kn && j < lane) ? Xb[(int64_t)j * ldl + lane] : czero<C>();
      }
      for (int col = 0; col < nrhs; ++col) {
        const C* Vb = V + col * m + k0;
        C acc = czero<C>();
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int j = wave + kSW * t;
          acc = cadd(acc, cmul(xv[t], j < kn ? Vb[j] : czero<C>()));
        }
        red[(col * kSW + wave) * kBW + lane] = acc;
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kn * nrhs; idx += kSweepThreads) {
      const int col = idx / kn, j = idx - col * kn;
      const C* rr = red + col * kSW * kBW + j;
      C acc = czero<C>();
#pragma unroll
      for (int q = 0; q < kSW; ++q) acc = cadd(acc, rr[q * kBW]);
      V[col * m + k0 + j] = cadd(V[col * m + k0 + j], acc);
    }
    __syncthreads();
    for (int rc = k1; rc < m; rc += kRowStep) {
      const int i = rc + 64 * rq + lane;
      C l[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int j = cg + 4 * t;
        const C* Lj = L + (int64_t)(k0 + min(j, kn - 1)) * ldl;
        l[t] = j < kn && i < m ? Lj[i] : czero<C>();
      }
      for (int col = 0; col < nrhs; ++col) {
        const C* Vb = V + col * m + k0;
        C acc = czero<C>();
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int j = cg + 4 * t;
          acc = cadd(acc, cmul(l[t], j < kn ? Vb[j] : czero<C>()));
        }
        red[(col * 4 + cg) * kRowStep + 64 * rq + lane] = acc;
      }
      __syncthreads();
      for (int idx = threadIdx.x; idx < kRowStep * nrhs; idx += kSweepThreads) {
        const int col = idx / kRowStep, r = idx - col * kRowStep, ii = rc + r;
        if (ii < m) {
          const C* rr = red + col * 4 * kRowStep + r;
          V[col * m + ii] =
              csub(V[col * m + ii], cadd(cadd(rr[0], rr[kRowStep]), cadd(rr[2 * kRowStep], rr[3 * kRowStep])));
        }
      }
      __syncthreads();
    }
  }
  for (int idx = threadIdx.x; idx < m * nrhs; idx += kSweepThreads) {
    const int col = idx / m, r = idx - col * m;
    if (r < p) {
      Y[(int64_t)col * a.N + pb + r] = cmul(V[col * m + r], cinv(L[(int64_t)r * ldl + r]));
      if (split) st_ag((C*)w.zv + (int64_t)s * nrhs * a.N + (int64_t)col * a.N + pb + r, V[col * m + r]);
    } else {
      st_ag(W + (int64_t)col * a.sum_u + a.upd_ptr[f] + (r - p), V[col * m + r]);
    }
  }
}

// Pivot block j of a block-split front in the forward sweep: V_j = the
// block's right-hand side rows + the children's update-vector entries, then
// V_j -= L[block j, block j'] z_j' for every earlier block j' as its item
// publishes z_j' (the block's L entries are loaded before each wait: the
// factor is final), then z_j = Xinv_j V_j with the stored inverted diagonal
// block, y_j = D^-1 z_j into y and z_j into zv for the later blocks and the
// update-row chunks.  Lane = row, wave w takes the columns w, w + kSW, ...
template <typename R>
__device__ void fwd_piv_block(const KArgs& a, const SweepArgs& w, const Queue& q, int ep, int s, int f, int j,
                              unsigned char* smem) {
  typedef typename Cx<R>::T C;
  constexpr int NT = kBW / kSW;
  const int p = a.npiv[f], u = a.nupd[f], ldl = p + u, pb = a.pbeg[f];
  const int k0 = j * kBW, kn = min(kBW, p - k0);
  const int nrhs = w.nrhs;
  C* red = reinterpret_cast<C*>(smem);  // nrhs x kSW x kBW partial sums
  C* V = red + kSW * kBW * nrhs;        // nrhs x kBW
  C* Z = V + kBW * nrhs;                // nrhs x kBW: z of the block being applied
  const C* L = (const C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  C* Y = (C*)w.y + (int64_t)s * nrhs * a.N;
  C* Zv = (C*)w.zv + (int64_t)s * nrhs * a.N;
  const C* W = (const C*)w.wv + (int64_t)s * nrhs * a.sum_u;
  const double2* B = w.src + (int64_t)s * w.io_ld;
  const int cb = a.child_ptr[f], nch = a.child_ptr[f + 1] - cb;
  const int32_t* g = a.gmap + a.gmap_ptr[f];
  for (int idx = threadIdx.x; idx < kn * nrhs; idx += kSweepThreads) {
    const int col = idx / kn, r = k0 + idx - col * kn;
    const int n = a.perm[pb + r];
    double2 bv = B[(int64_t)col * a.N + n];
    if (w.scale_src) bv = dmul(bv, sym_scale(a, s, n));
    C v = from_d2<C>(bv);
    for (int k = 0; k < nch; ++k) {
      const int gk = g[k * ldl + r];
      if (gk >= 0) v = cadd(v, ld_ag(W + (int64_t)col * a.sum_u + a.upd_ptr[a.child_list[cb + k]] + gk));
    }
    V[col * kBW + (r - k0)] = v;
  }
  for (int idx = threadIdx.x; idx < kSW * kBW * nrhs; idx += kSweepThreads) red[idx] = czero<C>();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // the stored strictly lower part of the block's inverted unit-lower
  // diagonal block, loaded ahead of the last wait of the chain
  const C* Xb = L + (int64_t)k0 * ldl + k0;
  C xv[NT];
  auto load_inv = [&]() {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int jj = wave + kSW * t;
      xv[t] = (lane < kn && jj < lane) ? Xb[(int64_t)jj * ldl + lane] : czero<C>();
    }
  };
  if (j == 0) load_inv();
  for (int jp = 0; jp < j; ++jp) {
    C l[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int c = jp * kBW + wave + kSW * t;
      l[t] = lane < kn ? L[(int64_t)c * ldl + k0 + lane] : czero<C>();
    }
    if (jp == j - 1) load_inv();
    if (threadIdx.x == 0) {
      wait_flag(q, ep, blk_flag(q, a, w, s, f, jp));
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kBW * nrhs; idx += kSweepThreads) {
      const int col = idx / kBW, r = idx - col * kBW;
      Z[idx] = ld_ag(Zv + (int64_t)col * a.N + pb + jp * kBW + r);
    }
    __syncthreads();
    for (int col = 0; col < nrhs; ++col) {
      C acc = czero<C>();
#pragma unroll
      for (int t = 0; t < NT; ++t) acc = cadd(acc, cmul(l[t], Z[col * kBW + wave + kSW * t]));
      C* rp = red + (col * kSW + wave) * kBW + lane;
      *rp = cadd(*rp, acc);
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < kn * nrhs; idx += kSweepThreads) {
    const int col = idx / kn, r = idx - col * kn;
    const C* rr = red + col * kSW * kBW + r;
    C acc = czero<C>();
#pragma unroll
    for (int qq = 0; qq < kSW; ++qq) acc = cadd(acc, rr[qq * kBW]);
    V[col * kBW + r] = csub(V[col * kBW + r], acc);
  }
  __syncthreads();
  {
    // V <- Xinv V
    for (int col = 0; col < nrhs; ++col) {
      C acc = czero<C>();
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int jj = wave + kSW * t;
        acc = cadd(acc, cmul(xv[t], jj < kn ? V[col * kBW + jj] : czero<C>()));
      }
      red[(col * kSW + wave) * kBW + lane] = acc;
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < kn * nrhs; idx += kSweepThreads) {
    const int col = idx / kn, r = idx - col * kn;
    const C* rr = red + col * kSW * kBW + r;
    C z = V[col * kBW + r];
#pragma unroll
    for (int qq = 0; qq < kSW; ++qq) z = cadd(z, rr[qq * kBW]);
    Y[(int64_t)col * a.N + pb + k0 + r] = cmul(z, cinv(L[(int64_t)(k0 + r) * ldl + k0 + r]));
    st_ag(Zv + (int64_t)col * a.N + pb + k0 + r, z);
  }
}

// One chunk of kChunkRows update rows R = [r0, r0 + nr) of a split front in
// the forward sweep: V_R = the children's update-vector entries of those rows
// (gathered before the front's pivot item is waited for), then
// V_R -= L[R, 0:p] z_p with z_p from that item, stored as rows R of the
// front's update vector.  Lane = row, wave w takes the columns w, w + kSW, ...
// (kSweepBatch loads per thread in flight); the partial sums of the waves
// accumulate in their own LDS slots and meet at the end.
template <typename R>
__device__ void fwd_chunk(const KArgs& a, const SweepArgs& w, const Queue& q, int ep, int s, int f, int j,
                          unsigned char* smem) {
  typedef typename Cx<R>::T C;
  const int p = a.npiv[f], u = a.nupd[f], m = p + u, pb = a.pbeg[f];
  const int r0 = p + kChunkRows * j, nr = min(kChunkRows, m - r0);
  const int nrhs = w.nrhs;
  C* red = reinterpret_cast<C*>(smem);   // nrhs x kSW x kChunkRows partial sums
  C* V = red + kSW * kChunkRows * nrhs;  // nrhs x nr
  C* Z = V + nr * nrhs;                  // nrhs x p
  const C* L = (const C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  C* W = (C*)w.wv + (int64_t)s * nrhs * a.sum_u;
  const int cb = a.child_ptr[f], nch = a.child_ptr[f + 1] - cb;
  const int32_t* g = a.gmap + a.gmap_ptr[f];
  for (int idx = threadIdx.x; idx < nr * nrhs; idx += kSweepThreads) {
    const int col = idx / nr, r = idx - col * nr;
    C v = czero<C>();
    for (int k = 0; k < nch; ++k) {
      const int gk = g[k * m + r0 + r];
      if (gk >= 0) v = cadd(v, ld_ag(W + (int64_t)col * a.sum_u + a.upd_ptr[a.child_list[cb + k]] + gk));
    }
    V[col * nr + r] = v;
  }
  for (int idx = threadIdx.x; idx < kSW * kChunkRows * nrhs; idx += kSweepThreads) red[idx] = czero<C>();
  const C* Zs = (const C*)w.zv + (int64_t)s * nrhs * a.N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool rowok = lane < nr;
  const C* Li = L + r0 + (rowok ? lane : 0);
  if (w.blk_base[f] >= 0) {
    // block-split front: take each pivot block's z as its item publishes it
    constexpr int NT = kBW / kSW;
    for (int jp = 0; jp * kBW < p; ++jp) {
      const int kb = jp * kBW, kn = min(kBW, p - kb);
      C l[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int c = wave + kSW * t;
        l[t] = rowok && c < kn ? Li[(int64_t)(kb + c) * m] : czero<C>();
      }
      if (threadIdx.x == 0) {
        wait_flag(q, ep, blk_flag(q, a, w, s, f, jp));
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      }
      __syncthreads();
      for (int idx = threadIdx.x; idx < kn * nrhs; idx += kSweepThreads) {
        const int col = idx / kn, r = idx - col * kn;
        Z[col * p + kb + r] = ld_ag(Zs + (int64_t)col * a.N + pb + kb + r);
      }
      __syncthreads();
      for (int col = 0; col < nrhs; ++col) {
        C* acc = red + (col * kSW + wave) * kChunkRows + lane;
        C v = *acc;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int c = wave + kSW * t;
          v = cadd(v, cmul(l[t], c < kn ? Z[col * p + kb + c] : czero<C>()));
        }
        *acc = v;
      }
    }
  } else {
  if (threadIdx.x == 0) {
    wait_flag(q, ep, q.done + (int64_t)s * a.nfronts + f);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < p * nrhs; idx += kSweepThreads) {
    const int col = idx / p, r = idx - col * p;
    Z[col * p + r] = ld_ag(Zs + (int64_t)col * a.N + pb + r);
  }
  __syncthreads();
  for (int t0 = wave; t0 < p; t0 += kSweepBatch * kSW) {
    C l[kSweepBatch];
#pragma unroll
    for (int t = 0; t < kSweepBatch; ++t) {
      const int c = t0 + kSW * t;
      l[t] = rowok && c < p ? Li[(int64_t)c * m] : czero<C>();
    }
    for (int col = 0; col < nrhs; ++col) {
      C* acc = red + (col * kSW + wave) * kChunkRows + lane;
      C v = *acc;
#pragma unroll
      for (int t = 0; t < kSweepBatch; ++t) {
        const int c = t0 + kSW * t;
        v = cadd(v, cmul(l[t], c < p ? Z[col * p + c] : czero<C>()));
      }
      *acc = v;
    }
  }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < nr * nrhs; idx += kSweepThreads) {
    const int col = idx / nr, r = idx - col * nr;
    const C* rr = red + col * kSW * kChunkRows + r;
    C acc = czero<C>();
#pragma unroll
    for (int q2 = 0; q2 < kSW; ++q2) acc = cadd(acc, rr[q2 * kChunkRows]);
    st_ag(W + (int64_t)col * a.sum_u + a.upd_ptr[f] + (r0 - p) + r, csub(V[col * nr + r], acc));
  }
}

template <typename C> __device__ __forceinline__ C wave_sum(C v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  return v;
}

// Column dot products of the backward sweep for NR right-hand sides: lane l
// of wave w owns column jj = 16 (w % 4) + (l & 15) of the block and, within
// the row quarter w / 4 of [r0, r1), the rows q0 + (l >> 4) + 4 t: one load
// instruction covers 16 columns x 4 consecutive rows, kDotBatch loads per
// thread are in flight per step, the four row phases of a column meet through
// two lane exchanges.  Returns the part's column sums in lanes l < 16.
// loads in flight per thread in bwd_dots: sixteen in both precisions (a
// deeper batch of complex64 entries, with the two right-hand-side columns'
// LDS reads it pulls forward, no longer fits the 256 registers a 512-thread
// workgroup leaves a lane, and spills)
template <typename C> constexpr int kDotBatch = 16;

template <int NR, typename C>
__device__ __forceinline__ void bwd_dots(const C* Lc, bool colok, const C* X, int m, int r0, int r1, C* acc) {
  // q is made opaque so that the row offsets q + 4t are formed in the call:
  // hoisted out of the persistent loop as 64-bit values, they were spilled,
  // and each reload waited for every load already in flight
  int q = (threadIdx.x & 63) >> 4;
  asm volatile("" : "+v"(q));
  const int rq = (threadIdx.x >> 6) >> 2;
  const int per = (r1 - r0 + kNQ - 1) / kNQ;
  const int q0 = r0 + rq * per, q1 = min(r1, q0 + per);
#pragma unroll
  for (int c = 0; c < NR; ++c) acc[c] = czero<C>();
  for (int i = q0 + q; i < q1; i += 4 * kDotBatch<C>) {
    const C* Li = Lc + i;
    const C* Xi = X + i;
    C l[kDotBatch<C>];
#pragma unroll
    for (int t = 0; t < kDotBatch<C>; ++t) l[t] = colok && i + 4 * t < q1 ? Li[4 * t] : czero<C>();
#pragma unroll
    for (int c = 0; c < NR; ++c)
#pragma unroll
      for (int t = 0; t < kDotBatch<C>; ++t)
        acc[c] = cadd(acc[c], cmul(l[t], i + 4 * t < q1 ? Xi[c * m + 4 * t] : czero<C>()));
  }
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    acc[c] = cadd(acc[c], shfl_xor_c(acc[c], 16));
    acc[c] = cadd(acc[c], shfl_xor_c(acc[c], 32));
  }
}

// Column sums of right-hand sides [c0, c0 + NR) over the below-block rows
// (diag = false) or, for column jj, the rows jj+1 .. kn-1 of the diagonal
// block's inverse (diag = true), per row part into red[c][part][jj].
template <int NR, typename C>
__device__ __forceinline__ void bwd_group(const C* L, int ldl, const C* X, C* red, int m, int k0, int kn, int k1,
                                          int r1, int c0, bool diag) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int jj = 16 * (wave & 3) + (lane & 15), rq = wave >> 2;
  const bool colok = jj < kn;
  C acc[NR];
  if (!diag) bwd_dots<NR>(L + (int64_t)(k0 + min(jj, kn - 1)) * ldl, colok, X + c0 * m, m, k1, r1, acc);
  else bwd_dots<NR>(L + (int64_t)(k0 + min(jj, kn - 1)) * ldl + k0, colok, X + c0 * m + k0, m, jj + 1, kn, acc);
  if (lane < 16)
#pragma unroll
    for (int c = 0; c < NR; ++c) red[((c0 + c) * kNQ + rq) * kBW + jj] = acc[c];
}

// L: the panel (leading dimension ldl); X: nrhs x m, rows [k1, r1) summed.
template <typename C>
__device__ __forceinline__ void bwd_block(const C* L, int ldl, const C* X, C* red, int m, int k0, int kn, int k1,
                                          int r1, int nrhs, bool diag) {
  for (int c0 = 0; c0 < nrhs; c0 += 2) {
    if (nrhs - c0 >= 2) bwd_group<2>(L, ldl, X, red, m, k0, kn, k1, r1, c0, diag);
    else bwd_group<1>(L, ldl, X, red, m, k0, kn, k1, r1, c0, diag);
  }
}

// A pivot block's column sums from a tile of at most 64 rows whose entries
// were loaded ahead (bwd_tile_load, before the wait for the right-hand side):
// the same lanes, rows and summation order as bwd_dots.
template <typename C>
__device__ __forceinline__ void bwd_tile_load(const C* Lc, bool colok, int r0, int r1, C (&l)[8]) {
  // q is made opaque so that the row offsets q + 4t are formed in the call:
  // hoisted out of the persistent loop as 64-bit values, they were spilled,
  // and each reload waited for every load already in flight
  int q = (threadIdx.x & 63) >> 4;
  asm volatile("" : "+v"(q));
  const int rq = (threadIdx.x >> 6) >> 2;
  const int per = (r1 - r0 + kNQ - 1) / kNQ;  // at most 32 rows: eight per thread
  const int q0 = r0 + rq * per, q1 = min(r1, q0 + per);
#pragma unroll
  for (int t = 0; t < 8; ++t) l[t] = colok && q0 + q + 4 * t < q1 ? Lc[q0 + q + 4 * t] : czero<C>();
}

template <int NR, typename C>
__device__ __forceinline__ void bwd_tile_group(const C (&l)[8], const C* X, C* red, int m, int r0, int r1, int c0) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, rq = wave >> 2, jj = 16 * (wave & 3) + (lane & 15);
  const int per = (r1 - r0 + kNQ - 1) / kNQ;
  const int q0 = r0 + rq * per, q1 = min(r1, q0 + per);
  C acc[NR];
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    acc[c] = czero<C>();
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int i = q0 + q + 4 * t;
      acc[c] = cadd(acc[c], cmul(l[t], i < q1 ? X[(c0 + c) * m + i] : czero<C>()));
    }
    acc[c] = cadd(acc[c], shfl_xor_c(acc[c], 16));
    acc[c] = cadd(acc[c], shfl_xor_c(acc[c], 32));
  }
  if (lane < 16)
#pragma unroll
    for (int c = 0; c < NR; ++c) red[((c0 + c) * kNQ + rq) * kBW + jj] = acc[c];
}

template <typename C>
__device__ __forceinline__ void bwd_tile(const C (&l)[8], const C* X, C* red, int m, int r0, int r1, int nrhs) {
  for (int c0 = 0; c0 < nrhs; c0 += 2) {
    if (nrhs - c0 >= 2) bwd_tile_group<2>(l, X, red, m, r0, r1, c0);
    else bwd_tile_group<1>(l, X, red, m, r0, r1, c0);
  }
}

// One front of the backward sweep.  X = [z_p; x(update rows)]; for kBW-wide
// blocks from the last: X_blk -= L_below,blk^T X_below, then
// X_blk <- Xinv^T X_blk (column dot products, bwd_dots; the row parts meet
// in LDS).  x_p goes to y and to the grid-order output.  Split fronts (nc
// chunks): the update rows' part of X_p -= L21^T x_u comes from the chunk
// items (bwd_chunk, summed in chunk order) and only the pivot rows remain.
template <typename R>
__device__ void bwd_front(const KArgs& a, const SweepArgs& w, int s, int f, int nc, unsigned char* smem) {
  typedef typename Cx<R>::T C;
  const bool split = nc > 0;
  const int p = a.npiv[f], u = a.nupd[f], m = split ? p : p + u, pb = a.pbeg[f];
  const int ldl = p + u;  // leading dimension of the panel
  const int nrhs = w.nrhs;
  C* red = reinterpret_cast<C*>(smem);  // nrhs x kNQ x kBW
  C* X = red + kNQ * nrhs * kBW;
  const C* L = (const C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  C* Y = (C*)w.y + (int64_t)s * nrhs * a.N;
  const int32_t* ui = a.upd_idx + a.upd_ptr[f];
  const C* PB = (const C*)w.pv + (int64_t)s * nrhs * w.part_total + (split ? w.part_base[f] : 0);
  for (int idx = threadIdx.x; idx < m * nrhs; idx += kSweepThreads) {
    const int col = idx / m, r = idx - col * m;
    C v = ld_ag(Y + (int64_t)col * a.N + (r < p ? pb + r : ui[r - p]));
    if (split) {
      // eight chunks' sums in flight at a time, added in chunk order
      const C* pr = PB + (int64_t)col * w.part_total + r;
      C acc = czero<C>();
      for (int j0 = 0; j0 < nc; j0 += 8) {
        C pj[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) pj[t] = j0 + t < nc ? ld_ag(pr + (int64_t)(j0 + t) * p) : czero<C>();
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (j0 + t < nc) acc = cadd(acc, pj[t]);
      }
      v = csub(v, acc);
    }
    X[col * m + r] = v;
  }
  __syncthreads();
  int k1 = p;
  while (k1 > 0) {
    const int k0 = ((k1 - 1) / kBW) * kBW;
    const int kn = k1 - k0;
    if (k1 < m) {
      bwd_block(L, ldl, X, red, m, k0, kn, k1, m, nrhs, false);
      __syncthreads();
      for (int idx = threadIdx.x; idx < kn * nrhs; idx += kSweepThreads) {
        const int col = idx / kn, j = idx - col * kn;
        const C* rr = red + col * kNQ * kBW + j;
        C acc = czero<C>();
#pragma unroll
        for (int q = 0; q < kNQ; ++q) acc = cadd(acc, rr[q * kBW]);
        X[col * m + k0 + j] = csub(X[col * m + k0 + j], acc);
      }
      __syncthreads();
    }
    bwd_block(L, ldl, X, red, m, k0, kn, k1, m, nrhs, true);
    __syncthreads();
    // x_blk = X_blk + the parts' sums (every read of X_blk above is done)
    for (int idx = threadIdx.x; idx < kn * nrhs; idx += kSweepThreads) {
      const int col = idx / kn, j = idx - col * kn;
      const C* rr = red + col * kNQ * kBW + j;
      C acc = czero<C>();
#pragma unroll
      for (int q = 0; q < kNQ; ++q) acc = cadd(acc, rr[q * kBW]);
      X[col * m + k0 + j] = cadd(X[col * m + k0 + j], acc);
    }
    __syncthreads();
    k1 = k0;
  }
  double2* O = w.out + (int64_t)s * w.io_ld;
  for (int idx = threadIdx.x; idx < p * nrhs; idx += kSweepThreads) {
    const int col = idx / p, r = idx - col * p;
    const C x = X[col * m + r];
    st_ag(Y + (int64_t)col * a.N + pb + r, x);
    double2* o = O + (int64_t)col * a.N + a.perm[pb + r];
    const double2 xv = to_d2(x);
    *o = w.accumulate ? dadd(*o, xv) : xv;
  }
}

// Pivot block j of a block-split front in the backward sweep (every chunk of
// the front has been waited for): X_j = y_j minus the chunks' partial column
// sums (in chunk order), then X_j -= L[block j', block j]^T x_j' for every
// later block j' as its item publishes x_j' (last block first), then
// x_j = Xinv_j^T X_j; x_j goes to y (for the other blocks and the children)
// and to the grid-order output.  X holds the front's rows (leading dimension
// m) as in bwd_front, filled only for block j and the block being applied.
template <typename R>
__device__ void bwd_piv_block(const KArgs& a, const SweepArgs& w, const Queue& q, int ep, int s, int f, int j, int nc,
                              unsigned char* smem) {
  typedef typename Cx<R>::T C;
  const int p = a.npiv[f], u = a.nupd[f], m = p + u, ldl = m, pb = a.pbeg[f];
  const int k0 = j * kBW, kn = min(kBW, p - k0);
  const int nrhs = w.nrhs;
  C* red = reinterpret_cast<C*>(smem);  // nrhs x kNQ x kBW
  C* X = red + kNQ * nrhs * kBW;        // nrhs x m
  const C* L = (const C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  C* Y = (C*)w.y + (int64_t)s * nrhs * a.N;
  const C* PB = (const C*)w.pv + (int64_t)s * nrhs * w.part_total + (nc > 0 ? w.part_base[f] : 0);
  for (int idx = threadIdx.x; idx < kn * nrhs; idx += kSweepThreads) {
    const int col = idx / kn, r = k0 + idx - col * kn;
    C v = ld_ag(Y + (int64_t)col * a.N + pb + r);
    if (nc > 0) {
      const C* pr = PB + (int64_t)col * w.part_total + r;
      C acc = czero<C>();
      for (int j0 = 0; j0 < nc; j0 += 8) {
        C pj[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) pj[t] = j0 + t < nc ? ld_ag(pr + (int64_t)(j0 + t) * p) : czero<C>();
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (j0 + t < nc) acc = cadd(acc, pj[t]);
      }
      v = csub(v, acc);
    }
    X[col * m + r] = v;
  }
  const int nbk = (p + kBW - 1) / kBW;
  // this thread's column of the block (bwd_dots' lane layout) and the tiles
  // of it that the chain waits on, loaded ahead of each wait: block jp's
  // rows before the wait for x_jp, the inverse's before the last wait
  const int jj = 16 * ((threadIdx.x >> 6) & 3) + (threadIdx.x & 15);
  const bool colok = jj < kn;
  const C* Lj = L + (int64_t)(k0 + min(jj, kn - 1)) * ldl;
  C li[8];
  if (nbk - 1 == j) bwd_tile_load(Lj + k0, colok, jj + 1, kn, li);
  for (int jp = nbk - 1; jp > j; --jp) {
    const int kb = jp * kBW, kbn = min(kBW, p - kb);
    C lt[8];
    bwd_tile_load(Lj, colok, kb, kb + kbn, lt);
    if (jp == j + 1) bwd_tile_load(Lj + k0, colok, jj + 1, kn, li);
    if (threadIdx.x == 0) {
      wait_flag(q, ep, blk_flag(q, a, w, s, f, jp));
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kbn * nrhs; idx += kSweepThreads) {
      const int col = idx / kbn, r = kb + idx - col * kbn;
      X[col * m + r] = ld_ag(Y + (int64_t)col * a.N + pb + r);
    }
    __syncthreads();
    bwd_tile(lt, X, red, m, kb, kb + kbn, nrhs);
    __syncthreads();
    for (int idx = threadIdx.x; idx < kn * nrhs; idx += kSweepThreads) {
      const int col = idx / kn, jj2 = idx - col * kn;
      const C* rr = red + col * kNQ * kBW + jj2;
      C acc = czero<C>();
#pragma unroll
      for (int qq = 0; qq < kNQ; ++qq) acc = cadd(acc, rr[qq * kBW]);
      X[col * m + k0 + jj2] = csub(X[col * m + k0 + jj2], acc);
    }
  }
  __syncthreads();
  bwd_tile(li, X + k0, red, m, jj + 1, kn, nrhs);
  __syncthreads();
  double2* O = w.out + (int64_t)s * w.io_ld;
  for (int idx = threadIdx.x; idx < kn * nrhs; idx += kSweepThreads) {
    const int col = idx / kn, jj = idx - col * kn;
    const C* rr = red + col * kNQ * kBW + jj;
    C x = X[col * m + k0 + jj];
#pragma unroll
    for (int qq = 0; qq < kNQ; ++qq) x = cadd(x, rr[qq * kBW]);
    st_ag(Y + (int64_t)col * a.N + pb + k0 + jj, x);
    double2* o = O + (int64_t)col * a.N + a.perm[pb + k0 + jj];
    const double2 xv = to_d2(x);
    *o = w.accumulate ? dadd(*o, xv) : xv;
  }
}

// One chunk of kChunkRows update rows R = [r0, r0 + nr) of a split front in
// the backward sweep: the partial column sums P_j[c] = sum_{r in R} L[r][c]
// x_r for all pivot columns c, x_r from the solution of the ancestors (in y),
// stored for the front's pivot item.  Lanes are 16 columns x 4 row phases
// (16 cache lines per load instruction), 16 loads per thread in flight, the
// waves take 16-column groups; the row phases meet through lane exchanges.
template <typename R>
__device__ void bwd_chunk(const KArgs& a, const SweepArgs& w, int s, int f, int j, unsigned char* smem) {
  typedef typename Cx<R>::T C;
  static_assert(kChunkRows == 64, "four row phases of sixteen rows");
  const int p = a.npiv[f], u = a.nupd[f], m = p + u;
  const int r0 = p + kChunkRows * j, nr = min(kChunkRows, m - r0);
  const int nrhs = w.nrhs;
  C* X = reinterpret_cast<C*>(smem);  // nrhs x kChunkRows
  const C* L = (const C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  const C* Y = (const C*)w.y + (int64_t)s * nrhs * a.N;
  const int32_t* ui = a.upd_idx + a.upd_ptr[f];
  for (int idx = threadIdx.x; idx < kChunkRows * nrhs; idx += kSweepThreads) {
    const int col = idx / kChunkRows, r = idx - col * kChunkRows;
    X[idx] = r < nr ? ld_ag(Y + (int64_t)col * a.N + ui[r0 - p + r]) : czero<C>();
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, q4 = lane >> 4;
  C* PB = (C*)w.pv + (int64_t)s * nrhs * w.part_total + w.part_base[f] + (int64_t)j * p;
  for (int c0 = 16 * wave; c0 < p; c0 += 16 * kSW) {
    const int c = c0 + (lane & 15);
    const bool cok = c < p;
    // one pointer per lane and immediate offsets: with the row indices
    // q4 + 4t as 64-bit values, the compiler hoisted all sixteen out of the
    // persistent loop, spilled them, and waited for each reload (and so for
    // every load already in flight) before the next load
    const C* Lq = L + (int64_t)(cok ? c : 0) * m + r0 + q4;
    C l[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) l[t] = cok && q4 + 4 * t < nr ? Lq[4 * t] : czero<C>();
    for (int col = 0; col < nrhs; ++col) {
      C acc = czero<C>();
#pragma unroll
      for (int t = 0; t < 16; ++t) acc = cadd(acc, cmul(l[t], X[col * kChunkRows + q4 + 4 * t]));
      acc = cadd(acc, shfl_xor_c(acc, 16));
      acc = cadd(acc, shfl_xor_c(acc, 32));
      if (lane < 16 && cok) st_ag(PB + (int64_t)col * w.part_total + c, acc);
    }
  }
}

// Forward sweep: items (front, part) in level order (leaves first), a front's
// pivot part before its update-row chunks; each waits for the children.
template <typename R>
__global__ __launch_bounds__(kSweepThreads) void k_fwd_sweep(KArgs a, SweepArgs w, Queue q, const int32_t* items) {
  if (done(w.flag)) return;
  sweep_status(w);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int sh;
  const int ep = launch_epoch(q);
  for (;;) {
    const int t = claim(q, &sh);
    if (t >= q.ntasks) break;
    const int it = t / a.nsys, s = t % a.nsys;
    const int f = items[2 * it], part = items[2 * it + 1];
    if (q.wait) {
      sweep_wait_children(q, ep, a, w, s, f, threadIdx.x, kSweepThreads);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      __syncthreads();
    }
    trace_mark(q, t, 1);
    if (part < 0 && w.blk_base[f] >= 0) {
      const int j = -1 - part;
      fwd_piv_block<R>(a, w, q, ep, s, f, j, smem_raw);
      publish(q, ep, (int64_t)a.nsys * (a.nfronts + w.nchunk) + (int64_t)s * w.nblk + w.blk_base[f] + j);
      // the front's own flag once its last block is done (every earlier block was waited for)
      if (j == (a.npiv[f] + kBW - 1) / kBW - 1 && threadIdx.x == 0)
        __hip_atomic_store(q.done + (int64_t)s * a.nfronts + f, ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (part < 0) {
      fwd_front<R>(a, w, s, f, w.nch[f] > 0, smem_raw);
      publish(q, ep, (int64_t)s * a.nfronts + f);
    } else {
      fwd_chunk<R>(a, w, q, ep, s, f, part, smem_raw);
      publish(q, ep, (int64_t)a.nsys * a.nfronts + (int64_t)s * w.nchunk + w.chunk_base[f] + part);
    }
    trace_mark(q, t, 2);
  }
  leave(q, ep);
}

// Backward sweep: items (front, part) in reverse level order (root first), a
// front's update-row chunks before its pivot part.  Chunks and unsplit fronts
// wait for the parent; the pivot part of a split front waits for its chunks.
template <typename R>
__global__ __launch_bounds__(kSweepThreads) void k_bwd_sweep(KArgs a, SweepArgs w, Queue q, const int32_t* items) {
  if (done(w.flag)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int sh;
  const int ep = launch_epoch(q);
  const int F = a.nfronts;
  for (;;) {
    const int t = claim(q, &sh);
    if (t >= q.ntasks) break;
    const int it = t / a.nsys, s = t % a.nsys;
    const int f = items[2 * it], part = items[2 * it + 1];
    const int nc = w.nch[f];
    if (q.wait) {
      if (threadIdx.x == 0) {
        if (part >= 0 || nc == 0) sweep_wait_parent(q, ep, a, w, s, f);
      }
      // the chunks of a split front, one thread each
      if (part < 0)
        for (int j = threadIdx.x; j < nc; j += kSweepThreads) wait_flag(q, ep, chunk_flag(q, a, w, s, f, j));
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      __syncthreads();
    }
    trace_mark(q, t, 1);
    if (part < 0 && w.blk_base[f] >= 0) {
      const int j = -1 - part;
      bwd_piv_block<R>(a, w, q, ep, s, f, j, nc, smem_raw);
      publish(q, ep, (int64_t)a.nsys * (F + w.nchunk) + (int64_t)s * w.nblk + w.blk_base[f] + j);
      // block 0 waited for every other block: the front is done
      if (j == 0 && threadIdx.x == 0)
        __hip_atomic_store(q.done + (int64_t)s * F + f, ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (part < 0) {
      bwd_front<R>(a, w, s, f, nc, smem_raw);
      publish(q, ep, (int64_t)s * F + f);
    } else {
      bwd_chunk<R>(a, w, s, f, part, smem_raw);
      publish(q, ep, (int64_t)a.nsys * F + (int64_t)s * w.nchunk + w.chunk_base[f] + part);
    }
    trace_mark(q, t, 2);
  }
  leave(q, ep);
}

// ---------------------------------------------------------------------------
// Sweeps over the bottom levels: one wavefront per front.  Those fronts are
// small (p <= kBW pivots, a few dozen rows), so a whole workgroup per front
// would leave most threads idle behind its barriers and run too few fronts at
// once.  Here each of the four waves of a workgroup takes one front of a
// four-item claim (one atomic per four fronts), lane = row, no workgroup
// barrier inside a front; the wave's own LDS slice holds the front vector.
// ---------------------------------------------------------------------------
// Loads in flight per lane in the wave sweeps: fewer than in the workgroup
// sweeps, so that four waves per SIMD stay resident (128 registers).
template <typename R> constexpr int kWaveBatch = sizeof(R) == 8 ? 4 : 8;


__device__ __forceinline__ void trace_wave(const Queue& q, int t, int slot) {
  if (q.trace && (threadIdx.x & 63) == 0 && t < q.ntasks) {
    q.trace[4 * (int64_t)t + slot] = (long long)wall_clock64();
    if (slot == 0) q.trace[4 * (int64_t)t + 3] = blockIdx.x;
  }
}


// Forward sweep of one small front by one wave (panel: D on the diagonal, the
// unit-lower L below).  V = [rhs_p; 0] + the children's update vectors is
// gathered into the wave's LDS; z = L11^-1 V_p by forward substitution with
// lane = row: lane i keeps its running value and, at step j, takes z_j from
// lane j (a register broadcast) times its own L_ij, loaded kWaveBatch columns
// at a time ahead of use; then V_u -= L21 z (lane = row, all loads
// independent), y_p = D^-1 z and the update vector is V_u.
template <typename R>
__device__ void fwd_front_wave(const KArgs& a, const SweepArgs& w, int s, int f, typename Cx<R>::T* V, int ldv) {
  typedef typename Cx<R>::T C;
  constexpr int WB = kWaveBatch<R>;
  constexpr int WB1 = 2 * WB;  // the merged pass: twice the batch
  const int lane = threadIdx.x & 63;
  const int p = a.npiv[f], u = a.nupd[f], m = p + u, pb = a.pbeg[f];
  const int nrhs = w.nrhs;
  const C* L = (const C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  C* Y = (C*)w.y + (int64_t)s * nrhs * a.N;
  C* W = (C*)w.wv + (int64_t)s * nrhs * a.sum_u;
  const double2* B = w.src + (int64_t)s * w.io_ld;
  const int cb = a.child_ptr[f], nch = a.child_ptr[f + 1] - cb;
  const int32_t* g = a.gmap + a.gmap_ptr[f];
  for (int col = 0; col < nrhs; ++col) {
    C* Vc = V + col * ldv;
#pragma unroll 1
    for (int r = lane; r < m; r += 64) {
      int gr[2];
      int64_t base[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        gr[k] = k < nch ? g[k * m + r] : -1;
        base[k] = k < nch ? (int64_t)col * a.sum_u + a.upd_ptr[a.child_list[cb + k]] : 0;
      }
      double2 bv = make_double2(0.0, 0.0);
      if (r < p) bv = B[(int64_t)col * a.N + a.perm[pb + r]];
      C cv[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) cv[k] = gr[k] >= 0 ? ld_ag(W + base[k] + gr[k]) : czero<C>();
      if (r < p && w.scale_src) bv = dmul(bv, sym_scale(a, s, a.perm[pb + r]));
      C v = cadd(from_d2<C>(bv), cadd(cv[0], cv[1]));
      for (int k = 2; k < nch; ++k) {
        const int gk = g[k * m + r];
        if (gk >= 0) v = cadd(v, ld_ag(W + (int64_t)col * a.sum_u + a.upd_ptr[a.child_list[cb + k]] + gk));
      }
      Vc[r] = v;
    }
  }
  wave_sync();
  const C dl = lane < p ? L[(int64_t)lane * m + lane] : czero<C>();
  if (m <= 128) {
    // One right-looking pass over the pivot columns for the pivot and the
    // update rows together (lane = row, rows lane and lane + 64): at step j,
    // z_j is final in lane j and every later row takes -L_ij z_j.  The pivot
    // rows end as z, the update rows as V_u - L21 z.
    const int r1 = lane + 64;
    const bool two = m > 64;
    for (int col = 0; col < nrhs; ++col) {
      C* Vc = V + col * ldv;
      C v0 = lane < m ? Vc[lane] : czero<C>();
      C v1 = two && r1 < m ? Vc[r1] : czero<C>();
#pragma unroll 1
      for (int j0 = 0; j0 < p; j0 += WB1) {
        C e0[WB1], e1[WB1];
#pragma unroll
        for (int t = 0; t < WB1; ++t) {
          const int j = j0 + t;
          e0[t] = j < p && j < lane && lane < m ? L[(int64_t)j * m + lane] : czero<C>();
          e1[t] = two && j < p && r1 < m ? L[(int64_t)j * m + r1] : czero<C>();
        }
#pragma unroll
        for (int t = 0; t < WB1; ++t) {
          const int j = j0 + t;
          if (j < p) {
            const C zj = bcast_c(v0, j);
            v0 = cfms(v0, e0[t], zj);
            if (two) v1 = cfms(v1, e1[t], zj);
          }
        }
      }
      C* Wf = W + (int64_t)col * a.sum_u + a.upd_ptr[f];
      if (lane < p) Y[(int64_t)col * a.N + pb + lane] = cmul(v0, cinv(dl));
      else if (lane < m) st_ag(Wf + (lane - p), v0);
      if (two && r1 < m) st_ag(Wf + (r1 - p), v1);
    }
    return;
  }
  for (int col = 0; col < nrhs; ++col) {
    C* Vc = V + col * ldv;
    // z = L11^-1 V_p, lane = row
    C zi = lane < p ? Vc[lane] : czero<C>();
#pragma unroll 1
    for (int j0 = 0; j0 < p; j0 += WB) {
      C e[WB];
#pragma unroll
      for (int t = 0; t < WB; ++t) {
        const int j = j0 + t;
        e[t] = j < lane && lane < p ? L[(int64_t)j * m + lane] : czero<C>();
      }
#pragma unroll
      for (int t = 0; t < WB; ++t) {
        const int j = j0 + t;
        if (j < p) zi = cfms(zi, e[t], bcast_c(zi, j));
      }
    }
    wave_sync();
    if (lane < p) Vc[lane] = zi;
    wave_sync();
    // V_u -= L21 z: rows p + lane, p + lane + 64, ...
#pragma unroll 1
    for (int r = p + lane; r < m; r += 64) {
      C acc = czero<C>();
#pragma unroll 1
      for (int j0 = 0; j0 < p; j0 += WB) {
        C e[WB];
#pragma unroll
        for (int t = 0; t < WB; ++t) e[t] = j0 + t < p ? L[(int64_t)(j0 + t) * m + r] : czero<C>();
#pragma unroll
        for (int t = 0; t < WB; ++t) acc = cadd(acc, cmul(e[t], j0 + t < p ? Vc[j0 + t] : czero<C>()));
      }
      st_ag(W + (int64_t)col * a.sum_u + a.upd_ptr[f] + (r - p), csub(Vc[r], acc));
    }
    if (lane < p) Y[(int64_t)col * a.N + pb + lane] = cmul(zi, cinv(dl));
    wave_sync();
  }
}

// Backward sweep of one small front by one wave: X = [y_p; x_u] in LDS;
// lane = column j: t_j = sum_{i>=p} L[i][j] x_i down the contiguous column,
// then back substitution x_j = y_j - t_j - sum_{j<i<p} L[i][j] x_i with x_i
// taken from lane i (a register broadcast) as soon as it is final, the
// column's L[i][j] loaded kWaveBatch rows at a time ahead of use.
template <typename R>
__device__ void bwd_front_wave(const KArgs& a, const SweepArgs& w, int s, int f, typename Cx<R>::T* X, int ldv) {
  typedef typename Cx<R>::T C;
  constexpr int WB = 2 * kWaveBatch<R>;  // two waves per SIMD: twice the batch
  const int lane = threadIdx.x & 63;
  const int p = a.npiv[f], u = a.nupd[f], m = p + u, pb = a.pbeg[f];
  const int nrhs = w.nrhs;
  const C* L = (const C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  C* Y = (C*)w.y + (int64_t)s * nrhs * a.N;
  const int32_t* ui = a.upd_idx + a.upd_ptr[f];
  const int prow = lane < p ? a.perm[pb + lane] : 0;  // grid cell of pivot row lane
  for (int col = 0; col < nrhs; ++col)
#pragma unroll 1
    for (int r = lane; r < m; r += 64)
      X[col * ldv + r] = ld_ag(Y + (int64_t)col * a.N + (r < p ? pb + r : ui[r - p]));
  wave_sync();
  const C* Lc = L + (int64_t)min(lane, max(p - 1, 0)) * m;
  // t_j = sum_{i >= p} L_ij x_i on G lanes per column, so that a front of few
  // pivots still keeps the wave's lanes loading: lane j + k p (k < G) takes
  // the rows p + k, p + k + G, ... of column j; lane j then adds the G sums.
  const int G = p > 0 && u > 0 ? max(1, min(64 / p, u)) : 1;
  const int jc = p > 0 ? lane % p : 0, kc = p > 0 ? lane / p : G;
  const int nr = kc < G ? (u - kc + G - 1) / G : 0;  // rows of this lane
  const int nr0 = (u + G - 1) / G;                    // rows of lane k = 0, the most
  // Loads past a lane's last row re-read that row (row p of column 0 for a
  // lane without rows; it exists whenever u > 0) and count as zero, so a batch
  // is one block of loads off a uniform base with 32-bit lane offsets.
  const int nrl = max(nr - 1, 0);
  const char* Lt = reinterpret_cast<const char*>(L + p);
  const uint32_t lofs = nr > 0 ? (uint32_t)(jc * m + kc) * (uint32_t)sizeof(C) : 0u;
  double2* O = w.out + (int64_t)s * w.io_ld;
  for (int col = 0; col < nrhs; ++col) {
    const C* Xc = X + col * ldv;
    const C* Xt = Xc + p + (nr > 0 ? kc : 0);
    C acc = czero<C>();
#pragma unroll 1
    for (int r0 = 0; r0 < nr0; r0 += WB) {
      C e[WB];
#pragma unroll
      for (int t = 0; t < WB; ++t)
        e[t] = *reinterpret_cast<const C*>(Lt + (uint32_t)(min(r0 + t, nrl) * G) * (uint32_t)sizeof(C) + lofs);
#pragma unroll
      for (int t = 0; t < WB; ++t) {
        const C prod = cmul(e[t], Xt[min(r0 + t, nrl) * G]);
        acc = r0 + t < nr ? cadd(acc, prod) : acc;
      }
    }
    for (int k = 1; k < G; ++k) {
      const C o = shfl_c(acc, min(lane + k * p, 63));
      acc = lane < p ? cadd(acc, o) : acc;
    }
    C xj = lane < p ? csub(Xc[lane], acc) : czero<C>();
    // rows i = p-1 down to 1: lane i's value is final, lanes j < i take it
#pragma unroll 1
    for (int i0 = p - 1; i0 > 0; i0 -= WB) {
      C e[WB];
#pragma unroll
      for (int t = 0; t < WB; ++t) {
        const int i = i0 - t;
        // a clamped row lies below the diagonal of the lane's column
        const C l = Lc[min(max(i, lane + 1), m - 1)];
        e[t] = i > lane && lane < p ? l : czero<C>();
      }
#pragma unroll
      for (int t = 0; t < WB; ++t) {
        const int i = i0 - t;
        if (i > 0) xj = cfms(xj, e[t], bcast_c(xj, i));
      }
    }
    if (lane < p) {
      st_ag(Y + (int64_t)col * a.N + pb + lane, xj);
      double2* o = O + (int64_t)col * a.N + prow;
      const double2 xv = to_d2(xj);
      *o = w.accumulate ? dadd(*o, xv) : xv;
    }
  }
  wave_sync();
}

// Wave-item launches: items claimed four at a time, wave w of the workgroup
// takes item t0 + w.  Waves of one workgroup only meet at the claim, so a wave
// may wait for a front that another wave of the same workgroup processes.
__device__ __forceinline__ int claim4(const Queue& q, int* sh) {
  __syncthreads();
  if (threadIdx.x == 0) *sh = atomicAdd(&q.counter[0], 4);
  __syncthreads();
  return *sh;
}

__device__ __forceinline__ void publish_wave(const Queue& q, int ep, int64_t idx) {
  drain_stores();
  if ((threadIdx.x & 63) == 0) __hip_atomic_store(q.done + idx, ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Items: seq[iptr[i] .. iptr[i+1]) -- a subtree of the bottom levels,
// children before parents, or a single front.  The wave sweeps the item's
// fronts in turn; the dependency flags are only used at the item's boundary
// (a single front waits, a subtree's root publishes).
template <typename R>
__global__ __launch_bounds__(kThreads, 4) void k_fwd_sweep_waves(KArgs a, SweepArgs w, Queue q, const int32_t* seq,
                                                                 const int32_t* iptr) {
  typedef typename Cx<R>::T C;
  if (done(w.flag)) return;
  sweep_status(w);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int sh;
  const int ep = launch_epoch(q);
  const int wave = threadIdx.x >> 6;
  C* V = reinterpret_cast<C*>(smem_raw) + wave * w.nrhs * w.wave_ld;
  for (;;) {
    const int t0 = claim4(q, &sh);
    if (t0 >= q.ntasks) break;
    const int t = t0 + wave;
    if (t < q.ntasks) {
      trace_wave(q, t, 0);
      const int it = t / a.nsys, s = t % a.nsys;
      const int e0 = iptr[it], e1 = iptr[it + 1];
      for (int e = e0; e < e1; ++e) {
        const int f = seq[e];
        // A multi-front item holds every descendant of its root, swept just
        // before by this wave: program order makes their update vectors
        // visible, so only a single front waits and only the root publishes.
        if (q.wait && e1 - e0 == 1) sweep_wait_children(q, ep, a, w, s, f, threadIdx.x & 63, 64);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (e == e0) trace_wave(q, t, 1);
        fwd_front_wave<R>(a, w, s, f, V, w.wave_ld);
        if (e == e1 - 1) publish_wave(q, ep, (int64_t)s * a.nfronts + f);
        else __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      }
      trace_wave(q, t, 2);
    }
  }
  leave(q, ep);
}

// The same items in reverse, each swept parents first.
template <typename R>
__global__ __launch_bounds__(kThreads, 4) void k_bwd_sweep_waves(KArgs a, SweepArgs w, Queue q, const int32_t* seq,
                                                                 const int32_t* iptr) {
  typedef typename Cx<R>::T C;
  if (done(w.flag)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int sh;
  const int ep = launch_epoch(q);
  const int wave = threadIdx.x >> 6;
  C* X = reinterpret_cast<C*>(smem_raw) + wave * w.nrhs * w.wave_ld;
  for (;;) {
    const int t0 = claim4(q, &sh);
    if (t0 >= q.ntasks) break;
    const int t = t0 + wave;
    if (t < q.ntasks) {
      trace_wave(q, t, 0);
      const int it = q.ntasks / a.nsys - 1 - t / a.nsys, s = t % a.nsys;
      const int e0 = iptr[it], e1 = iptr[it + 1];
      for (int e = e1 - 1; e >= e0; --e) {
        const int f = seq[e];
        // Below the root of a multi-front item every parent is the item's own,
        // swept just before by this wave; no other item waits for its fronts.
        if (q.wait && e == e1 - 1 && (threadIdx.x & 63) == 0) sweep_wait_parent(q, ep, a, w, s, f);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (e == e1 - 1) trace_wave(q, t, 1);
        bwd_front_wave<R>(a, w, s, f, X, w.wave_ld);
        if (e1 - e0 == 1) publish_wave(q, ep, (int64_t)s * a.nfronts + f);
        else __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      }
      trace_wave(q, t, 2);
    }
  }
  leave(q, ep);
}

// ---------------------------------------------------------------------------
// FP64 refinement: r = rhs_sym - (SA) x with per-workgroup partial norms
// (k_residual, one cell per thread), then one workgroup sums them in a fixed
// order, records the relative residual and raises the converged flag or the
// failure bits (k_residual_norm).  Two launches and no completion counter:
// a counter that every workgroup increments serialises thousands of atomics.
// ---------------------------------------------------------------------------
struct ResArgs {
  const double2* rhs;
  const double2* x;
  double2* res;
  double* partial;
  const int* flag;
  double tol;
  int32_t nrhs, scale_rhs, step, last;
};

__global__ __launch_bounds__(kThreads) void k_residual(KArgs a, ResArgs ra) {
  if (done(ra.flag)) return;
  const int col = blockIdx.y;
  const int s = col / ra.nrhs;
  const double2* X = ra.x + (int64_t)col * a.N;
  const double2* B = ra.rhs + (int64_t)col * a.N;
  double2* Rv = ra.res + (int64_t)col * a.N;
  double rr = 0.0, bb = 0.0;
  const int nx = a.nx, ny = a.ny;
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
       n += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % nx), j = (int)(n / nx);
    const Stencil S = stencil_at(a, s, (int)n);
    double2 ax = dmul(S.diag, X[n]);
    if (i > 0) ax = dadd(ax, dmul(S.c[0], X[n - 1]));
    if (i < nx - 1) ax = dadd(ax, dmul(S.c[1], X[n + 1]));
    if (j > 0) ax = dadd(ax, dmul(S.c[2], X[n - nx]));
    if (j < ny - 1) ax = dadd(ax, dmul(S.c[3], X[n + nx]));
    double2 b = B[n];
    if (ra.scale_rhs) b = dmul(b, sym_scale(a, s, (int)n));
    const double2 r = dsub(b, ax);
    Rv[n] = r;
    rr += r.x * r.x + r.y * r.y;
    bb += b.x * b.x + b.y * b.y;
  }
  __shared__ double red[2][kThreads];
  red[0][threadIdx.x] = rr;
  red[1][threadIdx.x] = bb;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* pp = ra.partial + ((int64_t)col * gridDim.x + blockIdx.x) * 2;
    pp[0] = red[0][0];
    pp[1] = red[1][0];
  }
}

// One workgroup: per column, thread t sums the partials of workgroups t,
// t + kThreads, ..., then a fixed tree (the result is reproducible).
__global__ __launch_bounds__(kThreads) void k_residual_norm(KArgs a, ResArgs ra, int nblk, int ncols) {
  if (done(ra.flag)) return;
  __shared__ double red[2][kThreads];
  double mx = 0.0;
  int anybad = 0;
  for (int c = 0; c < ncols; ++c) {
    double r2 = 0.0, b2 = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) {
      r2 += ra.partial[((int64_t)c * nblk + b) * 2];
      b2 += ra.partial[((int64_t)c * nblk + b) * 2 + 1];
    }
    __syncthreads();
    red[0][threadIdx.x] = r2;
    red[1][threadIdx.x] = b2;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) {
        red[0][threadIdx.x] += red[0][threadIdx.x + o];
        red[1][threadIdx.x] += red[1][threadIdx.x + o];
      }
      __syncthreads();
    }
    const double rel = red[1][0] > 0 ? sqrt(red[0][0] / red[1][0]) : sqrt(red[0][0]);
    if (!(rel <= DBL_MAX)) anybad = 1;
    mx = fmax(mx, rel);
  }
  if (threadIdx.x == 0) {
    DevStatus* st = a.st;
    st->ir_rel = anybad ? NAN : mx;
    st->ir_steps = ra.step;
    if (anybad) {
      st->nonfinite = 1;
      st->ir_failed = 1;
      st->ir_flag = 1;
    } else if (mx <= ra.tol) {
      st->ir_flag = 1;
    } else if (ra.last) {
      st->ir_failed = 1;
    }
  }
}

__global__ void k_ir_begin(DevStatus* st) {
  st->ir_flag = 0;
  st->ir_steps = 0;
  st->ir_failed = 0;
  st->ir_rel = -1.0;
}

__global__ void k_ir_end(DevStatus* st, int mode, int with_ir) {
  if (mode == 0) {
    st->ir_steps_solve = with_ir ? st->ir_steps : 0;
    st->rel_solve = with_ir ? st->ir_rel : -1.0;
    st->ir_failed_solve = with_ir ? st->ir_failed : 0;
  } else {
    st->ir_steps_adj = with_ir ? st->ir_steps : 0;
    st->rel_adj = with_ir ? st->ir_rel : -1.0;
    st->ir_failed_adj = with_ir ? st->ir_failed : 0;
  }
}

// lam = S lam' ; grad_n (+)= -2 w^2 sum_rhs Re(lam_n x_n), one system per grid row
// dF/deps_n of system s summed over the right-hand sides, from x and the
// symmetric adjoint solution lsym (lambda = S lsym); lambda goes to lam_out
// when asked for.
//   TM: -2 omega^2 Re(lambda_n x_n)                                  (Eq. 3)
//   TE: eps_n enters the four faces of cell n.  Through a face shared with
//       cell m it contributes -(c / eps_f) Re((x_m - x_n)(lsym_m - lsym_n)),
//       c the face's coupling in S*A and eps_f its permittivity (half of
//       the face's -2 Re(lambda^T dA/deps_f x), the face permittivity being
//       the mean of its two cells); through a grid-edge face, whose
//       permittivity is the cell's own, -(2 c / eps_f) Re(x_n lsym_n).
__device__ __forceinline__ double grad_cell(const KArgs& a, int s, int64_t n, const double2* x,
                                            const double2* lsym, int nrhs, double2* lam_out) {
  const double2 S = sym_scale(a, s, (int)n);
  double g = 0.0;
  if (!a.te) {
    const double w = a.omega[s];
    for (int r = 0; r < nrhs; ++r) {
      const int64_t o = ((int64_t)s * nrhs + r) * a.N + n;
      const double2 lam = dmul(S, lsym[o]);
      if (lam_out) lam_out[o] = lam;
      const double2 xv = x[o];
      g += lam.x * xv.x - lam.y * xv.y;
    }
    return -2.0 * w * w * g;
  }
  const Stencil st = stencil_at(a, s, (int)n);
  double ef[4];
  face_eps(a, s, (int)n, ef);
  const int nx = a.nx, i = (int)(n % nx), j = (int)(n / nx);
  const bool in[4] = {i > 0, i < nx - 1, j > 0, j < a.ny - 1};
  const int64_t step[4] = {-1, 1, -(int64_t)nx, (int64_t)nx};
  for (int r = 0; r < nrhs; ++r) {
    const int64_t o = ((int64_t)s * nrhs + r) * a.N + n;
    const double2 xn = x[o], ln = lsym[o];
    if (lam_out) lam_out[o] = dmul(S, ln);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double2 dx = in[k] ? dsub(x[o + step[k]], xn) : make_double2(-xn.x, -xn.y);
      const double2 dl = in[k] ? dsub(lsym[o + step[k]], ln) : make_double2(-ln.x, -ln.y);
      const double2 cw = make_double2(st.c[k].x / ef[k], st.c[k].y / ef[k]);
      const double2 p = dmul(cw, dmul(dx, dl));
      g -= (in[k] ? 1.0 : 2.0) * p.x;
    }
  }
  return g;
}

__global__ __launch_bounds__(kThreads) void k_gradient(KArgs a, const double2* x, const double2* lsym,
                                                        int nrhs, double2* lam_out, double* grad,
                                                        int accumulate) {
  const int s = blockIdx.y;
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
       n += (int64_t)gridDim.x * blockDim.x) {
    const double gv = grad_cell(a, s, n, x, lsym, nrhs, lam_out);
    double* gp = grad + (int64_t)s * a.N + n;
    *gp = accumulate ? *gp + gv : gv;
  }
}

// Sum over systems in fixed order (FDFD_GRAD_SUM_SYSTEMS).
__global__ __launch_bounds__(kThreads) void k_gradient_sum(KArgs a, const double2* x, const double2* lsym,
                                                            int nrhs, double2* lam_out, double* grad,
                                                            int accumulate) {
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
       n += (int64_t)gridDim.x * blockDim.x) {
    double tot = 0.0;
    for (int s = 0; s < a.nsys; ++s) tot += grad_cell(a, s, n, x, lsym, nrhs, lam_out);
    grad[n] = accumulate ? grad[n] + tot : tot;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
KArgs make_args(Plan& P) {
  KArgs a;
  a.pbeg = P.t.pbeg;
  a.npiv = P.t.npiv;
  a.nupd = P.t.nupd;
  a.child_ptr = P.t.child_ptr;
  a.child_list = P.t.child_list;
  a.upd_ptr = P.t.upd_ptr;
  a.upd_idx = P.t.upd_idx;
  a.gmap = P.t.gmap;
  a.nbr_row = P.t.nbr_row;
  a.perm = P.t.perm;
  a.iperm = P.t.iperm;
  a.parent = P.t.parent;
  a.height = P.t.height;
  a.fac_off = P.t.fac_off;
  a.upd_off = P.t.upd_off;
  a.gmap_ptr = P.t.gmap_ptr;
  a.nx = P.an.nx;
  a.ny = P.an.ny;
  a.N = (int32_t)P.an.N;
  a.nsys = P.desc.nsys;
  a.fac_total = P.an.fac_total;
  a.upd_total = P.an.upd_total;
  a.sum_u = P.an.upd_ptr.back();
  a.pml = P.pml;
  a.eps = P.eps;
  a.omega = P.omega;
  a.fac = P.fac;
  a.upd = P.upd;
  a.st = P.status;
  // pivot threshold tau * ||SA||_max, by default tau = sqrt(unit roundoff)
  a.tau = P.pivot_tau;
  a.nfronts = P.an.nfronts;
  a.te = (P.desc.flags & FDFD_POL_TE) ? 1 : 0;
  a.below_done = 0;
  return a;
}

inline unsigned grid1d(int64_t n, int64_t cap = 2048) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

Queue make_queue(Plan& P, int ntasks, int wait, int trace_kind = -1) {
  Queue q;
  q.counter = P.counters;
  q.done = P.done;
  q.st = P.status;
  q.trace = nullptr;
  if (trace_kind >= 0 && P.trace_buf[trace_kind] && ntasks <= P.trace_cap[trace_kind]) {
    q.trace = P.trace_buf[trace_kind];
    P.trace_n[trace_kind] = ntasks;
  }
  q.ntasks = ntasks;
  q.wait = wait;
  return q;
}

// FDFD_PROFILE: brackets one launch with events and records its algorithmic work.
struct Prof {
  Plan& P;
  hipStream_t st;
  int cls;
  double bytes, flops;
  hipEvent_t e0 = nullptr;
  Prof(Plan& P_, hipStream_t st_, int cls_, double b, double f) : P(P_), st(st_), cls(cls_), bytes(b), flops(f) {
    if (P.profile) {
      e0 = profile_event(P);
      (void)hipEventRecord(e0, st);
    }
  }
  ~Prof() {
    if (!e0) return;
    hipEvent_t e1 = profile_event(P);
    (void)hipEventRecord(e1, st);
    P.pending.push_back(PendingTiming{cls, e0, e1, bytes, flops});
  }
};

// Workgroups of a persistent launch: enough to fill every CU at the occupancy
// the LDS footprint allows, never more than the items.
unsigned persistent_grid(const Plan& P, size_t lds, int ntasks) {
  int per_cu = lds > 0 ? (int)(P.lds_limit / lds) : 8;
  per_cu = per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu);
  int g = P.n_cu * per_cu;
  if (g > ntasks) g = ntasks;
  return (unsigned)(g < 1 ? 1 : g);
}

// LDS of the task-graph kernel: the diagonal task's block and pivots, or the
// two 16-deep operand panels of the tile products, whichever is larger.
size_t tile_lds(const Plan& P) {
  return tile_lds_entries() * P.csize;
}

// Workgroups of a persistent launch: as many as can be resident at once for
// this kernel and LDS footprint, never more than the work items.
unsigned resident_grid(const Plan& P, const void* fn, size_t lds, int nitems, int threads = kThreads) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int g = P.n_cu * per_cu;
  if (g > nitems) g = nitems;
  return (unsigned)(g < 1 ? 1 : g);
}

template <typename R>
hipError_t refactor_impl(Plan& P, const double* eps, int64_t eps_stride, hipStream_t st) {
  const KArgs a = make_args(P);
  const int nsys = P.desc.nsys;
  Omegas om;
  for (int s = 0; s < kMaxSys; ++s) om.w[s] = s < nsys ? P.omega_host[s] : 0.0;
  {
    Prof pr(P, st, KC_SETUP, 24.0 * P.an.N * nsys, 0.0);
    hipLaunchKernelGGL(k_copy_eps, dim3(grid1d(P.an.N, 1024), nsys), dim3(kThreads), 0, st, a, eps,
                       eps_stride);
    hipLaunchKernelGGL(k_setup, dim3(nsys), dim3(kThreads), 0, st, a, om, P.desc.npml_x,
                       P.desc.npml_y);
    hipLaunchKernelGGL(k_anorm, dim3(grid1d(P.an.N, 512), nsys), dim3(kThreads), 0, st, a);
  }
  const int32_t* lf = P.t.level_fronts;
  // the small levels at the bottom of the tree, one launch per level: one
  // wavefront per front where a front fits one, else one workgroup per front
  if (P.small_prefix > 0) {
    // the bottom levels whose fronts fit one wavefront: one launch per level
    const int nwl = (int)P.wave_front_levels.size();
    for (int l = 0; l < nwl; ++l) {
      const LevelPlan& LP = P.levels[l];
      double fl = 0.0;
      for (int k = LP.first; k < LP.first + LP.count; ++k) fl += P.front_flops[P.an.level_fronts[k]];
      Prof pr(P, st, KC_FRONT_SMALL, 0.0, fl * nsys);
      const auto& WL = P.wave_front_levels[l];
      // fronts of up to 64 rows: four waves per workgroup; two rows per lane:
      // one wave per workgroup (its slice is larger; the LDS packs the CU)
      const int nitems = LP.count * nsys, wpg = WL.nr == 2 ? 1 : kThreads / 64;
      const dim3 grid((nitems + wpg - 1) / wpg), block(64 * wpg);
      const size_t lds = (size_t)wpg * WL.ldsw;
      const int32_t* ord = lf + LP.first;
      if (WL.nr == 1) {
        if (WL.pmax <= 8)
          hipLaunchKernelGGL((k_wave_fronts<R, 8, 1>), grid, block, lds, st, a, ord, nitems, WL.ldsw);
        else if (WL.pmax <= 16)
          hipLaunchKernelGGL((k_wave_fronts<R, 16, 1>), grid, block, lds, st, a, ord, nitems, WL.ldsw);
        else if (WL.pmax <= 24)
          hipLaunchKernelGGL((k_wave_fronts<R, 24, 1>), grid, block, lds, st, a, ord, nitems, WL.ldsw);
        else
          hipLaunchKernelGGL((k_wave_fronts<R, 40, 1>), grid, block, lds, st, a, ord, nitems, WL.ldsw);
      } else {
        if (WL.pmax <= 8)
          hipLaunchKernelGGL((k_wave_fronts<R, 8, 2>), grid, block, lds, st, a, ord, nitems, WL.ldsw);
        else
          hipLaunchKernelGGL((k_wave_fronts<R, 16, 2>), grid, block, lds, st, a, ord, nitems, WL.ldsw);
      }
    }
    // the other small levels: one launch per level, each with the LDS its
    // own largest front needs (the lower levels' small fronts then share a CU
    // several at a time), every child finished by an earlier launch
    for (int l = nwl; l < P.small_prefix; ++l) {
      const LevelPlan& LP = P.levels[l];
      KArgs as = a;
      as.below_done = l;
      const int n = LP.count * nsys;
      const Queue q = make_queue(P, n, 0, l == nwl ? 0 : -1);
      double fl = 0.0;
      for (int k = LP.first; k < LP.first + LP.count; ++k) fl += P.front_flops[P.an.level_fronts[k]];
      Prof pr(P, st, KC_FRONT_SMALL, 0.0, fl * nsys);
      const size_t lds = (LP.small_lds + 15) & ~size_t(15);
      hipLaunchKernelGGL(k_front_small<R>, dim3(resident_grid(P, (const void*)k_front_small<R>, lds, n)),
                         dim3(kThreads), lds, st, as, q, lf + LP.first);
    }
  }
  // every level above them: one persistent launch of the tile task graph
  if (P.ntile_tasks > 0) {
    const int64_t nstate = (int64_t)nsys * P.ntiles, ndone = (int64_t)nsys * P.an.nfronts;
    hipLaunchKernelGGL(k_tiles_reset, dim3(grid1d(nstate + ndone, 256)), dim3(kThreads), 0, st, P.tile_state,
                       nstate, P.tile_done, ndone);
    TileArgs ta;
    ta.tasks = P.t.tile_tasks;
    ta.state = P.tile_state;
    ta.done = P.tile_done;
    ta.tile_base = P.t.tile_base;
    ta.is_tiled = P.t.is_tiled;
    ta.ntiles = P.ntiles;
    const size_t lds = tile_lds(P);
    const int nt = P.ntile_tasks * nsys;
    Prof pr(P, st, KC_LARGE_TILES, 0.0, P.tiled_flops * nsys);
    hipLaunchKernelGGL(k_large_tiles<R>, dim3(persistent_grid(P, lds, nt)), dim3(kThreads), lds, st, a, ta,
                       make_queue(P, nt, 1, 1));
  }
  return hipGetLastError();
}

size_t sweep_lds(const Plan& P, int nrhs) {
  // forward: nrhs x 4 kRowStep partial sums + V; backward: nrhs x 4 kBW + X
  return ((size_t)4 * kRowStep * (nrhs > 1 ? nrhs : 1) + (size_t)P.an.max_front * nrhs) * P.csize;
}

// LDS of the wave-item sweeps: four waves, each with nrhs x wave_ld entries.
size_t sweep_wave_lds(const Plan& P, int nrhs) { return (size_t)4 * P.wave_ld * nrhs * P.csize; }


// Right-hand sides one sweep launch takes at once: the most whose LDS blocks
// fit (a front's right-hand-side block is held whole in LDS).
int sweep_group(const Plan& P, int nrhs) {
  const size_t lim = P.lds_limit - 512;
  int g = std::min(nrhs, P.rhs_cap);
  while (g > 1 && (sweep_lds(P, g) > lim || sweep_wave_lds(P, g) > lim)) --g;
  return g;
}

// One forward + backward sweep: dst (+)= (SA)^-1 (scale ? S : 1) src, over
// the columns in groups of sweep_group() (each group one forward and one
// backward pass over the factor, the work vectors laid out for the group).
// The bottom P.wave_levels levels run in the wave-item kernels (forward
// first, backward last), the levels above in the workgroup-per-front kernels.
template <typename R>
void sweep_cols(Plan& P, const SolveWork& wk, const KArgs& a, const double2* src, double2* dst, int64_t io_ld,
                int nrhs, int scale_in, int accumulate, const int* flag, hipStream_t st, int status_mode);

template <typename R>
void sweep(Plan& P, const SolveWork& wk, const KArgs& a, const double2* src, double2* dst, int nrhs, int scale_in,
           int accumulate, const int* flag, hipStream_t st, int status_mode = -1) {
  const int g = sweep_group(P, nrhs);
  const int64_t io_ld = (int64_t)nrhs * P.an.N;
  for (int c0 = 0; c0 < nrhs; c0 += g)
    sweep_cols<R>(P, wk, a, src + (int64_t)c0 * P.an.N, dst + (int64_t)c0 * P.an.N, io_ld, std::min(g, nrhs - c0),
                  scale_in, accumulate, flag, st, status_mode);
}

template <typename R>
void sweep_cols(Plan& P, const SolveWork& wk, const KArgs& a, const double2* src, double2* dst, int64_t io_ld,
                int nrhs, int scale_in, int accumulate, const int* flag, hipStream_t st, int status_mode) {
  const int nsys = P.desc.nsys;
  const size_t lds = sweep_lds(P, nrhs), wlds = sweep_wave_lds(P, nrhs);
  SweepArgs w;
  w.src = src;
  w.out = dst;
  w.io_ld = io_ld;
  w.y = wk.y;
  w.wv = wk.wv;
  w.flag = flag;
  w.nrhs = nrhs;
  w.scale_src = scale_in;
  w.accumulate = accumulate;
  w.st = P.status;
  w.status_mode = status_mode;
  w.wave_ld = P.wave_ld;
  w.items = P.t.fwd_items;
  w.nch = P.t.nch;
  w.chunk_base = P.t.chunk_base;
  w.zv = wk.zv;
  w.nchunk = P.nchunk;
  w.part_base = P.t.part_base;
  w.pv = wk.pv;
  w.part_total = P.part_total;
  w.blk_base = P.t.blk_base;
  w.nblk = P.nblk;
  const int nlev = (int)P.levels.size();
  const int lw = P.wave_levels;
  const int nlow = lw > 0 ? P.levels[lw - 1].first + P.levels[lw - 1].count : 0;
  const int nwi = P.wave_items;  // sweep items of those levels
  const int nhigh = P.an.nfronts - nlow;
  // algorithmic bytes: the lower-trapezoid factor once, the input vector read
  // in one precision and the output written in another
  const double vec_bytes = (double)P.an.N * nrhs * nsys * (16.0 + (double)P.csize);
  double low_bytes = 0.0;
  for (int l = 0; l < lw; ++l) low_bytes += P.levels[l].lbytes;
  const double fb_low = low_bytes * nsys + vec_bytes * nlow / P.an.nfronts;
  const double fb_high = (P.factor_lbytes - low_bytes) * nsys + vec_bytes * nhigh / P.an.nfronts;
  const void* fw = (const void*)k_fwd_sweep_waves<R>;
  const void* bw = (const void*)k_bwd_sweep_waves<R>;
  const void* fh = (const void*)k_fwd_sweep<R>;
  const void* bh = (const void*)k_bwd_sweep<R>;
  // forward: bottom levels, then the rest
  if (nlow > 0) {
    SweepArgs wl = w;
    wl.lev_lo = 0;
    wl.lev_hi = lw;
    const int n = nwi * nsys;
    Prof pr(P, st, KC_FWD_SWEEP, fb_low, 0.0);
    hipLaunchKernelGGL((k_fwd_sweep_waves<R>), dim3(resident_grid(P, fw, wlds, (n + 3) / 4)), dim3(kThreads), wlds,
                       st, a, wl, make_queue(P, n, 1, 2), P.t.wave_seq, P.t.wave_item_ptr);
    w.status_mode = -1;
  }
  if (nhigh > 0) {
    SweepArgs wh = w;
    wh.lev_lo = lw;
    wh.lev_hi = nlev;
    const int n = P.n_fwd_items * nsys;
    Prof pr(P, st, KC_FWD_SWEEP, fb_high, 0.0);
    hipLaunchKernelGGL((k_fwd_sweep<R>), dim3(resident_grid(P, fh, lds, n, kSweepThreads)), dim3(kSweepThreads), lds,
                       st, a, wh,
                       make_queue(P, n, 1, nlow > 0 || P.nchunk > 0 ? -1 : 2), P.t.fwd_items);
  }
  // backward: the top levels first
  if (nhigh > 0) {
    SweepArgs wh = w;
    wh.status_mode = -1;
    wh.lev_lo = lw;
    wh.lev_hi = nlev;
    const int n = P.n_bwd_items * nsys;
    Prof pr(P, st, KC_BWD_SWEEP, fb_high, 0.0);
    hipLaunchKernelGGL((k_bwd_sweep<R>), dim3(resident_grid(P, bh, lds, n, kSweepThreads)), dim3(kSweepThreads), lds,
                       st, a, wh,
                       make_queue(P, n, 1, P.nchunk > 0 ? -1 : 3), P.t.bwd_items);
  }
  if (nlow > 0) {
    SweepArgs wl = w;
    wl.status_mode = -1;
    wl.lev_lo = 0;
    wl.lev_hi = lw;
    const int n = nwi * nsys;
    Prof pr(P, st, KC_BWD_SWEEP, fb_low, 0.0);
    hipLaunchKernelGGL((k_bwd_sweep_waves<R>), dim3(resident_grid(P, bw, wlds, (n + 3) / 4)), dim3(kThreads), wlds,
                       st, a, wl, make_queue(P, n, 1, nhigh > 0 ? -1 : 3), P.t.wave_seq, P.t.wave_item_ptr);
  }
}

template <typename R>
hipError_t solve_impl(Plan& P, int mode, const double2* rhs, double2* x_out, int nrhs, int max_ir,
                      double tol, hipStream_t st, const SolveWork* work) {
  const KArgs a = make_args(P);
  SolveWork wk;
  if (work) {
    wk = *work;
  } else {
    wk.y = P.y;
    wk.wv = P.wv;
    wk.zv = P.zv;
    wk.pv = P.pv;
    wk.res = P.res;
    wk.partial = P.partial;
  }
  const int ncols = P.desc.nsys * nrhs;
  double2* xdst = mode == 0 ? x_out : P.xw;
  const int scale = mode == 0 ? 1 : 0;
  const int* flag = &P.status->ir_flag;
  if (max_ir <= 0) {
    // no refinement: the forward sweep records the solve's status itself
    sweep<R>(P, wk, a, rhs, xdst, nrhs, scale, 0, nullptr, st, mode);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_ir_begin, dim3(1), dim3(1), 0, st, P.status);
  sweep<R>(P, wk, a, rhs, xdst, nrhs, scale, 0, nullptr, st);
  ResArgs ra;
  ra.rhs = rhs;
  ra.x = xdst;
  ra.res = wk.res;
  ra.partial = wk.partial;
  ra.flag = flag;
  ra.tol = tol;
  ra.nrhs = nrhs;
  ra.scale_rhs = scale;
  // x, b, r (complex128) and eps per cell and column
  const double rbytes = (double)P.an.N * ncols * (16.0 * 3 + 8.0);
  for (int it = 1; it <= max_ir; ++it) {
    ra.step = it - 1;
    ra.last = 0;
    {
      Prof pr(P, st, KC_RESIDUAL, rbytes, 0.0);
      hipLaunchKernelGGL(k_residual, dim3(P.res_blocks, ncols), dim3(kThreads), 0, st, a, ra);
      hipLaunchKernelGGL(k_residual_norm, dim3(1), dim3(kThreads), 0, st, a, ra, P.res_blocks, ncols);
    }
    sweep<R>(P, wk, a, wk.res, xdst, nrhs, 0, 1, flag, st);
  }
  if (max_ir > 0) {
    ra.step = max_ir;
    ra.last = 1;
    Prof pr(P, st, KC_RESIDUAL, rbytes, 0.0);
    hipLaunchKernelGGL(k_residual, dim3(P.res_blocks, ncols), dim3(kThreads), 0, st, a, ra);
    hipLaunchKernelGGL(k_residual_norm, dim3(1), dim3(kThreads), 0, st, a, ra, P.res_blocks, ncols);
  }
  hipLaunchKernelGGL(k_ir_end, dim3(1), dim3(1), 0, st, P.status, mode, 1);
  return hipGetLastError();
}

template <typename R>
hipError_t set_lds_limits(int limit) {
  hipError_t e = hipSuccess;
  const void* fns[] = {(const void*)k_front_small<R>,     (const void*)k_wave_fronts<R, 8, 1>,
                       (const void*)k_wave_fronts<R, 16, 1>, (const void*)k_wave_fronts<R, 24, 1>,
                       (const void*)k_wave_fronts<R, 40, 1>, (const void*)k_wave_fronts<R, 8, 2>,
                       (const void*)k_wave_fronts<R, 16, 2>, (const void*)k_large_tiles<R>,
                       (const void*)k_fwd_sweep<R>,   (const void*)k_bwd_sweep<R>,
                       (const void*)k_fwd_sweep_waves<R>, (const void*)k_bwd_sweep_waves<R>};
  for (const void* fn : fns) {
    hipFuncAttributes fa;
    hipError_t r = hipFuncGetAttributes(&fa, fn);
    const int dyn = limit - (r == hipSuccess ? (int)fa.sharedSizeBytes : 1024);
    if (r == hipSuccess) r = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    if (r != hipSuccess && e == hipSuccess) e = r;
  }
  return e;
}

}  // namespace

hipError_t configure_kernels(Plan& P, int lds_limit) {
  return P.is_c64 ? set_lds_limits<float>(lds_limit) : set_lds_limits<double>(lds_limit);
}

size_t solve_lds_bytes(const Plan& P, int nrhs) { return std::max(sweep_lds(P, nrhs), sweep_wave_lds(P, nrhs)); }

int solve_rhs_group(const Plan& P, int nrhs) { return sweep_group(P, nrhs); }

hipError_t launch_refactor(Plan& P, const double* eps, int64_t eps_stride, hipStream_t st) {
  return P.is_c64 ? refactor_impl<float>(P, eps, eps_stride, st)
                  : refactor_impl<double>(P, eps, eps_stride, st);
}

hipError_t launch_solve(Plan& P, int mode, const double2* rhs, double2* x_out, int32_t nrhs,
                        int32_t max_ir, double tol, hipStream_t st, const SolveWork* work) {
  return P.is_c64 ? solve_impl<float>(P, mode, rhs, x_out, nrhs, max_ir, tol, st, work)
                  : solve_impl<double>(P, mode, rhs, x_out, nrhs, max_ir, tol, st, work);
}

hipError_t launch_gradient(Plan& P, const double2* x, const double2* lam_sym, int32_t nrhs,
                           double2* lam_out, double* grad, int32_t flags, hipStream_t st) {
  const KArgs a = make_args(P);
  const int acc = (flags & FDFD_GRAD_ACCUMULATE) ? 1 : 0;
  Prof pr(P, st, KC_GRADIENT, (double)P.an.N * P.desc.nsys * (nrhs * 32.0 + (lam_out ? nrhs * 16.0 : 0.0) + 8.0),
          0.0);
  if (flags & FDFD_GRAD_SUM_SYSTEMS)
    hipLaunchKernelGGL(k_gradient_sum, dim3(grid1d(P.an.N, 1024)), dim3(kThreads), 0, st, a, x, lam_sym,
                       nrhs, lam_out, grad, acc);
  else
    hipLaunchKernelGGL(k_gradient, dim3(grid1d(P.an.N, 1024), P.desc.nsys), dim3(kThreads), 0, st, a, x,
                       lam_sym, nrhs, lam_out, grad, acc);
  return hipGetLastError();
}


}  // namespace fdfd
