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
template <typename C> __device__ __forceinline__ C cinv(C d) {
  const auto s = d.x * d.x + d.y * d.y;
  C r;
  r.x = d.x / s;
  r.y = -d.y / s;
  return r;
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
  const int32_t *gmap, *nbr_row, *perm, *iperm, *mslot, *parent;
  const int64_t *fac_off, *upd_off, *gmap_ptr;
  int32_t nx, ny, N, nsys;
  int64_t fac_total, upd_total, sum_u;
  const double2* pml;
  const double* eps;
  const double* omega;
  void* fac;
  void* upd;
  void* mscr;
  DevStatus* st;
  double tau;
  int32_t nb, nmslot, nfronts;
};

// ---------------------------------------------------------------------------
// Operator coefficients of S*A (S = diag(sx_c sy_c)) at one cell.
// ---------------------------------------------------------------------------
struct Stencil {
  double2 diag, c[4];  // couplings to x-1, x+1, y-1, y+1
};

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
  const double e = a.eps[(int64_t)s * a.N + n];
  const double2 sc = dmul(sxc, syc);
  double2 d = make_double2(w * w * e * sc.x, w * w * e * sc.y);
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
template <typename C>
__device__ __forceinline__ C front_entry(const KArgs& a, int s, int f, int p, int m, int r, int c) {
  C val = czero<C>();
  if (c < p) {
    const int q = a.pbeg[f] + c;
    if (r == c) {
      val = from_d2<C>(stencil_at(a, s, a.perm[q]).diag);
    } else {
      const int32_t* nr = a.nbr_row + 4 * (int64_t)q;
      for (int d = 0; d < 4; ++d)
        if (nr[d] == r) val = from_d2<C>(stencil_at(a, s, a.perm[q]).c[d]);
    }
  }
  const int cb = a.child_ptr[f], ce = a.child_ptr[f + 1];
  const int32_t* g = a.gmap + a.gmap_ptr[f];
  const C* U = (const C*)a.upd + (int64_t)s * a.upd_total;
  for (int k = cb; k < ce; ++k, g += m) {
    const int gr = g[r];
    if (gr < 0) continue;
    const int gc = g[c];
    if (gc < 0) continue;
    const int ch = a.child_list[k];
    val = cadd(val, U[a.upd_off[ch] + (int64_t)gc * a.nupd[ch] + gr]);
  }
  return val;
}

// Static pivot perturbation: |d| < thr becomes d (1 + thr/|d|) (thr if d = 0).
template <typename C>
__device__ __forceinline__ C fix_pivot(C d, double thr, double anorm, int& npert, double& minr,
                                       int& nonfin) {
  const double ad = hypot((double)d.x, (double)d.y);
  if (!(ad <= DBL_MAX)) nonfin = 1;
  const double ratio = anorm > 0 ? ad / anorm : ad;
  minr = fmin(minr, ratio);
  if (ad < thr) {
    ++npert;
    if (ad == 0.0) {
      d.x = (decltype(d.x))thr;
      d.y = 0;
    } else {
      const double g = 1.0 + thr / ad;
      d.x = (decltype(d.x))(d.x * g);
      d.y = (decltype(d.y))(d.y * g);
    }
  }
  return d;
}

__device__ __forceinline__ void record_pivots(DevStatus* st, int npert, double minr, int nonfin) {
  if (npert) atomicAdd(&st->n_perturbed, npert);
  if (nonfin) atomicExch(&st->nonfinite, 1);
  if (minr < INFINITY)
    atomicMin(&st->min_ratio_bits, (unsigned long long)__double_as_longlong(minr));
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
  int32_t* counter;  // [0] next item, [1] workgroups that have left
  int32_t* done;     // [nsys][nfronts] epoch of the last completion
  DevStatus* st;
  int32_t epoch, ntasks, wait;
};

__device__ __forceinline__ int claim(const Queue& q, int* sh) {
  __syncthreads();
  if (threadIdx.x == 0) *sh = atomicAdd(&q.counter[0], 1);
  __syncthreads();
  return *sh;
}

__device__ __forceinline__ void leave(const Queue& q) {
  if (threadIdx.x == 0) {
    __threadfence();
    const int n = atomicAdd(&q.counter[1], 1);
    if (n == (int)(gridDim.x * gridDim.y * gridDim.z) - 1) {
      q.counter[0] = 0;
      q.counter[1] = 0;
    }
  }
}

// Polls with relaxed agent-scope loads (they read past the non-coherent
// caches without invalidating them); the caller issues one acquire fence once
// every awaited flag is seen.
__device__ __forceinline__ void wait_flag(const Queue& q, const int32_t* p) {
  int it = 0;
  while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != q.epoch) {
    if (++it > kSpinLimit) {
      atomicExch(&q.st->spin_timeout, 1);
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

__device__ __forceinline__ void wait_children(const Queue& q, const KArgs& a, int s, int f) {
  if (threadIdx.x == 0) {
    for (int k = a.child_ptr[f]; k < a.child_ptr[f + 1]; ++k)
      wait_flag(q, q.done + (int64_t)s * a.nfronts + a.child_list[k]);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

__device__ __forceinline__ void wait_parent(const Queue& q, const KArgs& a, int s, int f) {
  if (threadIdx.x == 0 && a.parent[f] >= 0) {
    wait_flag(q, q.done + (int64_t)s * a.nfronts + a.parent[f]);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

__device__ __forceinline__ void publish(const Queue& q, int64_t idx) {
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(q.done + idx, q.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Small fronts: one workgroup per (front, system), whole panel in LDS.
// Assembly, partial LDL^T of the pivot columns, Schur update of the u x u
// block straight into the front's update slot, panel write-back.
// ---------------------------------------------------------------------------
template <typename R>
__device__ void small_front(const KArgs& a, int s, int f, unsigned char* smem_raw) {
  typedef typename Cx<R>::T C;
  C* F = reinterpret_cast<C*>(smem_raw);
  const int p = a.npiv[f], u = a.nupd[f], m = p + u;
  C* dd = F + (int64_t)m * p;
  C* invd = dd + p;

  for (int idx = threadIdx.x; idx < m * p; idx += kThreads) {
    const int c = idx / m, r = idx - c * m;
    F[idx] = (r >= c) ? front_entry<C>(a, s, f, p, m, r, c) : czero<C>();
  }
  __syncthreads();

  const double anorm = anorm_of(a, s);
  const double thr = a.tau * anorm;
  int npert = 0, nonfin = 0;
  double minr = INFINITY;
  for (int k = 0; k < p; ++k) {
    // every thread derives the same (possibly perturbed) pivot
    const C d = fix_pivot(F[k * m + k], thr, anorm, npert, minr, nonfin);
    const C inv = cinv(d);
    if (threadIdx.x == 0) {
      dd[k] = d;
      invd[k] = inv;
    }
    const int Rn = m - k - 1, Cn = p - k - 1;
    const C* colk = F + k * m;
    for (int idx = threadIdx.x; idx < Rn * Cn; idx += kThreads) {
      const int jc = idx / Rn, ir = idx - jc * Rn;
      const int i = k + 1 + ir, j = k + 1 + jc;
      if (i >= j) F[j * m + i] = cfms(F[j * m + i], colk[i], cmul(colk[j], inv));
    }
    __syncthreads();
  }

  // Schur complement: U = F22 - W D^-1 W^T with W the unscaled columns.
  C* U = (C*)a.upd + (int64_t)s * a.upd_total + a.upd_off[f];
  for (int idx = threadIdx.x; idx < u * u; idx += kThreads) {
    const int jj = idx / u, ii = idx - jj * u;
    if (ii < jj) continue;
    C acc = front_entry<C>(a, s, f, p, m, p + ii, p + jj);
    for (int k = 0; k < p; ++k) acc = cfms(acc, F[k * m + p + ii], cmul(F[k * m + p + jj], invd[k]));
    U[(int64_t)jj * u + ii] = acc;
  }
  // Panel: unit-lower L with D on the diagonal.
  C* L = (C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  for (int idx = threadIdx.x; idx < m * p; idx += kThreads) {
    const int c = idx / m, r = idx - c * m;
    C v = czero<C>();
    if (r > c) v = cmul(F[idx], invd[c]);
    else if (r == c) v = dd[c];
    L[idx] = v;
  }
  if (threadIdx.x == 0) record_pivots(a.st, npert, minr, nonfin);
}

// Persistent launch over fronts order[0 .. ntasks/nsys): with q.wait set, a
// front first waits for its children (claimed earlier in the same launch).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_front_small(KArgs a, Queue q, const int32_t* order) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int sh;
  for (;;) {
    const int t = claim(q, &sh);
    if (t >= q.ntasks) break;
    const int f = order[t / a.nsys], s = t % a.nsys;
    if (q.wait) wait_children(q, a, s, f);
    small_front<R>(a, s, f, smem_raw);
    publish(q, s * a.nfronts + f);
  }
  leave(q);
}

// ---------------------------------------------------------------------------
// Large fronts: assembly into the panel / update slot, then per block column
// of width nb: diagonal-block factorisation (+ inverse of its unit-lower L11),
// panel solve as a product with that inverse, trailing update of every later
// column (pivot columns and the update block) with K = nb.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kThreads) void k_assemble_large(KArgs a, const int32_t* tasks) {
  typedef typename Cx<R>::T C;
  const int s = blockIdx.y;
  const int32_t* t = tasks + 3 * blockIdx.x;
  const int f = t[0], c0 = t[1], c1 = t[2];
  const int p = a.npiv[f], u = a.nupd[f], m = p + u;
  C* L = (C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  C* U = (C*)a.upd + (int64_t)s * a.upd_total + a.upd_off[f];
  for (int c = c0; c < c1; ++c) {
    if (c < p) {
      for (int r = threadIdx.x; r < m; r += kThreads)
        L[(int64_t)c * m + r] = (r >= c) ? front_entry<C>(a, s, f, p, m, r, c) : czero<C>();
    } else {
      for (int r = c + threadIdx.x; r < m; r += kThreads)
        U[(int64_t)(c - p) * u + (r - p)] = front_entry<C>(a, s, f, p, m, r, c);
    }
  }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_diag_large(KArgs a, const int32_t* fronts, int kb) {
  typedef typename Cx<R>::T C;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int NB = a.nb;
  C* B = reinterpret_cast<C*>(smem_raw);  // NB x NB, column major
  C* dd = B + NB * NB;
  C* invd = dd + NB;
  const int s = blockIdx.y;
  const int f = fronts[blockIdx.x];
  const int p = a.npiv[f], m = p + a.nupd[f];
  const int nb = min(NB, p - kb);
  C* L = (C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f] + (int64_t)kb * m + kb;
  for (int idx = threadIdx.x; idx < nb * nb; idx += kThreads) {
    const int c = idx / nb, r = idx - c * nb;
    B[c * NB + r] = (r >= c) ? L[(int64_t)c * m + r] : czero<C>();
  }
  __syncthreads();
  const double anorm = anorm_of(a, s);
  const double thr = a.tau * anorm;
  int npert = 0, nonfin = 0;
  double minr = INFINITY;
  for (int k = 0; k < nb; ++k) {
    const C d = fix_pivot(B[k * NB + k], thr, anorm, npert, minr, nonfin);
    const C inv = cinv(d);
    if (threadIdx.x == 0) {
      dd[k] = d;
      invd[k] = inv;
    }
    const int Rn = nb - k - 1;
    for (int idx = threadIdx.x; idx < Rn * Rn; idx += kThreads) {
      const int jc = idx / Rn, ir = idx - jc * Rn;
      const int i = k + 1 + ir, j = k + 1 + jc;
      if (i >= j) B[j * NB + i] = cfms(B[j * NB + i], B[k * NB + i], cmul(B[k * NB + j], inv));
    }
    __syncthreads();
  }
  // scale to unit-lower L11 and write back with D on the diagonal
  for (int idx = threadIdx.x; idx < nb * nb; idx += kThreads) {
    const int c = idx / nb, r = idx - c * nb;
    if (r > c) B[c * NB + r] = cmul(B[c * NB + r], invd[c]);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < nb * nb; idx += kThreads) {
    const int c = idx / nb, r = idx - c * nb;
    if (r > c) L[(int64_t)c * m + r] = B[c * NB + r];
    else if (r == c) L[(int64_t)c * m + r] = dd[c];
  }
  // X = L11^-1 (unit lower) in LDS by row elimination: X = I, then for every k
  // rows i > k take X[i][:] -= L[i][k] X[k][:] (only columns <= k are nonzero).
  C* Xl = invd + NB;  // NB x NB, column major
  for (int idx = threadIdx.x; idx < nb * nb; idx += kThreads) {
    const int c = idx / nb, r = idx - c * nb;
    C v = czero<C>();
    if (r == c) v.x = 1;
    Xl[c * NB + r] = v;
  }
  __syncthreads();
  for (int k = 0; k < nb - 1; ++k) {
    const int Rn = nb - k - 1, Cn = k + 1;
    for (int idx = threadIdx.x; idx < Rn * Cn; idx += kThreads) {
      const int j = idx / Rn, i = k + 1 + (idx - j * Rn);
      Xl[j * NB + i] = cfms(Xl[j * NB + i], B[k * NB + i], Xl[j * NB + k]);
    }
    __syncthreads();
  }
  C* X = (C*)a.mscr + ((int64_t)s * a.nmslot + a.mslot[f]) * NB * NB;
  for (int idx = threadIdx.x; idx < nb * NB; idx += kThreads) X[idx] = Xl[idx];
  if (threadIdx.x == 0) record_pivots(a.st, npert, minr, nonfin);
}

// Rows [r0, r0+64) below the diagonal block: L21 = F21 L11^-T D^-1.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_trsm_large(KArgs a, const int32_t* tasks, int kb) {
  typedef typename Cx<R>::T C;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int TR = 64;
  const int NB = a.nb;
  C* Xs = reinterpret_cast<C*>(smem_raw);  // NB x NB, Xs[j*NB + k] = (L11^-1)[k][j]... see below
  C* Ft = Xs + NB * NB;                   // TR x NB, row major
  C* invd = Ft + TR * NB;
  const int s = blockIdx.y;
  const int f = tasks[2 * blockIdx.x], r0 = tasks[2 * blockIdx.x + 1];
  const int p = a.npiv[f], m = p + a.nupd[f];
  const int nb = min(NB, p - kb);
  const int nr = min(TR, m - r0);
  C* L = (C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  const C* X = (const C*)a.mscr + ((int64_t)s * a.nmslot + a.mslot[f]) * NB * NB;
  for (int idx = threadIdx.x; idx < nb * NB; idx += kThreads) Xs[idx] = X[idx];
  for (int idx = threadIdx.x; idx < nr * nb; idx += kThreads) {
    const int k = idx / nr, r = idx - k * nr;
    Ft[r * NB + k] = L[(int64_t)(kb + k) * m + r0 + r];
  }
  for (int k = threadIdx.x; k < nb; k += kThreads)
    invd[k] = cinv(L[(int64_t)(kb + k) * m + kb + k]);
  __syncthreads();
  // out[r][j] = (sum_{k<=j} F[r][k] (L11^-1)[j][k]) / d_j ; (L11^-1)[j][k] = X[k*NB + j]
  for (int idx = threadIdx.x; idx < nr * nb; idx += kThreads) {
    const int j = idx / nr, r = idx - j * nr;
    C acc = czero<C>();
    for (int k = 0; k <= j; ++k) acc = cadd(acc, cmul(Ft[r * NB + k], Xs[k * NB + j]));
    L[(int64_t)(kb + j) * m + r0 + r] = cmul(acc, invd[j]);
  }
}

// Trailing update of a 64 x 64 lower tile: C[r][c] -= sum_k L[r][kb+k] d_k L[c][kb+k].
template <typename R>
__global__ __launch_bounds__(kThreads) void k_update_large(KArgs a, const int32_t* tasks, int kb) {
  typedef typename Cx<R>::T C;
  constexpr int TS = 64;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int NB = a.nb;
  C* As = reinterpret_cast<C*>(smem_raw);  // NB x TS (k major): As[k*TS + r]
  C* Bs = As + NB * TS;                   // NB x TS, premultiplied by d_k
  const int s = blockIdx.y;
  const int32_t* t = tasks + 3 * blockIdx.x;
  const int f = t[0], r0 = t[1], c0 = t[2];
  const int p = a.npiv[f], u = a.nupd[f], m = p + u;
  const int nb = min(NB, p - kb);
  const int nr = min(TS, m - r0), nc = min(TS, m - c0);
  C* L = (C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  C* U = (C*)a.upd + (int64_t)s * a.upd_total + a.upd_off[f];
  for (int idx = threadIdx.x; idx < nb * TS; idx += kThreads) {
    const int k = idx / TS, r = idx - k * TS;
    const C* col = L + (int64_t)(kb + k) * m;
    As[idx] = r < nr ? col[r0 + r] : czero<C>();
    Bs[idx] = r < nc ? cmul(col[c0 + r], col[kb + k]) : czero<C>();
  }
  __syncthreads();
  // 4 x 4 outputs per thread: rows tr*4.., cols tc*4.. with a 16 x 16 thread grid
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
  C acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = czero<C>();
  for (int k = 0; k < nb; ++k) {
    C av[4], bv[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) av[x] = As[k * TS + tr + 16 * x];
#pragma unroll
    for (int y = 0; y < 4; ++y) bv[y] = Bs[k * TS + tc + 16 * y];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = cadd(acc[x][y], cmul(av[x], bv[y]));
  }
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int r = r0 + tr + 16 * x;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int c = c0 + tc + 16 * y;
      if (r >= m || c >= m || r < c) continue;
      C* dst = (c < p) ? (L + (int64_t)c * m + r) : (U + (int64_t)(c - p) * u + (r - p));
      *dst = csub(*dst, acc[x][y]);
    }
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

template <typename C> __device__ __forceinline__ C shfl_c(C v, int lane) {
  v.x = __shfl(v.x, lane);
  v.y = __shfl(v.y, lane);
  return v;
}

struct SweepArgs {
  const double2* src;  // forward: right-hand sides, grid order
  double2* out;        // backward: solution, grid order
  void* y;
  void* wv;
  const int* flag;     // refinement converged: skip the launch
  int32_t nrhs, scale_src, accumulate;
};

// One front of the forward sweep: V = [rhs_p; 0] + children's update vectors,
// V <- L^-1 V over the pivot columns in BW-wide blocks (one wave solves the
// block triangle staged in LDS, all threads apply the rows below it), then
// y_p = D^-1 V_p and the front's update vector is V_u.
template <typename R, int BW>
__device__ void fwd_front(const KArgs& a, const SweepArgs& w, int s, int f, unsigned char* smem) {
  typedef typename Cx<R>::T C;
  const int p = a.npiv[f], u = a.nupd[f], m = p + u, pb = a.pbeg[f];
  const int nrhs = w.nrhs;
  C* T = reinterpret_cast<C*>(smem);  // BW x (BW+1)
  C* V = T + BW * (BW + 1);          // nrhs x m
  const C* L = (const C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  C* Y = (C*)w.y + (int64_t)s * nrhs * a.N;
  C* W = (C*)w.wv + (int64_t)s * nrhs * a.sum_u;
  const double2* B = w.src + (int64_t)s * nrhs * a.N;
  const int cb = a.child_ptr[f], ce = a.child_ptr[f + 1];
  const int32_t* g = a.gmap + a.gmap_ptr[f];
  for (int idx = threadIdx.x; idx < m * nrhs; idx += kThreads) {
    const int col = idx / m, r = idx - col * m;
    C v = czero<C>();
    if (r < p) {
      const int n = a.perm[pb + r];
      double2 bv = B[(int64_t)col * a.N + n];
      if (w.scale_src) bv = dmul(bv, sym_scale(a, s, n));
      v = from_d2<C>(bv);
    }
    for (int k = cb; k < ce; ++k) {
      const int gr = g[(k - cb) * m + r];
      if (gr >= 0) v = cadd(v, W[(int64_t)col * a.sum_u + a.upd_ptr[a.child_list[k]] + gr]);
    }
    V[col * m + r] = v;
  }
  __syncthreads();
  for (int k0 = 0; k0 < p; k0 += BW) {
    const int kn = min(BW, p - k0), k1 = k0 + kn;
    for (int idx = threadIdx.x; idx < kn * kn; idx += kThreads) {
      const int k = idx / kn, l = idx - k * kn;
      T[k * (BW + 1) + l] = L[(int64_t)(k0 + k) * m + k0 + l];
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      for (int col = 0; col < nrhs; ++col) {
        C v = lane < kn ? V[col * m + k0 + lane] : czero<C>();
        for (int k = 0; k < kn; ++k) {
          const C vk = shfl_c(v, k);
          if (lane > k && lane < kn) v = cfms(v, T[k * (BW + 1) + lane], vk);
        }
        if (lane < kn) V[col * m + k0 + lane] = v;
      }
    }
    __syncthreads();
    for (int i = k1 + threadIdx.x; i < m; i += kThreads) {
      for (int col = 0; col < nrhs; ++col) {
        C acc = V[col * m + i];
        for (int k = k0; k < k1; ++k) acc = cfms(acc, L[(int64_t)k * m + i], V[col * m + k]);
        V[col * m + i] = acc;
      }
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < m * nrhs; idx += kThreads) {
    const int col = idx / m, r = idx - col * m;
    if (r < p) Y[(int64_t)col * a.N + pb + r] = cmul(V[col * m + r], cinv(L[(int64_t)r * m + r]));
    else W[(int64_t)col * a.sum_u + a.upd_ptr[f] + (r - p)] = V[col * m + r];
  }
}

// One front of the backward sweep: X = [z_p; x(update rows)], then for BW-wide
// blocks from the last: X_blk -= L(rows below, blk)^T X(below) (one wave per
// column, lanes over rows) and one wave solves the transposed block triangle
// staged in LDS.  x_p goes to y and to the grid-order output.
template <typename R, int BW>
__device__ void bwd_front(const KArgs& a, const SweepArgs& w, int s, int f, unsigned char* smem) {
  typedef typename Cx<R>::T C;
  const int p = a.npiv[f], u = a.nupd[f], m = p + u, pb = a.pbeg[f];
  const int nrhs = w.nrhs;
  C* T = reinterpret_cast<C*>(smem);
  C* X = T + BW * (BW + 1);
  const C* L = (const C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  C* Y = (C*)w.y + (int64_t)s * nrhs * a.N;
  const int32_t* ui = a.upd_idx + a.upd_ptr[f];
  for (int idx = threadIdx.x; idx < m * nrhs; idx += kThreads) {
    const int col = idx / m, r = idx - col * m;
    X[col * m + r] = Y[(int64_t)col * a.N + (r < p ? pb + r : ui[r - p])];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = kThreads / 64;
  int k1 = p;
  while (k1 > 0) {
    const int k0 = ((k1 - 1) / BW) * BW;
    const int kn = k1 - k0;
    for (int k = k0 + wave; k < k1; k += NW) {
      for (int col = 0; col < nrhs; ++col) {
        C acc = czero<C>();
        for (int i = k1 + lane; i < m; i += 64) acc = cadd(acc, cmul(L[(int64_t)k * m + i], X[col * m + i]));
        for (int o = 32; o > 0; o >>= 1) {
          acc.x += __shfl_xor(acc.x, o);
          acc.y += __shfl_xor(acc.y, o);
        }
        if (lane == 0) X[col * m + k] = csub(X[col * m + k], acc);
      }
    }
    for (int idx = threadIdx.x; idx < kn * kn; idx += kThreads) {
      const int l = idx / kn, k = idx - l * kn;
      T[l * (BW + 1) + k] = L[(int64_t)(k0 + l) * m + k0 + k];
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      for (int col = 0; col < nrhs; ++col) {
        C v = lane < kn ? X[col * m + k0 + lane] : czero<C>();
        for (int k = kn - 1; k > 0; --k) {
          const C xk = shfl_c(v, k);
          if (lane < k) v = cfms(v, T[lane * (BW + 1) + k], xk);
        }
        if (lane < kn) X[col * m + k0 + lane] = v;
      }
    }
    __syncthreads();
    k1 = k0;
  }
  double2* O = w.out + (int64_t)s * nrhs * a.N;
  for (int idx = threadIdx.x; idx < p * nrhs; idx += kThreads) {
    const int col = idx / p, r = idx - col * p;
    const C x = X[col * m + r];
    Y[(int64_t)col * a.N + pb + r] = x;
    double2* o = O + (int64_t)col * a.N + a.perm[pb + r];
    const double2 xv = to_d2(x);
    *o = w.accumulate ? dadd(*o, xv) : xv;
  }
}

// Forward sweep: items in level order (leaves first), each waits for its children.
template <typename R, int BW>
__global__ __launch_bounds__(kThreads) void k_fwd_sweep(KArgs a, SweepArgs w, Queue q, const int32_t* order) {
  if (done(w.flag)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int sh;
  for (;;) {
    const int t = claim(q, &sh);
    if (t >= q.ntasks) break;
    const int f = order[t / a.nsys], s = t % a.nsys;
    if (q.wait) wait_children(q, a, s, f);
    fwd_front<R, BW>(a, w, s, f, smem_raw);
    publish(q, (int64_t)s * a.nfronts + f);
  }
  leave(q);
}

// Backward sweep: items in reverse level order (root first), each waits for its parent.
template <typename R, int BW>
__global__ __launch_bounds__(kThreads) void k_bwd_sweep(KArgs a, SweepArgs w, Queue q, const int32_t* order) {
  if (done(w.flag)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int sh;
  const int F = a.nfronts;
  for (;;) {
    const int t = claim(q, &sh);
    if (t >= q.ntasks) break;
    const int f = order[q.ntasks / a.nsys - 1 - t / a.nsys], s = t % a.nsys;
    if (q.wait) wait_parent(q, a, s, f);
    bwd_front<R, BW>(a, w, s, f, smem_raw);
    publish(q, (int64_t)s * F + f);
  }
  leave(q);
}

// ---------------------------------------------------------------------------
// FP64 refinement: r = rhs_sym - (SA) x with per-block partial norms; the last
// workgroup to finish reduces them in a fixed order, records the relative
// residual and raises the converged flag (or the failure bits).
// ---------------------------------------------------------------------------
struct ResArgs {
  const double2* rhs;
  const double2* x;
  double2* res;
  double* partial;
  int32_t* counter;
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
  __shared__ int last_block;
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
  const int nblk = gridDim.x, ncols = gridDim.y;
  if (threadIdx.x == 0) {
    double* pp = ra.partial + ((int64_t)col * nblk + blockIdx.x) * 2;
    pp[0] = red[0][0];
    pp[1] = red[1][0];
    __threadfence();
    last_block = atomicAdd(ra.counter, 1) == nblk * ncols - 1;
  }
  __syncthreads();
  if (!last_block) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double wmax = 0.0;
  int nf = 0;
  for (int c = threadIdx.x; c < ncols; c += kThreads) {
    double r2 = 0.0, b2 = 0.0;
    for (int b = 0; b < nblk; ++b) {
      r2 += ra.partial[((int64_t)c * nblk + b) * 2];
      b2 += ra.partial[((int64_t)c * nblk + b) * 2 + 1];
    }
    const double rel = b2 > 0 ? sqrt(r2 / b2) : sqrt(r2);
    if (!(rel <= DBL_MAX)) nf = 1;
    wmax = fmax(wmax, rel);
  }
  red[0][threadIdx.x] = wmax;
  red[1][threadIdx.x] = nf;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = 0.0;
    int anybad = 0;
    for (int t = 0; t < kThreads; ++t) {
      mx = fmax(mx, red[0][t]);
      anybad |= red[1][t] != 0.0;
    }
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
    *ra.counter = 0;
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
__global__ __launch_bounds__(kThreads) void k_gradient(KArgs a, const double2* x, const double2* lsym,
                                                        int nrhs, double2* lam_out, double* grad,
                                                        int accumulate) {
  const int s = blockIdx.y;
  const double w = a.omega[s];
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
       n += (int64_t)gridDim.x * blockDim.x) {
    const double2 S = sym_scale(a, s, (int)n);
    double gsum = 0.0;
    for (int r = 0; r < nrhs; ++r) {
      const int64_t o = ((int64_t)s * nrhs + r) * a.N + n;
      const double2 lam = dmul(S, lsym[o]);
      if (lam_out) lam_out[o] = lam;
      const double2 xv = x[o];
      gsum += lam.x * xv.x - lam.y * xv.y;
    }
    const double gv = -2.0 * w * w * gsum;
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
    for (int s = 0; s < a.nsys; ++s) {
      const double w = a.omega[s];
      const double2 S = sym_scale(a, s, (int)n);
      double gsum = 0.0;
      for (int r = 0; r < nrhs; ++r) {
        const int64_t o = ((int64_t)s * nrhs + r) * a.N + n;
        const double2 lam = dmul(S, lsym[o]);
        if (lam_out) lam_out[o] = lam;
        const double2 xv = x[o];
        gsum += lam.x * xv.x - lam.y * xv.y;
      }
      tot += -2.0 * w * w * gsum;
    }
    grad[n] = accumulate ? grad[n] + tot : tot;
  }
}

__global__ void k_status_reset(DevStatus* st) {
  st->ir_flag = 0;
  st->ir_steps_solve = 0;
  st->ir_steps_adj = 0;
  st->rel_solve = -1.0;
  st->rel_adj = -1.0;
  st->ir_failed_solve = 0;
  st->ir_failed_adj = 0;
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
  a.mslot = P.t.mslot;
  a.parent = P.t.parent;
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
  a.mscr = P.mscr;
  a.st = P.status;
  // pivot threshold tau * ||SA||_max with tau = sqrt(unit roundoff)
  a.tau = P.is_c64 ? 2.44140625e-4 : 1.0536712127723509e-8;
  a.nb = P.nb_large;
  a.nmslot = P.nmslot;
  a.nfronts = P.an.nfronts;
  return a;
}

inline unsigned grid1d(int64_t n, int64_t cap = 2048) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

Queue make_queue(Plan& P, int ntasks, int wait) {
  Queue q;
  q.counter = P.counters;
  q.done = P.done;
  q.st = P.status;
  q.epoch = ++P.epoch;
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

template <typename R>
hipError_t refactor_impl(Plan& P, const double* eps, int64_t eps_stride, hipStream_t st) {
  const KArgs a = make_args(P);
  const int nsys = P.desc.nsys;
  const size_t cs = P.csize;
  const int NB = P.nb_large;
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
  const int32_t* tk = P.t.tasks;
  const size_t nl = P.levels.size();
  size_t l = 0;
  // the small levels at the bottom of the tree: one persistent launch
  if (P.small_prefix > 0) {
    const int nf = P.levels[P.small_prefix - 1].first + P.levels[P.small_prefix - 1].count;
    const Queue q = make_queue(P, nf * nsys, 1);
    double fl = 0.0;
    for (int k = 0; k < nf; ++k) fl += P.front_flops[P.an.level_fronts[k]];
    Prof pr(P, st, KC_FRONT_SMALL, 0.0, fl * nsys);
    hipLaunchKernelGGL(k_front_small<R>, dim3(persistent_grid(P, P.small_lds_prefix, nf * nsys)),
                       dim3(kThreads), P.small_lds_prefix, st, a, q, lf);
    l = P.small_prefix;
  }
  for (; l < nl; ++l) {
    const LevelPlan& L = P.levels[l];
    if (L.small) {
      const Queue q = make_queue(P, L.count * nsys, 0);
      double fl = 0.0;
      for (int k = L.first; k < L.first + L.count; ++k) fl += P.front_flops[P.an.level_fronts[k]];
      Prof pr(P, st, KC_FRONT_SMALL, 0.0, fl * nsys);
      hipLaunchKernelGGL(k_front_small<R>, dim3(persistent_grid(P, L.small_lds, L.count * nsys)),
                         dim3(kThreads), L.small_lds, st, a, q, lf + L.first);
      continue;
    }
    {
      Prof pr(P, st, KC_ASSEMBLE_LARGE, L.asm_bytes * nsys, 0.0);
      hipLaunchKernelGGL(k_assemble_large<R>, dim3(L.nasm, nsys), dim3(kThreads), 0, st, a,
                         tk + L.asm_off);
    }
    for (const BlockStep& S : L.steps) {
      {
        Prof pr(P, st, KC_DIAG_LARGE, 0.0, S.diag_flops * nsys);
        hipLaunchKernelGGL(k_diag_large<R>, dim3(S.ndiag, nsys), dim3(kThreads),
                           (size_t)(2 * NB * NB + 2 * NB) * cs, st, a, tk + S.diag_off, S.kb);
      }
      if (S.ntrsm) {
        Prof pr(P, st, KC_TRSM_LARGE, 0.0, S.trsm_flops * nsys);
        hipLaunchKernelGGL(k_trsm_large<R>, dim3(S.ntrsm, nsys), dim3(kThreads),
                           (size_t)(NB * NB + 64 * NB + NB) * cs, st, a, tk + S.trsm_off, S.kb);
      }
      if (S.nupd) {
        Prof pr(P, st, KC_UPDATE_LARGE, 0.0, S.upd_flops * nsys);
        hipLaunchKernelGGL(k_update_large<R>, dim3(S.nupd, nsys), dim3(kThreads),
                           (size_t)(2 * NB * 64) * cs, st, a, tk + S.upd_off, S.kb);
      }
    }
  }
  return hipGetLastError();
}

template <typename R> constexpr int sweep_bw() { return sizeof(R) == 8 ? 32 : 64; }

size_t sweep_lds(const Plan& P, int nrhs, int bw) {
  return ((size_t)bw * (bw + 1) + (size_t)P.an.max_front * nrhs) * P.csize;
}

// One forward + backward sweep: dst (+)= (SA)^-1 (scale ? S : 1) src.
template <typename R>
void sweep(Plan& P, const KArgs& a, const double2* src, double2* dst, int nrhs, int scale_in,
           int accumulate, const int* flag, hipStream_t st) {
  constexpr int BW = sweep_bw<R>();
  const int nt = P.an.nfronts * P.desc.nsys;
  const size_t lds = sweep_lds(P, nrhs, BW);
  SweepArgs w;
  w.src = src;
  w.out = dst;
  w.y = P.y;
  w.wv = P.wv;
  w.flag = flag;
  w.nrhs = nrhs;
  w.scale_src = scale_in;
  w.accumulate = accumulate;
  const int32_t* lf = P.t.level_fronts;
  const int nsys = P.desc.nsys;
  // algorithmic bytes: the lower-trapezoid factor once, the input vector read
  // in one precision and the output written in another
  const double vec_bytes = (double)P.an.N * nrhs * nsys * (16.0 + (double)P.csize);
  if (P.sweep_levels) {
    // one launch per tree level: kernel boundaries order the levels
    for (const LevelPlan& L : P.levels) {
      const int n = L.count * nsys;
      Prof pr(P, st, KC_FWD_SWEEP, L.lbytes * nsys + vec_bytes * L.count / P.an.nfronts, 0.0);
      hipLaunchKernelGGL((k_fwd_sweep<R, BW>), dim3(persistent_grid(P, lds, n)), dim3(kThreads), lds, st, a, w,
                         make_queue(P, n, 0), lf + L.first);
    }
    for (size_t l = P.levels.size(); l-- > 0;) {
      const LevelPlan& L = P.levels[l];
      const int n = L.count * nsys;
      Prof pr(P, st, KC_BWD_SWEEP, L.lbytes * nsys + vec_bytes * L.count / P.an.nfronts, 0.0);
      hipLaunchKernelGGL((k_bwd_sweep<R, BW>), dim3(persistent_grid(P, lds, n)), dim3(kThreads), lds, st, a, w,
                         make_queue(P, n, 0), lf + L.first);
    }
    return;
  }
  const unsigned g = persistent_grid(P, lds, nt);
  const double fb = P.factor_lbytes * nsys + vec_bytes;
  {
    Prof pr(P, st, KC_FWD_SWEEP, fb, 0.0);
    hipLaunchKernelGGL((k_fwd_sweep<R, BW>), dim3(g), dim3(kThreads), lds, st, a, w, make_queue(P, nt, 1), lf);
  }
  {
    Prof pr(P, st, KC_BWD_SWEEP, fb, 0.0);
    hipLaunchKernelGGL((k_bwd_sweep<R, BW>), dim3(g), dim3(kThreads), lds, st, a, w, make_queue(P, nt, 1), lf);
  }
}

template <typename R>
hipError_t solve_impl(Plan& P, int mode, const double2* rhs, double2* x_out, int nrhs, int max_ir,
                      double tol, hipStream_t st) {
  const KArgs a = make_args(P);
  const int ncols = P.desc.nsys * nrhs;
  double2* xdst = mode == 0 ? x_out : P.xw;
  const int scale = mode == 0 ? 1 : 0;
  const int* flag = &P.status->ir_flag;
  hipLaunchKernelGGL(k_ir_begin, dim3(1), dim3(1), 0, st, P.status);
  sweep<R>(P, a, rhs, xdst, nrhs, scale, 0, nullptr, st);
  ResArgs ra;
  ra.rhs = rhs;
  ra.x = xdst;
  ra.res = P.res;
  ra.partial = P.partial;
  ra.counter = P.counters + 2;
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
    }
    sweep<R>(P, a, P.res, xdst, nrhs, 0, 1, flag, st);
  }
  if (max_ir > 0) {
    ra.step = max_ir;
    ra.last = 1;
    Prof pr(P, st, KC_RESIDUAL, rbytes, 0.0);
    hipLaunchKernelGGL(k_residual, dim3(P.res_blocks, ncols), dim3(kThreads), 0, st, a, ra);
  }
  hipLaunchKernelGGL(k_ir_end, dim3(1), dim3(1), 0, st, P.status, mode, max_ir > 0 ? 1 : 0);
  return hipGetLastError();
}

template <typename R>
hipError_t set_lds_limits(int limit) {
  constexpr int BW = sweep_bw<R>();
  hipError_t e = hipSuccess;
  const void* fns[] = {(const void*)k_front_small<R>, (const void*)k_diag_large<R>,
                       (const void*)k_trsm_large<R>, (const void*)k_update_large<R>,
                       (const void*)k_fwd_sweep<R, BW>, (const void*)k_bwd_sweep<R, BW>};
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

size_t solve_lds_bytes(const Plan& P, int nrhs) {
  return sweep_lds(P, nrhs, P.is_c64 ? sweep_bw<float>() : sweep_bw<double>());
}

hipError_t launch_refactor(Plan& P, const double* eps, int64_t eps_stride, hipStream_t st) {
  return P.is_c64 ? refactor_impl<float>(P, eps, eps_stride, st)
                  : refactor_impl<double>(P, eps, eps_stride, st);
}

hipError_t launch_solve(Plan& P, int mode, const double2* rhs, double2* x_out, int32_t nrhs,
                        int32_t max_ir, double tol, hipStream_t st) {
  return P.is_c64 ? solve_impl<float>(P, mode, rhs, x_out, nrhs, max_ir, tol, st)
                  : solve_impl<double>(P, mode, rhs, x_out, nrhs, max_ir, tol, st);
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

hipError_t launch_status_reset(Plan& P, hipStream_t st) {
  hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(1), 0, st, P.status);
  return hipGetLastError();
}

}  // namespace fdfd
